// CPU FP64 oracle for batched constant-pressure chemistry integration with the
// linearly implicit Rosenbrock solvers ROS4 (the default), ROS3, RODAS3, RODAS4,
// and the W-method ROS34PW2 with the Jacobian kept over several steps.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
// includes this file; only the tests, the smoke check and the CPU-baseline leg
// of the benchmark load it.  It shares no code with the HIP path: it has its
// own mechanism parser, its own thermochemistry, its own method tables.
//
// It is deliberately plain and slow: one cell at a time, textbook loops, no
// blocking or fusion; OpenMP runs independent cells on separate threads.
//
// What it computes, and where the paper defines it:
//   * state Phi = {T, V, n_1 .. n_{K-1}}, bath gas closed by the ideal-gas law
//     (Sec. 2.1, eqs. (state_vec) and (n_nsp));
//   * source terms f(Phi) (Sec. 2.1, eq. (dphidt)) with CHEMKIN-form rate laws:
//     Arrhenius, third body, Lindemann and Troe falloff, reverse rates through
//     equilibrium constants from NASA-7 Gibbs functions.  The paper delegates
//     these forms to its code generator; the oracle writes out the textbook
//     definitions;
//   * the Jacobian J_ij = df_i/dPhi_j (Sec. 2.1, eq. (jac)).  The oracle takes
//     the definition literally: forward-mode dual numbers differentiate f, one
//     column per pass (exact to rounding, no truncation error);
//   * the transformed Rosenbrock scheme (Sec. 2.3, eq. (ros) and the
//     u_i / a_ij / c_ij / m_j form that follows it), one LU per step, with the
//     coefficient sets of the solvers in Table T:solvers;
//   * adaptive step control from rtol/atol (Sec. 3.1), with the returned last
//     internal step reused as the next call's first step (Sec. 2.4.1);
//   * conversion (T, P, Y) <-> Phi through [C_i] = rho Y_i / W_i = n_i / V
//     (Sec. 2.4.2, eq. (conc_form1)), on a per-unit-mass basis.
//   * sensitivities of the final state to ln A_j (or to the initial state) along
//     the frozen accepted-step sequence, by forward-mode dual numbers through
//     every step (the tangent of the discrete map, exact to rounding).
//
// Readings where the paper is silent (rate-law forms, thermo, controller
// constants, error norm, failure policy) are the ones the library uses too;
// they are listed with the design notes.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>
#include <omp.h>

namespace {

const double RU = 8314.462618;     // J/(kmol K)
const double PATM = 101325.0;      // Pa
const double LN10 = 2.302585092994045684;

// ---------------------------------------------------------------- dual numbers
template <class T> struct Dual { T v, d; };

inline double val(double x) { return x; }
template <class T> inline double val(const Dual<T>& x) { return val(x.v); }

template <class T> Dual<T> operator+(Dual<T> a, Dual<T> b) { return {a.v + b.v, a.d + b.d}; }
template <class T> Dual<T> operator-(Dual<T> a, Dual<T> b) { return {a.v - b.v, a.d - b.d}; }
template <class T> Dual<T> operator-(Dual<T> a) { return {-a.v, -a.d}; }
template <class T> Dual<T> operator*(Dual<T> a, Dual<T> b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
template <class T> Dual<T> operator/(Dual<T> a, Dual<T> b) {
  T q = a.v / b.v;
  return {q, (a.d - q * b.d) / b.v};
}
template <class T> Dual<T> operator+(Dual<T> a, double b) { return {a.v + b, a.d}; }
template <class T> Dual<T> operator+(double b, Dual<T> a) { return {a.v + b, a.d}; }
template <class T> Dual<T> operator-(Dual<T> a, double b) { return {a.v - b, a.d}; }
template <class T> Dual<T> operator-(double b, Dual<T> a) { return {b - a.v, -a.d}; }
template <class T> Dual<T> operator*(Dual<T> a, double b) { return {a.v * b, a.d * b}; }
template <class T> Dual<T> operator*(double b, Dual<T> a) { return {a.v * b, a.d * b}; }
template <class T> Dual<T> operator/(Dual<T> a, double b) { return {a.v / b, a.d / b}; }
template <class T> Dual<T> operator/(double b, Dual<T> a) {
  T q = b / a.v;
  return {q, -q * a.d / a.v};
}
template <class T> Dual<T>& operator+=(Dual<T>& a, Dual<T> b) { a = a + b; return a; }
template <class T> Dual<T>& operator-=(Dual<T>& a, Dual<T> b) { a = a - b; return a; }
template <class T> Dual<T>& operator*=(Dual<T>& a, Dual<T> b) { a = a * b; return a; }
template <class T> Dual<T>& operator+=(Dual<T>& a, double b) { a.v += b; return a; }

inline double exp_(double x) { return std::exp(x); }
inline double log_(double x) { return std::log(x); }
inline double sqrt_(double x) { return std::sqrt(x); }
template <class T> Dual<T> exp_(Dual<T> a) { T e = exp_(a.v); return {e, e * a.d}; }
template <class T> Dual<T> log_(Dual<T> a) { return {log_(a.v), a.d / a.v}; }
template <class T> Dual<T> sqrt_(Dual<T> a) { T s = sqrt_(a.v); return {s, a.d / (2.0 * s)}; }

template <class S> struct Cst;
template <> struct Cst<double> { static double c(double x) { return x; } };
template <class T> struct Cst<Dual<T>> { static Dual<T> c(double x) { return {Cst<T>::c(x), Cst<T>::c(0.0)}; } };
template <class S> inline S C(double x) { return Cst<S>::c(x); }

// ---------------------------------------------------------------- mechanism
struct Rxn {
  char kind;                       // 'E', 'T', 'L', 'F'
  std::vector<int> ri, pi;         // reactant / product species
  std::vector<int> rn, pn;         // stoichiometric coefficients
  double lnA, b, theta;
  std::vector<int> ei;             // third-body efficiency overrides
  std::vector<double> ea;
  double lnA0 = 0, b0 = 0, theta0 = 0;
  double ta = 0, T3 = 0, T1 = 0, T2 = 0;
};

struct Mech {
  int E = 0, K = 0, Nr = 0;
  std::vector<std::string> names;
  std::vector<double> W;
  std::vector<int> comp;           // K x E
  std::vector<double> Tmid;
  std::vector<double> lo, hi;      // K x 7
  std::vector<Rxn> rx;
};

bool parse(const char* path, Mech& m) {
  std::ifstream f(path);
  if (!f) return false;
  std::string tok;
  int ver;
  if (!(f >> tok >> ver) || tok != "CHEMMECH" || ver != 1) return false;
  if (!(f >> tok >> m.E) || tok != "ELEMENTS") return false;
  for (int e = 0; e < m.E; ++e) f >> tok;
  if (!(f >> tok >> m.K) || tok != "SPECIES") return false;
  m.names.resize(m.K); m.W.resize(m.K); m.comp.resize(m.K * m.E); m.Tmid.resize(m.K);
  m.lo.resize(7 * m.K); m.hi.resize(7 * m.K);
  for (int k = 0; k < m.K; ++k) {
    f >> m.names[k] >> m.W[k];
    for (int e = 0; e < m.E; ++e) f >> m.comp[k * m.E + e];
    f >> m.Tmid[k];
    for (int i = 0; i < 7; ++i) f >> m.lo[7 * k + i];
    for (int i = 0; i < 7; ++i) f >> m.hi[7 * k + i];
  }
  if (!(f >> tok >> m.Nr) || tok != "REACTIONS") return false;
  m.rx.resize(m.Nr);
  for (int j = 0; j < m.Nr; ++j) {
    Rxn& r = m.rx[j];
    std::string kind;
    int n;
    f >> kind;
    r.kind = kind[0];
    f >> n; r.ri.resize(n); r.rn.resize(n);
    for (int i = 0; i < n; ++i) f >> r.ri[i] >> r.rn[i];
    f >> n; r.pi.resize(n); r.pn.resize(n);
    for (int i = 0; i < n; ++i) f >> r.pi[i] >> r.pn[i];
    f >> r.lnA >> r.b >> r.theta;
    f >> n; r.ei.resize(n); r.ea.resize(n);
    for (int i = 0; i < n; ++i) f >> r.ei[i] >> r.ea[i];
    if (r.kind == 'L' || r.kind == 'F') f >> r.lnA0 >> r.b0 >> r.theta0;
    if (r.kind == 'F') f >> r.ta >> r.T3 >> r.T1 >> r.T2;
  }
  return !f.fail();
}

// ---------------------------------------------------------------- thermo
// NASA 7-coefficient polynomials, molar: cp/R, h/(RT), s/R; the high range is
// used at T >= T_mid.
template <class S>
void thermo(const Mech& m, S T, S* cpR, S* hRT, S* sR) {
  S lnT = log_(T);
  for (int k = 0; k < m.K; ++k) {
    const double* a = (val(T) < m.Tmid[k]) ? &m.lo[7 * k] : &m.hi[7 * k];
    S T2 = T * T, T3 = T2 * T, T4 = T3 * T;
    cpR[k] = a[0] + a[1] * T + a[2] * T2 + a[3] * T3 + a[4] * T4;
    hRT[k] = a[0] + a[1] * T / 2.0 + a[2] * T2 / 3.0 + a[3] * T3 / 4.0 + a[4] * T4 / 5.0 + a[5] / T;
    sR[k] = a[0] * lnT + a[1] * T + a[2] * T2 / 2.0 + a[3] * T3 / 3.0 + a[4] * T4 / 4.0 + a[6];
  }
}

// ---------------------------------------------------------------- kinetics
// Rates of progress q_j and production rates wdot_k from T, P and all K molar
// concentrations.  lnA (nullable) replaces each reaction's ln A; for falloff
// reactions the low-pressure factor moves by the same amount, so ln A acts as
// a log-multiplier on the whole rate constant.
template <class S>
void kinetics(const Mech& m, S T, const S* Cc, const S* lnA, S* q, S* wdot,
              S* kf_out = nullptr, S* kr_out = nullptr) {
  const int K = m.K;
  std::vector<S> cpR(K), hRT(K), sR(K);
  thermo(m, T, cpR.data(), hRT.data(), sR.data());
  S lnT = log_(T);
  S ctot = C<S>(0.0);
  for (int k = 0; k < K; ++k) ctot += Cc[k];
  S lnPref = log_(PATM / (RU * T));      // ln of the standard-state concentration
  for (int k = 0; k < K; ++k) wdot[k] = C<S>(0.0);
  for (int j = 0; j < m.Nr; ++j) {
    const Rxn& r = m.rx[j];
    S la = lnA ? lnA[j] : C<S>(r.lnA);
    S kinf = exp_(la + r.b * lnT - r.theta / T);
    S keff = kinf;
    if (r.kind != 'E') {
      S M = ctot;
      for (size_t i = 0; i < r.ei.size(); ++i) M += (r.ea[i] - 1.0) * Cc[r.ei[i]];
      if (r.kind == 'T') {
        keff = kinf * M;
      } else {
        S k0 = exp_(la - r.lnA + r.lnA0 + r.b0 * lnT - r.theta0 / T);
        S Pr = k0 * M / kinf;
        S F = C<S>(1.0);
        if (r.kind == 'F') {
          S Fc = (1.0 - r.ta) * exp_(-T / r.T3) + r.ta * exp_(-T / r.T1);
          if (r.T2 > 0) Fc += exp_(-r.T2 / T);
          S lFc = log_(Fc) / LN10;
          S c = -0.4 - 0.67 * lFc;
          S n = 0.75 - 1.27 * lFc;
          S lPr = (val(Pr) > 1e-300) ? S(log_(Pr) / LN10) : C<S>(-300.0);
          S x = lPr + c;
          S y = x / (n - 0.14 * x);
          S lF = lFc / (1.0 + y * y);
          F = exp_(lF * LN10);
        }
        keff = kinf * (Pr / (1.0 + Pr)) * F;
      }
    }
    // equilibrium constant from the Gibbs functions
    S lnKp = C<S>(0.0);
    double dnu = 0;
    for (size_t i = 0; i < r.pi.size(); ++i) { lnKp += (double)r.pn[i] * (sR[r.pi[i]] - hRT[r.pi[i]]); dnu += r.pn[i]; }
    for (size_t i = 0; i < r.ri.size(); ++i) { lnKp -= (double)r.rn[i] * (sR[r.ri[i]] - hRT[r.ri[i]]); dnu -= r.rn[i]; }
    S lnKc = lnKp + dnu * lnPref;
    S kr = keff / exp_(lnKc);
    S fwd = keff, rev = kr;
    for (size_t i = 0; i < r.ri.size(); ++i)
      for (int p = 0; p < r.rn[i]; ++p) fwd *= Cc[r.ri[i]];
    for (size_t i = 0; i < r.pi.size(); ++i)
      for (int p = 0; p < r.pn[i]; ++p) rev *= Cc[r.pi[i]];
    q[j] = fwd - rev;
    if (kf_out) kf_out[j] = keff;
    if (kr_out) kr_out[j] = kr;
    for (size_t i = 0; i < r.ri.size(); ++i) wdot[r.ri[i]] -= (double)r.rn[i] * q[j];
    for (size_t i = 0; i < r.pi.size(); ++i) wdot[r.pi[i]] += (double)r.pn[i] * q[j];
  }
}

// f(Phi): Phi = (T, V, n_0 .. n_{K-2}); the last species is closed by the
// ideal-gas law.
template <class S>
void rhs(const Mech& m, double P, const S* phi, const S* lnA, S* f) {
  const int K = m.K;
  S T = phi[0], V = phi[1];
  std::vector<S> Cc(K), q(m.Nr), wdot(K), cpR(K), hRT(K), sR(K);
  S sum = C<S>(0.0);
  for (int k = 0; k < K - 1; ++k) { Cc[k] = phi[2 + k] / V; sum += Cc[k]; }
  Cc[K - 1] = P / (RU * T) - sum;
  kinetics(m, T, Cc.data(), lnA, q.data(), wdot.data());
  thermo(m, T, cpR.data(), hRT.data(), sR.data());
  S num = C<S>(0.0), den = C<S>(0.0), wsum = C<S>(0.0);
  for (int k = 0; k < K; ++k) {
    num += hRT[k] * RU * T * wdot[k];
    den += Cc[k] * cpR[k] * RU;
    wsum += wdot[k];
  }
  S Tdot = -num / den;
  f[0] = Tdot;
  f[1] = V * (Tdot / T + (RU * T / P) * wsum);
  for (int k = 0; k < K - 1; ++k) f[2 + k] = V * wdot[k];
}

// J_ij = d f_i / d Phi_j, one forward-mode pass per column.
template <class S>
void jacobian(const Mech& m, double P, const S* phi, const S* lnA, S* J) {
  const int N = m.K + 1;
  typedef Dual<S> D;
  std::vector<D> x(N), fx(N);
  std::vector<D> la;
  if (lnA) { la.resize(m.Nr); for (int j = 0; j < m.Nr; ++j) la[j] = D{lnA[j], C<S>(0.0)}; }
  for (int c = 0; c < N; ++c) {
    for (int i = 0; i < N; ++i) x[i] = D{phi[i], C<S>(i == c ? 1.0 : 0.0)};
    rhs<D>(m, P, x.data(), lnA ? la.data() : nullptr, fx.data());
    for (int i = 0; i < N; ++i) J[i * N + c] = fx[i].d;
  }
}

// ---------------------------------------------------------------- linear algebra
// In-place LU with partial pivoting (largest magnitude, ties to the lowest
// row position after the earlier swaps).  Returns 0, or 1 for a zero pivot, 2
// for a non-finite column.  margin (nullable) receives the smallest relative
// gap, over the steps, between the pivot's magnitude and the runner-up's
// ((best - second) / best; 1 where a column has one candidate): how far the
// pivot choices are from a tie.
template <class S>
int lu(int n, S* A, int* piv, double* margin = nullptr) {
  if (margin) *margin = 1.0;
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::fabs(val(A[k * n + k])), second = 0.0;
    bool finite = std::isfinite(best);
    for (int i = k + 1; i < n; ++i) {
      double v = std::fabs(val(A[i * n + k]));
      finite = finite && std::isfinite(v);
      if (v > best) { second = best; best = v; p = i; }
      else if (v > second) second = v;
    }
    if (!finite) return 2;
    if (!(best > 0.0)) return 1;
    if (margin && k + 1 < n) *margin = std::min(*margin, (best - second) / best);
    piv[k] = p;
    if (p != k)
      for (int j = 0; j < n; ++j) { S t = A[k * n + j]; A[k * n + j] = A[p * n + j]; A[p * n + j] = t; }
    for (int i = k + 1; i < n; ++i) {
      S l = A[i * n + k] / A[k * n + k];
      A[i * n + k] = l;
      for (int j = k + 1; j < n; ++j) A[i * n + j] -= l * A[k * n + j];
    }
  }
  return 0;
}

template <class S>
void lu_solve(int n, const S* LU, const int* piv, S* b) {
  for (int k = 0; k < n; ++k)
    if (piv[k] != k) { S t = b[k]; b[k] = b[piv[k]]; b[piv[k]] = t; }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) b[i] -= LU[i * n + j] * b[j];
  for (int i = n - 1; i >= 0; --i) {
    for (int j = i + 1; j < n; ++j) b[i] -= LU[i * n + j] * b[j];
    b[i] = b[i] / LU[i * n + i];
  }
}

// ---------------------------------------------------------------- Rosenbrock tables
// The four linearly implicit solvers of the paper's solver table (Table
// T:solvers), in the transformed form of Sec. 2.3: with u_i = sum_j gamma_ij k_j,
//   (I/(h gamma) - J) u_i = f(y + sum_{j<i} a_ij u_j) + sum_{j<i} (c_ij / h) u_j,
//   y_new = y + sum_j m_j u_j,   error estimate sum_j e_j u_j,
// where a = alpha Gamma^-1, C = diag(1/gamma) - Gamma^-1, m = b Gamma^-1 and
// e = (b - bhat) Gamma^-1 for the embedded weights bhat.  The coefficients are
// the published ones of the references the table gives: ROS3 and RODAS3 from
// Sandu et al. (1997), ROS4 (the L-stable set) and RODAS4 from Hairer and
// Wanner's Solving ODEs II.  `elo` is the order of the error estimate's
// leading term (embedded order + 1), the exponent of the step-size rule.
struct Method {
  const char* name;
  int s;
  double gamma;
  double a[6][6], c[6][6], m[6], e[6];
  double elo;
};

const Method ROS3 = {
    "ros3", 3, 0.43586652150845899941601945119356,
    {{0}, {1.0}, {1.0, 0.0}},
    {{0}, {-1.0156171083877702091975600115545},
     {4.0759956452537699824805835358067, 9.2076794298330791242156818474003}},
    {1.0, 6.1697947043828245592553615689730, -0.42772256543218573326238373806514},
    {0.5, -2.9079558716805469821718236208017, 0.22354069897811569627360909276199},
    3.0};

const Method ROS4 = {
    "ros4", 4, 0.57282,
    {{0}, {2.0}, {1.867943637803922, 0.2344449711399156},
     {1.867943637803922, 0.2344449711399156, 0.0}},
    {{0}, {-7.137615036412310}, {2.580708087951457, 0.6515950076447975},
     {-2.137148994382534, -0.3214669691237626, -0.6949742501781779}},
    {2.255570073418735, 0.2870493262186792, 0.4353179431840180, 1.093502252409163},
    {-0.2815431932141155, -0.07276199124938920, -0.1082196201495311, -1.093502252409163},
    4.0};

const Method RODAS3 = {
    "rodas3", 4, 0.5,
    {{0}, {0.0}, {2.0, 0.0}, {2.0, 0.0, 1.0}},
    {{0}, {4.0}, {1.0, -1.0}, {1.0, -1.0, -8.0 / 3.0}},
    {2.0, 0.0, 1.0, 1.0},
    {0.0, 0.0, 0.0, 1.0},
    3.0};

const Method RODAS4 = {
    "rodas4", 6, 0.25,
    {{0},
     {1.544},
     {0.9466785280815826, 0.2557011698983284},
     {3.314825187068521, 2.896124015972201, 0.9986419139977817},
     {1.221224509226641, 6.019134481288629, 12.53708332932087, -0.6878860361058950},
     {1.221224509226641, 6.019134481288629, 12.53708332932087, -0.6878860361058950, 1.0}},
    {{0},
     {-5.6688},
     {-2.430093356833875, -0.2063599157091915},
     {-0.1073529058151375, -9.594562251023355, -20.47028614809616},
     {7.496443313967647, -10.24680431464352, -33.99990352819905, 11.70890893206160},
     {8.083246795921522, -7.981132988064893, -31.52159432874371, 16.31930543123136,
      -6.058818238834054}},
    {1.221224509226641, 6.019134481288629, 12.53708332932087, -0.6878860361058950, 1.0, 1.0},
    {0.0, 0.0, 0.0, 0.0, 0.0, 1.0},
    4.0};

// The transformed coefficients from a method's standard form (alpha_ij,
// gamma_ij with gamma_ii = gamma, weights b and embedded weights bhat):
// a = alpha Gamma^-1, C = diag(1/gamma) - Gamma^-1, m = b Gamma^-1,
// e = (b - bhat) Gamma^-1, Gamma^-1 by forward substitution.
Method transformed(const char* name, int s, double gamma, const double al[6][6], const double ga[6][6],
                   const double* b, const double* bh, double elo) {
  double G[6][6] = {{0}}, Gi[6][6] = {{0}};
  for (int i = 0; i < s; ++i) {
    for (int j = 0; j < i; ++j) G[i][j] = ga[i][j];
    G[i][i] = gamma;
  }
  for (int c = 0; c < s; ++c)        // column c of Gamma^-1: Gamma x = e_c
    for (int i = 0; i < s; ++i) {
      double r = (i == c) ? 1.0 : 0.0;
      for (int j = 0; j < i; ++j) r -= G[i][j] * Gi[j][c];
      Gi[i][c] = r / G[i][i];
    }
  Method mt = {name, s, gamma, {{0}}, {{0}}, {0}, {0}, elo};
  for (int i = 0; i < s; ++i) {
    for (int j = 0; j < i; ++j) {
      double a = 0;
      for (int l = 0; l < s; ++l) a += al[i][l] * Gi[l][j];
      mt.a[i][j] = a;
      mt.c[i][j] = -Gi[i][j];
    }
  }
  for (int j = 0; j < s; ++j) {
    double m = 0, e = 0;
    for (int l = 0; l < s; ++l) {
      m += b[l] * Gi[l][j];
      e += (b[l] - bh[l]) * Gi[l][j];
    }
    mt.m[j] = m;
    mt.e[j] = e;
  }
  return mt;
}

// ROS34PW2 of Rang and Angermann (2005): a W-method - its order conditions
// hold for any matrix in the place of J, so a Jacobian kept from an earlier
// step leaves it of order 3 (embedded 2); stiffly accurate.  Published in the
// standard form.
Method make_ros34pw2() {
  const double g = 0.435866521508459;
  double al[6][6] = {{0}}, ga[6][6] = {{0}};
  al[1][0] = 0.87173304301691801;
  al[2][0] = 0.84457060015369423;
  al[2][1] = -0.11299064236484185;
  al[3][2] = 1.0;
  ga[1][0] = -0.87173304301691801;
  ga[2][0] = -0.90338057013044082;
  ga[2][1] = 0.054180672388095326;
  ga[3][0] = 0.24212380706095346;
  ga[3][1] = -1.2232505839045147;
  ga[3][2] = 0.54526025533510214;
  const double b[4] = {0.24212380706095346, -1.2232505839045147, 1.5452602553351020, 0.435866521508459};
  const double bh[4] = {0.37810903145819369, -0.096042292212423178, 0.5, 0.2179332607542295};
  return transformed("ros34pw2", 4, g, al, ga, b, bh, 3.0);
}
const Method ROS34PW2 = make_ros34pw2();

const Method* method_of(int id) {
  switch (id) {
    case 0: return &ROS4;
    case 1: return &ROS3;
    case 2: return &RODAS3;
    case 3: return &RODAS4;
    case 4: return &ROS34PW2;
    default: return nullptr;
  }
}

// A system for the integrator: dimension, f and J at a state.
struct ChemSys {
  const Mech* m;
  double P;
  int n() const { return m->K + 1; }
  template <class S> void f(const S* y, const S* lnA, S* out) const { rhs(*m, P, y, lnA, out); }
  template <class S> void jac(const S* y, const S* lnA, S* J) const { jacobian(*m, P, y, lnA, J); }
};

struct LinSys {            // y' = A y
  int dim;
  const double* A;
  int n() const { return dim; }
  template <class S> void f(const S* y, const S*, S* out) const {
    for (int i = 0; i < dim; ++i) { out[i] = C<S>(0.0); for (int j = 0; j < dim; ++j) out[i] += A[i * dim + j] * y[j]; }
  }
  template <class S> void jac(const S*, const S*, S* J) const {
    for (int i = 0; i < dim * dim; ++i) J[i] = C<S>(A[i]);
  }
};

struct CubicSys {          // y' = -y^3, y(t) = y0 / sqrt(1 + 2 y0^2 t)
  int n() const { return 1; }
  template <class S> void f(const S* y, const S*, S* out) const { out[0] = -(y[0] * y[0] * y[0]); }
  template <class S> void jac(const S* y, const S*, S* J) const { J[0] = -3.0 * (y[0] * y[0]); }
};

// Error estimates.  EST_EMBEDDED is the method's own: sum_j e_j u_j, the
// difference of the two solutions.  EST_FILTERED applies (I - h gamma J)^-1 to
// it, the filter Shampine proposed and Hairer and Wanner use in RADAU5: it
// keeps the leading h^elo term and takes the estimate of a strongly damped mode
// to zero, where the embedded solution of a 4-stage method of order 4 cannot
// damp it.
enum { EST_EMBEDDED = 0, EST_FILTERED = 1 };

// One step of size h from y with method `mt`.  Returns the LU's code (0 =
// success).  Stages whose argument equals the previous stage's (row i of a
// equal to row i-1) share that stage's f, as the methods are built for.
// Jac (optional) stands in for J(y): a Jacobian kept from an earlier state,
// which only a W-method tolerates without losing its order.
template <class Sys, class S>
int ros_step(const Sys& sys, const Method& mt, const S* y, const S* lnA, double h, int estimator,
             S* ynew, S* err, const S* Jac = nullptr) {
  const int n = sys.n(), s = mt.s;
  std::vector<S> J(n * n), Yi(n), F(n);
  std::vector<std::vector<S>> u(s, std::vector<S>(n));
  std::vector<int> piv(n);
  if (Jac)
    for (int i = 0; i < n * n; ++i) J[i] = Jac[i];
  else
    sys.jac(y, lnA, J.data());
  for (int i = 0; i < n * n; ++i) J[i] = -J[i];
  for (int i = 0; i < n; ++i) J[i * n + i] += 1.0 / (h * mt.gamma);
  int rc = lu(n, J.data(), piv.data());
  if (rc) return rc;
  for (int i = 0; i < s; ++i) {
    bool same = i > 0;
    for (int j = 0; j < i && same; ++j) same = mt.a[i][j] == (j < i - 1 ? mt.a[i - 1][j] : 0.0);
    if (!same) {
      for (int k = 0; k < n; ++k) {
        Yi[k] = y[k];
        for (int j = 0; j < i; ++j) Yi[k] += mt.a[i][j] * u[j][k];
      }
      sys.f(Yi.data(), lnA, F.data());
    }
    for (int k = 0; k < n; ++k) {
      S r = F[k];
      for (int j = 0; j < i; ++j) r += (mt.c[i][j] / h) * u[j][k];
      u[i][k] = r;
    }
    lu_solve(n, J.data(), piv.data(), u[i].data());
  }
  for (int k = 0; k < n; ++k) {
    ynew[k] = y[k];
    err[k] = C<S>(0.0);
    for (int j = 0; j < s; ++j) {
      ynew[k] += mt.m[j] * u[j][k];
      err[k] += mt.e[j] * u[j][k];
    }
  }
  if (estimator == EST_FILTERED) {
    // (I - h gamma J)^-1 = M^-1 / (h gamma), M = I/(h gamma) - J factored above
    lu_solve(n, J.data(), piv.data(), err);
    for (int k = 0; k < n; ++k) err[k] = err[k] / (h * mt.gamma);
  }
  return 0;
}

struct Ctl {
  double rtol, atol, h_min = 1e-20, safety = 0.9, fac_min = 0.2, fac_max = 6.0;
  int max_steps = 100000;
  int max_bad = 10;
  const Method* mt = &ROS4;
  int estimator = EST_EMBEDDED;
  int jac_every = 1;   // J evaluated at every jac_every-th accepted state, kept in between
};

struct Outcome { int accepted = 0, rejected = 0, status = 0; double h_next = 0; };

// Adaptive integration of y over [0, dt] (Sec. 3.1 tolerances; the constants
// are the readings listed with the design notes).  h0 <= 0 means h0 = dt.
// Records the accepted step sizes when ``hist`` is given.
template <class Sys>
Outcome integrate(const Sys& sys, double* y, double dt, double h0, const Ctl& c,
                  const double* lnA, std::vector<double>* hist = nullptr) {
  const int n = sys.n();
  std::vector<double> ynew(n), err(n), Jk(n * n);
  Outcome o;
  double h = (h0 > 0) ? h0 : dt;
  double rem = dt;
  bool last_rejected = false;
  int bad = 0;
  int attempts = 0;
  int since_jac = c.jac_every;   // accepted steps since J was evaluated
  while (rem > 0) {
    if (attempts >= c.max_steps) { o.status = 1; break; }
    if (h < c.h_min) { o.status = 2; break; }
    ++attempts;
    double hs = std::min(h, rem);
    if (since_jac >= c.jac_every) {   // a rejected step keeps the J of its state
      sys.jac(y, lnA, Jk.data());
      since_jac = 0;
    }
    int rc = ros_step(sys, *c.mt, y, lnA, hs, c.estimator, ynew.data(), err.data(), Jk.data());
    bool ok = rc == 0;
    double e = 0;
    if (ok) {
      for (int i = 0; i < n; ++i) {
        double sc = c.atol + c.rtol * std::max(std::fabs(y[i]), std::fabs(ynew[i]));
        e += (err[i] / sc) * (err[i] / sc);
      }
      e = std::sqrt(e / n);
    }
    if (!ok || !std::isfinite(e)) {
      ++o.rejected;
      if (++bad >= c.max_bad) { o.status = (rc == 1) ? 4 : 3; break; }
      h = hs * c.fac_min;
      last_rejected = true;
      continue;
    }
    bad = 0;
    double fac = (e > 0) ? c.safety * std::pow(e, -1.0 / c.mt->elo) : c.fac_max;
    if (e <= 1.0) {
      for (int i = 0; i < n; ++i) y[i] = ynew[i];
      rem -= hs;
      ++o.accepted;
      ++since_jac;
      if (hist) hist->push_back(hs);
      fac = std::min(c.fac_max, std::max(c.fac_min, fac));
      if (last_rejected) fac = std::min(fac, 1.0);
      last_rejected = false;
    } else {
      ++o.rejected;
      fac = std::min(1.0, std::max(c.fac_min, fac));
      last_rejected = true;
    }
    h = hs * fac;
  }
  o.h_next = h;
  return o;
}

// ---------------------------------------------------------------- conversions
// (T, P, Y) -> Phi per unit mass: V = R T / (P Wbar), n_k = Y_k / W_k.
template <class S>
void to_phi(const Mech& m, S T, double P, const S* Y, S* phi) {
  S inv = C<S>(0.0);
  for (int k = 0; k < m.K; ++k) inv += Y[k] / m.W[k];
  phi[0] = T;
  phi[1] = RU * T * inv / P;
  for (int k = 0; k < m.K - 1; ++k) phi[2 + k] = Y[k] / m.W[k];
}

// Phi -> (T, Y): n_K = P V / (R T) - sum n_k, Y_k = n_k W_k / sum_i n_i W_i.
template <class S>
void from_phi(const Mech& m, double P, const S* phi, S* T, S* Y) {
  const int K = m.K;
  std::vector<S> n(K);
  S s = C<S>(0.0);
  for (int k = 0; k < K - 1; ++k) { n[k] = phi[2 + k]; s += n[k]; }
  n[K - 1] = P * phi[1] / (RU * phi[0]) - s;
  S mass = C<S>(0.0);
  for (int k = 0; k < K; ++k) mass += n[k] * m.W[k];
  for (int k = 0; k < K; ++k) Y[k] = n[k] * m.W[k] / mass;
  *T = phi[0];
}

// Replays one cell's accepted steps in dual arithmetic: the derivative of the
// final (T, Y) along a direction in (ln A, T0, Y0).
void tangent(const Mech& m, const Method& mt, double P, double T0, const double* Y0, const double* lnA,
             const std::vector<double>& hs, const double* v_lnA, double dT0, const double* dY0,
             double* dT, double* dY) {
  typedef Dual<double> D;
  const int K = m.K, N = K + 1;
  ChemSys sys{&m, P};
  std::vector<D> la(m.Nr), Y(K), phi(N), ynew(N), err(N), Yo(K);
  for (int j = 0; j < m.Nr; ++j) la[j] = D{lnA ? lnA[j] : m.rx[j].lnA, v_lnA ? v_lnA[j] : 0.0};
  for (int k = 0; k < K; ++k) Y[k] = D{Y0[k], dY0 ? dY0[k] : 0.0};
  to_phi(m, D{T0, dT0}, P, Y.data(), phi.data());
  for (double h : hs) {
    ros_step(sys, mt, phi.data(), la.data(), h, EST_EMBEDDED, ynew.data(), err.data());
    phi = ynew;
  }
  D T;
  from_phi(m, P, phi.data(), &T, Yo.data());
  *dT = T.d;
  for (int k = 0; k < K; ++k) dY[k] = Yo[k].d;
}

}  // namespace

// ============================================================== C interface
// `method`: 0 ROS4, 1 ROS3, 2 RODAS3, 3 RODAS4, 4 ROS34PW2; `estimator`:
// 0 embedded, 1 filtered; `jac_every` (>= 1): J evaluated at every
// jac_every-th accepted state and kept in between.  Functions taking a method
// return -100 for an unknown one.
extern "C" {

void* or_mech_load(const char* path) {
  Mech* m = new Mech();
  if (!parse(path, *m)) { delete m; return nullptr; }
  return m;
}
void or_mech_free(void* h) { delete (Mech*)h; }
void or_mech_dims(void* h, int* K, int* Nr, int* E) {
  const Mech* m = (const Mech*)h;
  *K = m->K; *Nr = m->Nr; *E = m->E;
}
void or_mech_arrays(void* h, double* W, int* comp, double* lnA) {
  const Mech* m = (const Mech*)h;
  for (int k = 0; k < m->K; ++k) W[k] = m->W[k];
  for (int i = 0; i < m->K * m->E; ++i) comp[i] = m->comp[i];
  for (int j = 0; j < m->Nr; ++j) lnA[j] = m->rx[j].lnA;
}

void or_thermo(void* h, double T, double* cpR, double* hRT, double* sR) {
  thermo(*(const Mech*)h, T, cpR, hRT, sR);
}

void or_kinetics(void* h, double T, double P, const double* Cc, const double* lnA,
                 double* q, double* wdot, double* kf, double* kr) {
  (void)P;
  kinetics(*(const Mech*)h, T, Cc, lnA, q, wdot, kf, kr);
}

void or_rhs(void* h, double P, const double* phi, const double* lnA, double* f) {
  rhs(*(const Mech*)h, P, phi, lnA, f);
}

void or_jacobian(void* h, double P, const double* phi, const double* lnA, double* J) {
  jacobian(*(const Mech*)h, P, phi, lnA, J);
}

int or_lu_solve(int n, const double* A, const double* b, double* x) {
  std::vector<double> LU(A, A + n * n);
  std::vector<int> piv(n);
  if (lu(n, LU.data(), piv.data())) return -1;
  for (int i = 0; i < n; ++i) x[i] = b[i];
  lu_solve(n, LU.data(), piv.data(), x);
  return 0;
}

// LU of an n x n row-major matrix M: F receives the factors in pivot order
// (row k: L left of the diagonal, unit diagonal implied, U from it on), perm
// the row of M pivoted at each step (the swap sequence applied to 0..n-1),
// margin as lu's.  Returns lu's code; F and perm are complete only for 0.
int or_lu(int n, const double* M, double* F, int* perm, double* margin) {
  for (int i = 0; i < n * n; ++i) F[i] = M[i];
  std::vector<int> piv(n);
  const int rc = lu(n, F, piv.data(), margin);
  for (int i = 0; i < n; ++i) perm[i] = i;
  if (rc == 0)
    for (int k = 0; k < n; ++k) std::swap(perm[k], perm[piv[k]]);
  return rc;
}

// The transformed table of a method: t[0] = s, t[1] = gamma, t[2] = elo, then
// a[6][6], c[6][6], m[6], e[6] (t has 3 + 84 entries).
int or_method_table(int method, double* t) {
  const Method* mt = method_of(method);
  if (!mt) return -100;
  t[0] = mt->s; t[1] = mt->gamma; t[2] = mt->elo;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) { t[3 + 6 * i + j] = mt->a[i][j]; t[39 + 6 * i + j] = mt->c[i][j]; }
  for (int j = 0; j < 6; ++j) { t[75 + j] = mt->m[j]; t[81 + j] = mt->e[j]; }
  return 0;
}

int or_step(void* h, double P, const double* phi, double hs, double* phinew, double* err, int method,
            int estimator) {
  const Method* mt = method_of(method);
  if (!mt) return -100;
  ChemSys sys{(const Mech*)h, P};
  return ros_step(sys, *mt, phi, (const double*)nullptr, hs, estimator, phinew, err) ? -1 : 0;
}

void or_to_phi(void* h, double T, double P, const double* Y, double* phi) {
  to_phi(*(const Mech*)h, T, P, Y, phi);
}
void or_from_phi(void* h, double P, const double* phi, double* T, double* Y) {
  from_phi(*(const Mech*)h, P, phi, T, Y);
}

// Batched integration over one split step.  Y, Y_out are [K][ldY] (cell
// fastest).  h_io (nullable): in, first step (<= 0 -> dt); out, next step.
// Returns the number of threads used.
int or_integrate(void* hm, int64_t n, const double* T, const double* P, const double* Y, int64_t ldY,
                 double dt, double rtol, double atol, double* h_io, double* T_out, double* Y_out,
                 int32_t* n_acc, int32_t* n_rej, int32_t* status, const double* lnA, int max_steps,
                 int nthreads, int method, int estimator, int jac_every) {
  const Mech& m = *(const Mech*)hm;
  const Method* mt = method_of(method);
  if (!mt) return -100;
  if (nthreads <= 0) nthreads = omp_get_max_threads();
  Ctl c;
  c.rtol = rtol; c.atol = atol;
  c.mt = mt;
  c.estimator = estimator;
  c.jac_every = jac_every > 0 ? jac_every : 1;
  if (max_steps > 0) c.max_steps = max_steps;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
  for (int64_t cell = 0; cell < n; ++cell) {
    const int K = m.K, N = K + 1;
    std::vector<double> y(K), phi(N), Yo(K);
    for (int k = 0; k < K; ++k) y[k] = Y[k * ldY + cell];
    to_phi(m, T[cell], P[cell], y.data(), phi.data());
    ChemSys sys{&m, P[cell]};
    double h0 = h_io ? h_io[cell] : 0.0;
    Outcome o = integrate(sys, phi.data(), dt, h0, c, lnA);
    double To;
    from_phi(m, P[cell], phi.data(), &To, Yo.data());
    T_out[cell] = To;
    for (int k = 0; k < K; ++k) Y_out[k * ldY + cell] = Yo[k];
    if (h_io) h_io[cell] = o.h_next;
    if (n_acc) n_acc[cell] = o.accepted;
    if (n_rej) n_rej[cell] = o.rejected;
    if (status) status[cell] = o.status;
  }
  return nthreads;
}

// One cell: integrate and return the accepted step sizes (capacity cap).
int or_record_steps(void* hm, double T, double P, const double* Y, double dt, double rtol,
                    double atol, double h0, const double* lnA, double* hs, int cap, double* T_out,
                    double* Y_out, int method, int estimator, int jac_every) {
  const Mech& m = *(const Mech*)hm;
  const Method* mt = method_of(method);
  if (!mt) return -100;
  const int K = m.K, N = K + 1;
  std::vector<double> phi(N);
  to_phi(m, T, P, Y, phi.data());
  ChemSys sys{&m, P};
  Ctl c;
  c.rtol = rtol; c.atol = atol;
  c.mt = mt;
  c.estimator = estimator;
  c.jac_every = jac_every > 0 ? jac_every : 1;
  std::vector<double> hist;
  Outcome o = integrate(sys, phi.data(), dt, h0, c, lnA, &hist);
  from_phi(m, P, phi.data(), T_out, Y_out);
  if (o.status) return -o.status;
  int n = (int)hist.size();
  for (int i = 0; i < n && i < cap; ++i) hs[i] = hist[i];
  return n;
}

// One cell: replay a given sequence of step sizes (frozen steps, no control).
int or_replay(void* hm, double T, double P, const double* Y, const double* lnA, const double* hs,
              int nh, double* T_out, double* Y_out, int method) {
  const Mech& m = *(const Mech*)hm;
  const Method* mt = method_of(method);
  if (!mt) return -100;
  const int N = m.K + 1;
  std::vector<double> phi(N), ynew(N), err(N);
  to_phi(m, T, P, Y, phi.data());
  ChemSys sys{&m, P};
  for (int i = 0; i < nh; ++i) {
    if (ros_step(sys, *mt, phi.data(), lnA, hs[i], EST_EMBEDDED, ynew.data(), err.data())) return -1;
    phi = ynew;
  }
  from_phi(m, P, phi.data(), T_out, Y_out);
  return 0;
}

// One cell: directional derivative of the final (T, Y) along (v_lnA, dT0, dY0)
// through the frozen steps hs.
int or_tangent(void* hm, double T, double P, const double* Y, const double* lnA, const double* hs,
               int nh, const double* v_lnA, double dT0, const double* dY0, double* dT, double* dY,
               int method) {
  const Method* mt = method_of(method);
  if (!mt) return -100;
  std::vector<double> h(hs, hs + nh);
  tangent(*(const Mech*)hm, *mt, P, T, Y, lnA, h, v_lnA, dT0, dY0, dT, dY);
  return 0;
}

// Model problems for the integrator alone.  h_fixed > 0: fixed steps of that
// size (no control).  Returns accepted steps (negative status on failure).
int or_integrate_linear(int n, const double* A, double* y, double dt, double rtol, double atol,
                        double h_fixed, int method, int estimator) {
  const Method* mt = method_of(method);
  if (!mt) return -100;
  LinSys sys{n, A};
  if (h_fixed > 0) {
    std::vector<double> ynew(n), err(n);
    int steps = (int)std::llround(dt / h_fixed);
    for (int s = 0; s < steps; ++s) {
      ros_step(sys, *mt, y, (const double*)nullptr, h_fixed, estimator, ynew.data(), err.data());
      for (int i = 0; i < n; ++i) y[i] = ynew[i];
    }
    return steps;
  }
  Ctl c;
  c.rtol = rtol; c.atol = atol;
  c.mt = mt;
  c.estimator = estimator;
  Outcome o = integrate(sys, y, dt, 0.0, c, nullptr);
  return o.status ? -o.status : o.accepted;
}

// One step of y' = A y: the new state and the error estimate.  Ajac
// (nullable) stands in for the Jacobian A.
int or_linear_step(int n, const double* A, const double* y, double h, double* ynew, double* err,
                   int method, int estimator, const double* Ajac) {
  const Method* mt = method_of(method);
  if (!mt) return -100;
  LinSys sys{n, A};
  return ros_step(sys, *mt, y, (const double*)nullptr, h, estimator, ynew, err, Ajac) ? -1 : 0;
}

// y' = -y^3.  jac_every > 1: the Jacobian is evaluated at every jac_every-th
// step's state and kept in between (as the controller's reuse does).
int or_integrate_cubic(double* y, double dt, double rtol, double atol, double h_fixed, int method,
                       int estimator, int jac_every) {
  const Method* mt = method_of(method);
  if (!mt) return -100;
  CubicSys sys;
  if (jac_every < 1) jac_every = 1;
  if (h_fixed > 0) {
    double ynew, err, Jk = 0;
    int steps = (int)std::llround(dt / h_fixed);
    for (int s = 0; s < steps; ++s) {
      if (s % jac_every == 0) sys.jac(y, (const double*)nullptr, &Jk);
      ros_step(sys, *mt, y, (const double*)nullptr, h_fixed, estimator, &ynew, &err, &Jk);
      y[0] = ynew;
    }
    return steps;
  }
  Ctl c;
  c.rtol = rtol; c.atol = atol;
  c.mt = mt;
  c.estimator = estimator;
  c.jac_every = jac_every;
  Outcome o = integrate(sys, y, dt, 0.0, c, nullptr);
  return o.status ? -o.status : o.accepted;
}

}  // extern "C"
