// CPU FP64 oracle for batched constant-pressure chemistry integration with ROS4.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
// includes this file; only the tests, the smoke check and the CPU-baseline leg
// of the benchmark load it.  It shares no code with the HIP path: it has its
// own mechanism parser, its own thermochemistry, its own ROS4 table literals.
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
//     u_i / a_ij / c_ij / m_j form that follows it), 4 stages, one LU per step;
//     ROS4 with an L-stable 4(3) coefficient set (Table T:solvers);
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
// row).  Returns 0, or 1 for a zero pivot, 2 for a non-finite column.
template <class S>
int lu(int n, S* A, int* piv) {
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::fabs(val(A[k * n + k]));
    bool finite = std::isfinite(best);
    for (int i = k + 1; i < n; ++i) {
      double v = std::fabs(val(A[i * n + k]));
      finite = finite && std::isfinite(v);
      if (v > best) { best = v; p = i; }
    }
    if (!finite) return 2;
    if (!(best > 0.0)) return 1;
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

// ---------------------------------------------------------------- ROS4 table
// An L-stable 4-stage order-4 Rosenbrock method with an embedded order-3
// solution, in the transformed form u_i = sum_j gamma_ij k_j (Sec. 2.3).
// gamma = 1/x2, x2 the second root of the Laguerre polynomial L4, gives
// R(inf) = 0; alpha_4j = alpha_3j so stage 4 reuses stage 3's f.  The free
// parameters were fixed at alpha_21 = 2 gamma, alpha_3 = 0.45, b_4 = 0.4, and
// the embedded weights have bhat_4 = 0.
const double GAM = 0.57281606248213485541;
const double A21 = 2.0;
const double A31 = 1.491001215556513813960407;
const double A32 = 0.2283940090236591778889569;
const double C21 = -7.137649921358897064355991;
const double C31 = -6.196702482993044766389505;
const double C32 = -0.8558736500387530085234008;
const double C41 = 5.964333552759764215600564;
const double C42 = 0.4379266338878570570784905;
const double C43 = 2.525577246716920611308754;
const double M1 = 1.63885860954486232683164;
const double M2 = 0.474955117534000084335749;
const double M3 = -0.07416508734030706110427568;
const double M4 = 0.6983044404633386302747267;
const double E1 = 0.09734671529814985040858406;
const double E2 = 0.2866125685892372986834792;
const double E3 = 0.6849355088701844022099764;
const double E4 = 0.6983044404633386302747267;

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

struct RiccatiSys {        // y' = -y^2
  int n() const { return 1; }
  template <class S> void f(const S* y, const S*, S* out) const { out[0] = -(y[0] * y[0]); }
  template <class S> void jac(const S* y, const S*, S* J) const { J[0] = -2.0 * y[0]; }
};

// One ROS4 step of size h from y.  Returns the LU's code (0 = success).
template <class Sys, class S>
int ros4_step(const Sys& sys, const S* y, const S* lnA, double h, S* ynew, S* err) {
  const int n = sys.n();
  std::vector<S> J(n * n), u1(n), u2(n), u3(n), u4(n), Yi(n), F(n), F3(n);
  std::vector<int> piv(n);
  sys.jac(y, lnA, J.data());
  for (int i = 0; i < n * n; ++i) J[i] = -J[i];
  for (int i = 0; i < n; ++i) J[i * n + i] += 1.0 / (h * GAM);
  int rc = lu(n, J.data(), piv.data());
  if (rc) return rc;
  sys.f(y, lnA, u1.data());
  lu_solve(n, J.data(), piv.data(), u1.data());
  for (int i = 0; i < n; ++i) Yi[i] = y[i] + A21 * u1[i];
  sys.f(Yi.data(), lnA, F.data());
  for (int i = 0; i < n; ++i) u2[i] = F[i] + (C21 / h) * u1[i];
  lu_solve(n, J.data(), piv.data(), u2.data());
  for (int i = 0; i < n; ++i) Yi[i] = y[i] + A31 * u1[i] + A32 * u2[i];
  sys.f(Yi.data(), lnA, F3.data());
  for (int i = 0; i < n; ++i) u3[i] = F3[i] + (C31 * u1[i] + C32 * u2[i]) / h;
  lu_solve(n, J.data(), piv.data(), u3.data());
  for (int i = 0; i < n; ++i) u4[i] = F3[i] + (C41 * u1[i] + C42 * u2[i] + C43 * u3[i]) / h;
  lu_solve(n, J.data(), piv.data(), u4.data());
  for (int i = 0; i < n; ++i) {
    ynew[i] = y[i] + M1 * u1[i] + M2 * u2[i] + M3 * u3[i] + M4 * u4[i];
    err[i] = E1 * u1[i] + E2 * u2[i] + E3 * u3[i] + E4 * u4[i];
  }
  return 0;
}

struct Ctl {
  double rtol, atol, h_min = 1e-20, safety = 0.9, fac_min = 0.2, fac_max = 6.0;
  int max_steps = 100000;
  int max_bad = 10;
};

struct Outcome { int accepted = 0, rejected = 0, status = 0; double h_next = 0; };

// Adaptive integration of y over [0, dt].  h0 <= 0 means h0 = dt.  Records the
// accepted step sizes when ``hist`` is given.
template <class Sys>
Outcome integrate(const Sys& sys, double* y, double dt, double h0, const Ctl& c,
                  const double* lnA, std::vector<double>* hist = nullptr) {
  const int n = sys.n();
  std::vector<double> ynew(n), err(n);
  Outcome o;
  double h = (h0 > 0) ? h0 : dt;
  double rem = dt;
  bool last_rejected = false;
  int bad = 0;
  int attempts = 0;
  while (rem > 0) {
    if (attempts >= c.max_steps) { o.status = 1; break; }
    if (h < c.h_min) { o.status = 2; break; }
    ++attempts;
    double hs = std::min(h, rem);
    int rc = ros4_step(sys, y, lnA, hs, ynew.data(), err.data());
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
    double fac = (e > 0) ? c.safety * std::pow(e, -0.25) : c.fac_max;
    if (e <= 1.0) {
      for (int i = 0; i < n; ++i) y[i] = ynew[i];
      rem -= hs;
      ++o.accepted;
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
void tangent(const Mech& m, double P, double T0, const double* Y0, const double* lnA,
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
    ros4_step(sys, phi.data(), la.data(), h, ynew.data(), err.data());
    phi = ynew;
  }
  D T;
  from_phi(m, P, phi.data(), &T, Yo.data());
  *dT = T.d;
  for (int k = 0; k < K; ++k) dY[k] = Yo[k].d;
}

}  // namespace

// ============================================================== C interface
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

void or_ros4_table(double* t) {
  const double v[] = {GAM, A21, A31, A32, C21, C31, C32, C41, C42, C43, M1, M2, M3, M4, E1, E2, E3, E4};
  for (int i = 0; i < 18; ++i) t[i] = v[i];
}

int or_step(void* h, double P, const double* phi, double hs, double* phinew, double* err) {
  ChemSys sys{(const Mech*)h, P};
  return ros4_step(sys, phi, (const double*)nullptr, hs, phinew, err) ? -1 : 0;
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
                 int nthreads) {
  const Mech& m = *(const Mech*)hm;
  if (nthreads <= 0) nthreads = omp_get_max_threads();
  Ctl c;
  c.rtol = rtol; c.atol = atol;
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
                    double* Y_out) {
  const Mech& m = *(const Mech*)hm;
  const int K = m.K, N = K + 1;
  std::vector<double> phi(N);
  to_phi(m, T, P, Y, phi.data());
  ChemSys sys{&m, P};
  Ctl c;
  c.rtol = rtol; c.atol = atol;
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
              int nh, double* T_out, double* Y_out) {
  const Mech& m = *(const Mech*)hm;
  const int N = m.K + 1;
  std::vector<double> phi(N), ynew(N), err(N);
  to_phi(m, T, P, Y, phi.data());
  ChemSys sys{&m, P};
  for (int i = 0; i < nh; ++i) {
    if (ros4_step(sys, phi.data(), lnA, hs[i], ynew.data(), err.data())) return -1;
    phi = ynew;
  }
  from_phi(m, P, phi.data(), T_out, Y_out);
  return 0;
}

// One cell: directional derivative of the final (T, Y) along (v_lnA, dT0, dY0)
// through the frozen steps hs.
void or_tangent(void* hm, double T, double P, const double* Y, const double* lnA, const double* hs,
                int nh, const double* v_lnA, double dT0, const double* dY0, double* dT, double* dY) {
  std::vector<double> h(hs, hs + nh);
  tangent(*(const Mech*)hm, P, T, Y, lnA, h, v_lnA, dT0, dY0, dT, dY);
}

// Model problems for the integrator alone.  h_fixed > 0: fixed steps of that
// size (no control).  Returns accepted steps (negative status on failure).
int or_integrate_linear(int n, const double* A, double* y, double dt, double rtol, double atol,
                        double h_fixed) {
  LinSys sys{n, A};
  if (h_fixed > 0) {
    std::vector<double> ynew(n), err(n);
    int steps = (int)std::llround(dt / h_fixed);
    for (int s = 0; s < steps; ++s) {
      ros4_step(sys, y, (const double*)nullptr, h_fixed, ynew.data(), err.data());
      for (int i = 0; i < n; ++i) y[i] = ynew[i];
    }
    return steps;
  }
  Ctl c;
  c.rtol = rtol; c.atol = atol;
  Outcome o = integrate(sys, y, dt, 0.0, c, nullptr);
  return o.status ? -o.status : o.accepted;
}

int or_integrate_riccati(double* y, double dt, double rtol, double atol, double h_fixed) {
  RiccatiSys sys;
  if (h_fixed > 0) {
    double ynew, err;
    int steps = (int)std::llround(dt / h_fixed);
    for (int s = 0; s < steps; ++s) {
      ros4_step(sys, y, (const double*)nullptr, h_fixed, &ynew, &err);
      y[0] = ynew;
    }
    return steps;
  }
  Ctl c;
  c.rtol = rtol; c.atol = atol;
  Outcome o = integrate(sys, y, dt, 0.0, c, nullptr);
  return o.status ? -o.status : o.accepted;
}

}  // extern "C"
