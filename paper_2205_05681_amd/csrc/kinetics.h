// Device-side thermochemistry, source terms and analytical Jacobian for one
// cell per thread.  Per-cell vectors live in a structure-of-arrays workspace
// (element i of a cell at p[i * ld], consecutive cells adjacent), so every
// access of a wavefront is one coalesced transaction; the mechanism tables are
// read at wavefront-uniform indices and so go through scalar loads.  The rate
// law of one reaction (reaction_rate, templated on the scalar type for the
// dual numbers of the adjoint) is shared with the one-wavefront-per-cell
// kernels, which give each lane its own reaction.
//
// State (paper Sec. 2.1, eq. (state_vec)): Phi = (T, V, n_0 .. n_{K-2}) per
// unit mass; the bath gas K-1 is closed by the ideal-gas law (eq. (n_nsp)).
// Source terms (eq. (dphidt)), CHEMKIN-form rate laws:
//   C_k = n_k / V,  C_{K-1} = P/(R T) - sum_k C_k
//   k_f = A T^b exp(-theta/T);  third body k = k_f [M], [M] = sum alpha_k C_k;
//   falloff k = k_inf Pr/(1+Pr) F, Pr = k0 [M]/k_inf, F = 1 (Lindemann) or Troe;
//   K_c = exp(sum nu (s/R - h/RT)) (P_atm/(R T))^(sum nu);  k_r = k / K_c
//   q = k prod C^nu' - k_r prod C^nu'';  wdot_k = sum_j nu_kj q_j
//   dT/dt = -sum H_k wdot_k / sum C_k cp_k,  dV/dt = V (Tdot/T + R T/P sum wdot)
//   dn_k/dt = V wdot_k
// Jacobian (eq. (jac)), derived by hand:
//   G_km = d wdot_k / d C_m at fixed T, g_k = d wdot_k / dT at fixed C;
//   third-body and falloff terms enter G as a rank-one alpha_m * beta_j update,
//   split into a uniform part (a per-row sum) and the listed efficiencies;
//   the chain rule through C(Phi):  dC_k/dn_m = delta_km / V,
//   dC_{K-1}/dn_m = -1/V, dC_k/dV = -C_k/V, dC_{K-1}/dV = sum C_k / V,
//   dC_{K-1}/dT = -P/(R T^2);  the T and V rows are reductions over species.
#pragma once
#include <hip/hip_runtime.h>

#include "mech.h"

namespace chem {

template <class S>
struct LaneT {
  S* __restrict__ p;
  int64_t ld;
  __device__ __forceinline__ S& operator[](int i) const { return p[(int64_t)i * ld]; }
};
using Lane = LaneT<double>;

using ::exp;
using ::log;
using ::log10;

// Forward-mode dual number: value and derivative along one direction.  Used
// for directional derivatives of the Jacobian in the adjoint sweep.
struct Dd {
  double v, d;
};
__device__ __forceinline__ Dd dd(double v, double d = 0.0) { return Dd{v, d}; }
__device__ __forceinline__ Dd operator+(Dd a, Dd b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ Dd operator-(Dd a, Dd b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ Dd operator-(Dd a) { return {-a.v, -a.d}; }
__device__ __forceinline__ Dd operator*(Dd a, Dd b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ __forceinline__ Dd operator/(Dd a, Dd b) {
  const double q = a.v / b.v;
  return {q, (a.d - q * b.d) / b.v};
}
__device__ __forceinline__ Dd operator+(Dd a, double b) { return {a.v + b, a.d}; }
__device__ __forceinline__ Dd operator+(double b, Dd a) { return {a.v + b, a.d}; }
__device__ __forceinline__ Dd operator-(Dd a, double b) { return {a.v - b, a.d}; }
__device__ __forceinline__ Dd operator-(double b, Dd a) { return {b - a.v, -a.d}; }
__device__ __forceinline__ Dd operator*(Dd a, double b) { return {a.v * b, a.d * b}; }
__device__ __forceinline__ Dd operator*(double b, Dd a) { return {a.v * b, a.d * b}; }
__device__ __forceinline__ Dd operator/(Dd a, double b) { return {a.v / b, a.d / b}; }
__device__ __forceinline__ Dd operator/(double b, Dd a) {
  const double q = b / a.v;
  return {q, -q * a.d / a.v};
}
__device__ __forceinline__ Dd& operator+=(Dd& a, Dd b) { a = a + b; return a; }
__device__ __forceinline__ Dd& operator-=(Dd& a, Dd b) { a = a - b; return a; }
__device__ __forceinline__ Dd& operator*=(Dd& a, Dd b) { a = a * b; return a; }
__device__ __forceinline__ Dd& operator+=(Dd& a, double b) { a.v += b; return a; }
__device__ __forceinline__ Dd exp(Dd a) { const double e = exp(a.v); return {e, e * a.d}; }
__device__ __forceinline__ Dd log(Dd a) { return {log(a.v), a.d / a.v}; }
__device__ __forceinline__ Dd log10(Dd a) { return {log10(a.v), a.d / (a.v * 2.302585092994045684)}; }
__device__ __forceinline__ double val(double x) { return x; }
__device__ __forceinline__ double val(Dd x) { return x.v; }
template <class S> __device__ __forceinline__ S sc(double x);
template <> __device__ __forceinline__ double sc<double>(double x) { return x; }
template <> __device__ __forceinline__ Dd sc<Dd>(double x) { return Dd{x, 0.0}; }

// Workspace rows of one slot (in units of ld).  N = K + 1.
struct WsLayout {
  int N, K;
  __host__ __device__ int phi() const { return 0; }
  __host__ __device__ int ynew() const { return N; }
  __host__ __device__ int f1() const { return 2 * N; }
  __host__ __device__ int fs() const { return 3 * N; }
  __host__ __device__ int u(int i) const { return (4 + i) * N; }      // i = 0..5 (stages)
  __host__ __device__ int ys() const { return 10 * N; }
  __host__ __device__ int ah() const { return 11 * N; }
  __host__ __device__ int aw() const { return 12 * N; }
  __host__ __device__ int br() const { return 13 * N; }
  __host__ __device__ int conc() const { return 14 * N; }
  __host__ __device__ int wdot() const { return 14 * N + K; }
  __host__ __device__ int hrt() const { return 14 * N + 2 * K; }
  __host__ __device__ int cpr() const { return 14 * N + 3 * K; }
  __host__ __device__ int gibbs() const { return 14 * N + 4 * K; }
  __host__ __device__ int gb() const { return 14 * N + 5 * K; }
  __host__ __device__ int tb() const { return 14 * N + 6 * K; }
  __host__ __device__ int jac() const { return 14 * N + 7 * K; }
  __host__ __device__ int lu() const { return 14 * N + 7 * K + N * N; }
  __host__ __device__ int total() const { return 14 * N + 7 * K + 2 * N * N; }
};

// NASA-7 thermo of every species at T: hRT, cpR and g = s/R - h/(RT) into the
// workspace.  Returns sum_k C_k dcp_k/dT / R when conc is given (for dD/dT).
__device__ __forceinline__ double thermo(const MechView& M, double T, Lane hrt, Lane cpr,
                                         Lane gib, Lane conc, bool with_dcp) {
  const double lnT = log(T), iT = 1.0 / T;
  double sdcp = 0.0;
  for (int k = 0; k < M.K; ++k) {
    const double* c = M.nasa + 15 * k;
    const bool lo = T < c[0];
    const double a0 = lo ? c[1] : c[8], a1 = lo ? c[2] : c[9], a2 = lo ? c[3] : c[10],
                 a3 = lo ? c[4] : c[11], a4 = lo ? c[5] : c[12], a5 = lo ? c[6] : c[13],
                 a6 = lo ? c[7] : c[14];
    const double cp = a0 + T * (a1 + T * (a2 + T * (a3 + T * a4)));
    const double h = a0 + T * (a1 * 0.5 + T * (a2 * (1.0 / 3.0) + T * (a3 * 0.25 + T * a4 * 0.2))) + a5 * iT;
    const double s = a0 * lnT + T * (a1 + T * (a2 * 0.5 + T * (a3 * (1.0 / 3.0) + T * a4 * 0.25))) + a6;
    hrt[k] = h;
    cpr[k] = cp;
    gib[k] = s - h;
    if (with_dcp) sdcp += conc[k] * (a1 + T * (2.0 * a2 + T * (3.0 * a3 + T * 4.0 * a4)));
  }
  return sdcp;
}

// Rate data of one reaction at (T, C).
template <class S>
struct RateOutT {
  S q;        // rate of progress
  S kf_rf;    // k * prod C^nu'
  S kr_rr;    // k_r * prod C^nu''
  S kf;       // effective forward rate constant
  S kr;       // reverse rate constant
  S dlnk_dT;  // d ln k / dT at fixed C
  S dlnKc_dT; // d ln K_c / dT
  S beta;     // d q / d[M] (0 for elementary reactions)
};
using RateOut = RateOutT<double>;

// The per-reaction fields reaction_rate reads, loaded in one go so that a
// loop over reactions can fetch the next reaction's record while it works on
// the current one.
struct RxnRec {
  int type, nr, np, e0, e1, fo;
  int sp[6], nu[6];   // all six slots (unused ones hold 0)
  double lnA, b, th, dnu;
};

__device__ __forceinline__ RxnRec load_rxn(const MechView& M, int j, const double* __restrict__ lnA_over) {
  const int32_t* info = M.rinfo + 8 * j;
  const int32_t* sp = M.rspec + 6 * j;
  const int32_t* nu = M.rnu + 6 * j;
  const double* ar = M.arr + 4 * j;
  RxnRec r;
  r.type = info[0];
  r.nr = info[1];
  r.np = info[2];
  r.e0 = info[3];
  r.e1 = info[4];
  r.fo = info[5];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    r.sp[q] = sp[q];
    r.nu[q] = nu[q];
  }
  r.lnA = lnA_over ? lnA_over[M.rorig[j]] : ar[0];
  r.b = ar[1];
  r.th = ar[2];
  r.dnu = ar[3];
  return r;
}

// SIDE < MAX_SIDE: every reaction of the call has at most SIDE species on
// each side, and slots past SIDE are neither read nor used (the caller checks
// this for the whole wavefront; the result is the same as with MAX_SIDE).
template <class S, int SIDE = MAX_SIDE>
__device__ __forceinline__ RateOutT<S> reaction_rate(const MechView& M, const RxnRec& R, S T, S lnT, S iT,
                                                     S ctot, LaneT<S> conc, LaneT<S> gib,
                                                     LaneT<S> hrt, bool want_deriv) {
  int spv[6], nuv[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    spv[q] = R.sp[q];
    nuv[q] = R.nu[q];
  }
  const int type = R.type, nr = R.nr, np = R.np;
  const double lnA = R.lnA, b = R.b, th = R.th, dnu = R.dnu;
  S cq[6], gq[6], hq[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const bool used = (q % 3) < SIDE;
    cq[q] = used ? conc[spv[q]] : sc<S>(0.0);
    gq[q] = used ? gib[spv[q]] : sc<S>(0.0);
    hq[q] = (used && want_deriv) ? hrt[spv[q]] : sc<S>(0.0);
  }
  const S lnkinf = lnA + b * lnT - th * iT;
  const S kinf = exp(lnkinf);
  const S dlnkinf = (b + th * iT) * iT;
  S k = kinf, dlnk = dlnkinf, dk_dM = sc<S>(0.0);
  if (type != RX_ELEM) {
    // [M] = sum C + sum (alpha - 1) C over the listed efficiencies: the first
    // four unrolled - their table entries, then their concentrations, each
    // group issued together - any further ones in a loop
    S Mc = ctot;
    const int e0 = R.e0, e1 = R.e1;
    int ei[4];
    double ea[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = (e0 + t < e1) ? e0 + t : e0;   // in the table, or its padding when e0 == e1
      ei[t] = M.eff_idx[e];
      ea[t] = M.eff_am1[e];
    }
    S ec[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) ec[t] = conc[ei[t]];
#pragma unroll
    for (int t = 0; t < 4; ++t)
      if (e0 + t < e1) Mc += ea[t] * ec[t];
    for (int e = e0 + 4; e < e1; ++e) Mc += M.eff_am1[e] * conc[M.eff_idx[e]];
    if (type == RX_THIRD) {
      k = kinf * Mc;
      dk_dM = kinf;
    } else {
      const double* f = M.fo + 8 * R.fo;
      const S lnk0 = lnA + f[0] + f[1] * lnT - f[2] * iT;
      const S k0 = exp(lnk0);
      const S dlnk0 = (f[1] + f[2] * iT) * iT;
      const S Pr = k0 * Mc / kinf;
      S F = sc<S>(1.0), dlnF_dlnPr = sc<S>(0.0), dlnF_dT_fc = sc<S>(0.0);
      if (type == RX_TROE) {
        const double a = f[3], T3 = f[4], T1 = f[5], T2 = f[6];
        const S e3 = exp(-T * (1.0 / T3)), e1x = exp(-T * (1.0 / T1));
        const S e2 = T2 > 0.0 ? exp(-T2 * iT) : sc<S>(0.0);
        const S Fc = (1.0 - a) * e3 + a * e1x + e2;
        const S lFc = log10(Fc);
        const S c = -0.4 - 0.67 * lFc, n = 0.75 - 1.27 * lFc;
        const bool tiny = !(val(Pr) > 1e-300);
        const S lPr = tiny ? sc<S>(-300.0) : log10(Pr);
        const S x = lPr + c, den = n - 0.14 * x, y = x / den;
        const S opy = 1.0 + y * y;
        const S L = lFc / opy;
        F = exp(L * 2.302585092994045684);
        if (want_deriv) {
          const S dLdy = -2.0 * lFc * y / (opy * opy);
          const S dydx = n / (den * den), dydn = -x / (den * den);
          dlnF_dlnPr = tiny ? sc<S>(0.0) : dLdy * dydx;
          const S dLdlFc = 1.0 / opy + dLdy * (dydx * -0.67 + dydn * -1.27);
          const S dFc = -(1.0 - a) * (1.0 / T3) * e3 - a * (1.0 / T1) * e1x +
                        (T2 > 0.0 ? T2 * iT * iT * e2 : sc<S>(0.0));
          dlnF_dT_fc = dLdlFc * dFc / Fc;
        }
      }
      const S pfac = Pr / (1.0 + Pr);
      k = kinf * pfac * F;
      if (want_deriv) {
        const S phi = 1.0 / (1.0 + Pr) + dlnF_dlnPr;   // d ln k / d ln Pr
        dk_dM = k * phi / Mc;
        dlnk = dlnkinf + phi * (dlnk0 - dlnkinf) + dlnF_dT_fc;
      }
    }
  }
  // sums over the sides (reactants, then products, in slot order) and the
  // mass-action products; an unused slot contributes nothing.  Branch-free:
  // an unused slot's coefficient is 0 and its factor 1 (its species is a
  // valid one, so the terms it adds are exact zeros), and each power is
  // selected from C, C^2 and C^3 - per-lane branches here cost more than the
  // arithmetic they skip
  S sg = sc<S>(0.0), sh = sc<S>(0.0);
  S rf = sc<S>(1.0), rr = sc<S>(1.0);
#pragma unroll
  for (int i = 0; i < SIDE; ++i) {
    const bool on = i < nr;
    const double v = on ? (double)nuv[i] : 0.0;
    sg -= v * gq[i];
    if (want_deriv) sh -= v * hq[i];
    const S cs = cq[i], c2 = cs * cs, c3 = c2 * cs;
    const S pw = (nuv[i] == 1) ? cs : (nuv[i] == 2 ? c2 : c3);
    rf = on ? rf * pw : rf;
  }
#pragma unroll
  for (int i = 0; i < SIDE; ++i) {
    const bool on = i < np;
    const double v = on ? (double)nuv[3 + i] : 0.0;
    sg += v * gq[3 + i];
    if (want_deriv) sh += v * hq[3 + i];
    const S cs = cq[3 + i], c2 = cs * cs, c3 = c2 * cs;
    const S pw = (nuv[3 + i] == 1) ? cs : (nuv[3 + i] == 2 ? c2 : c3);
    rr = on ? rr * pw : rr;
  }
  const S lnKc = sg + dnu * log(PATM / (RU * T));
  const S kr = k * exp(-lnKc);
  RateOutT<S> o;
  o.kf = k;
  o.kr = kr;
  o.kf_rf = k * rf;
  o.kr_rr = kr * rr;
  o.q = o.kf_rf - o.kr_rr;
  o.dlnk_dT = dlnk;
  o.dlnKc_dT = (sh - dnu) * iT;
  o.beta = dk_dM * (rf - rr * exp(-lnKc));
  return o;
}

// The same for reaction j, its record loaded here.
template <class S>
__device__ __forceinline__ RateOutT<S> reaction_rate(const MechView& M, int j, S T, S lnT, S iT,
                                                     S ctot, LaneT<S> conc, LaneT<S> gib,
                                                     LaneT<S> hrt, const double* __restrict__ lnA_over,
                                                     bool want_deriv) {
  return reaction_rate(M, load_rxn(M, j, lnA_over), T, lnT, iT, ctot, conc, gib, hrt, want_deriv);
}

// Concentrations from Phi; returns the sum over all K species.
__device__ __forceinline__ double concentrations(const MechView& M, double P, Lane phi, Lane conc) {
  const double V = phi[1], iV = 1.0 / V;
  double s = 0.0;
  for (int k = 0; k < M.K - 1; ++k) {
    const double c = phi[2 + k] * iV;
    conc[k] = c;
    s += c;
  }
  const double cb = P / (RU * phi[0]) - s;
  conc[M.K - 1] = cb;
  return s + cb;
}

// f(Phi) into f.  ws supplies conc, wdot, hrt, cpr, gibbs.
__device__ void eval_rhs(const MechView& M, double P, Lane phi, Lane f, Lane conc, Lane wdot,
                         Lane hrt, Lane cpr, Lane gib, const double* __restrict__ lnA) {
  const int K = M.K;
  const double T = phi[0], V = phi[1];
  const double lnT = log(T), iT = 1.0 / T;
  const double ctot = concentrations(M, P, phi, conc);
  thermo(M, T, hrt, cpr, gib, conc, false);
  for (int k = 0; k < K; ++k) wdot[k] = 0.0;
  for (int j = 0; j < M.Nr; ++j) {
    const RateOut r = reaction_rate(M, j, T, lnT, iT, ctot, conc, gib, hrt, lnA, false);
    const int32_t* info = M.rinfo + 8 * j;
    const int32_t* sp = M.rspec + 6 * j;
    const int32_t* nu = M.rnu + 6 * j;
    for (int i = 0; i < info[1]; ++i) wdot[sp[i]] -= nu[i] * r.q;
    for (int i = 0; i < info[2]; ++i) wdot[sp[3 + i]] += nu[3 + i] * r.q;
  }
  double num = 0.0, den = 0.0, ws = 0.0;
  for (int k = 0; k < K; ++k) {
    const double w = wdot[k];
    num += hrt[k] * w;
    den += conc[k] * cpr[k];
    ws += w;
  }
  // H_k = hRT_k R T, cp_k = cpR_k R
  const double Tdot = -(num * T) / den;
  f[0] = Tdot;
  f[1] = V * (Tdot * iT + (RU * T / P) * ws);
  for (int k = 0; k < K - 1; ++k) f[2 + k] = V * wdot[k];
}

// f(Phi) into f and the dense Jacobian into J (row-major, element (i, c) at
// J[i * N + c]).  Uses the workspace rows of L.
__device__ void eval_rhs_jac(const MechView& M, double P, Lane phi, Lane f, Lane J, const WsLayout& L,
                             double* __restrict__ base, int64_t ld, const double* __restrict__ lnA) {
  const int K = M.K, N = M.N;
  Lane conc{base + L.conc() * ld, ld}, wdot{base + L.wdot() * ld, ld};
  Lane hrt{base + L.hrt() * ld, ld}, cpr{base + L.cpr() * ld, ld}, gib{base + L.gibbs() * ld, ld};
  Lane gb{base + L.gb() * ld, ld}, tb{base + L.tb() * ld, ld}, br{base + L.br() * ld, ld};
  Lane ah{base + L.ah() * ld, ld}, aw{base + L.aw() * ld, ld};
  const double T = phi[0], V = phi[1], iV = 1.0 / V;
  const double lnT = log(T), iT = 1.0 / T;
  const double ctot = concentrations(M, P, phi, conc);
  const double sdcp = thermo(M, T, hrt, cpr, gib, conc, true);
  // G (species block at fixed T, in C coordinates) accumulates in place:
  //   row k < K-1 -> J row k+2, columns m+2 for m < K-1 and column 0 for g_k;
  //   row K-1     -> br; column K-1 of every row -> gb; uniform third-body part -> tb.
  for (int k = 0; k < K; ++k) {
    wdot[k] = 0.0;
    gb[k] = 0.0;
    tb[k] = 0.0;
  }
  for (int k = 0; k < K - 1; ++k) {
    Lane row{J.p + (int64_t)(k + 2) * N * ld, ld};
    for (int c = 0; c < N; ++c) row[c] = 0.0;
  }
  for (int c = 0; c < N; ++c) br[c] = 0.0;
  for (int j = 0; j < M.Nr; ++j) {
    const RateOut r = reaction_rate(M, j, T, lnT, iT, ctot, conc, gib, hrt, lnA, true);
    const int32_t* info = M.rinfo + 8 * j;
    const int32_t* sp = M.rspec + 6 * j;
    const int32_t* nu = M.rnu + 6 * j;
    const int nr = info[1], np = info[2];
    const double dqdT = r.dlnk_dT * r.q + r.kr_rr * r.dlnKc_dT;
    // d q / d C_m of the participants (species part)
    double dq[6];
    int ms[6];
    int nm = 0;
    for (int i = 0; i < nr; ++i) {
      const int s = sp[i];
      double d = r.kf;
      for (int l = 0; l < nr; ++l) {
        const double c = conc[sp[l]];
        const int v = (l == i) ? nu[l] - 1 : nu[l];
        if (v >= 1) d *= c;
        if (v >= 2) d *= c;
        if (v >= 3) d *= c;
      }
      ms[nm] = s;
      dq[nm++] = d * nu[i];
    }
    for (int i = 0; i < np; ++i) {
      const int s = sp[3 + i];
      double d = r.kr;
      for (int l = 0; l < np; ++l) {
        const double c = conc[sp[3 + l]];
        const int v = (l == i) ? nu[3 + l] - 1 : nu[3 + l];
        if (v >= 1) d *= c;
        if (v >= 2) d *= c;
        if (v >= 3) d *= c;
      }
      ms[nm] = s;
      dq[nm++] = -d * nu[3 + i];
    }
    for (int side = 0; side < 2; ++side) {
      const int cnt = side ? np : nr;
      for (int i = 0; i < cnt; ++i) {
        const int k = sp[3 * side + i];
        const double vk = side ? (double)nu[3 + i] : -(double)nu[i];
        wdot[k] += vk * r.q;
        const bool bath = (k == K - 1);
        double* rowp = bath ? br.p : J.p + (int64_t)(k + 2) * N * ld;
        Lane row{rowp, ld};
        row[0] += vk * dqdT;
        for (int t = 0; t < nm; ++t) {
          const int m = ms[t];
          if (m == K - 1)
            gb[k] += vk * dq[t];
          else
            row[m + 2] += vk * dq[t];
        }
        if (info[0] != RX_ELEM) {
          tb[k] += vk * r.beta;
          for (int e = info[3]; e < info[4]; ++e) {
            const int m = M.eff_idx[e];
            const double d = vk * M.eff_am1[e] * r.beta;
            if (m == K - 1)
              gb[k] += d;
            else
              row[m + 2] += d;
          }
        }
      }
    }
  }
  // Phi coordinates, and the reductions the T and V rows need.
  const double dCb_dT = -P / (RU * T * T);
  for (int c = 0; c < N; ++c) {
    ah[c] = 0.0;
    aw[c] = 0.0;
  }
  double num = 0.0, den = 0.0, wsum = 0.0, wcp = 0.0;
  for (int k = 0; k < K; ++k) {
    const bool bath = (k == K - 1);
    Lane row{bath ? br.p : J.p + (int64_t)(k + 2) * N * ld, ld};
    const double t = tb[k];
    const double gbk = gb[k] + t;
    const double Hk = hrt[k] * RU * T;
    const double wk = wdot[k];
    num += Hk * wk;
    den += conc[k] * cpr[k] * RU;
    wsum += wk;
    wcp += wk * cpr[k] * RU;
    double dvs = 0.0;
    for (int m = 0; m < K - 1; ++m) {
      const double Gkm = row[m + 2] + t;
      const double dn = Gkm - gbk;              // V * d wdot_k / d n_m
      dvs -= dn * conc[m];                      // V * d wdot_k / d V
      ah[m + 2] += Hk * dn * iV;
      aw[m + 2] += dn * iV;
      if (!bath) row[m + 2] = dn;
    }
    const double dwdT = row[0] + gbk * dCb_dT;
    const double dwdV = dvs * iV;
    ah[0] += Hk * dwdT;
    aw[0] += dwdT;
    ah[1] += Hk * dwdV;
    aw[1] += dwdV;
    if (!bath) {
      row[0] = V * dwdT;
      row[1] = wk + dvs;
    }
  }
  const double Tdot = -num / den;
  const double cpb = cpr[K - 1] * RU;
  // dD/dPhi (D = sum C_k cp_k)
  double dD_T = sdcp * RU + cpb * dCb_dT;
  double dD_V = 0.0;
  for (int m = 0; m < K - 1; ++m) dD_V += (cpb - cpr[m] * RU) * conc[m];
  dD_V *= iV;
  Lane rowT{J.p, ld}, rowV{J.p + (int64_t)N * ld, ld};
  const double RTP = RU * T / P;
  const double dTdot_T = -(ah[0] + wcp) / den - Tdot * dD_T / den;
  const double dTdot_V = -ah[1] / den - Tdot * dD_V / den;
  rowT[0] = dTdot_T;
  rowT[1] = dTdot_V;
  rowV[0] = V * dTdot_T * iT - V * Tdot * iT * iT + (RU * V / P) * wsum + RTP * V * aw[0];
  rowV[1] = Tdot * iT + V * dTdot_V * iT + RTP * wsum + RTP * V * aw[1];
  for (int m = 0; m < K - 1; ++m) {
    const double dD_n = (cpr[m] * RU - cpb) * iV;
    const double dTd = -ah[m + 2] / den - Tdot * dD_n / den;
    rowT[m + 2] = dTd;
    rowV[m + 2] = V * dTd * iT + RTP * V * aw[m + 2];
  }
  f[0] = Tdot;
  f[1] = V * (Tdot * iT + RTP * wsum);
  for (int k = 0; k < K - 1; ++k) f[2 + k] = V * wdot[k];
}

}  // namespace chem
