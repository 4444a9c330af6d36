// One wavefront per cell ("team" kernels).
//
// Layout inside a wavefront (64 lanes, N = K + 1 <= 64):
//   * element i of every state-sized vector (Phi, f, ...) lives in lane i, one
//     register each; the stage vectors u_1..u_s of the integrator sit in a
//     small LDS area, each lane holding (and reading back) its own element;
//   * reactions are spread over lanes (reaction j on lane j mod 64); their
//     contributions to the production rates and to the Jacobian are scattered
//     into LDS with FP64 LDS atomics, then the chain rule through C(Phi) is
//     applied in one row-parallel and one column-parallel pass;
//   * the LU of M = I/(h gamma) - J loads row i into lane i's registers and
//     eliminates with implicit partial pivoting (rows stay in their lanes, the
//     pivot order is recorded; the pivot search is an exact wave max over the
//     IEEE words of |a| plus a ballot, the pivot row is broadcast by
//     v_readlane); the factors go back to LDS in pivot order for the
//     triangular solves;
//   * every controller decision is uniform over the wavefront.
// Work-groups are one wavefront, so a work-group barrier is a wave barrier.
#pragma once
#include <hip/hip_runtime.h>

#include "kinetics.h"
#include "mech.h"
#include "methods.h"

namespace chem {

__device__ __forceinline__ void wsync() { __syncthreads(); }

// Value of lane `src` (wave-uniform) through two v_readlane.
__device__ __forceinline__ double bcast(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

// Value of lane `src` for a per-lane source (LDS crossbar).
__device__ __forceinline__ double gather(double v, int src) { return __shfl(v, src, 64); }

// Cross-lane move inside 16-lane rows (DPP); CTRL is the DPP control word.
// The controls used here permute lanes inside a row, so every lane has a
// source (the bound-control setting never applies).  A move without an "old"
// operand lets the compiler fold it into the consuming ALU instruction.
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
constexpr int DPP_QUAD_1032 = 0xB1;   // quad_perm [1,0,3,2]
constexpr int DPP_QUAD_2301 = 0x4E;   // quad_perm [2,3,0,1]
constexpr int DPP_ROW_HALF_MIRROR = 0x141;
constexpr int DPP_ROW_MIRROR = 0x140;

// Sum over the 64 lanes (all lanes must be active), the same value in every
// lane: pairs, quads, octets and rows by DPP, then the four rows by readlane.
// The association order is fixed, so the result is deterministic.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp<DPP_QUAD_1032>(v);
  v += dpp<DPP_QUAD_2301>(v);
  v += dpp<DPP_ROW_HALF_MIRROR>(v);
  v += dpp<DPP_ROW_MIRROR>(v);
  return (bcast(v, 0) + bcast(v, 16)) + (bcast(v, 32) + bcast(v, 48));
}

__device__ __forceinline__ Dd wave_sum(Dd v) { return Dd{wave_sum(v.v), wave_sum(v.d)}; }
__device__ __forceinline__ Dd bcast(Dd v, int src) { return Dd{bcast(v.v, src), bcast(v.d, src)}; }

// LDS accumulation (FP64 LDS atomics); a dual number adds both components.
__device__ __forceinline__ void lds_add(double* p, double v) { atomicAdd(p, v); }
__device__ __forceinline__ void lds_add(Dd* p, Dd v) {
  atomicAdd(&p->v, v.v);
  atomicAdd(&p->d, v.d);
}

__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp<DPP_QUAD_1032>(v));
  v = fmax(v, dpp<DPP_QUAD_2301>(v));
  v = fmax(v, dpp<DPP_ROW_HALF_MIRROR>(v));
  v = fmax(v, dpp<DPP_ROW_MIRROR>(v));
  return fmax(fmax(bcast(v, 0), bcast(v, 16)), fmax(bcast(v, 32), bcast(v, 48)));
}

// Per-wavefront LDS scratch.  ldj = N + 1 (odd row stride).
template <class S>
struct TeamLdsT {
  S* J;      // [N][ldj]   Jacobian being assembled / factors of M
  S* brow;   // [ldj]      bath-gas row of d wdot / d Phi
  S* conc;   // [64]
  S* hrt;    // [64]
  S* cpr;    // [64]
  S* gib;    // [64]
  S* wdot;   // [64]
  S* gb;     // [64]       G column of the bath gas
  S* tb;     // [64]       uniform third-body part per row
  S* dwdT;   // [64]
  S* dwdV;   // [64]
  S* vec;    // [64]       staging of a lane-distributed vector
  S* ust;    // [MAX_STAGES][64] stage vectors of the integrator (bind() layout only)
  int* plane;            // [64]
  // Two layouts.  bind(): dwdT and dwdV first, then the matrix, brow, the
  // other vectors and the stage area, one block of doubles(N) doubles whose
  // last 32 hold plane.
  // bind2(): the matrix at Jb and brow plus every vector at Vb (the adjoint's
  // two matrix views share one vector block).
  // Elements of S besides the matrix: brow and ten 64-entry vectors.
  static __host__ __device__ size_t vec_elems(int N) { return (size_t)(N + 1) + 10 * 64; }
  static __host__ __device__ size_t doubles(int N) {
    return ((size_t)N * (N + 1) + vec_elems(N) + MAX_STAGES * 64) * (sizeof(S) / sizeof(double)) + 32;
  }
  __device__ void bind2(S* Jb, S* Vb, int* pl, int N) {
    J = Jb;
    brow = Vb;
    conc = brow + (N + 1);
    hrt = conc + 64;
    cpr = hrt + 64;
    gib = cpr + 64;
    wdot = gib + 64;
    gb = wdot + 64;
    tb = gb + 64;
    dwdT = tb + 64;
    dwdV = dwdT + 64;
    vec = dwdV + 64;
    ust = nullptr;
    plane = pl;
  }
  __device__ void bind(double* base, int N) {
    S* b = (S*)base;
    dwdT = b;
    dwdV = b + 64;
    J = b + 128;
    brow = J + (size_t)N * (N + 1);
    conc = brow + (N + 1);
    hrt = conc + 64;
    cpr = hrt + 64;
    gib = cpr + 64;
    wdot = gib + 64;
    gb = wdot + 64;
    tb = gb + 64;
    vec = tb + 64;
    ust = vec + 64;
    plane = (int*)(base + doubles(N) - 32);
  }
};
using TeamLds = TeamLdsT<double>;

// Lane-distributed LDS view with a fixed stride, to reuse reaction_rate().
struct LdsLane {
  double* p;
  __device__ __forceinline__ double& operator[](int i) const { return p[i]; }
};

// Concentrations and thermo of the state y (lane-distributed, element i in
// lane i).  Returns (T, V, sum C) uniform; fills conc/hrt/cpr/gib in LDS.
// sdcp (optional) receives sum_k C_k dcp_k/dT / R.
template <class S>
__device__ __forceinline__ void team_state(const MechView& M, double P, S y, TeamLdsT<S>& L, S& T,
                                           S& V, S& ctot, S* sdcp) {
  const int lane = threadIdx.x;
  const int K = M.K;
  T = bcast(y, 0);
  V = bcast(y, 1);
  L.vec[lane] = y;
  wsync();
  S c = sc<S>(0.0);
  if (lane < K - 1) c = L.vec[lane + 2] / V;
  const S s = wave_sum(c);
  if (lane == K - 1) c = P / (RU * T) - s;
  ctot = wave_sum(c);
  if (lane < K) L.conc[lane] = c;
  S dcp = sc<S>(0.0);
  if (lane < K) {
    // all fifteen coefficients read together, then the range selected
    double cf[15];
#pragma unroll
    for (int i = 0; i < 15; ++i) cf[i] = M.nasa[15 * lane + i];
    const bool lo = val(T) < cf[0];
    const double a0 = lo ? cf[1] : cf[8], a1 = lo ? cf[2] : cf[9], a2 = lo ? cf[3] : cf[10],
                 a3 = lo ? cf[4] : cf[11], a4 = lo ? cf[5] : cf[12], a5 = lo ? cf[6] : cf[13],
                 a6 = lo ? cf[7] : cf[14];
    const S lnT = log(T), iT = 1.0 / T;
    const S cp = a0 + T * (a1 + T * (a2 + T * (a3 + T * a4)));
    const S h = a0 + T * (a1 * 0.5 + T * (a2 * (1.0 / 3.0) + T * (a3 * 0.25 + T * a4 * 0.2))) + a5 * iT;
    const S sr = a0 * lnT + T * (a1 + T * (a2 * 0.5 + T * (a3 * (1.0 / 3.0) + T * a4 * 0.25))) + a6;
    L.hrt[lane] = h;
    L.cpr[lane] = cp;
    L.gib[lane] = sr - h;
    if (sdcp) dcp = c * (a1 + T * (2.0 * a2 + T * (3.0 * a3 + T * 4.0 * a4)));
  }
  if (sdcp) *sdcp = wave_sum(dcp);
  wsync();
}

// One reaction of the f loop: its rate and its scatter into wdot, slots up to
// SIDE per side.  An unused slot adds to this lane's own dummy cell (dwdT is
// used only by the Jacobian), so no per-lane branch.
template <int SIDE>
__device__ __forceinline__ void team_rhs_reaction(const MechView& M, const RxnRec& R, double T, double lnT,
                                                  double iT, double ctot, TeamLds& L) {
  const RateOut r = reaction_rate<double, SIDE>(M, R, T, lnT, iT, ctot, Lane{L.conc, 1}, Lane{L.gib, 1},
                                                Lane{L.hrt, 1}, false);
  double* const dummy = L.dwdT + threadIdx.x;
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    if (q % 3 >= SIDE) continue;
    const int sq = R.sp[q], nq = R.nu[q];
    const bool on = (q < 3) ? (q < R.nr) : (q - 3 < R.np);
    atomicAdd(on ? &L.wdot[sq] : dummy, (q < 3 ? -nq : nq) * r.q);
  }
}

// f(y) for lane-distributed y; returns f_i in lane i.
__device__ __forceinline__ double team_rhs(const MechView& M, double P, double y, TeamLds& L,
                           const double* __restrict__ lnA) {
  const int lane = threadIdx.x;
  const int K = M.K, N = M.N;
  double T, V, ctot;
  team_state<double>(M, P, y, L, T, V, ctot, nullptr);
  if (lane < K) L.wdot[lane] = 0.0;
  wsync();
  const double lnT = log(T), iT = 1.0 / T;
  // the next reaction's record is fetched while this one is worked on
  const int Nr = M.Nr;
  RxnRec nx = load_rxn(M, lane < Nr ? lane : Nr - 1, lnA);
  for (int j = lane; j < Nr; j += 64) {
    const RxnRec R = nx;
    nx = load_rxn(M, j + 64 < Nr ? j + 64 : j, lnA);
    // most passes hold two-by-two reactions only: then the third slot of each
    // side is left out (a wave-uniform choice, once per pass)
    if (__all(R.nr <= 2 && R.np <= 2))
      team_rhs_reaction<2>(M, R, T, lnT, iT, ctot, L);
    else
      team_rhs_reaction<MAX_SIDE>(M, R, T, lnT, iT, ctot, L);
  }
  wsync();
  double w = 0.0, num = 0.0, den = 0.0;
  if (lane < K) {
    w = L.wdot[lane];
    num = L.hrt[lane] * w;
    den = L.conc[lane] * L.cpr[lane];
  }
  num = wave_sum(num);
  den = wave_sum(den);
  const double ws = wave_sum(w);
  const double Tdot = -(num * T) / den;
  double f = 0.0;
  if (lane == 0) f = Tdot;
  if (lane == 1) f = V * (Tdot * iT + (RU * T / P) * ws);
  if (lane >= 2 && lane < N) f = V * L.wdot[lane - 2];
  wsync();
  return f;
}

// One reaction of the Jacobian loop: its rate with derivatives, d q / d(T, C)
// and the scatter into the rows of G, slots up to SIDE per side.  Unused
// slots send their updates to this lane's own dummy cell (dwdT is written
// only after the reaction loop).
template <class S, int SIDE>
__device__ __forceinline__ void team_jac_reaction(const MechView& M, const RxnRec& R, S T, S lnT, S iT,
                                                  S ctot, TeamLdsT<S>& L, int K, int ldj) {
  const RateOutT<S> r = reaction_rate<S, SIDE>(M, R, T, lnT, iT, ctot, LaneT<S>{L.conc, 1},
                                               LaneT<S>{L.gib, 1}, LaneT<S>{L.hrt, 1}, true);
  const int nr = R.nr, np = R.np;
  const S dqdT = r.dlnk_dT * r.q + r.kr_rr * r.dlnKc_dT;
  // participant slots 0..2 (reactants) and 3..5 (products), with compile-time
  // bounds: an unused slot has coefficient 0, and its updates go to this
  // lane's own dummy cell (dwdT is written only after this loop)
  S* const dummy = L.dwdT + threadIdx.x;
  int ks[6], nus[6];
  bool on[6];
  S cs[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    on[q] = (q % 3 < SIDE) && ((q < 3) ? (q < nr) : (q - 3 < np));
    ks[q] = R.sp[q];         // unused slots hold species 0 and coefficient 0
    nus[q] = R.nu[q];
    cs[q] = (q % 3 < SIDE) ? L.conc[ks[q]] : sc<S>(0.0);
  }
  // d q / d C of slot q: the mass-action product of its side with the power
  // of C_q lowered by one (the same multiplications, in the same order, as a
  // loop over the side's species)
  S dq[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const int s0 = q < 3 ? 0 : 3;
    S d = (q < 3) ? r.kf : r.kr;
#pragma unroll
    for (int l = 0; l < SIDE; ++l) {
      const int v = (s0 + l == q) ? nus[s0 + l] - 1 : nus[s0 + l];
      const S c = cs[s0 + l];
      d = (v >= 1) ? d * c : d;
      d = (v >= 2) ? d * c : d;
      d = (v >= 3) ? d * c : d;
    }
    dq[q] = d * (double)(q < 3 ? nus[q] : -nus[q]);
  }
  // scatter into row k = ks[q] of G (T column, species columns, bath column)
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    if (q % 3 >= SIDE) continue;
    const int k = ks[q];
    const double vk = (q < 3) ? -(double)nus[q] : (double)nus[q];
    S* row = (k == K - 1) ? L.brow : L.J + (k + 2) * ldj;
    lds_add(on[q] ? &L.wdot[k] : dummy, vk * r.q);
    lds_add(on[q] ? &row[0] : dummy, vk * dqdT);
#pragma unroll
    for (int t = 0; t < 6; ++t) {
      if (t % 3 >= SIDE) continue;
      const int m = ks[t];
      S* dst = (m == K - 1) ? &L.gb[k] : &row[m + 2];
      lds_add((on[q] && on[t]) ? dst : dummy, vk * dq[t]);
    }
  }
  if (R.type != RX_ELEM) {
    // third body and falloff: the uniform [M] part and the efficiency
    // columns; the first four efficiencies are read together up front, any
    // further ones in a loop
    const int e0 = R.e0, e1 = R.e1;
    int em[4];
    double ea[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = (e0 + t < e1) ? e0 + t : e0;   // in the table, or its padding when e0 == e1
      em[t] = M.eff_idx[e];
      ea[t] = M.eff_am1[e];
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      if (q % 3 >= SIDE) continue;
      const int k = ks[q];
      const double vk = (q < 3) ? -(double)nus[q] : (double)nus[q];
      S* row = (k == K - 1) ? L.brow : L.J + (k + 2) * ldj;
      lds_add(on[q] ? &L.tb[k] : dummy, vk * r.beta);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        S* dst = (em[t] == K - 1) ? &L.gb[k] : &row[em[t] + 2];
        lds_add((on[q] && e0 + t < e1) ? dst : dummy, (vk * ea[t]) * r.beta);
      }
      for (int e = e0 + 4; e < e1; ++e) {
        const int m = M.eff_idx[e];
        lds_add(on[q] ? ((m == K - 1) ? &L.gb[k] : &row[m + 2]) : dummy, (vk * M.eff_am1[e]) * r.beta);
      }
    }
  }
}

// f(y) and the Jacobian, assembled in L.J (row i at L.J[i*(N+1)]).  S is
// double, or the dual type for a directional derivative of f and J.
template <class S>
__device__ __forceinline__ S team_rhs_jac(const MechView& M, double P, S y, TeamLdsT<S>& L,
                          const double* __restrict__ lnA) {
  const int lane = threadIdx.x;
  const int K = M.K, N = M.N, ldj = N + 1;
  S T, V, ctot, sdcp;
  team_state(M, P, y, L, T, V, ctot, &sdcp);
  const S lnT = log(T), iT = 1.0 / T, iV = 1.0 / V;
  // clear: column `lane` of every species row, the bath row and the per-row sums
  if (lane < N) {
    for (int k = 0; k < K - 1; ++k) L.J[(k + 2) * ldj + lane] = sc<S>(0.0);
    L.brow[lane] = sc<S>(0.0);
  }
  if (lane < K) {
    L.wdot[lane] = sc<S>(0.0);
    L.gb[lane] = sc<S>(0.0);
    L.tb[lane] = sc<S>(0.0);
  }
  wsync();
  const int Nr = M.Nr;
  RxnRec nx = load_rxn(M, lane < Nr ? lane : Nr - 1, lnA);   // fetched one reaction ahead
  for (int j = lane; j < Nr; j += 64) {
    const RxnRec R = nx;
    nx = load_rxn(M, j + 64 < Nr ? j + 64 : j, lnA);
    // most passes hold two-by-two reactions only: then the third slot of each
    // side is left out (a wave-uniform choice, once per pass)
    if (__all(R.nr <= 2 && R.np <= 2))
      team_jac_reaction<S, 2>(M, R, T, lnT, iT, ctot, L, K, ldj);
    else
      team_jac_reaction<S, MAX_SIDE>(M, R, T, lnT, iT, ctot, L, K, ldj);
  }
  wsync();
  // pass 1, row-parallel (lane k = species row): Phi coordinates of row k
  const S dCb_dT = -P / (RU * T * T);
  S num = sc<S>(0.0), den = sc<S>(0.0), wsum = sc<S>(0.0), wcp = sc<S>(0.0), dDV = sc<S>(0.0);
  if (lane < K) {
    const int k = lane;
    S* row = (k == K - 1) ? L.brow : L.J + (k + 2) * ldj;
    const S t = L.tb[k];
    const S gbk = L.gb[k] + t;
    const S wk = L.wdot[k];
    const S cpk = L.cpr[k] * RU;
    num = L.hrt[k] * RU * T * wk;
    den = L.conc[k] * cpk;
    wsum = wk;
    wcp = wk * cpk;
    S dvs = sc<S>(0.0);
    // unrolled so that several LDS loads are in flight (latency-bound otherwise)
#pragma unroll 8
    for (int m = 0; m < K - 1; ++m) {
      const S dn = row[m + 2] + t - gbk;
      dvs -= dn * L.conc[m];
      row[m + 2] = dn;
    }
    const S dwdT = row[0] + gbk * dCb_dT;
    L.dwdT[k] = dwdT;
    L.dwdV[k] = dvs * iV;
    if (k < K - 1) {
      row[0] = V * dwdT;
      row[1] = wk + dvs;
      dDV = (L.cpr[K - 1] - L.cpr[k]) * RU * L.conc[k];
    }
  }
  num = wave_sum(num);
  den = wave_sum(den);
  wsum = wave_sum(wsum);
  wcp = wave_sum(wcp);
  dDV = wave_sum(dDV) * iV;
  wsync();
  // pass 2, column-parallel (lane c = column): the T and V rows
  const S Tdot = -num / den;
  const S RTP = RU * T / P;
  if (lane < N) {
    const int c = lane;
    S ah = sc<S>(0.0), aw = sc<S>(0.0);
    // d wdot_k / d Phi_c: column c of row k for the species columns (per unit
    // n, so times 1/V), dwdT / dwdV for the T and V columns; one loop for all
    // lanes, the address chosen per lane
    const S* src = (c == 0) ? L.dwdT : L.dwdV;
    const S scale = (c >= 2) ? iV : sc<S>(1.0);
#pragma unroll 8
    for (int k = 0; k < K; ++k) {
      const S* row = (k == K - 1) ? L.brow : L.J + (k + 2) * ldj;
      const S d = ((c >= 2) ? row[c] : src[k]) * scale;
      ah += L.hrt[k] * RU * T * d;
      aw += d;
    }
    const S cpb = L.cpr[K - 1] * RU;
    S dD, dTd, dVd;
    if (c == 0) {
      dD = sdcp * RU + cpb * dCb_dT;
      dTd = -(ah + wcp) / den - Tdot * dD / den;
      dVd = V * dTd * iT - V * Tdot * iT * iT + (RU * V / P) * wsum + RTP * V * aw;
    } else if (c == 1) {
      dD = dDV;
      dTd = -ah / den - Tdot * dD / den;
      dVd = Tdot * iT + V * dTd * iT + RTP * wsum + RTP * V * aw;
    } else {
      dD = (L.cpr[c - 2] * RU - cpb) * iV;
      dTd = -ah / den - Tdot * dD / den;
      dVd = V * dTd * iT + RTP * V * aw;
    }
    L.J[c] = dTd;
    L.J[ldj + c] = dVd;
  }
  S f = sc<S>(0.0);
  if (lane == 0) f = Tdot;
  if (lane == 1) f = V * (Tdot * iT + RTP * wsum);
  if (lane >= 2 && lane < N) f = V * L.wdot[lane - 2];
  wsync();
  return f;
}

// Largest of a non-negative 32-bit key over the 64 lanes: the row maximum by
// DPP inside each 16-lane row (every lane of a row ends with it), then the
// last lane of row 0 into row 1 and of row 2 into row 3 (row_bcast:15, rows 1
// and 3 written), then the last lane of row 1 into rows 2 and 3
// (row_bcast:31), so that lane 63 holds the wave maximum: one v_readlane
// instead of four and a scalar tree.
__device__ __forceinline__ unsigned umax32(unsigned a, unsigned b) { return a > b ? a : b; }
template <int CTRL>
__device__ __forceinline__ unsigned dpp32(unsigned v) {
  return (unsigned)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, true);
}
constexpr int DPP_ROW_BCAST15 = 0x142;
constexpr int DPP_ROW_BCAST31 = 0x143;
__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
  v = umax32(v, dpp32<DPP_QUAD_1032>(v));
  v = umax32(v, dpp32<DPP_QUAD_2301>(v));
  v = umax32(v, dpp32<DPP_ROW_HALF_MIRROR>(v));
  v = umax32(v, dpp32<DPP_ROW_MIRROR>(v));
  // rows not written by a broadcast keep their own value (the "old" operand)
  v = umax32(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, DPP_ROW_BCAST15, 0xA, 0xF, false));
  v = umax32(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, DPP_ROW_BCAST31, 0xC, 0xF, false));
  return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

// One column step of team_lu (column KC, a compile-time constant so that the
// row stays in registers), followed by the steps of the later columns.  No
// branches: the pivot row is broadcast by v_readlane and the failure code is
// accumulated, so the scheduler can overlap the next column's pivot search
// with the rest of this column's update.
template <int NMAX, int KC>
__device__ __forceinline__ void team_lu_col(double (&A)[NMAX], int& ord, double& rp_own, int& pv,
                                            int& rc) {
  if constexpr (KC < NMAX) {
    const int lane = threadIdx.x;
    const bool act = ord < 0;
    // the largest |A[KC]| over the rows not yet used, exactly: the IEEE words
    // of a non-negative double order like the value, high word first (the low
    // words are compared only when the high words tie)
    const double a = fabs(A[KC]);
    // every lane's reciprocal, computed while the pivot is searched (the
    // pivot lane's is 1 / pivot, the same division as after the search)
    const double ra = 1.0 / A[KC];
    const unsigned hi = act ? (unsigned)__double2hiint(a) : 0u;
    const unsigned lo = (unsigned)__double2loint(a);
    const unsigned mhi = wave_max_u32(hi);
    const bool cand = act && hi == mhi;
    unsigned long long sel = __ballot(cand);
    if (__builtin_popcountll(sel) > 1) {   // several rows share the high word: compare the low words
      const unsigned mlo = wave_max_u32(cand ? lo : 0u);
      sel = __ballot(cand && lo == mlo);
    }
    const int p = __builtin_amdgcn_readfirstlane(__ffsll(sel) - 1);   // ties: lowest lane
    const bool nonfinite = __any(act && hi >= 0x7FF00000u);
    const bool zero = (mhi == 0u) & (__builtin_amdgcn_readlane((int)lo, p) == 0);   // largest |a| is 0
    const int code = nonfinite ? 2 : (zero ? 1 : 0);
    rc = (rc == 0) ? code : rc;
    const double rp = bcast(ra, p);
    const bool is_p = lane == p;
    const bool upd = act && !is_p;
    const double l = upd ? A[KC] * rp : 0.0;
    A[KC] = upd ? l : A[KC];
    ord = is_p ? KC : ord;
    rp_own = is_p ? rp : rp_own;
    // lane KC records p (a v_writelane with a constant lane: no per-column
    // lane mask to keep live)
    asm("v_writelane_b32 %0, %1, %2" : "+v"(pv) : "s"(p), "i"(KC));
    // keep the step's bookkeeping here: left alone, the compiler sinks the
    // select chains of ord, rp_own and rc to their use after the last column
    // and keeps every column's inputs live until then
    asm volatile("" : "+v"(ord), "+v"(rp_own), "+v"(rc));
#pragma unroll
    for (int j = KC + 1; j < NMAX; ++j) A[j] -= l * bcast(A[j], p);
    team_lu_col<NMAX, KC + 1>(A, ord, rp_own, pv, rc);
  }
}

// LU with partial pivoting of M = d I - J, J the N x N matrix in LDS (row i at
// F[i * ldj]), N <= NMAX.  Lane i loads row i of M into NMAX registers (lanes
// N..NMAX-1 hold identity rows, so every column step is the same) and the
// elimination runs there with implicit pivoting: the pivot of column k is the
// largest |M[i][k]| over the rows not yet used (ties to the lowest original
// row).  The rows are then stored over J in pivot order: row k of F holds row k
// of L below the diagonal (unit diagonal implied) and row k of U from the
// diagonal on - the factors of the textbook LU with explicit row swaps.  perm
// (lane-distributed) receives the permutation (row k of the factors is row
// perm[k] of M); rdiag receives 1 / U_kk in lane k.  Returns 0, 1 (zero pivot)
// or 2 (non-finite pivot column), the first failure in column order; F is
// untouched unless 0 is returned.
template <int NMAX>
__device__ __forceinline__ int team_lu(double* __restrict__ F, int ldj, int N, double d, int& perm,
                                       double& rdiag) {
  const int lane = threadIdx.x;
  const bool own = lane < N;
  const double* row = F + (own ? lane : 0) * ldj;
  const int jn = own ? N : 0;   // entries of M in this lane's row
  double A[NMAX];
#pragma unroll
  for (int j = 0; j < NMAX; ++j) {
    // the load is in this work-group's LDS for every j < NMAX; a select on the
    // loaded value itself, without short-circuit terms, keeps the loads
    // unconditional and issued back to back
    const double f = (j < jn) ? row[j] : 0.0;
    const double dj = ((j == lane) & (j < jn)) ? d : 0.0;
    A[j] = ((lane >= N) & (j == lane)) ? 1.0 : dj - f;
  }
  int ord = lane < NMAX ? -1 : NMAX;          // pivot position of this lane's row; -1 while unused
  double rp_own = 0.0;                        // 1 / (this row's pivot)
  int pv = lane, rc = 0;                      // lane k: the row pivoted at step k
  team_lu_col<NMAX, 0>(A, ord, rp_own, pv, rc);
  wsync();
  if (rc) return rc;
  if (own) {
#pragma unroll
    for (int j = 0; j < NMAX; ++j)
      if (j < N) F[ord * ldj + j] = A[j];
  }
  wsync();
  perm = own ? pv : lane;
  rdiag = own ? gather(rp_own, pv) : 0.0;
  return 0;
}

// Factors of M held in registers: lane i keeps row i of M after elimination -
// the multipliers (row ord of L) in the columns before ord, row ord of U from
// column ord on, where ord is the step at which this row was the pivot.
// Lanes past N hold identity rows pivoted at their own index, lanes past NMAX
// zero rows that never pivot.
template <int NMAX>
struct RegLU {
  double A[NMAX];
  int ord;        // pivot step of this lane's row
  int pv;         // lane k: the lane (row of M) pivoted at step k
  double rown;    // 1 / (this row's pivot)
  double rdg;     // lane k: 1 / U_kk
};

// The elimination of team_lu, with the factors left in registers and J in LDS
// untouched, so that a rejected step can form M again from the same J.
// Returns 0, 1 (zero pivot) or 2 (non-finite pivot column).
template <int NMAX>
__device__ __forceinline__ int team_lu_reg(const double* __restrict__ J, int ldj, int N, double d,
                                           RegLU<NMAX>& F) {
  const int lane = threadIdx.x;
  const bool own = lane < N;
  const double* row = J + (own ? lane : 0) * ldj;
  const int jn = own ? N : 0;
#pragma unroll
  for (int j = 0; j < NMAX; ++j) {
    const double f = (j < jn) ? row[j] : 0.0;
    const double dj = ((j == lane) & (j < jn)) ? d : 0.0;
    F.A[j] = ((lane >= N) & (j == lane)) ? 1.0 : dj - f;
  }
  F.ord = lane < NMAX ? -1 : NMAX;
  F.rown = 0.0;
  F.pv = lane;
  int rc = 0;
  team_lu_col<NMAX, 0>(F.A, F.ord, F.rown, F.pv, rc);
  F.rdg = gather(F.rown, F.pv);
  return rc;
}

// Solve M x = b with the register factors of team_lu_reg.  b is
// lane-distributed by equation (element i in lane i = row i of M; lanes >= N
// hold 0) and so are the factor rows, so no permutation is applied up front.
// Forward, over the pivot steps k: y_k is the current value in the pivot lane
// p_k, and the rows pivoted later subtract L_(ord,k) y_k.  Backward, from the
// last step: x_k = z(p_k) / U_kk, and the rows pivoted earlier subtract
// U_(ord,k) x_k.  Every step is unrolled, so the factor entry is a register;
// p_k and 1/U_kk are read with constant lanes.  The result x_k is gathered
// into lane k.
template <int NMAX>
__device__ __forceinline__ double team_solve_reg(const RegLU<NMAX>& F, int N, double b) {
  const int lane = threadIdx.x;
  // the L/U selections are made here, in each solve: hoisted out of the
  // stage loop they became two masked copies of the factors (2 NMAX more
  // registers, spilled)
  int ord = F.ord;
  asm volatile("" : "+v"(ord));
#pragma unroll
  for (int k = 0; k < NMAX - 1; ++k) {
    const int p = __builtin_amdgcn_readlane(F.pv, k);
    const double yk = bcast(b, p);
    const double l = (ord > k) ? F.A[k] : 0.0;
    b -= l * yk;
  }
#pragma unroll
  for (int k = NMAX - 1; k > 0; --k) {
    const int p = __builtin_amdgcn_readlane(F.pv, k);
    const double xk = bcast(b, p) * bcast(F.rdg, k);
    const double u = (ord < k) ? F.A[k] : 0.0;
    b -= u * xk;
  }
  const double x = gather(b * F.rown, F.pv);
  return lane < N ? x : 0.0;
}

// Solve M x = b with the factors of team_lu (row k of F holds row k of L and
// of U in pivot order; perm and rdiag as returned).  b and x are
// lane-distributed (element i in lane i; lanes >= N hold 0).  Every column
// step is unrolled (NMAX >= N columns, the ones past N are zero), so the
// broadcast of the finished element is a v_readlane with a constant lane and
// the step's critical path is readlane -> FMA.  The row entries are read from
// LDS eight at a time and masked to the triangle being applied; the backward
// sweep applies columns of U scaled by 1/U_kk and multiplies by 1/U_ii at the
// end (lane i's element is final once column i is reached).
template <int NMAX>
__device__ __forceinline__ double team_solve(const double* __restrict__ F, int ldj, int N, int perm,
                                             double rdiag, double b) {
  const int lane = threadIdx.x;
  const bool own = lane < N;
  const double* row = F + (own ? lane : 0) * ldj;
  // Masks without short-circuit conditions: a select whose condition contains
  // own && ... becomes a branch around the LDS load, one full LDS round trip
  // per entry.  Rows past N take lim = 0 (no entry of L).
  const int lim = own ? lane : 0;
  b = gather(b, perm);                       // P b
  // forward: L y = P b (unit lower triangle)
#pragma unroll
  for (int k0 = 0; k0 < NMAX; k0 += 8) {
    double l[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int k = k0 + t;
      const double v = row[k];   // in this work-group's LDS for every k < NMAX; masked by a select
      l[t] = (k < lim) ? v : 0.0;
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int k = k0 + t;
      if (k < NMAX - 1) b -= l[t] * bcast(b, k);
    }
  }
  // backward: U x = y, with z_i -= (U_ik / U_kk) z_k and x_i = z_i / U_ii
#pragma unroll
  for (int k1 = NMAX - 1; k1 >= 0; k1 -= 8) {
    double u[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int k = k1 - t;
      const int kk = k >= 0 ? k : 0;
      const double v = row[kk] * bcast(rdiag, kk);
      u[t] = ((k > lane) & (k < N)) ? v : 0.0;   // lane < k < N: an own row
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int k = k1 - t;
      if (k > 0) b -= u[t] * bcast(b, k);
    }
  }
  return own ? b * rdiag : 0.0;
}

}  // namespace chem
