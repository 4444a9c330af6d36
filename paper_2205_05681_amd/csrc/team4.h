// Four wavefronts per cell ("team4" kernels), for mechanisms with state size
// 64 < N <= 128 (the 112-species mechanism: a 112 x 112 Jacobian per cell).
//
// Layout inside the work-group (256 threads, tid = 64 w + lane):
//   * every state-sized vector is held by every wavefront, as a pair of
//     registers per lane: element `lane` and element 64 + lane (V2).  The
//     four wavefronts run the same controller on the same values, so their
//     decisions agree without being broadcast; only the work below is split;
//   * the source terms and the Jacobian are shared work: species k on thread
//     k (thermo, concentrations, the chain-rule row pass), reactions over all
//     256 threads (reaction j on thread j mod 256) scattering into LDS with
//     FP64 LDS atomics, column c on thread c (the T and V rows); sums over
//     species are wave sums combined through LDS in a fixed order;
//   * the LU of M = I/(h gamma) - J is split over the wavefronts by columns
//     of the matrix padded to 128 x 128 with identity rows and columns, dealt
//     round-robin: wave w holds columns 4 j + w (j < 32) of every row, rows
//     lane and 64 + lane in 64 registers per lane, so the columns right of
//     any k are spread evenly over the four.  At column k the wavefront
//     holding it alone finds the largest |a| over the unused rows (exact, ties
//     to the lowest row) and the multipliers and puts them in LDS; after one
//     work-group barrier every wavefront updates its columns right of k,
//     reading the pivot row's entries from its own registers (v_readlane);
//     the wavefront holding column k + 1 updates that column first and
//     searches its pivot before the rest of its update;
//   * the triangular solves run in every wavefront on its own copy of the
//     vector (no barrier), reading the factors from LDS.
#pragma once
#include <hip/hip_runtime.h>

#include "kinetics.h"
#include "mech.h"
#include "methods.h"
#include "team.h"

namespace chem {

constexpr int T4_THREADS = 256;
constexpr int T4_NMAX = 128;

struct V2 {
  double a, b;   // element lane, element 64 + lane
};

// LDS of one cell (one work-group).  ldj = N + 1.
struct Team4Lds {
  double* J;      // [N][ldj]  Jacobian being assembled / factors of M
  double* brow;   // [ldj]     bath-gas row of d wdot / d Phi
  double* conc;   // [128]
  double* hrt;    // [128]
  double* cpr;    // [128]
  double* gib;    // [128]
  double* wdot;   // [128]
  double* gb;     // [128]     G column of the bath gas
  double* tb;     // [128]     uniform third-body part per row
  double* dwdT;   // [128]
  double* dwdV;   // [128]
  double* dummy;  // [256]     target of the unused participant slots of a reaction: the
                  //           LU's prow and lcol (the two are never in use together)
  double* red;    // [4][8]    per-wavefront partial sums
  double* prow;   // [128]     the LU's multipliers, even columns
  double* lcol;   // [128]     the LU's multipliers, odd columns (follows prow)
  double* rdg;    // [128]     1 / U_kk
  double* ust;    // [4][s][128] stage vectors, one copy per wavefront (s: the method's stages)
  unsigned* pslot;  // [16]    the LU's pivot row, by column parity; [4..7] each wavefront's first failure
  int* perm;        // [128]   the row pivoted at each step
  int* misc;        // [8]     work-queue position broadcast
  static __host__ __device__ size_t doubles(int N, int s) {
    return (size_t)N * (N + 1) + (N + 1) + 9 * 128 + 32 + 128 + 128 + 128 + 4 * (size_t)s * 128 +
           8 /* pslot */ + 64 /* perm */ + 4 /* misc */ + 1;
  }
  __device__ void bind(double* base, int N, int s) {
    J = base;
    brow = J + (size_t)N * (N + 1);
    conc = brow + (N + 1);
    hrt = conc + 128;
    cpr = hrt + 128;
    gib = cpr + 128;
    wdot = gib + 128;
    gb = wdot + 128;
    tb = gb + 128;
    dwdT = tb + 128;
    dwdV = dwdT + 128;
    red = dwdV + 128;
    prow = red + 32;
    lcol = prow + 128;
    dummy = prow;
    rdg = lcol + 128;
    ust = rdg + 128;
    pslot = (unsigned*)(ust + 4 * (size_t)s * 128);
    perm = (int*)(pslot + 16);
    misc = perm + 128;
  }
};

__device__ __forceinline__ int t4_tid() { return threadIdx.x; }
// The wavefront index, made visibly uniform (an SGPR value): branches on it
// are then scalar branches, not divergent ones that would keep both sides'
// register values live.
__device__ __forceinline__ int t4_wave() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }
__device__ __forceinline__ int t4_lane() { return threadIdx.x & 63; }

// Element e (uniform, < 128) of a pair vector.
__device__ __forceinline__ double v2_get(const V2& v, int e) { return bcast(e < 64 ? v.a : v.b, e & 63); }

// Per-lane element src (< 128) of a pair vector: both halves are gathered at
// the same lane index, then the half selected.
__device__ __forceinline__ double v2_gather(const V2& v, int src) {
  const double x = gather(v.a, src & 63), y = gather(v.b, src & 63);
  return src < 64 ? x : y;
}

// Sum over all 128 elements of a pair vector (every wavefront, the same value).
__device__ __forceinline__ double v2_sum(const V2& v) { return wave_sum(v.a + v.b); }

// Sums over the work-group of NS per-thread values (all threads must call it):
// wave sums, then the four wavefronts' partial sums in a fixed order.
template <int NS>
__device__ __forceinline__ void t4_sums(double (&v)[NS], Team4Lds& L) {
  const int w = t4_wave(), lane = t4_lane();
  double s[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) s[i] = wave_sum(v[i]);
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < NS; ++i) L.red[8 * w + i] = s[i];
  wsync();
#pragma unroll
  for (int i = 0; i < NS; ++i) v[i] = (L.red[i] + L.red[8 + i]) + (L.red[16 + i] + L.red[24 + i]);
  wsync();
}

// Concentrations and thermo of the state y.  Species k on thread k fills
// conc/hrt/cpr/gib in LDS; returns T, V, sum C (and sum_k C_k dcp_k/dT / R in
// *sdcp) in every thread.
__device__ __forceinline__ void t4_state(const MechView& M, double P, const V2& y, Team4Lds& L, double& T,
                                         double& V, double& ctot, double* sdcp) {
  const int tid = t4_tid();
  const int K = M.K;
  T = v2_get(y, 0);
  V = v2_get(y, 1);
  const double nk = v2_gather(y, (tid + 2) & 127);   // element tid + 2 (valid for tid < K - 1)
  double c = (tid < K - 1) ? nk / V : 0.0;
  double r1[1] = {c};
  t4_sums<1>(r1, L);
  if (tid == K - 1) c = P / (RU * T) - r1[0];
  double dcp = 0.0;
  if (tid < K) {
    L.conc[tid] = c;
    double cf[15];
#pragma unroll
    for (int i = 0; i < 15; ++i) cf[i] = M.nasa[15 * tid + i];
    const bool lo = T < cf[0];
    const double a0 = lo ? cf[1] : cf[8], a1 = lo ? cf[2] : cf[9], a2 = lo ? cf[3] : cf[10],
                 a3 = lo ? cf[4] : cf[11], a4 = lo ? cf[5] : cf[12], a5 = lo ? cf[6] : cf[13],
                 a6 = lo ? cf[7] : cf[14];
    const double lnT = log(T), iT = 1.0 / T;
    const double cp = a0 + T * (a1 + T * (a2 + T * (a3 + T * a4)));
    const double h = a0 + T * (a1 * 0.5 + T * (a2 * (1.0 / 3.0) + T * (a3 * 0.25 + T * a4 * 0.2))) + a5 * iT;
    const double sr = a0 * lnT + T * (a1 + T * (a2 * 0.5 + T * (a3 * (1.0 / 3.0) + T * a4 * 0.25))) + a6;
    L.hrt[tid] = h;
    L.cpr[tid] = cp;
    L.gib[tid] = sr - h;
    if (sdcp) dcp = c * (a1 + T * (2.0 * a2 + T * (3.0 * a3 + T * 4.0 * a4)));
  }
  double r2[2] = {tid < K ? c : 0.0, dcp};
  t4_sums<2>(r2, L);   // (its barriers also publish the LDS writes above)
  ctot = r2[0];
  if (sdcp) *sdcp = r2[1];
}

// The pair vector of f from wdot in LDS: f_0 = Tdot, f_1 = dV/dt, f_{2+k} = V wdot_k.
__device__ __forceinline__ V2 t4_pack_f(int N, double Tdot, double Vdot, double V, const double* wdot) {
  const int lane = t4_lane();
  V2 f;
  f.a = (lane == 0) ? Tdot : (lane == 1) ? Vdot : (lane < N ? V * wdot[lane - 2] : 0.0);
  f.b = (64 + lane < N) ? V * wdot[62 + lane] : 0.0;
  return f;
}

// The f scatter of one reaction, slots up to SIDE per side: an unused slot,
// or a thread past the last reaction, adds to the thread's own dummy cell (no
// per-lane branch).
template <int SIDE>
__device__ __forceinline__ void t4_rhs_scatter(const RxnRec& R, double q_rate, bool have, Team4Lds& L, int tid) {
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    if (q % 3 >= SIDE) continue;
    const int sq = R.sp[q], nq = R.nu[q];
    const bool on = have && ((q < 3) ? (q < R.nr) : (q - 3 < R.np));
    atomicAdd(on ? &L.wdot[sq] : L.dummy + tid, (q < 3 ? -nq : nq) * q_rate);
  }
}

// f(y).
__device__ __forceinline__ V2 t4_rhs(const MechView& M, double P, const V2& y, Team4Lds& L,
                                     const double* __restrict__ lnA) {
  const int tid = t4_tid();
  const int K = M.K, N = M.N;
  double T, V, ctot;
  t4_state(M, P, y, L, T, V, ctot, nullptr);
  if (tid < K) L.wdot[tid] = 0.0;
  wsync();
  const double lnT = log(T), iT = 1.0 / T;
  const int w = t4_wave();
  const int Nr = M.Nr;
  RxnRec nx = load_rxn(M, tid < Nr ? tid : 0, lnA);   // fetched one chunk ahead
  for (int j0 = 0; j0 < Nr; j0 += T4_THREADS) {
    // rates of 256 reactions in parallel, then their scatter one wavefront at a
    // time: the LDS additions of one wavefront come in a fixed order, those of
    // concurrent wavefronts would not, and the sums would vary from run to run
    const int j = j0 + tid;
    const bool have = j < Nr;
    const RxnRec R = nx;
    nx = load_rxn(M, j + T4_THREADS < Nr ? j + T4_THREADS : 0, lnA);
    // a wavefront whose reactions all have two species a side leaves the
    // third slots out (a wave-uniform choice)
    const bool two = __all(R.nr <= 2 && R.np <= 2);
    const RateOut r = two ? reaction_rate<double, 2>(M, R, T, lnT, iT, ctot, Lane{L.conc, 1}, Lane{L.gib, 1},
                                                     Lane{L.hrt, 1}, false)
                          : reaction_rate<double, MAX_SIDE>(M, R, T, lnT, iT, ctot, Lane{L.conc, 1},
                                                            Lane{L.gib, 1}, Lane{L.hrt, 1}, false);
    for (int ph = 0; ph < 4; ++ph) {
      if (w == ph) {
        if (two)
          t4_rhs_scatter<2>(R, r.q, have, L, tid);
        else
          t4_rhs_scatter<MAX_SIDE>(R, r.q, have, L, tid);
      }
      wsync();
    }
  }
  double wk = 0.0, num = 0.0, den = 0.0;
  if (tid < K) {
    wk = L.wdot[tid];
    num = L.hrt[tid] * wk;
    den = L.conc[tid] * L.cpr[tid];
  }
  double r3[3] = {num, den, wk};
  t4_sums<3>(r3, L);
  const double Tdot = -(r3[0] * T) / r3[1];
  const V2 f = t4_pack_f(N, Tdot, V * (Tdot * iT + (RU * T / P) * r3[2]), V, L.wdot);
  wsync();
  return f;
}

// The Jacobian scatter of one reaction into the rows of G, slots up to SIDE
// per side; an unused slot, or a thread past the last reaction, sends its
// updates to the thread's own dummy cell.
template <int SIDE>
__device__ __forceinline__ void t4_jac_scatter(const MechView& M, const RxnRec& R, const RateOut& r, double dqdT,
                                               const int (&ks)[6], const int (&nus)[6], const bool (&on_in)[6],
                                               const double (&dq)[6], bool have, Team4Lds& L, int K, int ldj,
                                               double* dummy) {
  bool on[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) on[q] = have && on_in[q];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    if (q % 3 >= SIDE) continue;
    const int k = ks[q];
    const double vk = (q < 3) ? -(double)nus[q] : (double)nus[q];
    double* row = (k == K - 1) ? L.brow : L.J + (k + 2) * ldj;
    lds_add(on[q] ? &L.wdot[k] : dummy, vk * r.q);
    lds_add(on[q] ? &row[0] : dummy, vk * dqdT);
#pragma unroll
    for (int t = 0; t < 6; ++t) {
      if (t % 3 >= SIDE) continue;
      const int mm = ks[t];
      double* dst = (mm == K - 1) ? &L.gb[k] : &row[mm + 2];
      lds_add((on[q] && on[t]) ? dst : dummy, vk * dq[t]);
    }
  }
  if (R.type != RX_ELEM) {
    const int e0 = R.e0, e1 = R.e1;
    int em[4];
    double ea[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = (e0 + t < e1) ? e0 + t : e0;
      em[t] = M.eff_idx[e];
      ea[t] = M.eff_am1[e];
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      if (q % 3 >= SIDE) continue;
      const int k = ks[q];
      const double vk = (q < 3) ? -(double)nus[q] : (double)nus[q];
      double* row = (k == K - 1) ? L.brow : L.J + (k + 2) * ldj;
      lds_add(on[q] ? &L.tb[k] : dummy, vk * r.beta);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        double* dst = (em[t] == K - 1) ? &L.gb[k] : &row[em[t] + 2];
        lds_add((on[q] && e0 + t < e1) ? dst : dummy, (vk * ea[t]) * r.beta);
      }
      for (int e = e0 + 4; e < e1; ++e) {
        const int mm = M.eff_idx[e];
        lds_add(on[q] ? ((mm == K - 1) ? &L.gb[k] : &row[mm + 2]) : dummy, (vk * M.eff_am1[e]) * r.beta);
      }
    }
  }
}

// f(y) and the Jacobian, assembled in L.J (row i at L.J[i*(N+1)]).  The same
// derivation as the one-wavefront kernel (team_rhs_jac), with species, columns
// and reactions over the work-group's threads.
__device__ __forceinline__ V2 t4_rhs_jac(const MechView& M, double P, const V2& y, Team4Lds& L,
                                         const double* __restrict__ lnA) {
  const int tid = t4_tid();
  const int K = M.K, N = M.N, ldj = N + 1;
  double T, V, ctot, sdcp;
  t4_state(M, P, y, L, T, V, ctot, &sdcp);
  const double lnT = log(T), iT = 1.0 / T, iV = 1.0 / V;
  if (tid < N) {
    for (int k = 0; k < K - 1; ++k) L.J[(k + 2) * ldj + tid] = 0.0;
    L.brow[tid] = 0.0;
  }
  if (tid < K) {
    L.wdot[tid] = 0.0;
    L.gb[tid] = 0.0;
    L.tb[tid] = 0.0;
  }
  wsync();
  const int w = t4_wave();
  const int Nr = M.Nr;
  RxnRec nx = load_rxn(M, tid < Nr ? tid : 0, lnA);   // fetched one chunk ahead
  for (int j0 = 0; j0 < Nr; j0 += T4_THREADS) {
    // rates of 256 reactions in parallel, then their scatter one wavefront at a
    // time (a fixed order of the LDS additions: deterministic sums)
    const int j = j0 + tid;
    const bool have = j < Nr;
    const RxnRec R = nx;
    nx = load_rxn(M, j + T4_THREADS < Nr ? j + T4_THREADS : 0, lnA);
    // a wavefront whose reactions all have two species a side leaves the
    // third slots out (a wave-uniform choice)
    const bool two = __all(R.nr <= 2 && R.np <= 2);
    const RateOut r = two ? reaction_rate<double, 2>(M, R, T, lnT, iT, ctot, Lane{L.conc, 1}, Lane{L.gib, 1},
                                                     Lane{L.hrt, 1}, true)
                          : reaction_rate<double, MAX_SIDE>(M, R, T, lnT, iT, ctot, Lane{L.conc, 1},
                                                            Lane{L.gib, 1}, Lane{L.hrt, 1}, true);
    const int nr = R.nr, np = R.np;
    const double dqdT = r.dlnk_dT * r.q + r.kr_rr * r.dlnKc_dT;
    double* const dummy = L.dummy + tid;
    int ks[6], nus[6];
    bool on[6];
    double cs[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      on[q] = (q < 3) ? (q < nr) : (q - 3 < np);
      ks[q] = R.sp[q];
      nus[q] = R.nu[q];
      cs[q] = L.conc[ks[q]];
    }
    double dq[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const int s0 = q < 3 ? 0 : 3;
      double d = (q < 3) ? r.kf : r.kr;
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        const int v = (s0 + l == q) ? nus[s0 + l] - 1 : nus[s0 + l];
        const double c = cs[s0 + l];
        d = (v >= 1) ? d * c : d;
        d = (v >= 2) ? d * c : d;
        d = (v >= 3) ? d * c : d;
      }
      dq[q] = d * (double)(q < 3 ? nus[q] : -nus[q]);
    }
    for (int ph = 0; ph < 4; ++ph) {
      if (w == ph) {
        if (two)
          t4_jac_scatter<2>(M, R, r, dqdT, ks, nus, on, dq, have, L, K, ldj, dummy);
        else
          t4_jac_scatter<MAX_SIDE>(M, R, r, dqdT, ks, nus, on, dq, have, L, K, ldj, dummy);
      }
      wsync();
    }
  }
  // pass 1, species row k on thread k
  const double dCb_dT = -P / (RU * T * T);
  double num = 0.0, den = 0.0, wsum = 0.0, wcp = 0.0, dDV = 0.0;
  if (tid < K) {
    const int k = tid;
    double* row = (k == K - 1) ? L.brow : L.J + (k + 2) * ldj;
    const double t = L.tb[k];
    const double gbk = L.gb[k] + t;
    const double wk = L.wdot[k];
    const double cpk = L.cpr[k] * RU;
    num = L.hrt[k] * RU * T * wk;
    den = L.conc[k] * cpk;
    wsum = wk;
    wcp = wk * cpk;
    double dvs = 0.0;
#pragma unroll 8
    for (int m = 0; m < K - 1; ++m) {
      const double dn = row[m + 2] + t - gbk;
      dvs -= dn * L.conc[m];
      row[m + 2] = dn;
    }
    const double dwdT = row[0] + gbk * dCb_dT;
    L.dwdT[k] = dwdT;
    L.dwdV[k] = dvs * iV;
    if (k < K - 1) {
      row[0] = V * dwdT;
      row[1] = wk + dvs;
      dDV = (L.cpr[K - 1] - L.cpr[k]) * RU * L.conc[k];
    }
  }
  double r5[5] = {num, den, wsum, wcp, dDV};
  t4_sums<5>(r5, L);
  num = r5[0];
  den = r5[1];
  wsum = r5[2];
  wcp = r5[3];
  dDV = r5[4] * iV;
  // pass 2, column c on thread c: the T and V rows
  const double Tdot = -num / den;
  const double RTP = RU * T / P;
  if (tid < N) {
    const int c = tid;
    double ah = 0.0, aw = 0.0;
    const double* src = (c == 0) ? L.dwdT : L.dwdV;
    const double scale = (c >= 2) ? iV : 1.0;
#pragma unroll 8
    for (int k = 0; k < K; ++k) {
      const double* row = (k == K - 1) ? L.brow : L.J + (k + 2) * ldj;
      const double d = ((c >= 2) ? row[c] : src[k]) * scale;
      ah += L.hrt[k] * RU * T * d;
      aw += d;
    }
    const double cpb = L.cpr[K - 1] * RU;
    double dD, dTd, dVd;
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
  const V2 f = t4_pack_f(N, Tdot, V * (Tdot * iT + RTP * wsum), V, L.wdot);
  wsync();
  return f;
}

// Column-cyclic LU: wave w holds column 4 jj + w (jj < 32) of rows lane and
// 64 + lane in A0[jj], A1[jj] (the matrix padded to 128 x 128 with identity
// rows and columns).  At column KC the wavefront owning it (KC % 4, local
// index KC / 4) alone finds the pivot (exact largest |a| over the unused rows,
// ties to the lowest row) and the multipliers, and publishes the pivot row
// index and the multipliers in LDS (two buffers, alternating with the column
// parity); after one work-group barrier every wavefront updates its columns
// right of KC, taking the pivot row's entries from its own registers by
// v_readlane.  The search for column KC + 1 runs in step KC, by its wavefront,
// right after that column's update and before its other columns.

// Rows lane, 64 + lane: A -= l u over the local columns J0..J1-1, u the
// pivot row (lane pl, second half when ph).
template <int J0, int J1 = 32>
__device__ __forceinline__ void t4c_update(double (&A0)[32], double (&A1)[32], double l0, double l1, int pl,
                                           bool ph) {
#pragma unroll
  for (int jj = J0; jj < J1; ++jj) {
    const double u = bcast(ph ? A1[jj] : A0[jj], pl);
    A0[jj] -= l0 * u;
    A1[jj] -= l1 * u;
  }
}

// Column KC's pivot and multipliers, by the wavefront holding the column
// (local index KC / 4): the exact largest |a| over the unused rows, ties to
// the lowest row (its first half, then its second); the multipliers replace
// the column, and the pivot row, the multipliers and 1 / pivot go to LDS
// (buffer KC & 1).  fk keeps the wavefront's first failure, 4 KC + code (its
// columns come in increasing order), T4_NOFAIL while there is none.
constexpr unsigned T4_NOFAIL = 4u * T4_NMAX;
template <int KC>
__device__ __forceinline__ void t4c_search(double (&A0)[32], double (&A1)[32], Team4Lds& L, int ord0, int ord1,
                                           int& p, double& l0, double& l1, unsigned& fk) {
  constexpr int KK = KC / 4;
  const int lane = t4_lane();
  double* lc = L.prow + 128 * (KC & 1);   // L.prow and L.lcol: two buffers of 128
  const bool act0 = ord0 < 0, act1 = ord1 < 0;
  const double a0 = fabs(A0[KK]), a1 = fabs(A1[KK]);
  // the IEEE words of a non-negative double order like the value
  const unsigned h0 = act0 ? (unsigned)__double2hiint(a0) : 0u, w0 = act0 ? (unsigned)__double2loint(a0) : 0u;
  const unsigned h1 = act1 ? (unsigned)__double2hiint(a1) : 0u, w1 = act1 ? (unsigned)__double2loint(a1) : 0u;
  const bool t1 = h1 > h0 || (h1 == h0 && w1 > w0);
  const unsigned bh = t1 ? h1 : h0, bl = t1 ? w1 : w0;
  const unsigned mhi = wave_max_u32(bh);
  const bool cand = bh == mhi;
  unsigned mlo;
  const unsigned long long sel = __ballot(cand);
  if (__builtin_popcountll(sel) > 1)   // several lanes share the high word
    mlo = wave_max_u32(cand ? bl : 0u);
  else
    mlo = (unsigned)__builtin_amdgcn_readlane((int)bl, __builtin_amdgcn_readfirstlane(__ffsll(sel) - 1));
  const unsigned long long s0 = __ballot(act0 && h0 == mhi && w0 == mlo);
  const unsigned long long s1 = __ballot(act1 && h1 == mhi && w1 == mlo);
  p = __builtin_amdgcn_readfirstlane(s0 ? __ffsll(s0) - 1 : 64 + __ffsll(s1) - 1);
  const bool nonfinite = __any((act0 && h0 >= 0x7FF00000u) || (act1 && h1 >= 0x7FF00000u));
  const int code = nonfinite ? 2 : ((mhi | mlo) == 0u ? 1 : 0);
  const double piv = bcast(p >= 64 ? A1[KK] : A0[KK], p & 63);
  const double rp = 1.0 / piv;
  const bool u0 = act0 && p != lane, u1 = act1 && p != 64 + lane;
  l0 = u0 ? A0[KK] * rp : 0.0;
  l1 = u1 ? A1[KK] * rp : 0.0;
  A0[KK] = u0 ? l0 : A0[KK];
  A1[KK] = u1 ? l1 : A1[KK];
  lc[lane] = l0;
  lc[64 + lane] = l1;
  if (lane == 0) {
    L.pslot[KC & 1] = (unsigned)p;
    L.perm[KC] = p;
    L.rdg[KC] = rp;
  }
  fk = (fk == T4_NOFAIL && code) ? 4u * KC + (unsigned)code : fk;
  // keep the column's values here (not sunk past the later columns)
  asm volatile("" : "+v"(l0), "+v"(l1));
}

// Elimination step KC.  On entry column KC's pivot and multipliers are in
// LDS (buffer KC & 1, behind a barrier) and, in the wavefront holding the
// column, in p, l0, l1.  Wavefront w's columns right of KC are its local
// columns from KC / 4 on when w > KC % 4, from KC / 4 + 1 otherwise.
template <int KC>
__device__ __forceinline__ void t4c_col(double (&A0)[32], double (&A1)[32], Team4Lds& L, int& ord0, int& ord1,
                                        int p, double l0, double l1, unsigned& fk, int N) {
  if constexpr (KC < T4_NMAX) {
    // the padding columns past N change no real row (their entries there are
    // zero): every wavefront stops at the same step (N is uniform)
    if constexpr (KC > 64)
      if (KC >= N) return;
    constexpr int W = KC % 4, KK = KC / 4;
    constexpr int W1 = (KC + 1) % 4, K1 = (KC + 1) / 4;   // the next column's wavefront and local index
    const int w = t4_wave(), lane = t4_lane();
    if (w != W) {
      const double* lc = L.prow + 128 * (KC & 1);
      p = (int)L.pslot[KC & 1];
      l0 = lc[lane];
      l1 = lc[64 + lane];
    }
    ord0 = (p == lane) ? KC : ord0;
    ord1 = (p == 64 + lane) ? KC : ord1;
    asm volatile("" : "+v"(ord0), "+v"(ord1));
    const int pl = p & 63;
    const bool ph = p >= 64;
    int pn = 0;
    double m0 = 0.0, m1 = 0.0;   // column KC + 1's pivot and multipliers (its wavefront)
    if constexpr (KC + 1 < T4_NMAX) {
      if (w == W1) {
        t4c_update<K1, K1 + 1>(A0, A1, l0, l1, pl, ph);
        t4c_search<KC + 1>(A0, A1, L, ord0, ord1, pn, m0, m1, fk);
        t4c_update<K1 + 1>(A0, A1, l0, l1, pl, ph);
      } else if (w > W) {
        t4c_update<KK>(A0, A1, l0, l1, pl, ph);
      } else {
        t4c_update<KK + 1>(A0, A1, l0, l1, pl, ph);
      }
      wsync();
    }
    t4c_col<KC + 1>(A0, A1, L, ord0, ord1, pn, m0, m1, fk, N);
  }
}

// LU with partial pivoting of M = d I - J, J the N x N matrix in LDS (row i
// at F[i * ldj]), 64 < N <= 128, by the four wavefronts (the layout at the
// top).  The pivot of column k is the largest |M[i][k]| over the rows not yet
// used, ties to the lowest original row.  The factors go back over J in pivot
// order (row k of F: row k of L below the diagonal, unit diagonal implied, and
// row k of U from the diagonal on), L.perm[k] receives the row of M pivoted at
// step k and L.rdg[k] = 1 / U_kk.  Returns 0, 1 (zero pivot) or 2
// (non-finite pivot column), the first failure in column order; F is
// untouched unless 0 is returned.
__device__ __forceinline__ int t4_lu(double* __restrict__ F, int ldj, int N, double d, Team4Lds& L) {
  const int w = t4_wave(), lane = t4_lane();
  const int r0 = lane, r1 = 64 + lane;
  const bool own0 = r0 < N, own1 = r1 < N;
  const double* row0 = F + (own0 ? r0 : 0) * ldj;
  const double* row1 = F + (own1 ? r1 : 0) * ldj;
  const int jn0 = own0 ? N : 0, jn1 = own1 ? N : 0;   // entries of M in each row
  double A0[32], A1[32];
#pragma unroll
  for (int jj = 0; jj < 32; ++jj) {
    const int c = 4 * jj + w;
    // unconditional loads (every address lies in this work-group's LDS), masked afterwards
    const double v0 = row0[c], v1 = row1[c];
    const double f0 = (c < jn0) ? v0 : 0.0, f1 = (c < jn1) ? v1 : 0.0;
    A0[jj] = ((!own0) & (c == r0)) ? 1.0 : (((c == r0) & own0) ? d : 0.0) - f0;
    A1[jj] = ((!own1) & (c == r1)) ? 1.0 : (((c == r1) & own1) ? d : 0.0) - f1;
  }
  int ord0 = -1, ord1 = -1;
  int p = 0;
  double l0 = 0.0, l1 = 0.0;
  unsigned fk = T4_NOFAIL;
  if (w == 0) t4c_search<0>(A0, A1, L, ord0, ord1, p, l0, l1, fk);
  wsync();
  t4c_col<0>(A0, A1, L, ord0, ord1, p, l0, l1, fk, N);
  // the first failure in column order over the four wavefronts
  if (lane == 0) L.pslot[4 + w] = fk;
  wsync();
  const unsigned f = min(min(L.pslot[4], L.pslot[5]), min(L.pslot[6], L.pslot[7]));
  const int rc = f == T4_NOFAIL ? 0 : (int)(f & 3u);
  if (rc) return rc;
#pragma unroll
  for (int jj = 0; jj < 32; ++jj) {
    const int c = 4 * jj + w;
    if (own0 && c < N) F[ord0 * ldj + c] = A0[jj];
    if (own1 && c < N) F[ord1 * ldj + c] = A1[jj];
  }
  wsync();
  return 0;
}

// Solve M x = b with the factors of t4_lu (F rows in pivot order, L.perm,
// L.rdg), in the calling wavefront only, on its own pair vector b (elements
// >= N hold 0).  Every column step is unrolled over the 128 padded columns, so
// the broadcast of the finished element is a v_readlane with a constant lane;
// the row entries are read from LDS eight at a time and masked to the
// triangle being applied.
__device__ __forceinline__ V2 t4_solve(const double* __restrict__ F, int ldj, int N, const Team4Lds& L,
                                       const V2& b_in) {
  const int lane = t4_lane();
  const int r0 = lane, r1 = 64 + lane;
  const bool own0 = r0 < N, own1 = r1 < N;
  const double* row0 = F + (own0 ? r0 : 0) * ldj;
  const double* row1 = F + (own1 ? r1 : 0) * ldj;
  const int lim0 = own0 ? r0 : 0, lim1 = own1 ? r1 : 0;
  const int p0 = own0 ? L.perm[r0] : r0, p1 = own1 ? L.perm[r1] : r1;
  // (the gathers run in every lane: a lane-crossing read needs its source active)
  const double g0 = v2_gather(b_in, p0 & 127), g1 = v2_gather(b_in, p1 & 127);
  V2 b;
  b.a = own0 ? g0 : 0.0;
  b.b = own1 ? g1 : 0.0;
  // forward: L y = P b (blocks of eight columns; those past N change nothing
  // and are skipped, a wave-uniform test)
#pragma unroll
  for (int k0 = 0; k0 < T4_NMAX; k0 += 8) {
    if (k0 >= N) break;
    double la[8], lb[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int k = k0 + t;
      const int kk = k < ldj ? k : 0;   // (row k of the factors has ldj entries)
      const double va = row0[kk], vb = row1[kk];
      la[t] = (k < lim0) ? va : 0.0;
      lb[t] = (k < lim1) ? vb : 0.0;
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int k = k0 + t;
      if (k < T4_NMAX - 1) {
        const double yk = bcast(k < 64 ? b.a : b.b, k & 63);
        if (k < 63) b.a -= la[t] * yk;
        b.b -= lb[t] * yk;
      }
    }
    __builtin_amdgcn_sched_barrier(0);   // eight columns' loads in flight, no more
  }
  // backward: U x = y, z_i -= (U_ik / U_kk) z_k, x_i = z_i / U_ii
  const double rd0 = own0 ? L.rdg[r0] : 0.0, rd1 = own1 ? L.rdg[r1] : 0.0;
  const V2 rd{rd0, rd1};
#pragma unroll
  for (int k1 = T4_NMAX - 1; k1 >= 0; k1 -= 8) {
    if (k1 - 7 >= N) continue;   // every column of the block past N
    double ua[8], ub[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int k = k1 - t;
      const int kk = (k >= 0 && k < ldj) ? k : 0;
      const double s = (k >= 0) ? v2_get(rd, k) : 0.0;
      const double va = row0[kk] * s, vb = row1[kk] * s;
      ua[t] = ((k > r0) & (k < N) & own0) ? va : 0.0;
      ub[t] = ((k > r1) & (k < N) & own1) ? vb : 0.0;
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int k = k1 - t;
      if (k > 0) {
        const double zk = bcast(k < 64 ? b.a : b.b, k & 63);
        b.a -= ua[t] * zk;
        if (k > 64) b.b -= ub[t] * zk;
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  return V2{own0 ? b.a * rd0 : 0.0, own1 ? b.b * rd1 : 0.0};
}

}  // namespace chem
