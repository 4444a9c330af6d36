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
//   * the LU of M = I/(h gamma) - J is split over the wavefronts in a 2 x 2
//     block layout of the matrix padded to 128 x 128 with identity rows and
//     columns: wave w holds rows 64 rb + lane (rb = w & 1) and columns
//     64 hc + j (hc = w >> 1, j < 64) in 64 registers per lane.  At column k
//     the two wavefronts holding column k each find the largest |a| over their
//     unused rows (exact, ties to the lowest row), the two candidates meet in
//     LDS, the pivot row's halves and every row's multiplier go through LDS,
//     and each wavefront updates its block: two work-group barriers per column;
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
  double* dummy;  // [256]     target of the unused participant slots of a reaction
  double* red;    // [4][8]    per-wavefront partial sums
  double* prow;   // [2][64]   the pivot row, by column half
  double* lcol;   // [2][64]   the multipliers, by row block
  double* rdg;    // [128]     1 / U_kk
  double* pval;   // [2]       signed pivot candidate of each row block
  double* ust;    // [4][MAX_STAGES][128] stage vectors, one copy per wavefront
  unsigned* pslot;  // [2][4]  pivot candidates: |a| high word, low word, row, non-finite flag
  int* perm;        // [128]   the row pivoted at each step
  int* misc;        // [8]     work-queue position broadcast
  static __host__ __device__ size_t doubles(int N) {
    return (size_t)N * (N + 1) + (N + 1) + 9 * 128 + 256 + 32 + 128 + 128 + 128 + 2 +
           4 * MAX_STAGES * 128 + 8 /* pslot */ + 64 /* perm */ + 4 /* misc */ + 1;
  }
  __device__ void bind(double* base, int N) {
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
    dummy = dwdV + 128;
    red = dummy + 256;
    prow = red + 32;
    lcol = prow + 128;
    rdg = lcol + 128;
    pval = rdg + 128;
    ust = pval + 2;
    pslot = (unsigned*)(ust + 4 * MAX_STAGES * 128);
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
  for (int j0 = 0; j0 < M.Nr; j0 += T4_THREADS) {
    // rates of 256 reactions in parallel, then their scatter one wavefront at a
    // time: the LDS additions of one wavefront come in a fixed order, those of
    // concurrent wavefronts would not, and the sums would vary from run to run
    const int j = j0 + tid;
    const bool have = j < M.Nr;
    const int jj = have ? j : 0;
    const RateOut r = reaction_rate(M, jj, T, lnT, iT, ctot, Lane{L.conc, 1}, Lane{L.gib, 1},
                                    Lane{L.hrt, 1}, lnA, false);
    const int32_t* info = M.rinfo + 8 * jj;
    const int32_t* sp = M.rspec + 6 * jj;
    const int32_t* nu = M.rnu + 6 * jj;
    for (int ph = 0; ph < 4; ++ph) {
      if (w == ph && have) {
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          const int sq = sp[q], nq = nu[q];
          if ((q < 3) ? (q < info[1]) : (q - 3 < info[2])) atomicAdd(&L.wdot[sq], (q < 3 ? -nq : nq) * r.q);
        }
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
  for (int j0 = 0; j0 < M.Nr; j0 += T4_THREADS) {
    // rates of 256 reactions in parallel, then their scatter one wavefront at a
    // time (a fixed order of the LDS additions: deterministic sums)
    const int j = j0 + tid;
    const bool have = j < M.Nr;
    const int jj = have ? j : 0;
    const RateOut r = reaction_rate(M, jj, T, lnT, iT, ctot, Lane{L.conc, 1}, Lane{L.gib, 1},
                                    Lane{L.hrt, 1}, lnA, true);
    const int32_t* info = M.rinfo + 8 * jj;
    const int32_t* sp = M.rspec + 6 * jj;
    const int32_t* nu = M.rnu + 6 * jj;
    const int nr = info[1], np = info[2];
    const double dqdT = r.dlnk_dT * r.q + r.kr_rr * r.dlnKc_dT;
    double* const dummy = L.dummy + tid;
    int ks[6], nus[6];
    bool on[6];
    double cs[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      on[q] = (q < 3) ? (q < nr) : (q - 3 < np);
      ks[q] = sp[q];
      nus[q] = nu[q];
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
    if (w == ph && have) {
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const int k = ks[q];
      const double vk = (q < 3) ? -(double)nus[q] : (double)nus[q];
      double* row = (k == K - 1) ? L.brow : L.J + (k + 2) * ldj;
      lds_add(on[q] ? &L.wdot[k] : dummy, vk * r.q);
      lds_add(on[q] ? &row[0] : dummy, vk * dqdT);
#pragma unroll
      for (int t = 0; t < 6; ++t) {
        const int mm = ks[t];
        double* dst = (mm == K - 1) ? &L.gb[k] : &row[mm + 2];
        lds_add((on[q] && on[t]) ? dst : dummy, vk * dq[t]);
      }
    }
    if (info[0] != RX_ELEM) {
      const int e0 = info[3], e1 = info[4];
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

// A[j] -= l * pr[j] for J0 <= j < 64, eight columns at a time: the eight
// loads of the pivot row, then their eight FMAs, with the scheduler kept from
// hoisting later loads (which would hold the whole pivot row in registers
// beside the block's row segment).
template <int J0>
__device__ __forceinline__ void t4_update(double (&A)[64], const double* pr, double l) {
#pragma unroll
  for (int j0 = J0; j0 < 64; j0 += 8) {
    double u[8];
#pragma unroll
    for (int t = 0; t < 8; ++t)
      if (j0 + t < 64) u[t] = pr[j0 + t];
#pragma unroll
    for (int t = 0; t < 8; ++t)
      if (j0 + t < 64) A[j0 + t] -= l * u[t];
    __builtin_amdgcn_sched_barrier(0);
  }
}

// One column step of t4_lu (column KC, a compile-time constant, so that the
// block's row segment stays in registers), then the later columns.
template <int KC>
__device__ __forceinline__ void t4_lu_col(double (&A)[64], Team4Lds& L, int& ord, double& rp_own, int& rc) {
  if constexpr (KC < T4_NMAX) {
    constexpr int HK = KC / 64, KK = KC % 64;
    const int w = t4_wave(), lane = t4_lane(), tid = t4_tid();
    const int rb = w & 1, hc = w >> 1;
    const bool act = ord < 0;
    // (1) the waves holding column KC: largest |a| over their unused rows
    if (hc == HK) {
      const double a = fabs(A[KK]);
      const unsigned hi = act ? (unsigned)__double2hiint(a) : 0u;
      const unsigned lo = act ? (unsigned)__double2loint(a) : 0u;
      const unsigned mhi = wave_max_u32(hi);
      const bool cand = act && hi == mhi;
      unsigned long long sel = __ballot(cand);
      if (__builtin_popcountll(sel) > 1) {
        const unsigned mlo = wave_max_u32(cand ? lo : 0u);
        sel = __ballot(cand && lo == mlo);
      }
      const bool nonfinite = __any(act && hi >= 0x7FF00000u);
      const int pl = sel ? __builtin_amdgcn_readfirstlane(__ffsll(sel) - 1) : 0;
      const unsigned plo = (unsigned)__builtin_amdgcn_readlane((int)lo, pl);
      const double pv = bcast(A[KK], pl);
      if (lane == 0) {
        L.pslot[4 * rb + 0] = sel ? mhi : 0u;
        L.pslot[4 * rb + 1] = sel ? plo : 0u;
        L.pslot[4 * rb + 2] = sel ? (unsigned)(64 * rb + pl) : 0xFFFFFFFFu;
        L.pslot[4 * rb + 3] = nonfinite ? 1u : 0u;
        L.pval[rb] = pv;
      }
    }
    wsync();
    // (2) the larger candidate (ties to row block 0, the lower rows)
    const unsigned h0 = L.pslot[0], l0 = L.pslot[1], r0 = L.pslot[2];
    const unsigned h1 = L.pslot[4], l1 = L.pslot[5], r1 = L.pslot[6];
    const bool nonfinite = (L.pslot[3] | L.pslot[7]) != 0u;
    const bool take1 = (r0 == 0xFFFFFFFFu) || (r1 != 0xFFFFFFFFu && (h1 > h0 || (h1 == h0 && l1 > l0)));
    const int p = (int)(take1 ? r1 : r0);
    const double piv = take1 ? L.pval[1] : L.pval[0];
    const bool zero = (take1 ? (h1 | l1) : (h0 | l0)) == 0u;
    const int code = nonfinite ? 2 : (zero ? 1 : 0);
    rc = (rc == 0) ? code : rc;
    const double rp = 1.0 / piv;
    const int myrow = 64 * rb + lane;
    const bool is_p = myrow == p;
    const bool upd = act && !is_p;
    double l = 0.0;
    if (hc == HK) {
      l = upd ? A[KK] * rp : 0.0;
      A[KK] = upd ? l : A[KK];
      L.lcol[64 * rb + lane] = l;
    }
    if (is_p) {
      // the pivot row's half of this wave, for the other row block's wave
#pragma unroll
      for (int j = 0; j < 64; ++j) L.prow[64 * hc + j] = A[j];
    }
    if (tid == 0) {
      L.perm[KC] = p;
      L.rdg[KC] = rp;
    }
    ord = is_p ? KC : ord;
    rp_own = is_p ? rp : rp_own;
    // keep the step's bookkeeping here: left alone, the compiler sinks these
    // select chains to their use after the last column and keeps every
    // column's pivot candidates live until then (hundreds of spilled registers)
    asm volatile("" : "+v"(ord), "+v"(rc), "+v"(rp_own));
    wsync();
    // (3) update this wave's block: the columns right of KC
    if (hc != HK) l = L.lcol[64 * rb + lane];
    const double* pr = L.prow + 64 * hc;
    if (hc == 0) {
      if constexpr (HK == 0) t4_update<KK + 1>(A, pr, l);
    } else {
      t4_update<(HK == 1 ? KK + 1 : 0)>(A, pr, l);
    }
    t4_lu_col<KC + 1>(A, L, ord, rp_own, rc);
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
  const int rb = w & 1, hc = w >> 1;
  const int r = 64 * rb + lane;
  const bool own = r < N;
  const double* row = F + (own ? r : 0) * ldj + 64 * hc;
  const int jn = own ? N - 64 * hc : 0;    // entries of M in this lane's segment
  double A[64];
#pragma unroll
  for (int j = 0; j < 64; ++j) {
    const int c = 64 * hc + j;
    // the load is unconditional (row[j] lies in this work-group's LDS for every
    // j < 64) and masked afterwards: a conditional load becomes a branch with a
    // full LDS wait per entry
    const double v = row[j];
    const double f = (j < jn) ? v : 0.0;
    const double dj = ((c == r) & own) ? d : 0.0;
    A[j] = ((!own) & (c == r)) ? 1.0 : dj - f;
  }
  int ord = -1;
  double rp_own = 0.0;
  int rc = 0;
  t4_lu_col<0>(A, L, ord, rp_own, rc);
  if (rc) return rc;
  if (own) {
#pragma unroll
    for (int j = 0; j < 64; ++j)
      if (64 * hc + j < N) F[ord * ldj + 64 * hc + j] = A[j];
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
  // forward: L y = P b
#pragma unroll
  for (int k0 = 0; k0 < T4_NMAX; k0 += 8) {
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
