// Discrete adjoint of the ROS4 step, one wavefront per cell.
//
// Forward step (transformed Rosenbrock form, paper Sec. 2.3), frozen h:
//   M = I/(h gamma) - J(Phi)
//   u1 = M^-1 f(Phi)
//   u2 = M^-1 (f(Phi + a21 u1) + c21/h u1)
//   u3 = M^-1 (F3 + (c31 u1 + c32 u2)/h),   F3 = f(Phi + a31 u1 + a32 u2)
//   u4 = M^-1 (F3 + (c41 u1 + c42 u2 + c43 u3)/h)
//   Phi+ = Phi + sum m_i u_i
// Reverse sweep for lambda = dL/dPhi+ (mu_i = M^-T ubar_i):
//   ubar_i = m_i lambda; Phibar = lambda
//   stage 4: mu4;  F3bar = mu4;  ubar_{1,2,3} += c4j/h mu4
//   stage 3: mu3;  F3bar += mu3; ubar_{1,2} += c3j/h mu3
//            y3bar = J(Y3)^T F3bar;  Phibar += y3bar;  ubar_{1,2} += a3j y3bar;
//            lnAbar += f_p(Y3)^T F3bar
//   stage 2: mu2;  y2bar = J(Y2)^T mu2; Phibar += y2bar; ubar_1 += a21 y2bar + c21/h mu2;
//            lnAbar += f_p(Y2)^T mu2
//   stage 1: mu1;  Phibar += J(Phi)^T mu1;  lnAbar += f_p(Phi)^T mu1
//   through M(Phi): Phibar += sum_i d/de [J(Phi + e u_i)^T mu_i],
//                   lnAbar += sum_i d/de [f_p(Phi + e u_i)^T mu_i]
// J(Y)^T mu and f_p(Y)^T mu are vector-Jacobian products (team_vjp: reverse
// mode through f, no Jacobian formed); the last two terms are their
// directional derivatives, evaluated exactly by running team_vjp on dual
// numbers.
// f_p^T mu for reaction j: ln A_j scales the whole rate constant (both
// directions, both falloff limits), so d f / d ln A_j = (d f / d q_j) q_j and
//   (f_p^T mu)_j = q_j sum_k nu_kj wbar_k,
//   wbar_k = mu_T (-H_k/D) + mu_V V (-H_k/(D T) + R T/P) + [k < K-1] mu_{n_k} V.
#pragma once
#include "team.h"

namespace chem {

// Solve M^T x = b with the factors of team_lu (P M = L U, perm, 1/U_ii) and
// invperm, the inverse of perm.  b, x lane-distributed (lanes >= N hold 0 and
// keep it).  As in team_solve, every column step is unrolled over NMAX >= N
// (the steps past N change nothing), rows are read eight at a time (row k of
// the factors, element `lane`, for every k < NMAX lies in this work-group's
// LDS) and masked by selects on the loaded values.
template <int NMAX>
__device__ __forceinline__ double team_solve_t(const double* __restrict__ F, int ldj, int N,
                                               int invperm, double rdiag, double b) {
  const int lane = threadIdx.x;
  const double* col = F + lane;
  // U^T z = b (lower triangular): column k of U^T is row k of U
#pragma unroll
  for (int k0 = 0; k0 < NMAX; k0 += 8) {
    double u[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int k = k0 + t;
      const double v = col[k * ldj];
      u[t] = ((lane > k) & (lane < N)) ? v : 0.0;
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int k = k0 + t;
      const double zk = (k < N) ? bcast(b, k) * bcast(rdiag, k) : 0.0;
      const double nb = b - u[t] * zk;
      b = ((lane == k) & (k < N)) ? zk : nb;
    }
  }
  // L^T w = z (unit upper triangular)
#pragma unroll
  for (int k1 = NMAX - 1; k1 >= 1; k1 -= 8) {
    double l[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int k = k1 - t;
      const double v = col[(k >= 0 ? k : 0) * ldj];
      l[t] = ((lane < k) & (k < N)) ? v : 0.0;
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int k = k1 - t;
      if (k >= 1) {
        const double wk = (k < N) ? bcast(b, k) : 0.0;
        b -= l[t] * wk;
      }
    }
  }
  // x = P^T w
  return gather(b, invperm);
}

__device__ __forceinline__ double der(double) { return 0.0; }
__device__ __forceinline__ double der(Dd c) { return c.d; }
__device__ __forceinline__ Dd gather(Dd v, int src) { return Dd{gather(v.v, src), gather(v.d, src)}; }

// One reaction of the vector-Jacobian product's loop, slots up to SIDE per
// side (SIDE < MAX_SIDE when every reaction of the wavefront's pass has at
// most SIDE species a side): qbar, the ln A gradient, and the scatter of
// wdot and of Cbar through the rates; tacc and bacc collect the lane's sums
// of qbar dq/dT and qbar beta.
template <class S, int SIDE>
__device__ __forceinline__ void vjp_reaction(const MechView& M, const RxnRec& R, int j, S T, S lnT, S iT, S ctot,
                                             TeamLdsT<S>& L, S* dummy, double* __restrict__ pbar, bool add_value,
                                             S& tacc, S& bacc) {
  const RateOutT<S> r = reaction_rate<S, SIDE>(M, R, T, lnT, iT, ctot, LaneT<S>{L.conc, 1},
                                               LaneT<S>{L.gib, 1}, LaneT<S>{L.hrt, 1}, true);
  const int nr = R.nr, np = R.np;
  int ks[6], nus[6];
  bool on[6];
  S cs[6], ws[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    on[q] = (q % 3 < SIDE) && ((q < 3) ? (q < nr) : (q - 3 < np));
    ks[q] = R.sp[q];            // unused slots hold species 0 and coefficient 0
    nus[q] = R.nu[q];
    cs[q] = (q % 3 < SIDE) ? L.conc[ks[q]] : sc<S>(0.0);
    ws[q] = (q % 3 < SIDE) ? L.tb[ks[q]] : sc<S>(0.0);
  }
  // qbar: reactants, then products, in slot order
  S qb = sc<S>(0.0);
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    if (q % 3 >= SIDE) continue;
    const double v = (q < 3) ? -(double)nus[q] : (double)nus[q];
    if (on[q]) qb += v * ws[q];
  }
  const S c = r.q * qb;
  pbar[j] += (add_value ? val(c) : 0.0) + der(c);
  // d q / d C of slot q, as in team_rhs_jac
  S dq[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const int s0 = q < 3 ? 0 : 3;
    S d = (q < 3) ? r.kf : r.kr;
#pragma unroll
    for (int l = 0; l < SIDE; ++l) {
      const int v = (s0 + l == q) ? nus[s0 + l] - 1 : nus[s0 + l];
      const S cc = cs[s0 + l];
      d = (v >= 1) ? d * cc : d;
      d = (v >= 2) ? d * cc : d;
      d = (v >= 3) ? d * cc : d;
    }
    dq[q] = d * (double)(q < 3 ? nus[q] : -nus[q]);
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    if (q % 3 >= SIDE) continue;
    const double vk = (q < 3) ? -(double)nus[q] : (double)nus[q];
    lds_add(on[q] ? &L.wdot[ks[q]] : dummy, vk * r.q);
    lds_add(on[q] ? &L.gb[ks[q]] : dummy, qb * dq[q]);
  }
  tacc += qb * (r.dlnk_dT * r.q + r.kr_rr * r.dlnKc_dT);
  if (R.type != RX_ELEM) {
    // [M] = sum C + sum (alpha - 1) C: the uniform part summed per lane, the
    // listed efficiencies scattered (the first four read together)
    const S qbb = qb * r.beta;
    bacc += qbb;
    const int e0 = R.e0, e1 = R.e1;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = (e0 + t < e1) ? e0 + t : e0;
      const int m = M.eff_idx[e];
      const double am1 = M.eff_am1[e];
      lds_add((e0 + t < e1) ? &L.gb[m] : dummy, qbb * am1);
    }
    for (int e = e0 + 4; e < e1; ++e) lds_add(&L.gb[M.eff_idx[e]], qbb * M.eff_am1[e]);
  }
}

// J(y)^T mu and f_p(y)^T mu (added to pbar) without forming J: reverse mode
// through f.  With G = mu^T f,
//   f_T = Tdot = -num/D,  num = sum_k h_k wdot_k,  D = sum_k C_k cp_k,
//   f_V = V (Tdot/T + (R T/P) W),  W = sum_k wdot_k,  f_(n_k) = V wdot_k,
//   wdot_k = sum_j nu_kj q_j(T, C),
//   C_k = n_k / V (k < K-1),  C_b = P/(R T) - sum_(k<K-1) C_k:
// * wbar_k = dG/dwdot_k (as in the comment at the top) and qbar_j =
//   sum_k nu_kj wbar_k; (f_p^T mu)_j = q_j qbar_j;
// * through the rates: Cbar_m += qbar_j dq_j/dC_m (the reaction's species
//   slots, and beta_j alpha_jm through [M]), Tbar += qbar_j dq_j/dT;
// * directly: with Tdbar = dG/dTdot = mu_T + mu_V V/T,
//   Tbar += Tdbar (-(sum cp_k wdot_k) - Tdot dD/dT)/D + mu_V V (-Tdot/T^2 + R W/P),
//   Cbar_k += Tdbar (-Tdot/D) cp_k,
//   Vbar = mu_V (Tdot/T + (R T/P) W) + sum_(k<K-1) mu_(n_k) wdot_k;
// * through the closure: nbar_k = (Cbar_k - Cbar_b)/V,
//   Vbar -= sum_(k<K-1) (Cbar_k - Cbar_b) C_k / V,  Tbar -= Cbar_b P/(R T^2).
// S = Dd gives, in the dual part, the derivative of both products along the
// dual part of y (mu is fixed).  Returns ybar lane-distributed (T, V, n_k);
// pbar[j] gets (add_value ? value : 0) + derivative.
template <class S>
__device__ S team_vjp(const MechView& M, double P, S y, double mu, TeamLdsT<S>& L,
                      const double* __restrict__ lnA, double* __restrict__ pbar, bool add_value) {
  const int lane = threadIdx.x;
  const int K = M.K, N = M.N;
  S T, V, ctot, sdcp;
  team_state<S>(M, P, y, L, T, V, ctot, &sdcp);
  S den = sc<S>(0.0);
  if (lane < K) den = L.conc[lane] * L.cpr[lane] * RU;
  den = wave_sum(den);
  const double muT = bcast(mu, 0), muV = bcast(mu, 1);
  const double mun = gather(mu, lane + 2 < 64 ? lane + 2 : 0);
  const S RTP = RU * T / P;
  if (lane < K) {
    const S Hk = L.hrt[lane] * RU * T;
    S wb = muT * (-Hk / den) + muV * V * (-Hk / (den * T) + RTP);
    if (lane < K - 1) wb += mun * V;
    L.tb[lane] = wb;             // wbar_k
    L.wdot[lane] = sc<S>(0.0);
    L.gb[lane] = sc<S>(0.0);     // Cbar_k through the rates
  }
  wsync();
  const S lnT = log(T), iT = 1.0 / T;
  S tacc = sc<S>(0.0), bacc = sc<S>(0.0);   // this lane's sums of qbar dq/dT and qbar beta
  S* const dummy = L.dwdT + lane;           // target of the updates of unused slots
  const int Nr = M.Nr;
  RxnRec nx = load_rxn(M, lane < Nr ? lane : Nr - 1, lnA);   // fetched one reaction ahead
  for (int j = lane; j < Nr; j += 64) {
    const RxnRec R = nx;
    nx = load_rxn(M, j + 64 < Nr ? j + 64 : j, lnA);
    // most passes hold two-by-two reactions only: then the third slot of each
    // side is left out (a wave-uniform choice, once per pass)
    if (__all(R.nr <= 2 && R.np <= 2))
      vjp_reaction<S, 2>(M, R, j, T, lnT, iT, ctot, L, dummy, pbar, add_value, tacc, bacc);
    else
      vjp_reaction<S, MAX_SIDE>(M, R, j, T, lnT, iT, ctot, L, dummy, pbar, add_value, tacc, bacc);
  }
  wsync();
  S num = sc<S>(0.0), cpw = sc<S>(0.0), W = sc<S>(0.0), muw = sc<S>(0.0);
  if (lane < K) {
    const S w = L.wdot[lane];
    num = L.hrt[lane] * RU * T * w;
    cpw = L.cpr[lane] * RU * w;
    W = w;
    if (lane < K - 1) muw = mun * w;
  }
  num = wave_sum(num);
  cpw = wave_sum(cpw);
  W = wave_sum(W);
  muw = wave_sum(muw);
  tacc = wave_sum(tacc);
  bacc = wave_sum(bacc);
  const S Tdot = -num / den;
  const S Tdb = muT + muV * V * iT;
  S Tb = tacc + Tdb * (-(cpw + Tdot * (sdcp * RU)) / den) + muV * V * (-Tdot * iT * iT + RU * W / P);
  S Vb = muV * (Tdot * iT + RTP * W) + muw;
  S cb = sc<S>(0.0);
  if (lane < K) cb = L.gb[lane] + bacc + Tdb * (-Tdot / den) * (L.cpr[lane] * RU);
  const S cbb = bcast(cb, K - 1);
  S nb = sc<S>(0.0), vp = sc<S>(0.0);
  if (lane < K - 1) {
    const S d = cb - cbb;
    nb = d / V;
    vp = d * L.conc[lane];
  }
  Vb -= wave_sum(vp) / V;
  Tb += cbb * (-P / (RU * T * T));
  const S nsh = gather(nb, lane >= 2 ? lane - 2 : 0);
  S out = sc<S>(0.0);
  if (lane == 0) out = Tb;
  if (lane == 1) out = Vb;
  if (lane >= 2 && lane < N) out = nsh;
  wsync();
  return out;
}

}  // namespace chem
