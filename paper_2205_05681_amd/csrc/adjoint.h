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
// The last two terms are directional derivatives of the Jacobian and of
// f_p^T mu, evaluated exactly with forward-mode dual numbers.
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

// (J^T mu)_c for the Jacobian held in LDS (lanes over columns); rows are read
// eight at a time (a loop over blocks of eight rows up to NMAX >= N, with the
// rows past N masked), so that eight loads are in flight at once.
template <int NMAX>
__device__ __forceinline__ double team_jt_mu(const double* __restrict__ J, int ldj, int N, double mu) {
  const int lane = threadIdx.x;
  const double* col = J + lane;
  double acc = 0.0;
#pragma unroll 1
  for (int r0 = 0; r0 < NMAX; r0 += 8) {
    double e[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int r = r0 + t;
      const double v = col[r * ldj];
      e[t] = ((lane < N) & (r < N)) ? v : 0.0;
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int r = r0 + t;
      const double m = (r < N) ? bcast(mu, r) : 0.0;
      acc += e[t] * m;
    }
  }
  return acc;
}

// (dJ^T mu)_c and (J^T mu)_c for a dual Jacobian (value and directional derivative).
template <int NMAX>
__device__ __forceinline__ void team_jt_mu_dual(const Dd* __restrict__ J, int ldj, int N, double mu,
                                                double& val_part, double& der_part) {
  const int lane = threadIdx.x;
  const Dd* col = J + lane;
  double a = 0.0, b = 0.0;
#pragma unroll 1
  for (int r0 = 0; r0 < NMAX; r0 += 8) {
    double ev[8], ed[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int r = r0 + t;
      const Dd e = col[r * ldj];
      const bool on = (lane < N) & (r < N);
      ev[t] = on ? e.v : 0.0;
      ed[t] = on ? e.d : 0.0;
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int r = r0 + t;
      const double m = (r < N) ? bcast(mu, r) : 0.0;
      a += ev[t] * m;
      b += ed[t] * m;
    }
  }
  val_part = a;
  der_part = b;
}

__device__ __forceinline__ double der(double) { return 0.0; }
__device__ __forceinline__ double der(Dd c) { return c.d; }

// Adds (f_p(y)^T mu)_j (if add_value) and its derivative along the dual part
// of y to pbar[j] (LDS, Nr entries; lane j mod 64 owns reaction j).
template <class S>
__device__ void team_pbar(const MechView& M, double P, S y, double mu, TeamLdsT<S>& L,
                          const double* __restrict__ lnA, double* __restrict__ pbar, bool add_value) {
  const int lane = threadIdx.x;
  const int K = M.K;
  S T, V, ctot;
  team_state<S>(M, P, y, L, T, V, ctot, (S*)nullptr);
  S den = sc<S>(0.0);
  if (lane < K) den = L.conc[lane] * L.cpr[lane] * RU;
  den = wave_sum(den);
  const double muT = bcast(mu, 0), muV = bcast(mu, 1);
  const double mun = gather(mu, lane + 2 < 64 ? lane + 2 : 0);
  if (lane < K) {
    const S Hk = L.hrt[lane] * RU * T;
    S wb = muT * (-Hk / den) + muV * V * (-Hk / (den * T) + RU * T / P);
    if (lane < K - 1) wb += mun * V;
    L.wdot[lane] = wb;
  }
  wsync();
  const S lnT = log(T), iT = 1.0 / T;
  for (int j = lane; j < M.Nr; j += 64) {
    const RateOutT<S> r = reaction_rate(M, j, T, lnT, iT, ctot, LaneT<S>{L.conc, 1},
                                        LaneT<S>{L.gib, 1}, LaneT<S>{L.hrt, 1}, lnA, false);
    const int32_t* info = M.rinfo + 8 * j;
    const int32_t* sp = M.rspec + 6 * j;
    const int32_t* nu = M.rnu + 6 * j;
    S s = sc<S>(0.0);
    for (int i = 0; i < info[1]; ++i) s -= (double)nu[i] * L.wdot[sp[i]];
    for (int i = 0; i < info[2]; ++i) s += (double)nu[3 + i] * L.wdot[sp[3 + i]];
    const S c = r.q * s;
    pbar[j] += (add_value ? val(c) : 0.0) + der(c);
  }
  wsync();
}

}  // namespace chem
