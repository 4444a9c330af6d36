// Batched Rosenbrock integration (ROS4 by default; ROS3, RODAS3, RODAS4), one
// cell per thread (plain and persistent launch) or one wavefront per cell, and
// the C ABI that drives them.
//
// Method (paper Sec. 2.3, transformed Rosenbrock form; Table T:solvers):
//   M = I/(h gamma) - J(Phi_n), one LU per step;
//   M u_i = f(Phi_n + sum_{j<i} a_ij u_j) + sum_{j<i} (c_ij / h) u_j, i = 1..s,
//   a stage whose argument equals the previous stage's reusing its f;
//   Phi_{n+1} = Phi_n + sum m_j u_j, error estimate sum e_j u_j (optionally
//   filtered by (I - h gamma J)^-1 = M^-1 / (h gamma)).
// Step control (Sec. 3.1 tolerances; constants are this library's reading):
//   err = RMS_i(err_i / (atol + rtol max(|Phi_n,i|, |Phi_n+1,i|)));
//   accept if err <= 1; h <- h clamp(0.9 err^(-1/elo), 0.2, 6), no growth
//   right after a rejection; the last step is clipped to the remaining time;
//   the final proposal is returned for reuse (Sec. 2.4.1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/chem.h"
#include "kinetics.h"
#include "mech.h"
#include "methods.h"
#include "team.h"
#include "team4.h"
#include "adjoint.h"

namespace chem {

struct IntParams {
  MechView M;
  int64_t n;
  const double* T_in;
  const double* P;
  const double* Y_in;
  int64_t ldY;
  double* T_out;
  double* Y_out;
  double dt, rtol, atol, h_min, safety, fac_min, fac_max, T_cut;
  int32_t max_steps;
  int32_t estimator;           // CHEM_EST_*
  int32_t jac_every;           // J at every jac_every-th accepted state, kept in between
  RosTable tab;                // the method's coefficients
  double* h_io;
  int32_t* n_steps;
  int32_t* status;
  const double* lnA;
  double* ws;
  int32_t* piv;
  int64_t ld;
  unsigned int* queue;
  const int32_t* order;        // nullable: queue position -> cell
  double* jsave;               // nullable: per work-group copy of J, [grid][N][N]
  unsigned long long* stats;   // nullable: attempts, accepted, rejected
  // adjoint checkpoint (ck_arena nullable): the (Phi_n, h_n) record of every
  // accepted step, in chunks of CK_CHUNK records claimed from a counter as a
  // cell needs them; a cell's chunks are linked backwards
  double* ck_arena;               // [ck_cap][CK_CHUNK][N+1]
  int64_t* ck_prev;               // [ck_cap] the cell's previous chunk, -1 for its first
  unsigned long long* ck_used;    // chunks claimed (past ck_cap: the arena overflowed)
  int64_t ck_cap;
  int64_t* ck_head;               // [n] chunk of the cell's last record (-1: none, -2: overflow)
  double* ck_final;               // [n][N+1] final Phi
  int32_t* ck_count;              // [n] accepted steps
};

constexpr int CK_CHUNK = 16;

// A new chunk for a cell whose current chunk is cur; -2 once the arena is full
// (the cell records nothing more and the host repeats the call with room).
__device__ __forceinline__ int64_t ck_claim(const IntParams& p, int64_t cur) {
  const unsigned long long c = atomicAdd(p.ck_used, 1ull);
  if (c >= (unsigned long long)p.ck_cap) return -2;
  p.ck_prev[c] = cur;
  return (int64_t)c;
}

// The chunk for record `accepted` of a cell (claimed by the calling lane when
// the record opens a chunk).
__device__ __forceinline__ int64_t ck_chunk_for(const IntParams& p, int64_t cur, int accepted) {
  if (cur == -2) return -2;
  return (accepted % CK_CHUNK == 0) ? ck_claim(p, cur) : cur;
}

// Wave-uniform chunk: lane 0 claims, every lane takes its answer.
__device__ __forceinline__ int64_t ck_chunk_wave(const IntParams& p, int64_t cur, int accepted) {
  int64_t c = cur;
  if (threadIdx.x % 64 == 0) c = ck_chunk_for(p, cur, accepted);
  const int lo = __shfl((int)(c & 0xffffffff), 0, 64), hi = __shfl((int)(c >> 32), 0, 64);
  return (int64_t)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// ------------------------------------------------------------------ per-lane linear algebra
// In-place LU with partial pivoting of the N x N matrix A (row-major, lane
// strided).  Ties go to the lowest row.  Returns 0, 1 (zero pivot) or
// 2 (non-finite column).
__device__ int lu_factor(Lane A, int32_t* __restrict__ piv, int64_t ld, int N) {
  for (int k = 0; k < N; ++k) {
    int p = k;
    double best = fabs(A[k * N + k]);
    bool finite = isfinite(best);
    for (int i = k + 1; i < N; ++i) {
      const double v = fabs(A[i * N + k]);
      finite = finite && isfinite(v);
      if (v > best) {
        best = v;
        p = i;
      }
    }
    if (!finite) return 2;
    if (!(best > 0.0)) return 1;
    piv[(int64_t)k * ld] = p;
    if (p != k) {
      for (int j = 0; j < N; ++j) {
        const double t = A[k * N + j];
        A[k * N + j] = A[p * N + j];
        A[p * N + j] = t;
      }
    }
    const double inv = 1.0 / A[k * N + k];
    for (int i = k + 1; i < N; ++i) {
      const double l = A[i * N + k] * inv;
      A[i * N + k] = l;
      if (l != 0.0)
        for (int j = k + 1; j < N; ++j) A[i * N + j] -= l * A[k * N + j];
    }
  }
  return 0;
}

__device__ void lu_solve(Lane A, const int32_t* __restrict__ piv, int64_t ld, int N, Lane b) {
  for (int k = 0; k < N; ++k) {
    const int p = piv[(int64_t)k * ld];
    if (p != k) {
      const double t = b[k];
      b[k] = b[p];
      b[p] = t;
    }
  }
  for (int i = 1; i < N; ++i) {
    double s = b[i];
    for (int j = 0; j < i; ++j) s -= A[i * N + j] * b[j];
    b[i] = s;
  }
  for (int i = N - 1; i >= 0; --i) {
    double s = b[i];
    for (int j = i + 1; j < N; ++j) s -= A[i * N + j] * b[j];
    b[i] = s / A[i * N + i];
  }
}

// ------------------------------------------------------------------ conversions
// (T, P, Y) -> Phi per unit mass (eq. (conc_form1)): V = R T / (P Wbar), n_k = Y_k/W_k.
__device__ void to_phi(const MechView& M, double T, double P, const double* __restrict__ Y,
                       int64_t ldY, int64_t cell, Lane phi) {
  double inv = 0.0;
  for (int k = 0; k < M.K; ++k) {
    const double y = Y[(int64_t)k * ldY + cell] / M.W[k];
    inv += y;
    if (k < M.K - 1) phi[2 + k] = y;
  }
  phi[0] = T;
  phi[1] = RU * T * inv / P;
}

// Phi -> (T, Y): n_K = P V/(R T) - sum n_k, Y_k = n_k W_k / sum n W.
__device__ void from_phi(const MechView& M, double P, Lane phi, double* __restrict__ Y, int64_t ldY,
                         int64_t cell, double* T_out) {
  const int K = M.K;
  double s = 0.0, mass = 0.0;
  for (int k = 0; k < K - 1; ++k) {
    s += phi[2 + k];
    mass += phi[2 + k] * M.W[k];
  }
  const double nb = P * phi[1] / (RU * phi[0]) - s;
  mass += nb * M.W[K - 1];
  const double im = 1.0 / mass;
  const double T = phi[0];
  for (int k = 0; k < K - 1; ++k) Y[(int64_t)k * ldY + cell] = phi[2 + k] * M.W[k] * im;
  Y[(int64_t)(K - 1) * ldY + cell] = nb * M.W[K - 1] * im;
  *T_out = T;
}

// ------------------------------------------------------------------ one-cell-per-thread integrator
template <bool PERSISTENT>
__global__ void __launch_bounds__(256) integrate_thread_kernel(IntParams p) {
  const MechView& M = p.M;
  const int N = M.N;
  const WsLayout L{N, M.K};
  const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ld = p.ld;
  if (slot >= ld) return;
  double* base = p.ws + slot;
  int32_t* piv = p.piv + slot;
  Lane phi{base + L.phi() * ld, ld}, ynew{base + L.ynew() * ld, ld};
  Lane f1{base + L.f1() * ld, ld}, fs{base + L.fs() * ld, ld}, ys{base + L.ys() * ld, ld};
  auto u = [&](int i) { return Lane{base + (int64_t)L.u(i) * ld, ld}; };   // stage vectors
  Lane J{base + (int64_t)L.jac() * ld, ld}, A{base + (int64_t)L.lu() * ld, ld};
  Lane conc{base + L.conc() * ld, ld}, wdot{base + L.wdot() * ld, ld};
  Lane hrt{base + L.hrt() * ld, ld}, cpr{base + L.cpr() * ld, ld}, gib{base + L.gibbs() * ld, ld};

  int64_t q = PERSISTENT ? (int64_t)atomicAdd(p.queue, 1u) : slot;   // queue position
  bool have = q < p.n;
  int64_t cell = have ? (p.order ? p.order[q] : q) : 0;
  // per-cell controller state
  double P = 0, h = 0, rem = 0;
  int attempts = 0, accepted = 0, bad = 0, status = 0;
  bool last_rej = false, need_f = false, done = false;
  int since_jac = 0, jac_evals = 0;   // accepted steps since J was evaluated; J evaluations
  int64_t ck_chunk = -1;

  auto init = [&](int64_t c) {
    P = p.P[c];
    const double T = p.T_in[c];
    to_phi(M, T, P, p.Y_in, p.ldY, c, phi);
    rem = p.dt;
    h = p.dt;
    if (p.h_io && p.h_io[c] > 0.0) h = p.h_io[c];
    attempts = accepted = bad = status = 0;
    last_rej = false;
    since_jac = p.jac_every;
    need_f = false;
    jac_evals = 0;
    done = !(T >= p.T_cut);     // T_cut = 0 integrates every cell (NaN T included)
    if (p.T_cut <= 0.0) done = false;
    ck_chunk = -1;
  };
  auto finish = [&](int64_t c) {
    if (p.ck_arena) {
      double* fin = p.ck_final + c * (int64_t)(N + 1);
      for (int i = 0; i < N; ++i) fin[i] = phi[i];
      fin[N] = 0.0;
      p.ck_head[c] = ck_chunk;
    }
    double T;
    from_phi(M, P, phi, p.Y_out, p.ldY, c, &T);
    p.T_out[c] = T;
    if (p.h_io) p.h_io[c] = h;
    if (p.n_steps) p.n_steps[c] = accepted;
    if (p.status) p.status[c] = status;
    if (p.ck_count) p.ck_count[c] = accepted;
    if (p.stats) {
      atomicAdd(&p.stats[0], (unsigned long long)attempts);
      atomicAdd(&p.stats[1], (unsigned long long)accepted);
      atomicAdd(&p.stats[2], (unsigned long long)(attempts - accepted));
      atomicAdd(&p.stats[3], (unsigned long long)jac_evals);
    }
  };
  if (have) init(cell);

  while (have) {
    if (!done) {
      if (attempts >= p.max_steps) {
        status = CHEM_CELL_MAX_STEPS;
        done = true;
      } else if (h < p.h_min) {
        status = CHEM_CELL_H_MIN;
        done = true;
      }
    }
    if (!done) {
      ++attempts;
      const double hs = fmin(h, rem);
      // J at every jac_every-th accepted state (and the first); in between
      // only f at the new state - a rejected step keeps both
      if (since_jac >= p.jac_every) {
        eval_rhs_jac(M, P, phi, f1, J, L, base, ld, p.lnA);
        since_jac = 0;
        need_f = false;
        ++jac_evals;
      } else if (need_f) {
        eval_rhs(M, P, phi, f1, conc, wdot, hrt, cpr, gib, p.lnA);
        need_f = false;
      }
      const RosTable& R = p.tab;
      const double d = 1.0 / (hs * R.gamma);
      for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) A[i * N + j] = (i == j ? d : 0.0) - J[i * N + j];
      const int rc = lu_factor(A, piv, ld, N);
      double err = 0.0;
      if (rc == 0) {
        // stage i: f at phi + sum_{j<i} a_ij u_j (or the previous stage's f
        // when the argument is the same), then M u_i = f + sum_{j<i} (c_ij/h) u_j
        for (int i = 0; i < R.s; ++i) {
          Lane ui = u(i);
          if (i == 0) {
            for (int k = 0; k < N; ++k) fs[k] = f1[k];
          } else if (R.newf[i]) {
            for (int k = 0; k < N; ++k) {
              double y = phi[k];
              for (int j = 0; j < i; ++j) y += R.a[i][j] * u(j)[k];
              ys[k] = y;
            }
            eval_rhs(M, P, ys, fs, conc, wdot, hrt, cpr, gib, p.lnA);
          }
          for (int k = 0; k < N; ++k) {
            double r = fs[k];
            for (int j = 0; j < i; ++j) r += (R.c[i][j] / hs) * u(j)[k];
            ui[k] = r;
          }
          lu_solve(A, piv, ld, N, ui);
        }
        // new state and error estimate (into ys; filtered in place if asked)
        for (int k = 0; k < N; ++k) {
          double yn = phi[k], e = 0.0;
          for (int j = 0; j < R.s; ++j) {
            const double uj = u(j)[k];
            yn += R.m[j] * uj;
            e += R.e[j] * uj;
          }
          ynew[k] = yn;
          ys[k] = e;
        }
        if (p.estimator == CHEM_EST_FILTERED) {
          lu_solve(A, piv, ld, N, ys);
          for (int k = 0; k < N; ++k) ys[k] = ys[k] / (hs * R.gamma);
        }
        for (int k = 0; k < N; ++k) {
          const double sc = p.atol + p.rtol * fmax(fabs(phi[k]), fabs(ynew[k]));
          const double r = ys[k] / sc;
          err += r * r;
        }
        err = sqrt(err / N);
      }
      if (rc != 0 || !isfinite(err)) {
        if (++bad >= 10) {
          status = (rc == 1) ? CHEM_CELL_SINGULAR : CHEM_CELL_NONFINITE;
          done = true;
        } else {
          h = hs * p.fac_min;
          last_rej = true;
        }
      } else {
        bad = 0;
        double fac = (err > 0.0) ? p.safety * pow(err, -1.0 / p.tab.elo) : p.fac_max;
        if (err <= 1.0) {
          if (p.ck_arena) {
            ck_chunk = ck_chunk_for(p, ck_chunk, accepted);
            if (ck_chunk >= 0) {
              double* rec = p.ck_arena + (ck_chunk * CK_CHUNK + accepted % CK_CHUNK) * (int64_t)(N + 1);
              for (int i = 0; i < N; ++i) rec[i] = phi[i];
              rec[N] = hs;
            }
          }
          for (int i = 0; i < N; ++i) phi[i] = ynew[i];
          rem -= hs;
          ++accepted;
          fac = fmin(p.fac_max, fmax(p.fac_min, fac));
          if (last_rej) fac = fmin(fac, 1.0);
          last_rej = false;
          ++since_jac;
          need_f = true;
          if (rem <= 0.0) done = true;
        } else {
          fac = fmin(1.0, fmax(p.fac_min, fac));
          last_rej = true;
        }
        h = hs * fac;
      }
    }
    if (done) {
      finish(cell);
      if (PERSISTENT) {
        q = atomicAdd(p.queue, 1u);
        have = q < p.n;
        if (have) {
          cell = p.order ? p.order[q] : q;
          init(cell);
        }
      } else {
        have = false;
      }
    }
  }
}


// ------------------------------------------------------------------ one-wavefront-per-cell integrator
template <int NMAX>
__global__ void __launch_bounds__(64) integrate_team_kernel(IntParams p, bool PERSISTENT) {
  extern __shared__ double lds_raw[];
  const MechView& M = p.M;
  const int N = M.N, K = M.K, ldj = N + 1;
  const int lane = threadIdx.x;
  TeamLds L;
  L.bind(lds_raw, N);
  int64_t q;   // queue position
  if (PERSISTENT) {
    unsigned c0 = 0;
    if (lane == 0) c0 = atomicAdd(p.queue, 1u);
    q = (unsigned)__shfl((int)c0, 0, 64);
  } else {
    q = blockIdx.x;
  }
  while (q < p.n) {
    const int64_t cell = p.order ? p.order[q] : q;
    // ---- input conversion (eq. (conc_form1)), element i of Phi in lane i
    const double P = p.P[cell];
    const double T0 = p.T_in[cell];
    double yk = 0.0;
    if (lane < K) yk = p.Y_in[(int64_t)lane * p.ldY + cell] / M.W[lane];
    const double inv = wave_sum(yk);
    const double ysh = gather(yk, lane >= 2 ? lane - 2 : 0);
    double phi = 0.0;
    if (lane == 0) phi = T0;
    if (lane == 1) phi = RU * T0 * inv / P;
    if (lane >= 2 && lane < N) phi = ysh;
    double rem = p.dt, h = p.dt;
    if (p.h_io && p.h_io[cell] > 0.0) h = p.h_io[cell];
    int attempts = 0, accepted = 0, bad = 0, status = 0;
    bool last_rej = false, need_f = false;   // need_f: Phi changed since f1 was evaluated
    int since_jac = p.jac_every, jac_evals = 0;   // accepted steps since J was evaluated
    bool done = (p.T_cut > 0.0) && !(T0 >= p.T_cut);
    int64_t ck_chunk = -1;
    double f1 = 0.0;
    while (!done) {
      if (attempts >= p.max_steps) {
        status = CHEM_CELL_MAX_STEPS;
        break;
      }
      if (h < p.h_min) {
        status = CHEM_CELL_H_MIN;
        break;
      }
      ++attempts;
      const double hs = fmin(h, rem);
      // J(Phi) into LDS at every jac_every-th accepted state (and the first),
      // in between only f at the new state; a rejected step keeps both (same
      // Phi; the factors live in registers, J is not overwritten)
      if (since_jac >= p.jac_every) {
        f1 = team_rhs_jac(M, P, phi, L, p.lnA);
        since_jac = 0;
        need_f = false;
        ++jac_evals;
      } else if (need_f) {
        f1 = team_rhs(M, P, phi, L, p.lnA);
        need_f = false;
      }
      // factors of M = I/(h gamma) - J, row i in lane i's registers
      RegLU<NMAX> F;
      const RosTable& R = p.tab;
      const int rc = team_lu_reg<NMAX>(L.J, ldj, N, 1.0 / (hs * R.gamma), F);
      double err = 0.0, ynew = 0.0;
      if (rc == 0) {
        // stage i: f at phi + sum_{j<i} a_ij u_j (or the previous stage's f
        // when the argument is the same), then M u_i = f + sum_{j<i} (c_ij/h)
        // u_j.  Lane i keeps element i of every stage vector in the LDS stage
        // area (a per-lane array indexed by the stage, read back by the same
        // lane only, so no barrier is needed).
        double fs = f1;
#pragma unroll 1
        for (int i = 0; i < R.s; ++i) {
          if (i > 0 && R.newf[i]) {
            double y = phi;
            for (int j = 0; j < i; ++j) y += R.a[i][j] * L.ust[64 * j + lane];
            fs = team_rhs(M, P, y, L, p.lnA);
          }
          double r = fs;
          for (int j = 0; j < i; ++j) r += (R.c[i][j] / hs) * L.ust[64 * j + lane];
          L.ust[64 * i + lane] = team_solve_reg<NMAX>(F, N, r);
        }
        double e = 0.0;
        ynew = phi;
        for (int j = 0; j < R.s; ++j) {
          const double uj = L.ust[64 * j + lane];
          ynew += R.m[j] * uj;
          e += R.e[j] * uj;
        }
        if (p.estimator == CHEM_EST_FILTERED)
          e = team_solve_reg<NMAX>(F, N, e) / (hs * R.gamma);
        const double sc = p.atol + p.rtol * fmax(fabs(phi), fabs(ynew));
        const double r = (lane < N) ? e / sc : 0.0;
        err = sqrt(wave_sum(r * r) / N);
      }
      if (rc != 0 || !isfinite(err)) {
        if (++bad >= 10) {
          status = (rc == 1) ? CHEM_CELL_SINGULAR : CHEM_CELL_NONFINITE;
          break;
        }
        h = hs * p.fac_min;
        last_rej = true;
        continue;
      }
      bad = 0;
      double fac = (err > 0.0) ? p.safety * pow(err, -1.0 / p.tab.elo) : p.fac_max;
      if (err <= 1.0) {
        if (p.ck_arena) {
          ck_chunk = ck_chunk_wave(p, ck_chunk, accepted);
          if (ck_chunk >= 0) {
            double* rec = p.ck_arena + (ck_chunk * CK_CHUNK + accepted % CK_CHUNK) * (int64_t)(N + 1);
            if (lane < N) rec[lane] = phi;
            if (lane == 0) rec[N] = hs;
          }
        }
        phi = ynew;
        ++since_jac;
        need_f = true;
        rem -= hs;
        ++accepted;
        fac = fmin(p.fac_max, fmax(p.fac_min, fac));
        if (last_rej) fac = fmin(fac, 1.0);
        last_rej = false;
        h = hs * fac;
        if (rem <= 0.0) break;
      } else {
        fac = fmin(1.0, fmax(p.fac_min, fac));
        last_rej = true;
        h = hs * fac;
      }
    }
    if (p.ck_arena) {
      double* fin = p.ck_final + cell * (int64_t)(N + 1);
      if (lane < N) fin[lane] = phi;
      if (lane == 0) {
        fin[N] = 0.0;
        p.ck_head[cell] = ck_chunk;
      }
    }
    // ---- output conversion: n_K from the ideal-gas closure, Y_k = n_k W_k / mass
    {
      const double T = bcast(phi, 0), V = bcast(phi, 1);
      const double nk = gather(phi, lane + 2 < 64 ? lane + 2 : 0);
      const double n_here = (lane < K - 1) ? nk : 0.0;
      const double s = wave_sum(n_here);
      const double nb = P * V / (RU * T) - s;
      const double nn = (lane < K - 1) ? n_here : (lane == K - 1 ? nb : 0.0);
      const double mass = wave_sum(lane < K ? nn * M.W[lane] : 0.0);
      if (lane < K) p.Y_out[(int64_t)lane * p.ldY + cell] = nn * M.W[lane] / mass;
      if (lane == 0) {
        p.T_out[cell] = T;
        if (p.h_io) p.h_io[cell] = h;
        if (p.n_steps) p.n_steps[cell] = accepted;
        if (p.status) p.status[cell] = status;
        if (p.ck_count) p.ck_count[cell] = accepted;
        if (p.stats) {
          atomicAdd(&p.stats[0], (unsigned long long)attempts);
          atomicAdd(&p.stats[1], (unsigned long long)accepted);
          atomicAdd(&p.stats[2], (unsigned long long)(attempts - accepted));
          atomicAdd(&p.stats[3], (unsigned long long)jac_evals);
        }
      }
    }
    if (PERSISTENT) {
      unsigned c1 = 0;
      if (lane == 0) c1 = atomicAdd(p.queue, 1u);
      q = (unsigned)__shfl((int)c1, 0, 64);
    } else {
      break;
    }
  }
}


// ------------------------------------------------------------------ four wavefronts per cell (64 < N <= 128)
// The same integrator as integrate_team_kernel, on a work-group of four
// wavefronts per cell (team4.h).  Every wavefront holds the state and stage
// vectors and runs the same controller, so all its decisions are uniform over
// the work-group; source terms, Jacobian and LU are split over the 256 threads.
__global__ void __launch_bounds__(256) integrate_team4_kernel(IntParams p, bool PERSISTENT) {
  extern __shared__ double lds_raw[];
  const MechView& M = p.M;
  const int N = M.N, K = M.K, ldj = N + 1;
  const int tid = t4_tid(), w = t4_wave(), lane = t4_lane();
  Team4Lds L;
  L.bind(lds_raw, N, p.tab.s);
  double* const ust = L.ust + w * (p.tab.s * 128);   // this wavefront's stage vectors
  double* const jsv = p.jsave ? p.jsave + (int64_t)blockIdx.x * N * N : nullptr;
  int64_t q;
  if (PERSISTENT) {
    if (tid == 0) L.misc[0] = (int)atomicAdd(p.queue, 1u);
    wsync();
    q = (unsigned)L.misc[0];
    wsync();
  } else {
    q = blockIdx.x;
  }
  while (q < p.n) {
    const int64_t cell = p.order ? p.order[q] : q;
    // ---- input conversion (eq. (conc_form1)), every wavefront
    const double P = p.P[cell];
    const double T0 = p.T_in[cell];
    const double y0 = (lane < K) ? p.Y_in[(int64_t)lane * p.ldY + cell] / M.W[lane] : 0.0;
    const double y1 = (64 + lane < K) ? p.Y_in[(int64_t)(64 + lane) * p.ldY + cell] / M.W[64 + lane] : 0.0;
    const V2 yw{y0, y1};
    const double inv = v2_sum(yw);
    V2 phi;
    {
      const double s0 = v2_gather(yw, (lane + 126) & 127);   // element lane - 2 (lanes >= 2)
      const double s1 = v2_gather(yw, 62 + lane);             // element 62 + lane
      phi.a = (lane == 0) ? T0 : (lane == 1) ? RU * T0 * inv / P : s0;
      phi.b = (64 + lane < N) ? s1 : 0.0;
    }
    double rem = p.dt, h = p.dt;
    if (p.h_io && p.h_io[cell] > 0.0) h = p.h_io[cell];
    int attempts = 0, accepted = 0, bad = 0, status = 0;
    bool last_rej = false, need_f = false;
    int since_jac = p.jac_every, jac_evals = 0;
    bool done = (p.T_cut > 0.0) && !(T0 >= p.T_cut);
    int64_t ck_chunk = -1;   // kept by wavefront 0, which writes the records
    V2 f1{0.0, 0.0};
    while (!done) {
      if (attempts >= p.max_steps) {
        status = CHEM_CELL_MAX_STEPS;
        break;
      }
      if (h < p.h_min) {
        status = CHEM_CELL_H_MIN;
        break;
      }
      ++attempts;
      const double hs = fmin(h, rem);
      // J at every jac_every-th accepted state (and the first), saved; the
      // LU overwrites it, so in between and after a rejection it is reloaded
      // (without a saved copy - jac_every is then 1 - evaluated again at the
      // same state), with f alone at a new state
      if (since_jac >= p.jac_every || !jsv) {
        f1 = t4_rhs_jac(M, P, phi, L, p.lnA);
        since_jac = 0;
        need_f = false;
        ++jac_evals;
        if (jsv && tid < N)
          for (int i = 0; i < N; ++i) jsv[i * N + tid] = L.J[i * ldj + tid];
      } else {
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");   // own stores done, L1 invalidated
        if (tid < N)
          for (int i = 0; i < N; ++i) L.J[i * ldj + tid] = jsv[i * N + tid];
        wsync();
        if (need_f) {
          f1 = t4_rhs(M, P, phi, L, p.lnA);
          need_f = false;
        }
      }
      const RosTable& R = p.tab;
      const int rc = t4_lu(L.J, ldj, N, 1.0 / (hs * R.gamma), L);
      double err = 0.0;
      V2 ynew{0.0, 0.0};
      if (rc == 0) {
        const double* F = L.J;
        V2 fs = f1;
#pragma unroll 1
        for (int i = 0; i < R.s; ++i) {
          if (i > 0 && R.newf[i]) {
            V2 y = phi;
            for (int j = 0; j < i; ++j) {
              y.a += R.a[i][j] * ust[128 * j + lane];
              y.b += R.a[i][j] * ust[128 * j + 64 + lane];
            }
            fs = t4_rhs(M, P, y, L, p.lnA);
          }
          V2 r = fs;
          for (int j = 0; j < i; ++j) {
            r.a += (R.c[i][j] / hs) * ust[128 * j + lane];
            r.b += (R.c[i][j] / hs) * ust[128 * j + 64 + lane];
          }
          const V2 u = t4_solve(F, ldj, N, L, r);
          ust[128 * i + lane] = u.a;
          ust[128 * i + 64 + lane] = u.b;
        }
        V2 e{0.0, 0.0};
        ynew = phi;
        for (int j = 0; j < R.s; ++j) {
          const double ua = ust[128 * j + lane], ub = ust[128 * j + 64 + lane];
          ynew.a += R.m[j] * ua;
          ynew.b += R.m[j] * ub;
          e.a += R.e[j] * ua;
          e.b += R.e[j] * ub;
        }
        if (p.estimator == CHEM_EST_FILTERED) {
          const V2 ef = t4_solve(F, ldj, N, L, e);
          e.a = ef.a / (hs * R.gamma);
          e.b = ef.b / (hs * R.gamma);
        }
        const double sa = p.atol + p.rtol * fmax(fabs(phi.a), fabs(ynew.a));
        const double sb = p.atol + p.rtol * fmax(fabs(phi.b), fabs(ynew.b));
        const double ra = (lane < N) ? e.a / sa : 0.0;
        const double rb = (64 + lane < N) ? e.b / sb : 0.0;
        err = sqrt(wave_sum(ra * ra + rb * rb) / N);
      }
      if (rc != 0 || !isfinite(err)) {
        if (++bad >= 10) {
          status = (rc == 1) ? CHEM_CELL_SINGULAR : CHEM_CELL_NONFINITE;
          break;
        }
        h = hs * p.fac_min;
        last_rej = true;
        continue;
      }
      bad = 0;
      double fac = (err > 0.0) ? p.safety * pow(err, -1.0 / p.tab.elo) : p.fac_max;
      if (err <= 1.0) {
        if (p.ck_arena && w == 0) {
          ck_chunk = ck_chunk_wave(p, ck_chunk, accepted);
          if (ck_chunk >= 0) {
            double* rec = p.ck_arena + (ck_chunk * CK_CHUNK + accepted % CK_CHUNK) * (int64_t)(N + 1);
            rec[lane] = phi.a;
            if (64 + lane < N) rec[64 + lane] = phi.b;
            if (lane == 0) rec[N] = hs;
          }
        }
        phi = ynew;
        ++since_jac;
        need_f = true;
        rem -= hs;
        ++accepted;
        fac = fmin(p.fac_max, fmax(p.fac_min, fac));
        if (last_rej) fac = fmin(fac, 1.0);
        last_rej = false;
        h = hs * fac;
        if (rem <= 0.0) break;
      } else {
        fac = fmin(1.0, fmax(p.fac_min, fac));
        last_rej = true;
        h = hs * fac;
      }
    }
    if (w == 0) {
      if (p.ck_arena) {
        double* fin = p.ck_final + cell * (int64_t)(N + 1);
        fin[lane] = phi.a;
        if (64 + lane < N) fin[64 + lane] = phi.b;
        if (lane == 0) {
          fin[N] = 0.0;
          p.ck_head[cell] = ck_chunk;
        }
      }
      // ---- output conversion: n_K from the ideal-gas closure, Y_k = n_k W_k / mass
      const double T = v2_get(phi, 0), V = v2_get(phi, 1);
      const double n0 = v2_gather(phi, lane + 2);          // species lane
      const double n1 = v2_gather(phi, (66 + lane) & 127); // species 64 + lane
      const double h0 = (lane < K - 1) ? n0 : 0.0;
      const double h1 = (64 + lane < K - 1) ? n1 : 0.0;
      const double s = wave_sum(h0 + h1);
      const double nb = P * V / (RU * T) - s;
      const double nn0 = (lane < K - 1) ? h0 : (lane == K - 1 ? nb : 0.0);
      const double nn1 = (64 + lane < K - 1) ? h1 : (64 + lane == K - 1 ? nb : 0.0);
      const double m0 = (lane < K) ? nn0 * M.W[lane] : 0.0;
      const double m1 = (64 + lane < K) ? nn1 * M.W[64 + lane] : 0.0;
      const double mass = wave_sum(m0 + m1);
      if (lane < K) p.Y_out[(int64_t)lane * p.ldY + cell] = m0 / mass;
      if (64 + lane < K) p.Y_out[(int64_t)(64 + lane) * p.ldY + cell] = m1 / mass;
      if (lane == 0) {
        p.T_out[cell] = T;
        if (p.h_io) p.h_io[cell] = h;
        if (p.n_steps) p.n_steps[cell] = accepted;
        if (p.status) p.status[cell] = status;
        if (p.ck_count) p.ck_count[cell] = accepted;
        if (p.stats) {
          atomicAdd(&p.stats[0], (unsigned long long)attempts);
          atomicAdd(&p.stats[1], (unsigned long long)accepted);
          atomicAdd(&p.stats[2], (unsigned long long)(attempts - accepted));
          atomicAdd(&p.stats[3], (unsigned long long)jac_evals);
        }
      }
    }
    if (PERSISTENT) {
      wsync();   // every wavefront is done with this cell's LDS
      if (tid == 0) L.misc[0] = (int)atomicAdd(p.queue, 1u);
      wsync();
      q = (unsigned)L.misc[0];
      wsync();
    } else {
      break;
    }
  }
}


// ------------------------------------------------------------------ discrete adjoint, one wavefront per cell
struct AdjParams {
  MechView M;
  int64_t n;
  const double* ck_arena;  // the checkpoint's record chunks (as in IntParams)
  const int64_t* ck_prev;
  const int64_t* ck_head;
  const double* ck_final;
  const int32_t* ck_count;
  const int32_t* order;    // [n] work-group -> cell
  const double* P;         // [n]
  const double* T0;        // [n] initial state (copy)
  const double* Y0;        // [K][n]
  const double* gT;        // [n]
  const double* gY;        // [K][ldY]
  int64_t ldY;
  const double* lnA;       // nullable, as in the forward call
  double* g_cell;          // [Nr][n] per-cell d L / d ln A, file order
  double* gT0;             // nullable [n]
  double* gY0;             // nullable [K][ldY]
};

template <int NMAX>
__global__ void __launch_bounds__(64) adjoint_team_kernel(AdjParams a) {
  extern __shared__ double lds_raw[];
  const MechView& M = a.M;
  const int N = M.N, K = M.K, ldj = N + 1;
  const int lane = threadIdx.x;
  // LDS: J and its factors, the vector block (doubles), the vector block of
  // the dual products, the pivot staging, this cell's d L / d ln A
  const size_t mat = (size_t)N * ldj, ve = TeamLdsT<double>::vec_elems(N);
  double* vb = lds_raw + mat;
  Dd* vbd = (Dd*)(vb + ve);
  int* plane = (int*)(vb + 3 * ve);
  double* pbar = vb + 3 * ve + 32;   // [Nr]
  TeamLdsT<double> LA;
  TeamLdsT<Dd> LD;
  LA.bind2(lds_raw, vb, plane, N);
  LD.bind2(nullptr, vbd, plane, N);
  if ((int64_t)blockIdx.x >= a.n) return;
  const int64_t cell = a.order[blockIdx.x];
  const double P = a.P[cell];
  const int64_t cnt = a.ck_count[cell];

  // ---- output conversion adjoint: L = gT T + sum_k gY_k Y_k,
  //      Y_i = a_i / m, a_k = n_k W_k, a_b = n_b W_b, n_b = P V/(R T) - sum n_k
  double lam;
  {
    const double* fin = a.ck_final + cell * (int64_t)(N + 1);
    const double phi = (lane < N) ? fin[lane] : 0.0;
    const double T = bcast(phi, 0), V = bcast(phi, 1);
    const double nk = gather(phi, lane + 2 < 64 ? lane + 2 : 0);
    const double n_here = (lane < K - 1) ? nk : 0.0;
    const double nb = P * V / (RU * T) - wave_sum(n_here);
    const double ai = (lane < K - 1) ? n_here * M.W[lane] : (lane == K - 1 ? nb * M.W[K - 1] : 0.0);
    const double mass = wave_sum(ai);
    const double gy = (lane < K) ? a.gY[(int64_t)lane * a.ldY + cell] : 0.0;
    const double sgy = wave_sum(gy * ai) / mass;
    const double abar = (lane < K) ? (gy - sgy) / mass : 0.0;     // d L / d a_lane
    const double abW = bcast(abar, K - 1) * M.W[K - 1];
    const double abk = gather(abar, lane >= 2 ? lane - 2 : 0);
    lam = 0.0;
    if (lane == 0) lam = a.gT[cell] - abW * P * V / (RU * T * T);
    if (lane == 1) lam = abW * P / (RU * T);
    if (lane >= 2 && lane < N) lam = abk * M.W[lane - 2] - abW;
  }
  for (int j = lane; j < M.Nr; j += 64) pbar[j] = 0.0;
  wsync();

  int64_t chunk = a.ck_head[cell];
  for (int64_t s = cnt - 1; s >= 0; --s) {
    if (s % CK_CHUNK == CK_CHUNK - 1 && s != cnt - 1) chunk = a.ck_prev[chunk];   // into the previous chunk
    const double* rec = a.ck_arena + (chunk * CK_CHUNK + s % CK_CHUNK) * (int64_t)(N + 1);
    const double x = (lane < N) ? rec[lane] : 0.0;
    const double h = rec[N];
    // ---- recompute the forward step
    const double f1 = team_rhs_jac<double>(M, P, x, LA, a.lnA);
    int perm;
    double rdiag;
    team_lu<NMAX>(LA.J, ldj, N, 1.0 / (h * ROS4_GAMMA), perm, rdiag);
    if (lane < N) plane[perm] = lane;
    wsync();
    const int invperm = (lane < N) ? plane[lane] : lane;
    wsync();
    const double ih = 1.0 / h;
    const double* F = LA.J;
    const double u1 = team_solve<NMAX>(F, ldj, N, perm, rdiag, f1);
    const double y2 = x + ROS4_A21 * u1;
    const double F2 = team_rhs(M, P, y2, LA, a.lnA);
    const double u2 = team_solve<NMAX>(F, ldj, N, perm, rdiag, F2 + (ROS4_C21 * ih) * u1);
    const double y3 = x + ROS4_A31 * u1 + ROS4_A32 * u2;
    const double F3 = team_rhs(M, P, y3, LA, a.lnA);
    const double u3 = team_solve<NMAX>(F, ldj, N, perm, rdiag, F3 + (ROS4_C31 * u1 + ROS4_C32 * u2) * ih);
    const double u4 = team_solve<NMAX>(F, ldj, N, perm, rdiag,
                                 F3 + (ROS4_C41 * u1 + ROS4_C42 * u2 + ROS4_C43 * u3) * ih);
    // ---- reverse
    double phib = lam;
    double ub1 = ROS4_M1 * lam, ub2 = ROS4_M2 * lam, ub3 = ROS4_M3 * lam;
    const double ub4 = ROS4_M4 * lam;
    const double mu4 = team_solve_t<NMAX>(F, ldj, N, invperm, rdiag, ub4);
    double F3b = mu4;
    ub1 += ROS4_C41 * ih * mu4;
    ub2 += ROS4_C42 * ih * mu4;
    ub3 += ROS4_C43 * ih * mu4;
    const double mu3 = team_solve_t<NMAX>(F, ldj, N, invperm, rdiag, ub3);
    F3b += mu3;
    ub1 += ROS4_C31 * ih * mu3;
    ub2 += ROS4_C32 * ih * mu3;
    const double y3b = team_vjp<double>(M, P, y3, F3b, LA, a.lnA, pbar, true);
    phib += y3b;
    ub1 += ROS4_A31 * y3b;
    ub2 += ROS4_A32 * y3b;
    const double mu2 = team_solve_t<NMAX>(F, ldj, N, invperm, rdiag, ub2);
    ub1 += ROS4_C21 * ih * mu2;
    const double y2b = team_vjp<double>(M, P, y2, mu2, LA, a.lnA, pbar, true);
    phib += y2b;
    ub1 += ROS4_A21 * y2b;
    const double mu1 = team_solve_t<NMAX>(F, ldj, N, invperm, rdiag, ub1);
    wsync();
    // ---- J(Phi)^T mu1 and the terms through M(Phi): dual products along u_i
#pragma unroll 1
    for (int i = 0; i < 4; ++i) {
      const double ui = (i == 0) ? u1 : (i == 1) ? u2 : (i == 2) ? u3 : u4;
      const double mui = (i == 0) ? mu1 : (i == 1) ? mu2 : (i == 2) ? mu3 : mu4;
      const Dd r = team_vjp<Dd>(M, P, Dd{x, (lane < N) ? ui : 0.0}, mui, LD, a.lnA, pbar, i == 0);
      phib += r.d;
      if (i == 0) phib += r.v;
    }
    lam = (lane < N) ? phib : 0.0;
  }

  // ---- input conversion adjoint: Phi0 = (T0, R T0 S / P, Y_k / W_k), S = sum Y_k / W_k
  if (a.gT0 || a.gY0) {
    const double T0 = a.T0[cell];
    const double yw = (lane < K) ? a.Y0[(int64_t)lane * a.n + cell] / M.W[lane] : 0.0;
    const double S = wave_sum(yw);
    const double lT = bcast(lam, 0), lV = bcast(lam, 1);
    const double ln = gather(lam, lane + 2 < 64 ? lane + 2 : 0);
    if (a.gT0 && lane == 0) a.gT0[cell] = lT + lV * RU * S / P;
    if (a.gY0 && lane < K) {
      double g = lV * RU * T0 / (P * M.W[lane]);
      if (lane < K - 1) g += ln / M.W[lane];
      a.gY0[(int64_t)lane * a.ldY + cell] = g;
    }
  }
  for (int j = lane; j < M.Nr; j += 64) a.g_cell[(int64_t)M.rorig[j] * a.n + cell] = pbar[j];
}

// g[j] = sum over cells of g_cell[j][cell], in a fixed order (deterministic).
__global__ void __launch_bounds__(256) reduce_cells_kernel(const double* __restrict__ g_cell, int64_t n,
                                                           double* __restrict__ g) {
  __shared__ double part[256];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int64_t c = threadIdx.x; c < n; c += 256) s += g_cell[(int64_t)j * n + c];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) g[j] = part[0];
}

// f and J at given states, for tests of the pieces.
__global__ void eval_kernel(MechView M, int64_t n, const double* __restrict__ phi_in, int64_t ldp,
                            const double* __restrict__ P, const double* __restrict__ lnA,
                            double* __restrict__ f_out, double* __restrict__ J_out, double* ws,
                            int64_t ld) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int N = M.N;
  const WsLayout L{N, M.K};
  double* base = ws + c;
  Lane phi{base + L.phi() * ld, ld}, f{base + L.f1() * ld, ld};
  Lane J{base + (int64_t)L.jac() * ld, ld};
  for (int i = 0; i < N; ++i) phi[i] = phi_in[(int64_t)i * ldp + c];
  if (J_out) {
    eval_rhs_jac(M, P[c], phi, f, J, L, base, ld, lnA);
    for (int i = 0; i < N * N; ++i) J_out[(int64_t)i * ldp + c] = J[i];
  } else {
    Lane conc{base + L.conc() * ld, ld}, wdot{base + L.wdot() * ld, ld};
    Lane hrt{base + L.hrt() * ld, ld}, cpr{base + L.cpr() * ld, ld}, gib{base + L.gibbs() * ld, ld};
    eval_rhs(M, P[c], phi, f, conc, wdot, hrt, cpr, gib, lnA);
  }
  for (int i = 0; i < N; ++i) f_out[(int64_t)i * ldp + c] = f[i];
}

// ---- the factorisation of a stage matrix alone, M = d I - A, by each
// launch's own routine; matrix c's element (i, j) at [(i * N + j) * ld + c].
// The factors leave in pivot order, perm[k] the row of M pivoted at step k.

// One matrix per thread (lu_factor: explicit row swaps), the swap sequence
// turned into the permutation afterwards.
__global__ void lu_thread_kernel(int64_t n, int N, const double* __restrict__ A, int64_t ld, double d,
                                 double* __restrict__ F, int32_t* __restrict__ perm,
                                 int32_t* __restrict__ status) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  Lane a{F + c, ld};
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) a[i * N + j] = (i == j ? d : 0.0) - A[(int64_t)(i * N + j) * ld + c];
  const int rc = lu_factor(a, perm + c, ld, N);
  status[c] = rc;
  if (rc) return;
  int q[MAX_SPECIES + 1];
  for (int k = 0; k < N; ++k) q[k] = k;
  for (int k = 0; k < N; ++k) {
    const int s = perm[(int64_t)k * ld + c], t = q[k];
    q[k] = q[s];
    q[s] = t;
  }
  for (int k = 0; k < N; ++k) perm[(int64_t)k * ld + c] = q[k];
}

// One wavefront per matrix (team_lu_reg), N <= NMAX <= 64: J staged in LDS
// with the integrator's row stride N + 1.
template <int NMAX>
__global__ void __launch_bounds__(64) lu_team_kernel(int64_t n, int N, const double* __restrict__ A,
                                                     int64_t ld, double d, double* __restrict__ F,
                                                     int32_t* __restrict__ perm, int32_t* __restrict__ status) {
  extern __shared__ double lds_raw[];
  const int lane = threadIdx.x, ldj = N + 1;
  const int64_t c = blockIdx.x;
  for (int e = lane; e < N * N; e += 64) lds_raw[(e / N) * ldj + e % N] = A[(int64_t)e * ld + c];
  wsync();
  RegLU<NMAX> R;
  const int rc = team_lu_reg<NMAX>(lds_raw, ldj, N, d, R);
  if (lane == 0) status[c] = rc;
  if (rc) return;
  if (lane < N) {   // every row of M was pivoted at a step < N
#pragma unroll
    for (int j = 0; j < NMAX; ++j)
      if (j < N) F[(int64_t)(R.ord * N + j) * ld + c] = R.A[j];
    perm[(int64_t)lane * ld + c] = R.pv;
  }
}

// A work-group of four wavefronts per matrix (t4_lu), 64 < N <= 128.
__global__ void __launch_bounds__(256) lu_team4_kernel(int64_t n, int N, const double* __restrict__ A,
                                                       int64_t ld, double d, double* __restrict__ F,
                                                       int32_t* __restrict__ perm, int32_t* __restrict__ status) {
  extern __shared__ double lds_raw[];
  Team4Lds L;
  L.bind(lds_raw, N, 1);
  const int tid = t4_tid(), ldj = N + 1;
  const int64_t c = blockIdx.x;
  for (int e = tid; e < N * N; e += T4_THREADS) L.J[(e / N) * ldj + e % N] = A[(int64_t)e * ld + c];
  wsync();
  const int rc = t4_lu(L.J, ldj, N, d, L);
  if (tid == 0) status[c] = rc;
  if (rc) return;
  for (int e = tid; e < N * N; e += T4_THREADS) F[(int64_t)e * ld + c] = L.J[(e / N) * ldj + e % N];
  for (int k = tid; k < N; k += T4_THREADS) perm[(int64_t)k * ld + c] = L.perm[k];
}

__global__ void reset_counter_kernel(unsigned int* q) { *q = 0u; }

// ---- dispatch order: counting sort of the cells by a temperature bucket,
// hottest first.  bins[0..255] counts, bins[256..511] cursors.  The order
// inside a bucket depends on atomics; no result depends on it.
constexpr int ORDER_BINS = 256;
__device__ __forceinline__ int order_bucket(double T) {
  if (!(T >= 0.0)) return 0;
  if (T >= 12.0 * (ORDER_BINS - 1)) return ORDER_BINS - 1;
  return (int)(T * (1.0 / 12.0));
}

__global__ void __launch_bounds__(ORDER_BINS) order_clear_kernel(unsigned int* bins) {
  bins[threadIdx.x] = 0u;
  bins[ORDER_BINS + threadIdx.x] = 0u;
}

__global__ void __launch_bounds__(256) order_count_kernel(int64_t n, const double* __restrict__ T,
                                                          unsigned int* bins) {
  __shared__ unsigned int c[ORDER_BINS];
  c[threadIdx.x] = 0u;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) atomicAdd(&c[order_bucket(T[i])], 1u);
  __syncthreads();
  if (c[threadIdx.x]) atomicAdd(&bins[threadIdx.x], c[threadIdx.x]);
}

// cursor[b] = number of cells in hotter buckets (one block of ORDER_BINS threads)
__global__ void __launch_bounds__(ORDER_BINS) order_scan_kernel(unsigned int* bins) {
  __shared__ unsigned int s[ORDER_BINS];
  const int t = threadIdx.x;
  s[t] = bins[ORDER_BINS - 1 - t];          // s[t]: count of the t-th hottest bucket
  __syncthreads();
  for (int d = 1; d < ORDER_BINS; d <<= 1) {
    const unsigned int v = (t >= d) ? s[t - d] : 0u;
    __syncthreads();
    s[t] += v;
    __syncthreads();
  }
  // exclusive prefix of the t-th hottest bucket
  bins[ORDER_BINS + (ORDER_BINS - 1 - t)] = s[t] - bins[ORDER_BINS - 1 - t];
}

__global__ void __launch_bounds__(256) order_scatter_kernel(int64_t n, const double* __restrict__ T,
                                                            unsigned int* bins, int32_t* __restrict__ order) {
  __shared__ unsigned int c[ORDER_BINS], base[ORDER_BINS];
  c[threadIdx.x] = 0u;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int b = 0;
  unsigned int r = 0u;
  if (i < n) {
    b = order_bucket(T[i]);
    r = atomicAdd(&c[b], 1u);
  }
  __syncthreads();
  if (c[threadIdx.x]) base[threadIdx.x] = atomicAdd(&bins[ORDER_BINS + threadIdx.x], c[threadIdx.x]);
  __syncthreads();
  if (i < n) order[base[b] + r] = (int32_t)i;
}

// Strided sample of a batch: cell i of the sample is cell i * stride.
__global__ void sample_cells_kernel(int64_t ns, int64_t stride, int K, const double* __restrict__ T,
                                    const double* __restrict__ P, const double* __restrict__ Y,
                                    int64_t ldY, double* __restrict__ Ts, double* __restrict__ Ps,
                                    double* __restrict__ Ys) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ns) return;
  const int64_t c = i * stride;
  Ts[i] = T[c];
  Ps[i] = P[c];
  for (int k = 0; k < K; ++k) Ys[(int64_t)k * ns + i] = Y[(int64_t)k * ldY + c];
}

// Scratch of chem_integrate_noalloc: the work-queue counter (word 0), the
// dispatch-order bins (words 64 .. 64 + 2 ORDER_BINS) and the queue position ->
// cell map (NOALLOC_MAX_CELLS words).  One copy per device, held until the
// process ends; host code reaches it only through the address that
// hipGetSymbolAddress returns for the device.
constexpr int64_t NOALLOC_MAX_CELLS = 1 << 20;
constexpr size_t NOALLOC_ORDER_WORD = 64 + 2 * ORDER_BINS;
constexpr size_t NOALLOC_WORDS = NOALLOC_ORDER_WORD + NOALLOC_MAX_CELLS;
static __device__ __align__(256) unsigned int scratch[NOALLOC_WORDS];

}  // namespace chem

// ====================================================================== host side
using namespace chem;

struct Workspace {
  double* ws = nullptr;
  int32_t* piv = nullptr;
  unsigned int* queue = nullptr;   // [0] work-queue counter, [64..575] dispatch-order bins
  int32_t* order = nullptr;        // queue position -> cell
  double* jsave = nullptr;         // persistent one-wavefront-per-cell mode: J copy per work-group
  size_t ws_bytes = 0, piv_bytes = 0, order_bytes = 0, jsave_bytes = 0;
};

struct chem_mech_s {
  HostMech host;
  MechView view;
  void* blob = nullptr;
  int device = 0;
  int n_cu = 0;
  size_t max_lds = 0;               // LDS of a CU: the most one work-group can take
  std::mutex mu;
  std::map<hipStream_t, Workspace> ws;
  std::map<int, chem_opts> tuned;   // batch-size bucket -> autotuned options
  bool cache_read = false;
  double ck_per_cell = 48.0;        // records per cell of the last checkpointed call (arena sizing)
};

struct chem_graph_s {
  int device = 0;
  hipStream_t stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

struct chem_ckpt_s {
  chem_mech_t mech = nullptr;
  int32_t method = CHEM_METHOD_ROS4;
  hipStream_t stream = nullptr;
  int64_t n = 0;
  // (Phi_n, h_n) of every accepted step in chunks of CK_CHUNK records, each
  // cell's chunks linked backwards from head; the final Phi per cell
  double* arena = nullptr;       // [cap][CK_CHUNK][N+1]
  int64_t* prev = nullptr;       // [cap]
  unsigned long long* used = nullptr;
  int64_t cap = 0;
  int64_t* head = nullptr;       // [n]
  double* final_phi = nullptr;   // [n][N+1]
  int32_t* count = nullptr;      // [n] accepted steps
  std::vector<int32_t> count_host;
  double* P = nullptr;           // copy of the pressures [n]
  double* T0 = nullptr;          // copy of the initial state: T [n], Y [K][n]
  double* Y0 = nullptr;
  double* lnA = nullptr;         // [Nr] copy of the ln A override, or null
  int64_t total = 0;             // records
  int32_t* order = nullptr;      // [n] cells by decreasing record count (adjoint dispatch order)
  std::vector<int32_t> order_host;
};

namespace {

#define HIPCHECK(x)                    \
  do {                                 \
    hipError_t e_ = (x);               \
    if (e_ != hipSuccess) return CHEM_EHIP; \
  } while (0)

int grow(void** p, size_t* have, size_t need) {
  if (*have >= need && *p) return CHEM_OK;
  if (*p) {
    if (hipFree(*p) != hipSuccess) return CHEM_EHIP;
    *p = nullptr;
    *have = 0;
  }
  if (hipMalloc(p, need) != hipSuccess) {
    *p = nullptr;
    return CHEM_ENOMEM;
  }
  *have = need;
  return CHEM_OK;
}

constexpr size_t QUEUE_BYTES = (64 + 2 * ORDER_BINS) * sizeof(unsigned int);

int get_workspace(chem_mech_t m, hipStream_t s, int64_t slots, Workspace** out) {
  std::lock_guard<std::mutex> g(m->mu);
  Workspace& w = m->ws[s];
  const WsLayout L{m->view.N, m->view.K};
  if (slots == 0) {
    if (!w.queue && hipMalloc(&w.queue, QUEUE_BYTES) != hipSuccess) return CHEM_ENOMEM;
    *out = &w;
    return CHEM_OK;
  }
  int rc = grow((void**)&w.ws, &w.ws_bytes, (size_t)L.total() * slots * sizeof(double));
  if (rc) return rc;
  rc = grow((void**)&w.piv, &w.piv_bytes, (size_t)m->view.N * slots * sizeof(int32_t));
  if (rc) return rc;
  if (!w.queue) {
    if (hipMalloc(&w.queue, QUEUE_BYTES) != hipSuccess) return CHEM_ENOMEM;
  }
  *out = &w;
  return CHEM_OK;
}

int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

int size_bucket(int64_t n) {
  int b = 0;
  while ((int64_t)1 << (b + 1) <= n) ++b;
  return b;
}

std::string tune_key(chem_mech_t m, int bucket) {
  std::ostringstream k;
  k << "N" << m->view.N << " Nr" << m->view.Nr << " cu" << m->n_cu << " b" << bucket;
  return k.str();
}

// Reads CHEM_AUTOTUNE_CACHE once per handle (lines: "<key> mode wg waves").
void tune_cache_read(chem_mech_t m) {
  if (m->cache_read) return;
  m->cache_read = true;
  const char* path = getenv("CHEM_AUTOTUNE_CACHE");
  if (!path) return;
  std::ifstream in(path);
  std::string line;
  const std::string pre = "N" + std::to_string(m->view.N) + " Nr" + std::to_string(m->view.Nr) +
                          " cu" + std::to_string(m->n_cu) + " b";
  while (std::getline(in, line)) {
    if (line.compare(0, pre.size(), pre) != 0) continue;
    std::istringstream is(line.substr(pre.size()));
    int b, mode, wg, waves;
    if (is >> b >> mode >> wg >> waves) {
      chem_opts o;
      chem_opts_default(&o);
      o.mode = mode;
      o.wg_size = wg;
      o.waves_per_cu = waves;
      m->tuned[b] = o;          // later lines win
    }
  }
}

bool tuned_lookup(chem_mech_t m, int64_t n, chem_opts* out) {
  std::lock_guard<std::mutex> g(m->mu);
  tune_cache_read(m);
  auto it = m->tuned.find(size_bucket(n));
  if (it == m->tuned.end()) return false;
  *out = it->second;
  return true;
}

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
unsigned int* g_scratch[MAX_DEVICES];   // device address of `scratch` on each device

// Device address of this device's scratch array (the device must be current).
int scratch_address(int device, unsigned int** out) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (device < 0 || device >= MAX_DEVICES) return CHEM_EUNSUPPORTED;
  if (!g_scratch[device]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return CHEM_EHIP;
    g_scratch[device] = (unsigned int*)ptr;
  }
  *out = g_scratch[device];
  return CHEM_OK;
}

typedef void (*TeamKernel)(IntParams, bool);

// One wavefront per cell holds a state vector element per lane: N <= 64.
TeamKernel team_kernel(int N) {
  if (N <= 16) return integrate_team_kernel<16>;
  if (N <= 32) return integrate_team_kernel<32>;
  if (N <= 48) return integrate_team_kernel<48>;
  if (N <= 56) return integrate_team_kernel<56>;
  if (N <= 64) return integrate_team_kernel<64>;
  return nullptr;
}

// Whether a team launch (one or four wavefronts per cell) can run a method of
// s stages: N <= 128, and the work-group's LDS within a CU's (the four-wavefront
// layout holds four copies of the s stage vectors besides the N x (N + 1) J).
bool team_fits(chem_mech_t m, int s) {
  const int N = m->view.N;
  if (N > T4_NMAX) return false;
  const size_t lds = (N > 64 ? Team4Lds::doubles(N, s) : TeamLds::doubles(N)) * sizeof(double);
  return lds <= m->max_lds;
}

}  // namespace

extern "C" {

void chem_opts_default(chem_opts* o) {
  if (!o) return;
  o->rtol = 1e-6;
  o->atol = 1e-10;
  o->h_min = 1e-20;
  o->safety = 0.9;
  o->fac_min = 0.2;
  o->fac_max = 6.0;
  o->T_cut = 0.0;
  o->max_steps = 100000;
  o->mode = CHEM_MODE_AUTO;
  o->wg_size = 0;
  o->waves_per_cu = 0;
  o->order = CHEM_ORDER_HOT_FIRST;
  o->method = CHEM_METHOD_ROS4;
  o->estimator = CHEM_EST_EMBEDDED;
  o->team_waves = 0;
  o->jac_every = 1;
  o->stats = nullptr;
}

const char* chem_error_string(int code) {
  switch (code) {
    case CHEM_OK: return "ok";
    case CHEM_EINVAL: return "invalid argument";
    case CHEM_EPARSE: return "mechanism parse error";
    case CHEM_EHIP: return "HIP runtime error";
    case CHEM_ENOMEM: return "device out of memory";
    case CHEM_EUNSUPPORTED: return "mechanism exceeds compiled limits, or method not supported here";
    case CHEM_ENONDET: return "checkpointed integration: the recording pass did not repeat the counted steps";
    default: return "unknown error";
  }
}

int chem_mech_load(const char* path, int device, chem_mech_t* out) {
  if (!path || !out) return CHEM_EINVAL;
  *out = nullptr;
  chem_mech_t m = new (std::nothrow) chem_mech_s();
  if (!m) return CHEM_ENOMEM;
  int rc = parse_mechanism(path, m->host);
  if (rc) {
    delete m;
    return rc;
  }
  group_reactions_by_type(m->host);
  if (hipSetDevice(device) != hipSuccess) {
    delete m;
    return CHEM_EHIP;
  }
  m->device = device;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    delete m;
    return CHEM_EHIP;
  }
  m->n_cu = prop.multiProcessorCount;
  m->max_lds = prop.maxSharedMemoryPerMultiProcessor;
  {
    unsigned int* sp;   // set up the no-allocation entry point's scratch on this device
    (void)scratch_address(device, &sp);
  }
  const HostMech& h = m->host;
  // one blob, each array 256-byte aligned
  struct Part { const void* src; size_t bytes; size_t off; };
  std::vector<Part> parts = {
      {h.W.data(), h.W.size() * 8, 0},          {h.nasa.data(), h.nasa.size() * 8, 0},
      {h.rinfo.data(), h.rinfo.size() * 4, 0},  {h.rspec.data(), h.rspec.size() * 4, 0},
      {h.rnu.data(), h.rnu.size() * 4, 0},      {h.arr.data(), h.arr.size() * 8, 0},
      {h.eff_idx.data(), h.eff_idx.size() * 4, 0}, {h.eff_am1.data(), h.eff_am1.size() * 8, 0},
      {h.fo.data(), h.fo.size() * 8, 0},         {h.rorig.data(), h.rorig.size() * 4, 0}};
  size_t total = 0;
  for (auto& p : parts) {
    p.off = total;
    total += (p.bytes + 255) / 256 * 256 + 256;
  }
  if (hipMalloc(&m->blob, total) != hipSuccess) {
    delete m;
    return CHEM_ENOMEM;
  }
  std::vector<char> staging(total, 0);
  for (auto& p : parts)
    if (p.bytes) memcpy(staging.data() + p.off, p.src, p.bytes);
  if (hipMemcpy(m->blob, staging.data(), total, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(m->blob);
    delete m;
    return CHEM_EHIP;
  }
  char* b = (char*)m->blob;
  MechView& v = m->view;
  v.K = h.K;
  v.Nr = h.Nr;
  v.N = h.K + 1;
  v.W = (const double*)(b + parts[0].off);
  v.nasa = (const double*)(b + parts[1].off);
  v.rinfo = (const int32_t*)(b + parts[2].off);
  v.rspec = (const int32_t*)(b + parts[3].off);
  v.rnu = (const int32_t*)(b + parts[4].off);
  v.arr = (const double*)(b + parts[5].off);
  v.eff_idx = (const int32_t*)(b + parts[6].off);
  v.eff_am1 = (const double*)(b + parts[7].off);
  v.fo = (const double*)(b + parts[8].off);
  v.rorig = (const int32_t*)(b + parts[9].off);
  *out = m;
  return CHEM_OK;
}

int chem_mech_info(chem_mech_t m, int32_t* K, int32_t* Nr, int32_t* E) {
  if (!m) return CHEM_EINVAL;
  if (K) *K = m->host.K;
  if (Nr) *Nr = m->host.Nr;
  if (E) *E = m->host.E;
  return CHEM_OK;
}

void chem_mech_free(chem_mech_t m) {
  if (!m) return;
  (void)hipSetDevice(m->device);
  (void)hipDeviceSynchronize();
  for (auto& kv : m->ws) {
    if (kv.second.ws) (void)hipFree(kv.second.ws);
    if (kv.second.piv) (void)hipFree(kv.second.piv);
    if (kv.second.queue) (void)hipFree(kv.second.queue);
    if (kv.second.order) (void)hipFree(kv.second.order);
    if (kv.second.jsave) (void)hipFree(kv.second.jsave);
  }
  if (m->blob) (void)hipFree(m->blob);
  delete m;
}

int chem_eval(chem_mech_t m, int64_t n, const double* phi, int64_t ld, const double* P,
              const double* lnA, double* f, double* J, hipStream_t stream) {
  if (!m || n < 0 || !phi || !P || !f || ld < n) return CHEM_EINVAL;
  if (n == 0) return CHEM_OK;
  HIPCHECK(hipSetDevice(m->device));
  Workspace* w;
  const int64_t slots = round_up(n, 64);
  int rc = get_workspace(m, stream, slots, &w);
  if (rc) return rc;
  const int wg = 64;
  hipLaunchKernelGGL(eval_kernel, dim3((unsigned)((n + wg - 1) / wg)), dim3(wg), 0, stream, m->view,
                     n, phi, ld, P, lnA, f, J, w->ws, slots);
  HIPCHECK(hipGetLastError());
  return CHEM_OK;
}

int chem_lu(int64_t n, int32_t N, const double* A, int64_t ld, double d, double* F, int32_t* perm,
            int32_t* status, int32_t launch, hipStream_t stream) {
  if (n < 0 || n > INT32_MAX || N < 1 || ld < n || (launch != 0 && launch != 1)) return CHEM_EINVAL;
  if (n > 0 && (!A || !F || !perm || !status)) return CHEM_EINVAL;
  if (N > (launch == 0 ? T4_NMAX : MAX_SPECIES + 1)) return CHEM_EUNSUPPORTED;
  if (n == 0) return CHEM_OK;
  if (launch == 1) {
    hipLaunchKernelGGL(lu_thread_kernel, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, stream, n, (int)N, A,
                       ld, d, F, perm, status);
  } else if (N <= 64) {
    decltype(&lu_team_kernel<64>) kern = N <= 16   ? lu_team_kernel<16>
                                        : N <= 32 ? lu_team_kernel<32>
                                        : N <= 48 ? lu_team_kernel<48>
                                        : N <= 56 ? lu_team_kernel<56>
                                                  : lu_team_kernel<64>;
    hipLaunchKernelGGL(kern, dim3((unsigned)n), dim3(64), (size_t)N * (N + 1) * sizeof(double), stream, n,
                       (int)N, A, ld, d, F, perm, status);
  } else {
    const size_t lds = Team4Lds::doubles(N, 1) * sizeof(double);
    HIPCHECK(hipFuncSetAttribute((const void*)lu_team4_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)lds));
    hipLaunchKernelGGL(lu_team4_kernel, dim3((unsigned)n), dim3(T4_THREADS), lds, stream, n, (int)N, A, ld, d,
                       F, perm, status);
  }
  HIPCHECK(hipGetLastError());
  return CHEM_OK;
}

static int integrate_impl(chem_mech_t m, int64_t n, const double* T_in, const double* P,
                          const double* Y_in, int64_t ldY, double* T_out, double* Y_out, double dt,
                          double rtol, double atol, double* h_io, int32_t* n_steps, int32_t* status,
                          const double* lnA, const chem_opts* opts, const chem_ckpt_s* ck,
                          hipStream_t stream);

// The options a call runs with: the caller's (or the defaults), with the
// autotuner's choice for this batch size in place of CHEM_MODE_AUTO.
static int resolve_opts(chem_mech_t m, int64_t n, const chem_opts* opts, chem_opts* out) {
  chem_opts o;
  chem_opts_default(&o);
  if (opts) o = *opts;
  if (o.mode == CHEM_MODE_AUTO) {
    chem_opts t;
    if (tuned_lookup(m, n, &t)) {
      o.mode = t.mode;
      o.wg_size = t.wg_size;
      o.waves_per_cu = t.waves_per_cu;
    }
  }
  *out = o;
  return CHEM_OK;
}

static void set_checkpoint(IntParams& p, const chem_ckpt_s* ck) {
  if (!ck) return;
  p.ck_arena = ck->arena;
  p.ck_prev = ck->prev;
  p.ck_used = ck->used;
  p.ck_cap = ck->cap;
  p.ck_head = ck->head;
  p.ck_final = ck->final_phi;
  p.ck_count = ck->count;
}

int chem_integrate(chem_mech_t m, int64_t n, const double* T_in, const double* P, const double* Y_in,
                   int64_t ldY, double* T_out, double* Y_out, double dt, double rtol, double atol,
                   double* h_io, int32_t* n_steps, int32_t* status, const double* lnA,
                   const chem_opts* opts, chem_ckpt_t* ckpt_out, hipStream_t stream) {
  if (!ckpt_out)
    return integrate_impl(m, n, T_in, P, Y_in, ldY, T_out, Y_out, dt, rtol, atol, h_io, n_steps,
                          status, lnA, opts, nullptr, stream);
  *ckpt_out = nullptr;
  if (!m || n <= 0 || !T_in || !P || !Y_in || !T_out || !Y_out || ldY < n) return CHEM_EINVAL;
  HIPCHECK(hipSetDevice(m->device));
  const int K = m->view.K, N = m->view.N;
  // One pass records every accepted step into an arena sized from the last
  // checkpointed call.  If it fills up, the counts of that pass give the exact
  // size and the call runs once more from the saved inputs (the integration is
  // deterministic, so it repeats the same steps).
  double* h0 = nullptr;   // the caller's initial h (or 0)
  chem_ckpt_t c = new (std::nothrow) chem_ckpt_s();
  if (!c) return CHEM_ENOMEM;
  c->mech = m;
  c->stream = stream;
  c->n = n;
  auto fail = [&](int rc) {
    if (h0) (void)hipFree(h0);
    chem_ckpt_free(c);
    return rc;
  };
  if (hipMalloc(&h0, n * 8) || hipMalloc(&c->P, n * 8) || hipMalloc(&c->T0, n * 8) ||
      hipMalloc(&c->Y0, (size_t)K * n * 8) || hipMalloc(&c->head, n * 8) ||
      hipMalloc(&c->final_phi, (size_t)n * (N + 1) * 8) || hipMalloc(&c->count, n * 4) ||
      hipMalloc(&c->used, 8))
    return fail(CHEM_ENOMEM);
  if (lnA) {
    if (hipMalloc(&c->lnA, (size_t)m->view.Nr * 8)) return fail(CHEM_ENOMEM);
    if (hipMemcpyAsync(c->lnA, lnA, (size_t)m->view.Nr * 8, hipMemcpyDeviceToDevice, stream)) return fail(CHEM_EHIP);
  }
  if (hipMemcpyAsync(c->P, P, n * 8, hipMemcpyDeviceToDevice, stream) ||
      hipMemcpyAsync(c->T0, T_in, n * 8, hipMemcpyDeviceToDevice, stream) ||
      hipMemcpy2DAsync(c->Y0, n * 8, Y_in, ldY * 8, n * 8, K, hipMemcpyDeviceToDevice, stream))
    return fail(CHEM_EHIP);
  if (h_io) {
    if (hipMemcpyAsync(h0, h_io, n * 8, hipMemcpyDeviceToDevice, stream)) return fail(CHEM_EHIP);
  } else if (hipMemsetAsync(h0, 0, n * 8, stream)) {
    return fail(CHEM_EHIP);
  }
  // every pass runs the same resolved options (an autotuner update between
  // passes must not change the launch, which could change the rounding)
  chem_opts ro;
  int rc = resolve_opts(m, n, opts, &ro);
  if (rc) return fail(rc);
  c->method = ro.method;
  if (ro.jac_every > 1) return fail(CHEM_EUNSUPPORTED);   // the adjoint re-evaluates J at every record
  double per_cell;
  {
    std::lock_guard<std::mutex> g(m->mu);
    per_cell = m->ck_per_cell;
  }
  const size_t chunk_bytes = (size_t)CK_CHUNK * (N + 1) * 8;
  int64_t cap = (int64_t)((double)n * (per_cell * 1.25 / CK_CHUNK + 1.0));
  {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess)
      cap = std::min<int64_t>(cap, (int64_t)(free_b / 4 / (chunk_bytes + 8)));
    cap = std::max<int64_t>(cap, 1);
  }
  std::vector<int32_t> counts;
  for (int pass = 0; pass < 2; ++pass) {
    if (c->arena) (void)hipFree(c->arena);
    if (c->prev) (void)hipFree(c->prev);
    c->arena = nullptr;
    c->prev = nullptr;
    c->cap = cap;
    if (hipMalloc(&c->arena, (size_t)cap * chunk_bytes) || hipMalloc(&c->prev, (size_t)cap * 8))
      return fail(CHEM_ENOMEM);
    if (hipMemsetAsync(c->used, 0, 8, stream)) return fail(CHEM_EHIP);
    double* h = h_io ? h_io : nullptr;
    if (h_io && pass > 0 && hipMemcpyAsync(h_io, h0, n * 8, hipMemcpyDeviceToDevice, stream))
      return fail(CHEM_EHIP);
    rc = integrate_impl(m, n, c->T0, c->P, c->Y0, n, T_out, Y_out, dt, rtol, atol, h, n_steps, status,
                        c->lnA, &ro, c, stream);
    if (rc) return fail(rc);
    unsigned long long used = 0;
    std::vector<int32_t> cnt(n);
    if (hipMemcpyAsync(&used, c->used, 8, hipMemcpyDeviceToHost, stream) ||
        hipMemcpyAsync(cnt.data(), c->count, n * 4, hipMemcpyDeviceToHost, stream) ||
        hipStreamSynchronize(stream))
      return fail(CHEM_EHIP);
    if (pass > 0 && cnt != counts) return fail(CHEM_ENONDET);
    counts.swap(cnt);
    if (used <= (unsigned long long)cap) break;
    if (pass > 0) return fail(CHEM_ENONDET);
    // exact size from this pass's counts
    cap = 0;
    for (int64_t i = 0; i < n; ++i) cap += (counts[i] + CK_CHUNK - 1) / CK_CHUNK;
    cap = std::max<int64_t>(cap, 1);
  }
  c->count_host = counts;
  c->total = 0;
  for (int64_t i = 0; i < n; ++i) c->total += counts[i] + 1;
  {
    std::lock_guard<std::mutex> g(m->mu);
    m->ck_per_cell = std::max(4.0, (double)(c->total - n) / (double)n);
  }
  // the adjoint's cost per cell is its record count: longest first
  c->order_host.resize(n);
  for (int64_t i = 0; i < n; ++i) c->order_host[i] = (int32_t)i;
  std::stable_sort(c->order_host.begin(), c->order_host.end(),
                   [&](int32_t a, int32_t b) { return counts[a] > counts[b]; });
  if (hipMalloc(&c->order, n * 4)) return fail(CHEM_ENOMEM);
  if (hipMemcpyAsync(c->order, c->order_host.data(), n * 4, hipMemcpyHostToDevice, stream) ||
      hipStreamSynchronize(stream))
    return fail(CHEM_EHIP);
  (void)hipFree(h0);
  h0 = nullptr;
  *ckpt_out = c;
  return CHEM_OK;
}

static int resolve_opts(chem_mech_t m, int64_t n, const chem_opts* opts, chem_opts* out);
static int team_launch(chem_mech_t m, const chem_opts& o, IntParams p, bool persistent,
                       unsigned int* queue, Workspace* jsave_ws, hipStream_t stream);
static int launch_order(int64_t n, const double* T_in, unsigned int* bins, int32_t* order,
                        hipStream_t stream);
static bool wants_order(int32_t mode, int64_t n);
static IntParams make_params(chem_mech_t m, const chem_opts& o, int64_t n, const double* T_in,
                             const double* P, const double* Y_in, int64_t ldY, double* T_out,
                             double* Y_out, double dt, double rtol, double atol, double* h_io,
                             int32_t* n_steps, int32_t* status, const double* lnA);

int chem_integrate_noalloc(chem_mech_t m, int64_t n, const double* T_in, const double* P,
                           const double* Y_in, int64_t ldY, double* T_out, double* Y_out, double dt,
                           double rtol, double atol, double* h_io, int32_t* n_steps, int32_t* status,
                           const double* lnA, const chem_opts* opts, hipStream_t stream) {
  if (!m || n < 0 || n > NOALLOC_MAX_CELLS) return CHEM_EINVAL;
  if (n > 0 && (!T_in || !P || !Y_in || !T_out || !Y_out)) return CHEM_EINVAL;
  if (!(dt > 0) || !(rtol > 0) || !(atol >= 0) || ldY < n) return CHEM_EINVAL;
  chem_opts o;
  resolve_opts(m, n, opts, &o);
  if (o.mode < CHEM_MODE_AUTO || o.mode > CHEM_MODE_TEAM_PERSISTENT) return CHEM_EINVAL;
  if (o.mode == CHEM_MODE_PLAIN || o.mode == CHEM_MODE_PERSISTENT) {
    // an autotuned one-cell-per-thread choice needs a workspace: use the team launch
    if (opts && (opts->mode == CHEM_MODE_PLAIN || opts->mode == CHEM_MODE_PERSISTENT)) return CHEM_EUNSUPPORTED;
    o.mode = CHEM_MODE_TEAM_PERSISTENT;
  }
  if (o.mode == CHEM_MODE_AUTO) o.mode = CHEM_MODE_TEAM_PERSISTENT;
  if (o.max_steps <= 0 || !(o.fac_min > 0) || !(o.fac_max >= 1) || !(o.safety > 0)) return CHEM_EINVAL;
  if (o.order != CHEM_ORDER_INDEX && o.order != CHEM_ORDER_HOT_FIRST) return CHEM_EINVAL;
  if (o.method < 0 || o.method >= N_METHODS) return CHEM_EINVAL;
  if (o.estimator != CHEM_EST_EMBEDDED && o.estimator != CHEM_EST_FILTERED) return CHEM_EINVAL;
  if (o.team_waves != 0 && o.team_waves != 1 && o.team_waves != 4) return CHEM_EINVAL;
  if (o.jac_every < 0) return CHEM_EINVAL;
  if (!team_fits(m, TABLES[o.method].s)) return CHEM_EUNSUPPORTED;
  if ((o.team_waves == 1 && m->view.N > 64) || (o.team_waves == 4 && m->view.N <= 64)) return CHEM_EUNSUPPORTED;
  if (o.wg_size < 0 || o.wg_size > 256 || (o.wg_size % 64) != 0) return CHEM_EINVAL;
  if (n == 0) return CHEM_OK;
  HIPCHECK(hipSetDevice(m->device));
  unsigned int* sp = nullptr;
  int rc = scratch_address(m->device, &sp);
  if (rc) return rc;
  IntParams p = make_params(m, o, n, T_in, P, Y_in, ldY, T_out, Y_out, dt, rtol, atol, h_io, n_steps,
                            status, lnA);
  if (wants_order(o.order, n)) {
    int32_t* order = (int32_t*)(sp + NOALLOC_ORDER_WORD);
    rc = launch_order(n, T_in, sp + 64, order, stream);
    if (rc) return rc;
    p.order = order;
  }
  return team_launch(m, o, p, o.mode == CHEM_MODE_TEAM_PERSISTENT, sp, nullptr, stream);
}

// Dispatch order of the cells (hottest first) into w->order; *order receives
// it, or null when the cells go in index order.  Four small kernels, no memset.
// The four ordering kernels: bins[0..2*ORDER_BINS) are counts and cursors,
// order[n] receives the queue position -> cell map.
static int launch_order(int64_t n, const double* T_in, unsigned int* bins, int32_t* order,
                        hipStream_t stream) {
  const unsigned blocks = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(order_clear_kernel, dim3(1), dim3(ORDER_BINS), 0, stream, bins);
  hipLaunchKernelGGL(order_count_kernel, dim3(blocks), dim3(256), 0, stream, n, T_in, bins);
  hipLaunchKernelGGL(order_scan_kernel, dim3(1), dim3(ORDER_BINS), 0, stream, bins);
  hipLaunchKernelGGL(order_scatter_kernel, dim3(blocks), dim3(256), 0, stream, n, T_in, bins, order);
  HIPCHECK(hipGetLastError());
  return CHEM_OK;
}

static bool wants_order(int32_t mode, int64_t n) { return mode == CHEM_ORDER_HOT_FIRST && n >= 1024; }

static int build_order(chem_mech_t m, Workspace* w, int64_t n, const double* T_in, int32_t mode,
                       hipStream_t stream, const int32_t** order) {
  *order = nullptr;
  if (!wants_order(mode, n)) return CHEM_OK;
  {
    std::lock_guard<std::mutex> g(m->mu);
    const int rc = grow((void**)&w->order, &w->order_bytes, (size_t)n * sizeof(int32_t));
    if (rc) return rc;
  }
  const int rc = launch_order(n, T_in, w->queue + 64, w->order, stream);
  if (rc) return rc;
  *order = w->order;
  return CHEM_OK;
}

// Parameters common to every launch.
static IntParams make_params(chem_mech_t m, const chem_opts& o, int64_t n, const double* T_in,
                             const double* P, const double* Y_in, int64_t ldY, double* T_out,
                             double* Y_out, double dt, double rtol, double atol, double* h_io,
                             int32_t* n_steps, int32_t* status, const double* lnA) {
  IntParams p;
  memset(&p, 0, sizeof(p));
  p.M = m->view;
  p.n = n;
  p.T_in = T_in;
  p.P = P;
  p.Y_in = Y_in;
  p.ldY = ldY;
  p.T_out = T_out;
  p.Y_out = Y_out;
  p.dt = dt;
  p.rtol = rtol;
  p.atol = atol;
  p.h_min = o.h_min;
  p.safety = o.safety;
  p.fac_min = o.fac_min;
  p.fac_max = o.fac_max;
  p.T_cut = o.T_cut;
  p.max_steps = o.max_steps;
  p.estimator = o.estimator;
  p.jac_every = o.jac_every > 0 ? o.jac_every : 1;
  p.tab = TABLES[o.method];
  p.h_io = h_io;
  p.n_steps = n_steps;
  p.status = status;
  p.lnA = lnA;
  p.stats = o.stats;
  return p;
}

// One-wavefront-per-cell launch.  persistent: resident grid over the work
// queue at `queue` (reset here by a kernel); jsave (nullable): per-work-group
// J copies of the persistent grid, sized by jsave_grow (null: a rejected step
// re-evaluates J at the same state, which gives the same J).
static int team_launch(chem_mech_t m, const chem_opts& o, IntParams p, bool persistent,
                       unsigned int* queue, Workspace* jsave_ws, hipStream_t stream) {
  const int N = m->view.N;
  const bool four = N > 64;             // four wavefronts per cell (N <= 128)
  TeamKernel kern = four ? integrate_team4_kernel : team_kernel(N);
  if (!kern) return CHEM_EUNSUPPORTED;
  // four wavefronts per cell keep J only through the persistent grid's saved copies
  if (four && p.jac_every > 1 && !(persistent && jsave_ws)) return CHEM_EUNSUPPORTED;
  const int threads = four ? T4_THREADS : 64;
  const size_t lds = (four ? Team4Lds::doubles(N, p.tab.s) : TeamLds::doubles(N)) * sizeof(double);
  if (lds > 65536)   // above the default dynamic-LDS limit of a launch
    HIPCHECK(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  unsigned grid = (unsigned)p.n;
  p.queue = queue;
  if (persistent) {
    int per_cu = 0;
    HIPCHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, lds));
    if (o.waves_per_cu > 0) per_cu = std::min(per_cu, std::max(1, o.waves_per_cu * 64 / threads));
    if (per_cu < 1) per_cu = 1;
    grid = (unsigned)std::min<int64_t>((int64_t)m->n_cu * per_cu, p.n);
    if (jsave_ws && four) {   // the one-wavefront kernel keeps J in LDS across a rejection
      std::lock_guard<std::mutex> g(m->mu);
      const int rc = grow((void**)&jsave_ws->jsave, &jsave_ws->jsave_bytes,
                          (size_t)grid * N * N * sizeof(double));
      if (rc) return rc;
      p.jsave = jsave_ws->jsave;
    }
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, stream, queue);
  }
  hipLaunchKernelGGL(kern, dim3(grid), dim3(threads), lds, stream, p, persistent);
  HIPCHECK(hipGetLastError());
  return CHEM_OK;
}

static int integrate_impl(chem_mech_t m, int64_t n, const double* T_in, const double* P,
                          const double* Y_in, int64_t ldY, double* T_out, double* Y_out, double dt,
                          double rtol, double atol, double* h_io, int32_t* n_steps, int32_t* status,
                          const double* lnA, const chem_opts* opts, const chem_ckpt_s* ck,
                          hipStream_t stream) {

  if (!m || n < 0 || n > INT32_MAX) return CHEM_EINVAL;
  if (n > 0 && (!T_in || !P || !Y_in || !T_out || !Y_out)) return CHEM_EINVAL;
  if (!(dt > 0) || !(rtol > 0) || !(atol >= 0) || ldY < n) return CHEM_EINVAL;
  chem_opts o;
  resolve_opts(m, n, opts, &o);
  if (o.mode < CHEM_MODE_AUTO || o.mode > CHEM_MODE_TEAM_PERSISTENT) return CHEM_EINVAL;
  if (o.wg_size < 0 || o.wg_size > 256 || (o.wg_size % 64) != 0) return CHEM_EINVAL;
  if (o.max_steps <= 0 || !(o.fac_min > 0) || !(o.fac_max >= 1) || !(o.safety > 0)) return CHEM_EINVAL;
  if (o.order != CHEM_ORDER_INDEX && o.order != CHEM_ORDER_HOT_FIRST) return CHEM_EINVAL;
  if (o.method < 0 || o.method >= N_METHODS) return CHEM_EINVAL;
  if (o.estimator != CHEM_EST_EMBEDDED && o.estimator != CHEM_EST_FILTERED) return CHEM_EINVAL;
  if (o.team_waves != 0 && o.team_waves != 1 && o.team_waves != 4) return CHEM_EINVAL;
  if (o.jac_every < 0) return CHEM_EINVAL;
  if (n == 0) return CHEM_OK;
  HIPCHECK(hipSetDevice(m->device));
  int mode = o.mode;
  // one or four wavefronts per cell need N <= 128 and their LDS within a CU's;
  // other mechanisms use one cell per thread
  const bool team_ok = team_fits(m, TABLES[o.method].s);
  if (o.team_waves != 0 && !team_ok) return CHEM_EUNSUPPORTED;
  if (o.team_waves == 1 && m->view.N > 64) return CHEM_EUNSUPPORTED;
  if (o.team_waves == 4 && m->view.N <= 64) return CHEM_EUNSUPPORTED;
  if (mode == CHEM_MODE_AUTO) mode = team_ok ? CHEM_MODE_TEAM_PERSISTENT : CHEM_MODE_PERSISTENT;
  if (!team_ok && mode == CHEM_MODE_TEAM) mode = CHEM_MODE_PLAIN;
  if (!team_ok && mode == CHEM_MODE_TEAM_PERSISTENT) mode = CHEM_MODE_PERSISTENT;
  const bool persistent = (mode == CHEM_MODE_PERSISTENT || mode == CHEM_MODE_TEAM_PERSISTENT);
  const bool team = (mode == CHEM_MODE_TEAM || mode == CHEM_MODE_TEAM_PERSISTENT);
  if (team) {
    Workspace* w;
    int rc = get_workspace(m, stream, 0, &w);
    if (rc) return rc;
    const int32_t* order;
    rc = build_order(m, w, n, T_in, o.order, stream, &order);
    if (rc) return rc;
    IntParams p = make_params(m, o, n, T_in, P, Y_in, ldY, T_out, Y_out, dt, rtol, atol, h_io, n_steps,
                              status, lnA);
    p.order = order;
    set_checkpoint(p, ck);
    return team_launch(m, o, p, persistent, w->queue, w, stream);
  }
  const int wg = o.wg_size ? o.wg_size : 64;
  int64_t slots;
  if (persistent) {
    int per_cu = 0;
    HIPCHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, integrate_thread_kernel<true>, wg, 0));
    if (o.waves_per_cu > 0) per_cu = std::min(per_cu, std::max(1, o.waves_per_cu * 64 / wg));
    if (per_cu < 1) per_cu = 1;
    slots = (int64_t)m->n_cu * per_cu * wg;
    slots = std::min(slots, round_up(n, wg));
  } else {
    slots = round_up(n, wg);
  }
  Workspace* w;
  int rc = get_workspace(m, stream, slots, &w);
  if (rc) return rc;
  const int32_t* order;
  rc = build_order(m, w, n, T_in, o.order, stream, &order);
  if (rc) return rc;
  IntParams p = make_params(m, o, n, T_in, P, Y_in, ldY, T_out, Y_out, dt, rtol, atol, h_io, n_steps,
                            status, lnA);
  p.order = order;
  p.ws = w->ws;
  p.piv = w->piv;
  p.ld = slots;
  p.queue = w->queue;
  p.stats = o.stats;
  set_checkpoint(p, ck);
  const unsigned grid = (unsigned)(slots / wg);
  if (persistent) {
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, stream, w->queue);
    hipLaunchKernelGGL(integrate_thread_kernel<true>, dim3(grid), dim3(wg), 0, stream, p);
  } else {
    hipLaunchKernelGGL(integrate_thread_kernel<false>, dim3(grid), dim3(wg), 0, stream, p);
  }
  HIPCHECK(hipGetLastError());
  return CHEM_OK;
}

int chem_integrate_adjoint(chem_mech_t m, chem_ckpt_t ckpt, const double* gT, const double* gY,
                           int64_t ldY, double* g_lnA, int32_t per_cell, double* gT0, double* gY0,
                           hipStream_t stream) {
  if (!m || !ckpt || ckpt->mech != m || !gT || !gY || !g_lnA || ldY < ckpt->n) return CHEM_EINVAL;
  const int N = m->view.N, Nr = m->view.Nr;
  const int64_t n = ckpt->n;
  if (N > 64 || ckpt->method != CHEM_METHOD_ROS4) return CHEM_EUNSUPPORTED;
  const size_t lds = ((size_t)N * (N + 1) + 3 * TeamLdsT<double>::vec_elems(N) + 32 + Nr) * 8;
  HIPCHECK(hipSetDevice(m->device));
  int lds_max = 0;
  HIPCHECK(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, m->device));
  if (lds > (size_t)lds_max) return CHEM_EUNSUPPORTED;
  double* g_cell = per_cell ? g_lnA : nullptr;
  if (!per_cell && hipMalloc(&g_cell, (size_t)Nr * n * 8)) return CHEM_ENOMEM;
  AdjParams a;
  a.M = m->view;
  a.n = n;
  a.ck_arena = ckpt->arena;
  a.ck_prev = ckpt->prev;
  a.ck_head = ckpt->head;
  a.ck_final = ckpt->final_phi;
  a.ck_count = ckpt->count;
  a.order = ckpt->order;
  a.P = ckpt->P;
  a.T0 = ckpt->T0;
  a.Y0 = ckpt->Y0;
  a.gT = gT;
  a.gY = gY;
  a.ldY = ldY;
  a.lnA = ckpt->lnA;
  a.g_cell = g_cell;
  a.gT0 = gT0;
  a.gY0 = gY0;
  void (*kern)(AdjParams) = N <= 16   ? adjoint_team_kernel<16>
                            : N <= 32 ? adjoint_team_kernel<32>
                            : N <= 48 ? adjoint_team_kernel<48>
                            : N <= 56 ? adjoint_team_kernel<56>
                                      : adjoint_team_kernel<64>;
  if (lds > 65536)   // above the default dynamic-LDS limit of a launch
    HIPCHECK(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(kern, dim3((unsigned)n), dim3(64), lds, stream, a);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && !per_cell) {
    hipLaunchKernelGGL(reduce_cells_kernel, dim3(Nr), dim3(256), 0, stream, g_cell, n, g_lnA);
    e = hipGetLastError();
  }
  if (!per_cell) {
    // the reduction must finish before the scratch is released
    if (hipStreamSynchronize(stream) != hipSuccess) e = hipErrorUnknown;
    (void)hipFree(g_cell);
  }
  return e == hipSuccess ? CHEM_OK : CHEM_EHIP;
}

int chem_ckpt_export(chem_ckpt_t c, int64_t* off, double* records) {
  if (!c) return CHEM_EINVAL;
  const int64_t n = c->n;
  if (off) {
    off[0] = 0;
    for (int64_t i = 0; i < n; ++i) off[i + 1] = off[i] + c->count_host[i] + 1;
  }
  if (records) {
    // walk each cell's chunks back from its head, then lay the records out
    // cell by cell (accepted steps in order, the final state last)
    const int N = c->mech->view.N;
    const size_t rl = (size_t)N + 1;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return CHEM_EHIP;
    std::vector<int64_t> head(n), prev(c->cap);
    std::vector<double> arena((size_t)c->cap * CK_CHUNK * rl), fin((size_t)n * rl);
    if (hipMemcpy(head.data(), c->head, n * 8, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(prev.data(), c->prev, c->cap * 8, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(arena.data(), c->arena, arena.size() * 8, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(fin.data(), c->final_phi, fin.size() * 8, hipMemcpyDeviceToHost) != hipSuccess)
      return CHEM_EHIP;
    double* out = records;
    std::vector<int64_t> chunks;
    for (int64_t i = 0; i < n; ++i) {
      const int64_t cnt = c->count_host[i];
      chunks.assign((size_t)((cnt + CK_CHUNK - 1) / CK_CHUNK), -1);
      int64_t ch = head[i];
      for (int64_t k = (int64_t)chunks.size() - 1; k >= 0; --k) {
        if (ch < 0 || ch >= c->cap) return CHEM_EINVAL;
        chunks[(size_t)k] = ch;
        ch = prev[(size_t)ch];
      }
      for (int64_t s = 0; s < cnt; ++s) {
        const double* r = &arena[((size_t)chunks[(size_t)(s / CK_CHUNK)] * CK_CHUNK + s % CK_CHUNK) * rl];
        std::copy(r, r + rl, out);
        out += rl;
      }
      std::copy(&fin[(size_t)i * rl], &fin[(size_t)i * rl] + rl, out);
      out += rl;
    }
  }
  return CHEM_OK;
}

int64_t chem_ckpt_records(chem_ckpt_t c) { return c ? c->total : -1; }

int chem_autotune(chem_mech_t m, int64_t n, const double* T_in, const double* P, const double* Y_in,
                  int64_t ldY, double dt, double rtol, double atol, chem_opts* chosen, double* ms,
                  hipStream_t stream) {
  if (!m || n <= 0 || !T_in || !P || !Y_in || ldY < n) return CHEM_EINVAL;
  HIPCHECK(hipSetDevice(m->device));
  const int K = m->view.K, N = m->view.N;
  // The sample must load the device the way the batch will: with a few cells
  // per resident slot, every candidate waits on the sample's slowest cell and
  // the timings cannot tell the occupancies apart (measured: a 4,096-cell
  // sample of the batching mix picked 2 waves per CU, half the throughput of
  // 4 on the full batch).  Sixteen cells per resident wavefront at the
  // largest occupancy tried, at least 4,096.
  const int64_t ns = std::min<int64_t>(n, std::max<int64_t>(4096, 16 * 4 * (int64_t)m->n_cu));
  const int64_t stride = n / ns;
  double *Ts = nullptr, *Ps = nullptr, *Ys = nullptr, *To = nullptr, *Yo = nullptr;
  auto cleanup = [&]() {
    for (double* q : {Ts, Ps, Ys, To, Yo})
      if (q) (void)hipFree(q);
  };
  if (hipMalloc(&Ts, ns * 8) || hipMalloc(&Ps, ns * 8) || hipMalloc(&Ys, (size_t)K * ns * 8) ||
      hipMalloc(&To, ns * 8) || hipMalloc(&Yo, (size_t)K * ns * 8)) {
    cleanup();
    return CHEM_ENOMEM;
  }
  hipLaunchKernelGGL(sample_cells_kernel, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, stream, ns,
                     stride, K, T_in, P, Y_in, ldY, Ts, Ps, Ys);
  std::vector<chem_opts> cand;
  auto add = [&](int mode, int wg, int waves) {
    chem_opts o;
    chem_opts_default(&o);
    o.mode = mode;
    o.wg_size = wg;
    o.waves_per_cu = waves;
    cand.push_back(o);
  };
  if (N <= 64) {
    add(CHEM_MODE_TEAM, 0, 0);
    for (int w : {0, 2, 3, 4}) add(CHEM_MODE_TEAM_PERSISTENT, 0, w);
  } else if (team_fits(m, TABLES[METHOD_ROS4].s)) {
    // four wavefronts per cell, one work-group per CU (its LDS)
    add(CHEM_MODE_TEAM, 0, 0);
    add(CHEM_MODE_TEAM_PERSISTENT, 0, 0);
  }
  if (N <= 16 || !team_fits(m, TABLES[METHOD_ROS4].s)) {
    add(CHEM_MODE_PLAIN, 64, 0);
    add(CHEM_MODE_PLAIN, 256, 0);
    add(CHEM_MODE_PERSISTENT, 64, 0);
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) || hipEventCreate(&e1)) {
    cleanup();
    return CHEM_EHIP;
  }
  double best = 1e300;
  int best_i = -1;
  int rc = CHEM_OK;
  for (size_t i = 0; i < cand.size() && rc == CHEM_OK; ++i) {
    double t_best = 1e300;
    for (int rep = 0; rep < 3 && rc == CHEM_OK; ++rep) {
      (void)hipEventRecord(e0, stream);
      rc = integrate_impl(m, ns, Ts, Ps, Ys, ns, To, Yo, dt, rtol, atol, nullptr, nullptr, nullptr,
                          nullptr, &cand[i], nullptr, stream);
      (void)hipEventRecord(e1, stream);
      float t = 0;
      if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess)
        rc = CHEM_EHIP;
      if (rep > 0) t_best = std::min(t_best, (double)t);   // the first run warms up
    }
    if (ms && i < 8) ms[i] = t_best;
    if (t_best < best) {
      best = t_best;
      best_i = (int)i;
    }
  }
  if (ms)
    for (size_t i = cand.size(); i < 8; ++i) ms[i] = -1.0;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  cleanup();
  if (rc) return rc;
  const int bucket = size_bucket(n);
  {
    std::lock_guard<std::mutex> g(m->mu);
    tune_cache_read(m);
    m->tuned[bucket] = cand[best_i];
  }
  if (const char* path = getenv("CHEM_AUTOTUNE_CACHE")) {
    std::ofstream out(path, std::ios::app);
    out << tune_key(m, bucket) << " " << cand[best_i].mode << " " << cand[best_i].wg_size << " "
        << cand[best_i].waves_per_cu << "\n";
  }
  if (chosen) *chosen = cand[best_i];
  return CHEM_OK;
}

int chem_graph_create(chem_mech_t m, int64_t n, const double* T_in, const double* P, const double* Y_in,
                      int64_t ldY, double* T_out, double* Y_out, double dt, double rtol, double atol,
                      double* h_io, int32_t* n_steps, int32_t* status, const double* lnA,
                      const chem_opts* opts, chem_graph_t* out) {
  if (!m || !out || n <= 0) return CHEM_EINVAL;
  *out = nullptr;
  HIPCHECK(hipSetDevice(m->device));
  chem_graph_t g = new (std::nothrow) chem_graph_s();
  if (!g) return CHEM_ENOMEM;
  g->device = m->device;
  if (hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking) != hipSuccess) {
    delete g;
    return CHEM_EHIP;
  }
  // relaxed capture: a first call may allocate the stream's workspace (that
  // allocation runs immediately and is not part of the graph)
  if (hipStreamBeginCapture(g->stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
    chem_graph_free(g);
    return CHEM_EHIP;
  }
  const int rc = integrate_impl(m, n, T_in, P, Y_in, ldY, T_out, Y_out, dt, rtol, atol, h_io, n_steps,
                                status, lnA, opts, nullptr, g->stream);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(g->stream, &graph);
  if (rc || e != hipSuccess || !graph) {
    if (graph) (void)hipGraphDestroy(graph);
    chem_graph_free(g);
    return rc ? rc : CHEM_EHIP;
  }
  g->graph = graph;
  if (hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    chem_graph_free(g);
    return CHEM_EHIP;
  }
  *out = g;
  return CHEM_OK;
}

int chem_graph_launch(chem_graph_t g, hipStream_t stream) {
  if (!g || !g->exec) return CHEM_EINVAL;
  HIPCHECK(hipSetDevice(g->device));
  HIPCHECK(hipGraphLaunch(g->exec, stream));
  return CHEM_OK;
}

void chem_graph_free(chem_graph_t g) {
  if (!g) return;
  (void)hipSetDevice(g->device);
  (void)hipDeviceSynchronize();
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->stream) (void)hipStreamDestroy(g->stream);
  delete g;
}

void chem_ckpt_free(chem_ckpt_t c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  if (c->arena) (void)hipFree(c->arena);
  if (c->prev) (void)hipFree(c->prev);
  if (c->used) (void)hipFree(c->used);
  if (c->head) (void)hipFree(c->head);
  if (c->final_phi) (void)hipFree(c->final_phi);
  if (c->count) (void)hipFree(c->count);
  if (c->P) (void)hipFree(c->P);
  if (c->T0) (void)hipFree(c->T0);
  if (c->Y0) (void)hipFree(c->Y0);
  if (c->lnA) (void)hipFree(c->lnA);
  if (c->order) (void)hipFree(c->order);
  delete c;
}

}  // extern "C"
