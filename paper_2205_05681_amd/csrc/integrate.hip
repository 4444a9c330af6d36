// Batched ROS4 integration, one cell per thread (plain and persistent launch)
// and the C ABI that drives it.
//
// Method (paper Sec. 2.3, transformed Rosenbrock form; Table T:solvers, ROS4):
//   M = I/(h gamma) - J(Phi_n), one LU per step;
//   M u_i = f(Phi_n + sum_{j<i} a_ij u_j) + sum_{j<i} (c_ij / h) u_j, i = 1..4,
//   with a_4j = a_3j so the fourth stage reuses the third f;
//   Phi_{n+1} = Phi_n + sum m_j u_j, error estimate sum e_j u_j.
// Step control (Sec. 3.1 tolerances; constants are this library's reading):
//   err = RMS_i(err_i / (atol + rtol max(|Phi_n,i|, |Phi_n+1,i|)));
//   accept if err <= 1; h <- h clamp(0.9 err^(-1/4), 0.2, 6), no growth right
//   after a rejection; the last step is clipped to the remaining time; the
//   final proposal is returned for reuse (Sec. 2.4.1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/chem.h"
#include "kinetics.h"
#include "mech.h"
#include "ros4.h"
#include "team.h"

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
  double* h_io;
  int32_t* n_steps;
  int32_t* status;
  const double* lnA;
  double* ws;
  int32_t* piv;
  int64_t ld;
  unsigned int* queue;
  unsigned long long* stats;   // nullable: attempts, accepted, rejected
  // adjoint checkpoint (nullable): per cell, accepted (Phi_n, h) records
  double* ck_data;          // [rec][N+1] per record, cell-major blocks
  const int64_t* ck_off;    // [n+1] record offsets per cell
  int32_t* ck_count;        // [n] steps counted (pass 1) or written (pass 2)
};

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
  Lane u1{base + L.u(0) * ld, ld}, u2{base + L.u(1) * ld, ld}, u3{base + L.u(2) * ld, ld},
      u4{base + L.u(3) * ld, ld};
  Lane J{base + (int64_t)L.jac() * ld, ld}, A{base + (int64_t)L.lu() * ld, ld};
  Lane conc{base + L.conc() * ld, ld}, wdot{base + L.wdot() * ld, ld};
  Lane hrt{base + L.hrt() * ld, ld}, cpr{base + L.cpr() * ld, ld}, gib{base + L.gibbs() * ld, ld};

  int64_t cell;
  if (PERSISTENT)
    cell = atomicAdd(p.queue, 1u);
  else
    cell = slot;
  bool have = cell < p.n;
  // per-cell controller state
  double P = 0, h = 0, rem = 0;
  int attempts = 0, accepted = 0, bad = 0, status = 0;
  bool last_rej = false, need_jac = true, done = false;
  int64_t ck_rec = 0;

  auto init = [&](int64_t c) {
    P = p.P[c];
    const double T = p.T_in[c];
    to_phi(M, T, P, p.Y_in, p.ldY, c, phi);
    rem = p.dt;
    h = p.dt;
    if (p.h_io && p.h_io[c] > 0.0) h = p.h_io[c];
    attempts = accepted = bad = status = 0;
    last_rej = false;
    need_jac = true;
    done = !(T >= p.T_cut);     // T_cut = 0 integrates every cell (NaN T included)
    if (p.T_cut <= 0.0) done = false;
    ck_rec = p.ck_off ? p.ck_off[c] : 0;
  };
  auto finish = [&](int64_t c) {
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
      if (need_jac) {
        eval_rhs_jac(M, P, phi, f1, J, L, base, ld, p.lnA);
        need_jac = false;
      }
      const double d = 1.0 / (hs * ROS4_GAMMA);
      for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) A[i * N + j] = (i == j ? d : 0.0) - J[i * N + j];
      const int rc = lu_factor(A, piv, ld, N);
      double err = 0.0;
      if (rc == 0) {
        const double ih = 1.0 / hs;
        for (int i = 0; i < N; ++i) u1[i] = f1[i];
        lu_solve(A, piv, ld, N, u1);
        for (int i = 0; i < N; ++i) ys[i] = phi[i] + ROS4_A21 * u1[i];
        eval_rhs(M, P, ys, fs, conc, wdot, hrt, cpr, gib, p.lnA);
        for (int i = 0; i < N; ++i) u2[i] = fs[i] + (ROS4_C21 * ih) * u1[i];
        lu_solve(A, piv, ld, N, u2);
        for (int i = 0; i < N; ++i) ys[i] = phi[i] + ROS4_A31 * u1[i] + ROS4_A32 * u2[i];
        eval_rhs(M, P, ys, fs, conc, wdot, hrt, cpr, gib, p.lnA);
        for (int i = 0; i < N; ++i) u3[i] = fs[i] + (ROS4_C31 * u1[i] + ROS4_C32 * u2[i]) * ih;
        lu_solve(A, piv, ld, N, u3);
        for (int i = 0; i < N; ++i)
          u4[i] = fs[i] + (ROS4_C41 * u1[i] + ROS4_C42 * u2[i] + ROS4_C43 * u3[i]) * ih;
        lu_solve(A, piv, ld, N, u4);
        for (int i = 0; i < N; ++i) {
          const double y0 = phi[i];
          const double yn = y0 + ROS4_M1 * u1[i] + ROS4_M2 * u2[i] + ROS4_M3 * u3[i] + ROS4_M4 * u4[i];
          const double e = ROS4_E1 * u1[i] + ROS4_E2 * u2[i] + ROS4_E3 * u3[i] + ROS4_E4 * u4[i];
          ynew[i] = yn;
          const double sc = p.atol + p.rtol * fmax(fabs(y0), fabs(yn));
          const double r = e / sc;
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
        double fac = (err > 0.0) ? p.safety * pow(err, -0.25) : p.fac_max;
        if (err <= 1.0) {
          if (p.ck_data) {
            double* rec = p.ck_data + (ck_rec + accepted) * (int64_t)(N + 1);
            for (int i = 0; i < N; ++i) rec[i] = phi[i];
            rec[N] = hs;
          }
          for (int i = 0; i < N; ++i) phi[i] = ynew[i];
          rem -= hs;
          ++accepted;
          fac = fmin(p.fac_max, fmax(p.fac_min, fac));
          if (last_rej) fac = fmin(fac, 1.0);
          last_rej = false;
          need_jac = true;
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
        cell = atomicAdd(p.queue, 1u);
        have = cell < p.n;
        if (have) init(cell);
      } else {
        have = false;
      }
    }
  }
}


// ------------------------------------------------------------------ one-wavefront-per-cell integrator
__global__ void __launch_bounds__(64) integrate_team_kernel(IntParams p, bool PERSISTENT) {
  extern __shared__ double lds_raw[];
  const MechView& M = p.M;
  const int N = M.N, K = M.K, ldj = N + 1;
  const int lane = threadIdx.x;
  TeamLds L;
  L.bind(lds_raw, N);
  int64_t cell;
  if (PERSISTENT) {
    unsigned c0 = 0;
    if (lane == 0) c0 = atomicAdd(p.queue, 1u);
    cell = __shfl((int)c0, 0, 64);
  } else {
    cell = blockIdx.x;
  }
  while (cell < p.n) {
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
    bool last_rej = false, need_jac = true;
    bool done = (p.T_cut > 0.0) && !(T0 >= p.T_cut);
    const int64_t ck_rec = p.ck_off ? p.ck_off[cell] : 0;
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
      if (need_jac) {
        f1 = team_rhs_jac(M, P, phi, L, p.lnA);
        need_jac = false;
      }
      // M = I/(h gamma) - J in place of J (J is re-evaluated after a rejection)
      const double d = 1.0 / (hs * ROS4_GAMMA);
      if (lane < N)
        for (int i = 0; i < N; ++i) L.J[i * ldj + lane] = (i == lane ? d : 0.0) - L.J[i * ldj + lane];
      need_jac = true;
      wsync();
      int perm;
      double rdiag;
      const int rc = team_lu(L.J, ldj, N, perm, rdiag);
      double err = 0.0, ynew = 0.0;
      if (rc == 0) {
        const double ih = 1.0 / hs;
        const double* F = L.J;
        const double u1 = team_solve(F, ldj, N, perm, rdiag, f1);
        double fs = team_rhs(M, P, phi + ROS4_A21 * u1, L, p.lnA);
        const double u2 = team_solve(F, ldj, N, perm, rdiag, fs + (ROS4_C21 * ih) * u1);
        fs = team_rhs(M, P, phi + ROS4_A31 * u1 + ROS4_A32 * u2, L, p.lnA);
        const double u3 = team_solve(F, ldj, N, perm, rdiag, fs + (ROS4_C31 * u1 + ROS4_C32 * u2) * ih);
        const double u4 = team_solve(F, ldj, N, perm, rdiag,
                                           fs + (ROS4_C41 * u1 + ROS4_C42 * u2 + ROS4_C43 * u3) * ih);
        ynew = phi + ROS4_M1 * u1 + ROS4_M2 * u2 + ROS4_M3 * u3 + ROS4_M4 * u4;
        const double e = ROS4_E1 * u1 + ROS4_E2 * u2 + ROS4_E3 * u3 + ROS4_E4 * u4;
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
      double fac = (err > 0.0) ? p.safety * pow(err, -0.25) : p.fac_max;
      if (err <= 1.0) {
        if (p.ck_data) {
          double* rec = p.ck_data + (ck_rec + accepted) * (int64_t)(N + 1);
          if (lane < N) rec[lane] = phi;
          if (lane == 0) rec[N] = hs;
        }
        phi = ynew;
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
        }
      }
    }
    if (PERSISTENT) {
      unsigned c1 = 0;
      if (lane == 0) c1 = atomicAdd(p.queue, 1u);
      cell = __shfl((int)c1, 0, 64);
    } else {
      break;
    }
  }
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

__global__ void reset_counter_kernel(unsigned int* q) { *q = 0u; }

}  // namespace chem

// ====================================================================== host side
using namespace chem;

struct Workspace {
  double* ws = nullptr;
  int32_t* piv = nullptr;
  unsigned int* queue = nullptr;
  size_t ws_bytes = 0, piv_bytes = 0;
};

struct chem_mech_s {
  HostMech host;
  MechView view;
  void* blob = nullptr;
  int device = 0;
  int n_cu = 0;
  std::mutex mu;
  std::map<hipStream_t, Workspace> ws;
};

struct chem_ckpt_s {
  chem_mech_t mech = nullptr;
  hipStream_t stream = nullptr;
  int64_t n = 0, ldY = 0;
  double* data = nullptr;        // records (Phi_n, h) for every accepted step
  int64_t* off = nullptr;        // [n+1]
  double* P = nullptr;           // copy of the pressures [n]
  double* T0 = nullptr;          // copy of the initial state: T [n], Y [K][n]
  double* Y0 = nullptr;
  double* lnA = nullptr;         // [Nr] the ln A used
  int64_t total = 0;
  double rtol = 0, atol = 0;
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

int get_workspace(chem_mech_t m, hipStream_t s, int64_t slots, Workspace** out) {
  std::lock_guard<std::mutex> g(m->mu);
  Workspace& w = m->ws[s];
  const WsLayout L{m->view.N, m->view.K};
  if (slots == 0) {
    if (!w.queue && hipMalloc(&w.queue, 256) != hipSuccess) return CHEM_ENOMEM;
    *out = &w;
    return CHEM_OK;
  }
  int rc = grow((void**)&w.ws, &w.ws_bytes, (size_t)L.total() * slots * sizeof(double));
  if (rc) return rc;
  rc = grow((void**)&w.piv, &w.piv_bytes, (size_t)m->view.N * slots * sizeof(int32_t));
  if (rc) return rc;
  if (!w.queue) {
    if (hipMalloc(&w.queue, 256) != hipSuccess) return CHEM_ENOMEM;
  }
  *out = &w;
  return CHEM_OK;
}

int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

typedef void (*TeamKernel)(IntParams, bool);

// One wavefront per cell holds a state vector element per lane: N <= 64.
TeamKernel team_kernel(int N) { return N <= 64 ? integrate_team_kernel : nullptr; }

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
  o->mode = CHEM_MODE_PLAIN;
  o->wg_size = 0;
  o->waves_per_cu = 0;
  o->stats = nullptr;
}

const char* chem_error_string(int code) {
  switch (code) {
    case CHEM_OK: return "ok";
    case CHEM_EINVAL: return "invalid argument";
    case CHEM_EPARSE: return "mechanism parse error";
    case CHEM_EHIP: return "HIP runtime error";
    case CHEM_ENOMEM: return "device out of memory";
    case CHEM_EUNSUPPORTED: return "mechanism exceeds compiled limits";
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

int chem_integrate(chem_mech_t m, int64_t n, const double* T_in, const double* P, const double* Y_in,
                   int64_t ldY, double* T_out, double* Y_out, double dt, double rtol, double atol,
                   double* h_io, int32_t* n_steps, int32_t* status, const double* lnA,
                   const chem_opts* opts, chem_ckpt_t* ckpt_out, hipStream_t stream) {
  if (!m || n < 0) return CHEM_EINVAL;
  if (n > 0 && (!T_in || !P || !Y_in || !T_out || !Y_out)) return CHEM_EINVAL;
  if (!(dt > 0) || !(rtol > 0) || !(atol >= 0) || ldY < n) return CHEM_EINVAL;
  chem_opts o;
  chem_opts_default(&o);
  if (opts) o = *opts;
  if (o.mode < CHEM_MODE_AUTO || o.mode > CHEM_MODE_TEAM_PERSISTENT) return CHEM_EINVAL;
  if (o.wg_size < 0 || o.wg_size > 256 || (o.wg_size % 64) != 0) return CHEM_EINVAL;
  if (o.max_steps <= 0 || !(o.fac_min > 0) || !(o.fac_max >= 1) || !(o.safety > 0)) return CHEM_EINVAL;
  if (ckpt_out) *ckpt_out = nullptr;
  if (n == 0) return CHEM_OK;
  HIPCHECK(hipSetDevice(m->device));
  int mode = o.mode;
  if (mode == CHEM_MODE_AUTO) mode = (m->view.N <= 64) ? CHEM_MODE_TEAM_PERSISTENT : CHEM_MODE_PERSISTENT;
  // one wavefront per cell needs N <= 64; larger mechanisms use one cell per thread
  if (m->view.N > 64 && mode == CHEM_MODE_TEAM) mode = CHEM_MODE_PLAIN;
  if (m->view.N > 64 && mode == CHEM_MODE_TEAM_PERSISTENT) mode = CHEM_MODE_PERSISTENT;
  const bool persistent = (mode == CHEM_MODE_PERSISTENT || mode == CHEM_MODE_TEAM_PERSISTENT);
  const bool team = (mode == CHEM_MODE_TEAM || mode == CHEM_MODE_TEAM_PERSISTENT);
  if (team) {
    Workspace* w;
    int rc = get_workspace(m, stream, 0, &w);
    if (rc) return rc;
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
    p.h_io = h_io;
    p.n_steps = n_steps;
    p.status = status;
    p.lnA = lnA;
    p.queue = w->queue;
    p.stats = o.stats;
    TeamKernel kern = team_kernel(m->view.N);
    const size_t lds = TeamLds::doubles(m->view.N) * sizeof(double);
    unsigned grid = (unsigned)n;
    if (persistent) {
      int per_cu = 0;
      HIPCHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64, lds));
      if (o.waves_per_cu > 0) per_cu = std::min(per_cu, o.waves_per_cu);
      if (per_cu < 1) per_cu = 1;
      grid = (unsigned)std::min<int64_t>((int64_t)m->n_cu * per_cu, n);
      hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, stream, w->queue);
    }
    hipLaunchKernelGGL(kern, dim3(grid), dim3(64), lds, stream, p, persistent);
    HIPCHECK(hipGetLastError());
    return CHEM_OK;
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
  IntParams p;
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
  p.h_io = h_io;
  p.n_steps = n_steps;
  p.status = status;
  p.lnA = lnA;
  p.ws = w->ws;
  p.piv = w->piv;
  p.ld = slots;
  p.queue = w->queue;
  p.stats = o.stats;
  p.ck_data = nullptr;
  p.ck_off = nullptr;
  p.ck_count = nullptr;
  const unsigned grid = (unsigned)(slots / wg);
  if (persistent) {
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, stream, w->queue);
    hipLaunchKernelGGL(integrate_thread_kernel<true>, dim3(grid), dim3(wg), 0, stream, p);
  } else {
    hipLaunchKernelGGL(integrate_thread_kernel<false>, dim3(grid), dim3(wg), 0, stream, p);
  }
  HIPCHECK(hipGetLastError());
  (void)ckpt_out;
  return CHEM_OK;
}

int chem_integrate_adjoint(chem_mech_t m, chem_ckpt_t ckpt, const double* gT, const double* gY,
                           int64_t ldY, double* g_lnA, int32_t per_cell, double* gT0, double* gY0,
                           hipStream_t stream) {
  (void)m; (void)ckpt; (void)gT; (void)gY; (void)ldY; (void)g_lnA; (void)per_cell; (void)gT0;
  (void)gY0; (void)stream;
  return CHEM_EINVAL;
}

void chem_ckpt_free(chem_ckpt_t c) { delete c; }

}  // extern "C"
