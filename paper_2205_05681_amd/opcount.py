"""Algorithmic operation counts of one ROS4 step for a given mechanism.

The roofline of the integrator is priced in *algorithmic* FP64 operations:
what the method needs, independent of how a kernel organises it.  Additions,
subtractions, multiplications and divisions count 1, a fused multiply-add 2;
exp/log/log10 are counted separately (they are not part of the flop count).

Per attempted step an s-stage method needs (paper Sec. 2.3, one LU per
step):
  * M = I/(h gamma) - J and its LU with partial pivoting;
  * s forward/backward substitutions (one more for the filtered estimate);
  * the new source-term evaluations of stages 2..s (a stage whose argument
    equals the previous stage's reuses its f: ROS4 needs 2, ROS3 1, RODAS3 2,
    RODAS4 5);
  * the stage combinations and the error norm.
Per accepted step it also needs f and the analytical Jacobian at the new
state; a rejected step reuses them.  With the Jacobian kept over several
steps (a W-method), a new state without a new J needs f alone.  So for a
batch with E Jacobian evaluations:
  flops = E * F_fJ + (accepted - E) * F_f
          + attempts * (F_M + F_LU + n_sol F_sol + n_f F_f + F_vec).
"""

from __future__ import annotations

# stages, new f evaluations per attempt (stage 1 uses the f evaluated with J)
METHOD_SHAPE = {"ros4": (4, 2), "ros3": (3, 1), "rodas3": (4, 2), "rodas4": (6, 5), "ros34pw2": (4, 3)}


def _thermo(K, with_dcp):
    # cp (8), h/RT (11), s/R (10), g = s - h (1); dcp/dT (8) for the Jacobian
    return K * (30 + (8 if with_dcp else 0)) + 2


def _reaction(r, jac):
    nr, np_ = len(r.reac), len(r.prod)
    nu_r = sum(n for _, n in r.reac)
    nu_p = sum(n for _, n in r.prod)
    f = 5                                       # ln k = lnA + b lnT - theta/T
    if r.kind != "E":
        f += 1 + 2 * len(r.eff)                 # [M]
        f += 1 if r.kind == "T" else 0
    if r.kind in "LF":
        f += 5 + 3                              # k0, Pr, Pr/(1+Pr) k_inf
    if r.kind == "F":
        f += 12 + 10 + 2                        # Fcent, c, n, x, y, log F, F
    f += 2 * (nr + np_) + 3                     # ln Kc, k_r
    f += max(nu_r - 1, 0) + max(nu_p - 1, 0) + 3   # products and q
    f += 2 * (nr + np_)                         # wdot scatter (FMA)
    if jac:
        f += 6                                  # dq/dT
        f += (nr + np_) * (nr + np_)            # dq/dC of the participants
        f += 2 * (nr + np_) * (1 + nr + np_)    # scatter into G and the T column
        if r.kind != "E":
            f += 4 + 2 * (nr + np_) * (1 + len(r.eff))
        if r.kind == "F":
            f += 30                             # Troe derivatives
    return f


def _transcendentals(r):
    t = 1                                       # exp(ln k)
    if r.kind in "LF":
        t += 1
    if r.kind == "F":
        t += 3 + 2 + 1                          # three exp in Fcent, two log10, F
    t += 1                                      # exp(-ln Kc)
    return t


def step_counts(mech, method="ros4", estimator="embedded"):
    """Dict of per-piece algorithmic flop counts for a synth.Mechanism."""
    K = mech.n_species
    N = K + 1
    rx = mech.reactions
    f_rhs = (2 * K + 3) + _thermo(K, False) + sum(_reaction(r, False) for r in rx) + 6 * K + 12 + K
    f_fj = (2 * K + 3) + _thermo(K, True) + sum(_reaction(r, True) for r in rx) + 6 * K + 12 + K
    f_fj += K * (K - 1) * 4 + K * 6                 # Phi coordinates of the species rows
    f_fj += (N - 2) * K * 4 + N * 20 + (K - 1) * 3  # T and V rows
    f_m = N * N + 2
    f_lu = sum((N - k - 1) + 2 * (N - k - 1) ** 2 for k in range(N))
    f_sol = N * (N - 1) + N * (N - 1) + N
    s, nf = METHOD_SHAPE[method]
    n_sol = s + (1 if estimator == "filtered" else 0)
    # stage arguments and right-hand sides (2 FMA per earlier stage each),
    # the new state and the estimate (2 FMA per stage each), the error norm
    f_vec = N * (2 * s * (s - 1) + 4 * s + 6) + 2
    t_rhs = sum(_transcendentals(r) for r in rx) + 2
    return dict(N=N, rhs=f_rhs, rhs_jac=f_fj, matrix=f_m, lu=f_lu, solve=f_sol, vector=f_vec,
                per_attempt=f_m + f_lu + n_sol * f_sol + nf * f_rhs + f_vec, per_accept=f_fj,
                transcendentals_per_rhs=t_rhs, f_per_attempt=nf)


def batch_flops(mech, attempts, accepted, method="ros4", estimator="embedded", jac_evals=None):
    """Algorithmic FP64 flops and transcendental calls of a batch (jac_evals:
    Jacobian evaluations, one per accepted step unless J is kept)."""
    c = step_counts(mech, method, estimator)
    je = accepted if jac_evals is None else jac_evals
    flops = je * c["per_accept"] + (accepted - je) * c["rhs"] + attempts * c["per_attempt"]
    trans = (accepted + c["f_per_attempt"] * attempts) * c["transcendentals_per_rhs"]
    return flops, trans
