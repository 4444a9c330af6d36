"""Benchmark: cells integrated per second over one operator-splitting step.

Headline workload (the metric's configuration that fits one GPU at its
largest): the batching mix of the CH4-shaped synthetic mechanism (53 species,
325 reversible reactions, 30 third-body, 25 Troe), 1,048,576 cells - 85 %
cold (T < 800 K), 10 % stoichiometric at 1100-1400 K, 5 % burnt gas -
dt = 1e-5 s, FP64, rtol 1e-6, atol 1e-10.  The library's autotuner runs once
on the batch; one step is then one chem_integrate call (default launch) over
every cell with the inputs resident in HBM.

Prints one JSON line.  Besides the contract's keys:
  "roofline"      the dominant kernel of the headline call: algorithmic FP64
                  flops per launch (op-count model x the call's own step
                  counts) over its average launch time, from HIP events on the
                  launch stream;
  "cpu_baseline"  the CPU oracle on a stratified 4,096-cell sample of the
                  headline batch on this host's cores, with per-configuration
                  samples and a single-core rate under "per_config";
  "plain_vs_persistent"  the headline batch in the plain one-cell-per-thread
                  launch and in the one-wavefront-per-cell launches (plain grid,
                  persistent queue), all at full size;
  "mixing"        the 65,536-cell mixing-layer case (dt = 1e-6 s) and each
                  launch mode on it;
  "large"         the 111-species mechanism (N = 112) on its mixing states;
  "small"         the 10-species mechanism on 256 cells: per-call time of the
                  plain, persistent and team launches and of a replayed
                  captured graph (launch-overhead regime);
  "methods"       the other solvers and the filtered error estimate on the
                  mixing case;
  "adjoint"       discrete-adjoint vs forward time on the 16,384-cell
                  differentiation case.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 vector: 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
# the sources of the headline kernel (the one-wavefront-per-cell integrator):
# the traffic file's counters stay valid while none of them changes
KERNEL_SOURCES = ["paper_2205_05681_amd/csrc/integrate.hip", "paper_2205_05681_amd/csrc/team.h",
                  "paper_2205_05681_amd/csrc/kinetics.h", "paper_2205_05681_amd/csrc/methods.h",
                  "paper_2205_05681_amd/csrc/mech.h", "paper_2205_05681_amd/csrc/mech.cpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_team_kernel_batching_1048576.json")
METRIC = "cells/s per split step at rtol 1e-6 (plain vs persistent); adjoint/forward cost"


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class Ctx:
    def __init__(self, torch, np, chem, synth, opcount, dev, mech_dir):
        self.torch, self.np, self.chem, self.synth, self.opcount = torch, np, chem, synth, opcount
        self.dev, self.mech_dir = dev, mech_dir

    def d(self, x):
        return self.torch.from_numpy(self.np.ascontiguousarray(x)).to(self.dev)

    def sync(self):
        self.torch.cuda.synchronize()


def timed(c, fn, reps=1):
    c.sync()
    t = time.perf_counter()
    for _ in range(reps):
        fn()
    c.sync()
    return (time.perf_counter() - t) / reps


def run_stats(c, mech, m, Tt, Pt, Yt, dt, with_jac=False, **kw):
    """One call with step counters: (attempts, accepted, rejected, n_steps,
    status), and the Jacobian evaluations last when with_jac is set."""
    stats = c.torch.zeros(4, dtype=c.torch.int64, device=c.dev)
    r = c.chem.integrate(mech, Tt, Pt, Yt, dt, opts=c.chem.default_opts(stats=stats, **kw))
    c.sync()
    a, acc, rej, je = (int(x) for x in stats.cpu().numpy())
    out = (a, acc, rej, r[3].cpu().numpy(), r[4].cpu().numpy())
    return out + (je,) if with_jac else out


def headline(c, a):
    """The batching mix at full size: autotune, then W warm-up and K timed
    calls of the default launch."""
    np, chem, synth = c.np, c.chem, c.synth
    path, m = synth.mechanism_file("ch4", c.mech_dir)
    T, P, Y, kind = synth.states_batching(m, a.cells, 203)
    n = T.size
    mech = chem.Mechanism(path, device=0)
    Tt, Pt, Yt = c.d(T), c.d(P), c.d(Y)
    T1, Y1 = c.torch.empty_like(Tt), c.torch.empty_like(Yt)
    h = c.torch.zeros(n, dtype=c.torch.float64, device=c.dev)
    ns = c.torch.empty(n, dtype=c.torch.int32, device=c.dev)
    st = c.torch.empty(n, dtype=c.torch.int32, device=c.dev)
    log("headline: autotune")
    chosen, cand_ms = chem.autotune(mech, Tt, Pt, Yt, 1e-5)
    opts = chem.default_opts()
    for _ in range(a.warmup):
        h.zero_()
        chem.integrate(mech, Tt, Pt, Yt, 1e-5, h=h, opts=opts, out=(T1, Y1), n_steps=ns, status=st)
    c.sync()
    log("headline: timed steps")
    stream = c.torch.cuda.current_stream()
    ev = [(c.torch.cuda.Event(enable_timing=True), c.torch.cuda.Event(enable_timing=True))
          for _ in range(a.steps)]
    t0 = time.perf_counter()
    for i in range(a.steps):
        h.zero_()
        ev[i][0].record(stream)
        chem.integrate(mech, Tt, Pt, Yt, 1e-5, h=h, opts=opts, out=(T1, Y1), n_steps=ns, status=st)
        ev[i][1].record(stream)
    c.sync()
    wall = time.perf_counter() - t0
    launch_ms = [s.elapsed_time(e) for s, e in ev]
    status = st.cpu().numpy()
    steps = ns.cpu().numpy()
    att, acc, rej, _, _ = run_stats(c, mech, m, Tt, Pt, Yt, 1e-5)
    flops, trans = c.opcount.batch_flops(m, att, acc)
    avg_s = float(np.mean(launch_ms)) / 1e3
    achieved = flops / avg_s / 1e12
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        tf = json.load(open(TRAFFIC_FILE))
        if tf.get("kernel_hash") == kernel_hash() and tf.get("cells") == n:
            traffic = tf.get("hbm_bytes_per_launch")
    modes = {1: "plain", 2: "persistent", 3: "team", 4: "team_persistent"}
    roofline = {"bound": "alu", "achieved": round(achieved, 4), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP64_PEAK_TFLOPS, 6), "traffic": traffic,
                "kernel": "integrate_team_kernel<56>" if chosen.mode in (3, 4) else "integrate_thread_kernel",
                "flops_per_launch": flops, "transcendentals_per_launch": trans,
                "attempted_steps": att, "accepted_steps": acc, "rejected_steps": rej,
                "avg_launch_ms": round(avg_s * 1e3, 4)}
    out = dict(value=n / (wall / a.steps), ms_per_step=wall * 1e3 / a.steps, roofline=roofline,
               config={"workload": "batching mix: CH4-shaped synthetic mechanism (53 species, 325 reactions: "
                                   "30 third-body, 25 Troe), 1,048,576 cells (85% cold <800 K, 10% stoichiometric "
                                   "1100-1400 K, 5% burnt gas), dt=1e-5 s, rtol 1e-6, atol 1e-10, ROS4, "
                                   "autotuned launch" if n == 1048576 else "batching mix, %d cells" % n,
                       "cells": n, "species": m.n_species, "reactions": len(m.reactions), "dt": 1e-5,
                       "rtol": 1e-6, "atol": 1e-10, "method": "ros4",
                       "autotuned": {"mode": modes.get(chosen.mode, chosen.mode),
                                     "waves_per_cu": chosen.waves_per_cu, "candidates_ms": cand_ms},
                       "failed_cells": int((status != 0).sum()),
                       "accepted_steps": {k: {"mean": round(float(steps[kind == i].mean()), 2),
                                              "max": int(steps[kind == i].max())}
                                          for i, k in enumerate(("cold", "igniting", "burnt"))},
                       "step_spread": int(steps.max()) / max(1, int(steps.min()))})
    # plain vs persistent at full size
    pvp = {}
    if not a.quick:
        for label, mode in (("team_plain_grid", "team"), ("team_persistent", "team_persistent"),
                            ("thread_plain", "plain")):
            log("headline: %s" % label)
            o = chem.default_opts(mode=mode)
            t = timed(c, lambda: chem.integrate(mech, Tt, Pt, Yt, 1e-5, opts=o, out=(T1, Y1)))
            pvp[label] = round(n / t, 1)
        pvp["autotuned_default"] = round(out["value"], 1)
        pvp["persistent_over_plain_team"] = round(pvp["team_persistent"] / pvp["team_plain_grid"], 3)
        pvp["default_over_thread_plain"] = round(out["value"] / pvp["thread_plain"], 2)
    out["plain_vs_persistent"] = pvp
    mech.close()
    return out, (path, m, T, P, Y, kind)


def mixing(c, a):
    """The 65,536-cell mixing-layer case, each launch mode."""
    chem, synth = c.chem, c.synth
    path, m = synth.mechanism_file("ch4", c.mech_dir)
    T, P, Y = synth.states_mixing(m, 65536, 202)
    n = T.size
    mech = chem.Mechanism(path, device=0)
    Tt, Pt, Yt = c.d(T), c.d(P), c.d(Y)
    out = {"workload": "CH4-shaped mechanism, 65,536 mixing-layer cells, P~U[1,5] atm, Z~Beta(2,5), dt=1e-6 s",
           "cells_per_s": {}}
    for mode in ("auto", "team", "team_persistent", "plain", "persistent"):
        o = chem.default_opts(mode=mode)
        chem.integrate(mech, Tt, Pt, Yt, 1e-6, opts=o)
        reps = 1 if mode in ("plain", "persistent") else 3
        t = timed(c, lambda: chem.integrate(mech, Tt, Pt, Yt, 1e-6, opts=o), reps)
        out["cells_per_s"][mode] = round(n / t, 1)
        if mode == "auto":
            out["ms_per_call"] = round(t * 1e3, 3)
    att, acc, rej, ns, _ = run_stats(c, mech, m, Tt, Pt, Yt, 1e-6)
    out.update(attempted_steps=att, accepted_steps=acc, rejected_steps=rej,
               accepted_steps_max=int(ns.max()))
    mech.close()
    return out


def methods(c, a):
    """Cells/s of each solver and of the filtered estimate on the mixing case
    (default launch), with their step counts; the W-method ROS34PW2 also with
    the Jacobian kept for 2, 4 and 8 accepted steps."""
    chem, synth = c.chem, c.synth
    path, m = synth.mechanism_file("ch4", c.mech_dir)
    T, P, Y = synth.states_mixing(m, 65536, 202)
    n = T.size
    mech = chem.Mechanism(path, device=0)
    Tt, Pt, Yt = c.d(T), c.d(P), c.d(Y)
    out = {}
    cases = [(meth, est, 1) for meth in ("ros4", "ros3", "rodas3", "rodas4", "ros34pw2")
             for est in ("embedded", "filtered")]
    cases += [("ros34pw2", "embedded", k) for k in (2, 4, 8)]
    for meth, est, k in cases:
        o = chem.default_opts(method=meth, estimator=est, jac_every=k)
        chem.integrate(mech, Tt, Pt, Yt, 1e-6, opts=o)
        t = timed(c, lambda: chem.integrate(mech, Tt, Pt, Yt, 1e-6, opts=o), 2)
        att, acc, rej, _, _, je = run_stats(c, mech, m, Tt, Pt, Yt, 1e-6, with_jac=True, method=meth,
                                            estimator=est, jac_every=k)
        key = "%s_%s" % (meth, est) + ("_jac%d" % k if k > 1 else "")
        out[key] = {"cells_per_s": round(n / t, 1), "accepted": acc, "rejected": rej, "jacobians": je}
    mech.close()
    return out


def large(c, a):
    """The 111-species mechanism (N = 112) on its mixing-layer states."""
    chem, synth = c.chem, c.synth
    path, m = synth.mechanism_file("large", c.mech_dir)
    T, P, Y = synth.states_mixing(m, 262144, 204)
    n = min(a.large_cells, T.size)
    T, P, Y = T[:n], P[:n], Y[:, :n]
    mech = chem.Mechanism(path, device=0)
    Tt, Pt, Yt = c.d(T), c.d(P), c.d(Y)
    chem.integrate(mech, Tt[:64], Pt[:64], Yt[:, :64].contiguous(), 1e-5)
    t = timed(c, lambda: chem.integrate(mech, Tt, Pt, Yt, 1e-5))
    att, acc, rej, ns, st = run_stats(c, mech, m, Tt, Pt, Yt, 1e-5)
    flops, _ = c.opcount.batch_flops(m, att, acc)
    mech.close()
    return {"workload": "111-species mechanism (784 reactions: 60 third-body, 40 Troe), %s of the "
                        "262,144 mixing-layer cells, dt=1e-5 s, default launch (four wavefronts per cell)"
                        % ("all" if n == 262144 else "the first %d" % n),
            "cells": n, "cells_per_s": round(n / t, 1), "ms_per_call": round(t * 1e3, 3),
            "attempted_steps": att, "accepted_steps": acc, "failed_cells": int((st != 0).sum()),
            "fp64_tflops": round(flops / t / 1e12, 4), "frac": round(flops / t / 1e12 / FP64_PEAK_TFLOPS, 6)}


def small(c, a):
    """10 species, 256 cells, dt = 1e-6 s: per-call times of the launches and of a
    replayed captured graph (the default launch)."""
    chem, synth = c.chem, c.synth
    path, m = synth.mechanism_file("small", c.mech_dir)
    T, P, Y = synth.states_small(m, 256, 201)
    mech = chem.Mechanism(path, device=0)
    Tt, Pt, Yt = c.d(T), c.d(P), c.d(Y)
    out = {"workload": "H2/O2-shaped mechanism (10 species, 25 reactions), 256 cells, dt=1e-6 s", "ms_per_call": {}}
    for mode in ("plain", "persistent", "team", "team_persistent", "auto"):
        o = chem.default_opts(mode=mode)
        chem.integrate(mech, Tt, Pt, Yt, 1e-6, opts=o)
        out["ms_per_call"][mode] = round(timed(c, lambda: chem.integrate(mech, Tt, Pt, Yt, 1e-6, opts=o), 20) * 1e3, 4)
    T1, Y1 = c.torch.empty_like(Tt), c.torch.empty_like(Yt)
    g = chem.Graph(mech, Tt, Pt, Yt, 1e-6, out=(T1, Y1))
    g.launch()
    out["ms_per_call"]["graph_auto"] = round(timed(c, g.launch, 20) * 1e3, 4)
    g.close()
    mech.close()
    return out


def adjoint_cost(c, a):
    """Differentiation case: 16,384 mixing-layer cells, dt = 1e-5 s, loss
    T_final + sum_k w_k Y_k; times of the plain forward call, the checkpointed
    forward call (two passes) and the discrete adjoint (gradients with respect
    to every ln A summed over cells, and the initial state)."""
    chem, synth, np = c.chem, c.synth, c.np
    path, m = synth.mechanism_file("ch4", c.mech_dir)
    n = a.adjoint_cells
    T, P, Y = synth.states_mixing(m, n, 205)
    w = synth.loss_weights(m)
    mech = chem.Mechanism(path, device=0)
    Tt, Pt, Yt = c.d(T), c.d(P), c.d(Y)
    gT = c.torch.ones(n, dtype=c.torch.float64, device=c.dev)
    gY = c.d(np.repeat(w[:, None], n, 1))
    chem.integrate(mech, Tt[:256], Pt[:256], Yt[:, :256].contiguous(), 1e-5)
    t_fwd = min(timed(c, lambda: chem.integrate(mech, Tt, Pt, Yt, 1e-5)) for _ in range(2))
    res = {}

    def fwd_ck():
        res["ck"] = chem.integrate(mech, Tt, Pt, Yt, 1e-5, checkpoint=True)[5]
    t_ck = timed(c, fwd_ck)
    ck = res["ck"]
    recs = int(ck.records())
    t_adj = timed(c, lambda: chem.adjoint(mech, ck, gT, gY, per_cell=False, initial=True))
    ck.close()
    mech.close()
    return {"workload": "CH4-shaped mechanism, %d mixing-layer cells, dt=1e-5 s, d(T_final + sum w_k Y_k)"
                        "/d(ln A_j, T0, Y0)" % n,
            "cells": n, "forward_ms": round(t_fwd * 1e3, 3), "forward_checkpointed_ms": round(t_ck * 1e3, 3),
            "adjoint_ms": round(t_adj * 1e3, 3), "checkpoint_records": recs,
            "adjoint_over_forward": round(t_adj / t_fwd, 3),
            "gradient_over_forward": round((t_ck + t_adj) / t_fwd, 3)}


def work_precision(c, a):
    """The paper's verification study (Sec. 3.1) on synthetic states: each
    solver at tolerances 1e-4 .. 1e-12 (rtol = atol), error against a tight
    reference in the norm of eqs. (ivp_norm)/(error_norm) - per cell the
    2-norm over (T, Y) of |y_ref - y| / (1e-10 + 1e-6 |y_ref|), then the
    largest over cells - and GPU time per call.  States: a sample of the
    65,536 mixing-layer cells (the 64 with the most steps and the rest at
    random), dt = 1e-6 s.  Reference: the CPU oracle with RODAS4 at
    rtol = 1e-14, atol = 1e-18 (the paper uses CVODES at 1e-15 / 1e-20; with
    atol 1e-20 the hottest cell takes 347,169 steps, and the atol 1e-18 and
    1e-20 references differ by 3e-5 in this norm, the FP64 rounding of such
    long integrations - the floor of the comparison)."""
    import oracle
    np, chem, synth = c.np, c.chem, c.synth
    path, m = synth.mechanism_file("ch4", c.mech_dir)
    T, P, Y = synth.states_mixing(m, 65536, 202)
    mech = chem.Mechanism(path, device=0)
    Tt, Pt, Yt = c.d(T), c.d(P), c.d(Y)
    ns = chem.integrate(mech, Tt, Pt, Yt, 1e-6)[3].cpu().numpy()
    top = np.argsort(-ns)[:64]
    rng = np.random.default_rng(11)
    idx = np.unique(np.r_[top, rng.choice(np.setdiff1d(np.arange(T.size), top), a.wp_cells - 64, replace=False)])
    T, P, Y = T[idx], P[idx], np.ascontiguousarray(Y[:, idx])
    log("work-precision: reference on %d cells" % idx.size)
    t0 = time.time()
    ora = oracle.Oracle(path)
    parts, threads = [], 0
    ref_status = []
    for s0 in range(0, idx.size, 64):
        s = slice(s0, min(s0 + 64, idx.size))
        ref = ora.integrate(T[s], P[s], np.ascontiguousarray(Y[:, s]), 1e-6, rtol=1e-14, atol=1e-18,
                            method="rodas4", max_steps=10 ** 7)
        parts.append(np.vstack([ref["T"], ref["Y"]]))
        ref_status.append(ref["status"])
        threads = ref["threads"]
        log("work-precision: reference %d/%d cells, %.0f s" % (s.stop, idx.size, time.time() - t0))
    t_ref = time.time() - t0
    yref = np.hstack(parts)
    ref_ok = np.concatenate(ref_status) == 0
    Tt, Pt, Yt = c.d(T), c.d(P), c.d(Y)
    pts = []
    cases = [(meth, est, 1) for meth in ("ros3", "ros4", "rodas3", "rodas4", "ros34pw2")
             for est in ("embedded", "filtered")]
    cases += [("ros34pw2", "embedded", 4)]
    for meth, est, k in cases:
        for e in range(4, 13):
            tol = 10.0 ** -e
            o = chem.default_opts(method=meth, estimator=est, jac_every=k)
            r = chem.integrate(mech, Tt, Pt, Yt, 1e-6, rtol=tol, atol=tol, opts=o)
            t = timed(c, lambda: chem.integrate(mech, Tt, Pt, Yt, 1e-6, rtol=tol, atol=tol, opts=o))
            y = np.vstack([r[0].cpu().numpy(), r[1].cpu().numpy()])
            ok = ref_ok & (r[4].cpu().numpy() == 0)
            E = np.sqrt((((yref - y) / (1e-10 + 1e-6 * np.abs(yref))) ** 2).sum(0))[ok]
            pts.append({"method": meth, "estimator": est, "jac_every": k, "tol": tol,
                        "error_norm": float(E.max()) if E.size else None,
                        "error_norm_median": float(np.median(E)) if E.size else None, "ms": round(t * 1e3, 3),
                        "failed": int((r[4] != 0).sum().item())})
        log("work-precision: %s %s jac_every=%d done" % (meth, est, k))
    mech.close()
    return {"workload": "%d of the 65,536 CH4 mixing-layer cells (64 with the most steps), dt=1e-6 s" % idx.size,
            "reference": "oracle RODAS4, rtol 1e-14, atol 1e-18, %.1f s on %d threads; %d of %d cells "
                         "finished" % (t_ref, threads, int(ref_ok.sum()), ref_ok.size),
            "norm": "max over cells of the 2-norm over (T, Y) of |y_ref - y| / (1e-10 + 1e-6 |y_ref|); "
                    "cells a solver did not finish are counted in 'failed' and left out of the norm",
            "points": pts}


def oracle_rate(oracle, path, T, P, Y, dt, budget_s, threads=0, chunk=256):
    """The oracle (as it is) on the given cells in order, in chunks, until about
    budget_s seconds of wall time; returns (cells/s, cells done, seconds, threads)."""
    import numpy as np
    o = oracle.Oracle(path)
    done, t0, thr = 0, time.time(), 0
    n = T.size
    while done < n and (time.time() - t0) < budget_s:
        s = slice(done, min(done + chunk, n))
        r = o.integrate(T[s], P[s], np.ascontiguousarray(Y[:, s]), dt, nthreads=threads)
        thr = r["threads"]
        done = s.stop
    el = time.time() - t0
    return done / el, done, el, thr


def cpu_baseline(c, a, head):
    """The oracle on a stratified 4,096-cell sample of the headline batch (the
    85/10/5 mix kept, cells shuffled), on all host threads; per configuration
    the oracle on a bounded sample of that workload, and one core."""
    import oracle
    np, synth = c.np, c.synth
    path, m, T, P, Y, kind = head
    rng = np.random.default_rng(7)
    idx = np.concatenate([rng.choice(np.flatnonzero(kind == k), int(round(f * 4096)), replace=False)
                          for k, f in ((0, 0.85), (1, 0.10), (2, 0.05))])
    idx = rng.permutation(idx)
    v, done, el, thr = oracle_rate(oracle, path, T[idx], P[idx], Y[:, idx], 1e-5, 1e9)
    out = {"value": round(v, 1), "unit": "cells/s", "cores": int(thr), "kind": "oracle",
           "sample": "stratified 4,096 cells of the 1,048,576-cell batching mix (3,482 cold, 410 igniting, "
                     "205 burnt; shuffled), %.1f s wall on %d threads" % (el, thr), "per_config": {}}
    pc = out["per_config"]
    v1, d1, e1, _ = oracle_rate(oracle, path, T[idx], P[idx], Y[:, idx], 1e-5, a.cpu_seconds / 2, threads=1,
                                chunk=32)
    pc["batching_single_core"] = {"cells_per_s": round(v1, 2), "cells": d1, "seconds": round(e1, 1)}
    p2, m2 = synth.mechanism_file("ch4", c.mech_dir)
    T2, P2, Y2 = synth.states_mixing(m2, 65536, 202)
    v, d_, e_, t_ = oracle_rate(oracle, p2, T2, P2, Y2, 1e-6, a.cpu_seconds)
    pc["mixing_65536"] = {"cells_per_s": round(v, 1), "cells": d_, "seconds": round(e_, 1), "threads": t_,
                          "sample": "first cells of the batch"}
    p1, m1 = synth.mechanism_file("small", c.mech_dir)
    T1, P1, Y1 = synth.states_small(m1, 256, 201)
    v, d_, e_, t_ = oracle_rate(oracle, p1, T1, P1, Y1, 1e-6, 1e9)
    pc["small_256"] = {"cells_per_s": round(v, 1), "cells": d_, "seconds": round(e_, 1), "threads": t_}
    p4, m4 = synth.mechanism_file("large", c.mech_dir)
    T4, P4, Y4 = synth.states_mixing(m4, 262144, 204)
    sel = np.random.default_rng(9).permutation(T4.size)[:8192]
    v, d_, e_, t_ = oracle_rate(oracle, p4, T4[sel], P4[sel], Y4[:, sel], 1e-5, a.cpu_seconds, chunk=64)
    pc["large_262144"] = {"cells_per_s": round(v, 1), "cells": d_, "seconds": round(e_, 1), "threads": t_,
                          "sample": "random cells of the batch"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cells", type=int, default=1048576, help="headline batch size")
    ap.add_argument("--large-cells", type=int, default=262144)
    ap.add_argument("--adjoint-cells", type=int, default=16384)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--quick", action="store_true", help="headline only")
    ap.add_argument("--skip", default="", help="comma list of legs to skip: mixing,methods,large,small,adjoint")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one 256 MiB device-to-device copy (reference for HBM byte counters)")
    ap.add_argument("--work-precision", default="",
                    help="run only the work-precision sweep and write its JSON to this file")
    ap.add_argument("--wp-cells", type=int, default=256)
    ap.add_argument("--only", default="", help="run only this leg (mixing, methods, large, small, adjoint) "
                                               "and print its JSON (for profiling one workload)")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py measures one GPU; --gpus %d is not supported "
              "(cells are independent: several GPUs would each take a contiguous share of the batch)" % a.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2205_05681_amd import chem, opcount, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    c = Ctx(torch, np, chem, synth, opcount, dev, tempfile.mkdtemp(prefix="chem_bench_"))
    if a.calibrate_copy:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        c.sync()
        del src, dst
    if a.work_precision:
        wp = work_precision(c, a)
        with open(a.work_precision, "w") as f:
            json.dump(wp, f)
        print(json.dumps({"work_precision": a.work_precision, "points": len(wp["points"])}), flush=True)
        return
    if a.only:
        fn = {"mixing": mixing, "methods": methods, "large": large, "small": small, "adjoint": adjoint_cost}[a.only]
        print(json.dumps({a.only: fn(c, a)}), flush=True)
        return
    head, head_data = headline(c, a)
    skip = set(a.skip.split(",")) if a.skip else set()
    if a.quick:
        skip |= {"mixing", "methods", "large", "small", "adjoint"}
    legs = {}
    for name, fn in (("mixing", mixing), ("methods", methods), ("large", large), ("small", small),
                     ("adjoint", adjoint_cost)):
        if name not in skip:
            log("leg: %s" % name)
            legs[name] = fn(c, a)
    cpu = None if a.no_cpu else cpu_baseline(c, a, head_data)
    out = {
        "metric": METRIC,
        "value": round(head["value"], 1),
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": head["config"],
        "roofline": head["roofline"],
        "cpu_baseline": cpu,
        "plain_vs_persistent": head["plain_vs_persistent"],
    }
    out.update(legs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
