"""Benchmark: cells integrated per second over one operator-splitting step.

Workload (default): the CH4-shaped synthetic mechanism (53 species, 325
reversible reactions, 30 third-body, 25 Troe) over 65,536 mixing-layer cells
(P ~ U[1, 5] atm, Z ~ Beta(2, 5), T = linear mix of 300 K fuel and 800 K air
plus N(0, 200^2) K), dt = 1e-6 s, FP64, rtol 1e-6, atol 1e-10.  One step = one
chem_integrate call over every cell with the inputs resident in HBM.

Prints one JSON line (rank 0).  Extra keys: "roofline" for the integrator
kernel (algorithmic FP64 flops per launch over its average launch duration,
measured with HIP events on the launch stream), "cpu_baseline" (the CPU
oracle on a bounded sample of the same cells, on this host's cores), "modes"
(cells/s of each launch mode of the library on this workload), "batching"
(plain vs persistent launches on the batching mix, whose step counts differ
by ~1000x between cells) and "adjoint" (discrete-adjoint vs forward time on
the differentiation case).
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
KERNEL_SOURCES = ["paper_2205_05681_amd/csrc/integrate.hip", "paper_2205_05681_amd/csrc/team.h",
                  "paper_2205_05681_amd/csrc/kinetics.h", "paper_2205_05681_amd/csrc/ros4.h",
                  "paper_2205_05681_amd/csrc/mech.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_team_kernel_ch4_65536.json")


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def workload(name, synth, mech_dir):
    if name == "ch4_mixing":
        path, m = synth.mechanism_file("ch4", mech_dir)
        T, P, Y = synth.states_mixing(m, 65536, 202)
        desc = ("CH4-shaped synthetic mechanism (53 species, 325 reactions: 30 third-body, 25 Troe), "
                "65,536 mixing-layer cells, P~U[1,5] atm, Z~Beta(2,5), dt=1e-6 s, rtol 1e-6, atol 1e-10")
        return path, m, T, P, Y, 1e-6, desc
    if name == "ch4_batching":
        path, m = synth.mechanism_file("ch4", mech_dir)
        T, P, Y, _ = synth.states_batching(m, 1048576, 203)
        desc = ("CH4-shaped synthetic mechanism, 1,048,576 cells: 85% cold (<800 K), 10% stoichiometric "
                "1100-1400 K, 5% burnt gas; dt=1e-5 s, rtol 1e-6, atol 1e-10")
        return path, m, T, P, Y, 1e-5, desc
    if name == "small":
        path, m = synth.mechanism_file("small", mech_dir)
        T, P, Y = synth.states_small(m, 256, 201)
        desc = "H2/O2-shaped synthetic mechanism (10 species, 25 reactions), 256 cells, dt=1e-6 s"
        return path, m, T, P, Y, 1e-6, desc
    raise SystemExit("unknown workload %s" % name)


def timed(fn, torch):
    torch.cuda.synchronize()
    t = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t


def batching(chem, synth, torch, np, mech_dir, n, dev):
    """The batching mix (85 % cold, 10 % near ignition at stoichiometric
    mixture fraction, 5 % burnt gas; dt = 1e-5 s) on n cells: cells/s of the
    plain and persistent one-cell-per-thread launches (cells in index order
    and hottest first) and of the one-wavefront-per-cell launches, one timed
    call each after a warm-up call on 256 cells."""
    path, m = synth.mechanism_file("ch4", mech_dir)
    T, P, Y, kind = synth.states_batching(m, n, 203)
    mech = chem.Mechanism(path, device=0)
    d = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    Tt, Pt, Yt = d(T), d(P), d(Y)
    out = {"workload": "CH4-shaped mechanism, %d cells drawn with the 1,048,576-cell batching recipe "
                       "(85%% cold <800 K, 10%% stoichiometric 1100-1400 K, 5%% burnt gas), dt=1e-5 s" % n,
           "cells": n, "cells_per_s": {}}
    ns = None
    runs = (("plain", 0), ("persistent", 0), ("plain", 1), ("persistent", 1), ("team", 1),
            ("team_persistent", 1))
    for mode, order in runs:
        o = chem.default_opts(mode=mode, order=order)
        chem.integrate(mech, Tt[:256], Pt[:256], Yt[:, :256].contiguous(), 1e-5, opts=o)
        res = {}

        def run():
            res["r"] = chem.integrate(mech, Tt, Pt, Yt, 1e-5, opts=o)
        el = timed(run, torch)
        out["cells_per_s"][mode + ("" if order else "_index_order")] = round(n / el, 1)
        ns = res["r"][3].cpu().numpy()
        assert int((res["r"][4] != 0).sum()) == 0, "failed cells in the batching mix"
    out["accepted_steps"] = {k: {"mean": round(float(ns[kind == i].mean()), 2), "max": int(ns[kind == i].max())}
                             for i, k in enumerate(("cold", "igniting", "burnt"))}
    cps = out["cells_per_s"]
    # one cell per thread in index order is the plain baseline of the comparison
    base = cps["plain_index_order"]
    out["over_plain_index_order"] = {k: round(v / base, 3) for k, v in cps.items()}
    mech.close()
    return out


def adjoint_cost(chem, synth, torch, np, mech_dir, n, dev):
    """Differentiation case: n mixing-layer cells, dt = 1e-5 s, losses final T
    and sum_k w_k Y_k; times of the plain forward call, the checkpointed
    forward call (two passes) and the discrete adjoint (gradients with
    respect to every ln A summed over cells, and the initial state)."""
    path, m = synth.mechanism_file("ch4", mech_dir)
    T, P, Y = synth.states_mixing(m, n, 205)
    w = synth.loss_weights(m)
    mech = chem.Mechanism(path, device=0)
    d = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    Tt, Pt, Yt = d(T), d(P), d(Y)
    gT = torch.ones(n, dtype=torch.float64, device=dev)
    gY = d(np.repeat(w[:, None], n, 1))
    chem.integrate(mech, Tt[:256], Pt[:256], Yt[:, :256].contiguous(), 1e-5)
    t_fwd = min(timed(lambda: chem.integrate(mech, Tt, Pt, Yt, 1e-5), torch) for _ in range(2))
    res = {}

    def fwd_ck():
        res["ck"] = chem.integrate(mech, Tt, Pt, Yt, 1e-5, checkpoint=True)[5]
    t_ck = timed(fwd_ck, torch)
    ck = res["ck"]
    recs = int(ck.records())
    t_adj = timed(lambda: chem.adjoint(mech, ck, gT, gY, per_cell=False, initial=True), torch)
    ck.close()
    mech.close()
    return {"workload": "CH4-shaped mechanism, %d mixing-layer cells, dt=1e-5 s, d(T_final + sum w_k Y_k)"
                        "/d(ln A_j, T0, Y0)" % n,
            "cells": n, "forward_ms": round(t_fwd * 1e3, 3), "forward_checkpointed_ms": round(t_ck * 1e3, 3),
            "adjoint_ms": round(t_adj * 1e3, 3), "checkpoint_records": recs,
            "adjoint_over_forward": round(t_adj / t_fwd, 3),
            "gradient_over_forward": round((t_ck + t_adj) / t_fwd, 3)}


def cpu_baseline(oracle, path, T, P, Y, dt, budget_s):
    """The oracle (as it is) on the first cells of the workload, in chunks of
    512, until about budget_s seconds of CPU work."""
    import numpy as np
    o = oracle.Oracle(path)
    done, t0, threads = 0, time.time(), 0
    n = T.size
    while done < n and (time.time() - t0) < budget_s:
        c = slice(done, min(done + 512, n))
        r = o.integrate(T[c], P[c], np.ascontiguousarray(Y[:, c]), dt)
        threads = r["threads"]
        done = c.stop
    el = time.time() - t0
    return {"value": done / el, "unit": "cells/s", "cores": int(threads), "kind": "oracle",
            "sample": "first %d of the %d cells, %.1f s wall on %d threads" % (done, n, el, threads)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="ch4_mixing")
    ap.add_argument("--mode", default="auto", help="headline launch mode")
    ap.add_argument("--compare", default="team,plain,persistent",
                    help="other modes to time (thread-per-cell modes take one step)")
    ap.add_argument("--order", default="hot", choices=["hot", "index"],
                    help="dispatch order of the cells: hottest first (library default) or index order")
    ap.add_argument("--batching-cells", type=int, default=65536,
                    help="cells of the batching-mix comparison (0: skip)")
    ap.add_argument("--adjoint-cells", type=int, default=16384,
                    help="cells of the adjoint/forward cost measurement (0: skip)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one 256 MiB device copy (reference for HBM byte counters)")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py measures one GPU; --gpus %d is not supported "
              "(cells are independent: several GPUs would each take a contiguous share of the batch)" % a.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2205_05681_amd import chem, opcount, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    mech_dir = tempfile.mkdtemp(prefix="chem_bench_")
    path, m, T, P, Y, dt, desc = workload(a.workload, synth, mech_dir)
    n = T.size
    mech = chem.Mechanism(path, device=0)
    d = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    Tt, Pt, Yt = d(T), d(P), d(Y)
    T1 = torch.empty_like(Tt)
    Y1 = torch.empty_like(Yt)
    h = torch.zeros(n, dtype=torch.float64, device=dev)
    ns = torch.empty(n, dtype=torch.int32, device=dev)
    st = torch.empty(n, dtype=torch.int32, device=dev)

    order = {"hot": 1, "index": 0}[a.order]

    def step(mode):
        h.zero_()
        chem.integrate(mech, Tt, Pt, Yt, dt, h=h, opts=chem.default_opts(mode=mode, order=order),
                       out=(T1, Y1), n_steps=ns, status=st)

    if a.calibrate_copy:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # ---- headline mode: W warmup steps, then K timed steps
    for _ in range(a.warmup):
        step(a.mode)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(a.steps)]
    opts = chem.default_opts(mode=a.mode, order=order)
    t0 = time.perf_counter()
    for i in range(a.steps):
        h.zero_()
        ev[i][0].record(stream)
        chem.integrate(mech, Tt, Pt, Yt, dt, h=h, opts=opts, out=(T1, Y1), n_steps=ns, status=st)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_ms = [s.elapsed_time(e) for s, e in ev]
    ms_per_step = wall * 1e3 / a.steps
    value = n / (wall / a.steps)
    status = st.cpu().numpy()
    steps_acc = ns.cpu().numpy()

    # ---- step statistics of the same call (deterministic), for the op count
    stats = torch.zeros(3, dtype=torch.int64, device=dev)
    h.zero_()
    chem.integrate(mech, Tt, Pt, Yt, dt, h=h, opts=chem.default_opts(mode=a.mode, order=order, stats=stats), out=(T1, Y1))
    torch.cuda.synchronize()
    attempts, accepted, rejected = (int(x) for x in stats.cpu().numpy())
    flops, trans = opcount.batch_flops(m, attempts, accepted)
    avg_launch_s = float(np.mean(launch_ms)) / 1e3
    achieved = flops / avg_launch_s / 1e12
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        tf = json.load(open(TRAFFIC_FILE))
        if tf.get("kernel_hash") == kernel_hash() and tf.get("workload") == a.workload:
            traffic = tf.get("hbm_bytes_per_launch")
    roofline = {"bound": "alu", "achieved": round(achieved, 4), "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 6), "traffic": traffic,
                "kernel": "integrate_team_kernel" if a.mode in ("auto", "team", "team_persistent") else
                "integrate_thread_kernel",
                "flops_per_launch": flops, "transcendentals_per_launch": trans,
                "attempted_steps": attempts, "accepted_steps": accepted,
                "avg_launch_ms": round(avg_launch_s * 1e3, 4)}

    # ---- warm start: each cell's last internal step carried over as its next
    # initial step (the coupling's reuse of h between split steps), same inputs
    hw = torch.zeros(n, dtype=torch.float64, device=dev)
    chem.integrate(mech, Tt, Pt, Yt, dt, h=hw, opts=opts, out=(T1, Y1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        chem.integrate(mech, Tt, Pt, Yt, dt, h=hw, opts=opts, out=(T1, Y1))
    torch.cuda.synchronize()
    warm_wall = time.perf_counter() - t0
    wstats = torch.zeros(3, dtype=torch.int64, device=dev)
    chem.integrate(mech, Tt, Pt, Yt, dt, h=hw, opts=chem.default_opts(mode=a.mode, order=order, stats=wstats),
                   out=(T1, Y1))
    torch.cuda.synchronize()
    w_att, w_acc, _ = (int(x) for x in wstats.cpu().numpy())
    warm = {"value": round(n / (warm_wall / a.steps), 1), "unit": "cells/s",
            "ms_per_step": round(warm_wall * 1e3 / a.steps, 4),
            "attempted_steps": w_att, "accepted_steps": w_acc,
            "note": "same inputs, h_io carried over from the previous call"}

    # ---- other launch modes on the same cells
    modes = {a.mode: round(value, 1)}
    for mode in [x for x in a.compare.split(",") if x and x != a.mode]:
        reps = 1 if mode in ("plain", "persistent") else max(1, a.steps // 2)
        step(mode)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            step(mode)
        torch.cuda.synchronize()
        modes[mode] = round(n / ((time.perf_counter() - t) / reps), 1)

    mech.close()
    batch = batching(chem, synth, torch, np, mech_dir, a.batching_cells, dev) if a.batching_cells else None
    adj = adjoint_cost(chem, synth, torch, np, mech_dir, a.adjoint_cells, dev) if a.adjoint_cells else None

    cpu = None
    if not a.no_cpu:
        import oracle
        cpu = cpu_baseline(oracle, path, T, P, Y, dt, a.cpu_seconds)

    out = {
        "metric": "cells/s per split step at rtol 1e-6 (plain vs persistent); adjoint/forward cost",
        "value": round(value, 1),
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "cells": n, "species": m.n_species, "reactions": len(m.reactions),
                   "dt": dt, "rtol": 1e-6, "atol": 1e-10, "mode": a.mode, "order": a.order,
                   "failed_cells": int((status != 0).sum()),
                   "accepted_steps_mean": round(float(steps_acc.mean()), 3),
                   "accepted_steps_max": int(steps_acc.max())},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "modes": modes,
        "warm_start": warm,
        "batching": batch,
        "adjoint": adj,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
