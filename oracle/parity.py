"""The parity rule of the GPU tests, measured on the oracle itself.

TEST INFRASTRUCTURE ONLY (used by the GPU tests and the smoke check).

Bar, per cell: |T - T_or| <= 1e-6 T_or and |Y_k - Y_or,k| <= 1e-6 |Y_or,k| +
1e-10 (rtol 1e-6 on T and Y; atol 1e-10).  Both sides run the same algorithm
and constants; they differ by rounding only (contracted multiply-adds, the
order of sums, device exp/log).  Cells that run hundreds of steps through a
thermal runaway amplify such differences past the bar: measured on the
oracle, changes at the rounding level - the same source built with
multiply-adds contracted, and the input temperature moved by one or two ulp -
each put 5 to 13 of the 256 cells of the small H2/O2-shaped case beyond the
bar (up to 38 times it) and change the accepted-step count of 10 to 14 % of
them (by up to 20 steps); on the CH4 mixing states one cell in 4096 moves
past the bar.  So the rule compares the GPU with what rounding does to the
oracle, cell by cell:

 R1  a cell off the bar must be rounding-sensitive: one of nine rounding-level
     variants of the oracle (the contracted build; either build with T moved by
     -2, -1, +1, +2 ulp) moves that cell by at least 1e-3 of the bar, an
     amplification of a one-ulp change by 1e7 or more;
 R2  its deviation must stay within three times the bar plus the largest of
     those moves, component by component (the moves are heavy-tailed: one
     accept/reject decision that goes the other way moves a cell by about the
     bar while the other variants move it by 1e-3 of it);
 R3  at most twice as many cells may be off the bar as the worst single
     variant puts off it, plus two.
Accepted-step counts follow the same logic:
 S1  at most twice as many cells may differ from the oracle's count as for the
     worst variant, plus two;
 S2  a count may differ by at most 2, or, on a rounding-sensitive cell, by at
     most 8 % (the variants move counts by up to 4 %).
Applied to each of the nine variants in turn, with the other eight as its
envelope, the rule passes all nine on the small case.
"""
from __future__ import annotations

import numpy as np

import oracle

ULPS = (-2, -1, 1, 2)
SENSITIVE = 1e-3      # a variant moves the cell by this fraction of the bar
STEP_SPREAD = 0.08    # twice the largest relative step-count change of a variant


def fma_twin(o):
    """The same mechanism in the FMA-contracted build of the oracle."""
    if not hasattr(o, "_fma"):
        import os
        if not os.path.exists(oracle.LIB_FMA) or os.path.getmtime(oracle.LIB_FMA) < os.path.getmtime(oracle.SRC):
            oracle.build(out=oracle.LIB_FMA, flags=oracle.FMA_FLAGS)
        o._fma = oracle.Oracle(o.path, library=oracle.lib(oracle.LIB_FMA))
    return o._fma


def variants(o, T, P, Y, dt, h=None, **kw):
    """Results of the nine rounding-level variants on the given cells."""
    u = np.finfo(float).eps
    f = fma_twin(o)
    out = []
    for src, shifts in ((f, (0,) + ULPS), (o, ULPS)):
        for k in shifts:
            out.append(src.integrate(T * (1.0 + k * u), P, np.ascontiguousarray(Y), dt,
                                     h=None if h is None else h.copy(), **kw))
    return out


def _ratio(T, Y, ref):
    barT = 1e-6 * np.abs(ref["T"])
    barY = 1e-6 * np.abs(ref["Y"]) + 1e-10
    return np.maximum(np.abs(T - ref["T"]) / barT, (np.abs(Y - ref["Y"]) / barY).max(0))


def check(Tg, Yg, ng, ref, var, label, steps=True, worst=None, worst_n=None):
    """Apply R1-R3 (and S1, S2 when ``steps``) to GPU results against the
    oracle's ``ref`` and its rounding variants ``var`` (all on the same
    cells).  ``worst``/``worst_n`` replace the variants' counts of off-bar
    cells and of cells with another step count when ``var`` covers only some
    of the cells (a large batch: the counts then come from one variant run
    over the whole batch).  Returns a short summary string."""
    barT = 1e-6 * np.abs(ref["T"])
    barY = 1e-6 * np.abs(ref["Y"]) + 1e-10
    envT = np.max([np.abs(v["T"] - ref["T"]) for v in var], axis=0)
    envY = np.max([np.abs(v["Y"] - ref["Y"]) for v in var], axis=0)
    sens_all = (envT > SENSITIVE * barT) | (envY > SENSITIVE * barY).any(0)
    rg = _ratio(Tg, Yg, ref)
    off = np.flatnonzero(rg > 1.0)
    if worst is None:
        worst = max(int((_ratio(v["T"], v["Y"], ref) > 1.0).sum()) for v in var)
    assert off.size <= 2 * worst + 2, "%s: %d cells off the bar, a rounding variant puts %d off (first %s)" % (
        label, off.size, worst, off[:5])
    sens = sens_all[off]
    assert sens.all(), "%s: cells %s off the bar (%s x) but not rounding-sensitive" % (
        label, off[~sens], rg[off[~sens]])
    dT = np.abs(Tg - ref["T"])[off]
    dY = np.abs(Yg - ref["Y"])[:, off]
    okT = dT <= 3 * (barT[off] + envT[off])
    okY = (dY <= 3 * (barY[:, off] + envY[:, off])).all(0)
    assert (okT & okY).all(), "%s: cells %s beyond three times the bar plus the rounding envelope" % (
        label, off[~(okT & okY)])
    msg = "%s: %d cells, %d off the bar (rounding variants: up to %d)" % (label, rg.size, off.size, worst)
    if steps:
        no = ref["n_acc"].astype(np.int64)
        d = np.abs(ng.astype(np.int64) - no)
        vn = np.array([v["n_acc"] for v in var], np.int64)
        if worst_n is None:
            worst_n = int((vn != no).sum(1).max())
        assert (d > 0).sum() <= 2 * worst_n + 2, "%s: steps differ on %d cells, a rounding variant on %d" % (
            label, (d > 0).sum(), worst_n)
        lim = np.where(sens_all, np.maximum(2, np.ceil(STEP_SPREAD * no)), 2)
        bad = np.flatnonzero(d > lim)
        assert bad.size == 0, "%s: step counts of cells %s: %s against the oracle's %s" % (
            label, bad, ng[bad], no[bad])
        msg += ", steps differ on %d (variants: up to %d)" % ((d > 0).sum(), worst_n)
    return msg


def check_batch(o, T, P, Y, dt, Tg, Yg, ng, label, h=None, steps=True, **kw):
    """The rule on a whole batch: the oracle and its FMA-contracted twin run on
    every cell (the twin's counts stand for the variants' in R3 and S1), and
    the nine variants run on the cells that are off the bar or whose step
    count differs."""
    ref = o.integrate(T, P, Y, dt, h=None if h is None else h.copy(), **kw)
    fma = fma_twin(o).integrate(T, P, Y, dt, h=None if h is None else h.copy(), **kw)
    worst = int((_ratio(fma["T"], fma["Y"], ref) > 1.0).sum())
    worst_n = int((fma["n_acc"] != ref["n_acc"]).sum())
    rg = _ratio(Tg, Yg, ref)
    sel = np.flatnonzero((rg > 1.0) | (ng != ref["n_acc"]))
    if sel.size == 0:
        return ref, "%s: %d cells, none off the bar, equal step counts" % (label, T.size)
    sub = lambda r: {k: (v[..., sel] if isinstance(v, np.ndarray) and v.shape[-1] == T.size else v)
                     for k, v in r.items()}
    var = variants(o, T[sel], P[sel], Y[:, sel], dt, h=None if h is None else h[sel], **kw)
    msg = check(Tg[sel], Yg[:, sel], ng[sel], sub(ref), var, label, steps=steps, worst=worst,
                worst_n=worst_n)
    return ref, msg + " (of %d cells; rounding variants on the %d that differ)" % (T.size, sel.size)
