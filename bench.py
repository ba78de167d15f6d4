#!/usr/bin/env python3
"""Throughput of the VIP fractional step on one MI355X.

Workload (the configuration the headline metric is quoted on): flow past a
circular cylinder D = 1 in [-10, 20] x [-10, 10] with h = D/128 (lattice nodes
outside the body plus 256 surface nodes), together with the equilateral
triangular lid-driven cavity (side 1, lid on top) at the same h; Re = 200,
dt = h/10 (local CFL about 0.2 at the cylinder's shoulders, where |u| ~ 2),
pressure Poisson solved to an FP64 relative residual of 1e-8.  One step = one
fractional step of both domains.

Paths timed on the same node sets, each from the same impulsive start:
  * learned: FP32 inner Krylov (SpMV + vectors) inside FP64 iterative
             refinement; Poisson start vector phi_n + alpha (phi_n - phi_(n-1))
             + beta c with c the learned network's correction;
  * mixed:   the same precision split, start vector phi_n;
  * fp64:    plain FP64 Krylov, start vector phi_n;
  (optional: extrap = mixed with the extrapolation alone, fp64zero = FP64 from
  a zero start vector).
Every timed path starts from the same flow: the state after --spinup (500)
untimed fractional steps from the impulsive start, so that the timed steps
stand for the bulk of a long run (the workload runs 2000 steps) rather than its
first steps, where the pressure transient of the impulsive start makes the
solves several times more expensive; the first path and fp64 are also timed
from the impulsive start and reported under `transient`.
The network is trained before any timing on snapshots the solver generates on
small training node sets (one-off, outside the timed region).  `value` is the
learned path.  The roofline entry is the kernel of that path with the most time
per step among those timed with HIP events inside the library over the timed
steps (all of them under `rooflines`).  The CPU baseline runs the FP64 oracle
(SciPy, Krylov mode, same tolerance) on a window of the workload.

Prints one JSON line.  `--summarize-trace DIR [SKIP]` and `--summarize-counter DIR
COUNTER` instead print markdown summaries of rocprofv3 CSV output of this script.
`--network-only` times the learned start vector's fused network launch alone on a
synthetic image of the cylinder lattice (for profiler runs of that kernel).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1401_6513_amd import nodesets as ns  # noqa: E402

METRIC = "node-updates/s per fractional step (Poisson to 1e-8), learned+FP32 vs plain FP64"
HBM_PEAK_GBS = 8000.0
# committed HBM counter profiles per timed kernel, and the sources each kernel is built from
# (hashed together, in this order)
HBM_PROFILES = {
    "pres_spmv": ("hbm_counters_pressure_spmv_cylinder_h128.md", ("krylov.hip", "tile.h")),
    "pred_t": ("hbm_counters_predictor_t_cylinder_h128.md", ("krylov.hip", "tile.h")),
    "pred_x": ("hbm_counters_predictor_x_cylinder_h128.md", ("krylov.hip",)),
    "pred_e": ("hbm_counters_predictor_e_cylinder_h128.md", ("krylov.hip",)),
    "pred_ts": ("hbm_counters_predictor_ts_cylinder_h128.md", ("krylov.hip", "tile.h")),
    "pred_spmv": ("hbm_counters_predictor_spmv_cylinder_h128.md", ("krylov.hip", "tile.h")),
    "pred_spmv1": ("hbm_counters_predictor_spmv1_cylinder_h128.md", ("krylov.hip", "tile.h")),
    "sweep0": ("hbm_counters_finest_sweep_cylinder_h128.md", ("amg.hip", "tile.h")),
    "pred_rhs": ("hbm_counters_predictor_rhs_cylinder_h128.md", ("step.hip", "tile.h")),
}


def measured_traffic(kernel="pres_spmv"):
    """Calibrated HBM bytes per launch of a kernel from its committed counter profile, or None
    when there is none or the kernel's sources have changed since the counters were taken."""
    import hashlib
    if kernel not in HBM_PROFILES:
        return None
    fname, srcs = HBM_PROFILES[kernel]
    try:
        fields = dict(line.split(": ", 1) for line in open(os.path.join(ROOT, "profiles", fname)).read().splitlines()
                      if line.startswith(("traffic_bytes_per_launch:", "source_sha256:")))
        cur = hashlib.sha256(b"".join(open(os.path.join(ROOT, "paper_1401_6513_amd", "csrc", f), "rb").read()
                                      for f in srcs)).hexdigest()
        if fields.get("source_sha256", "").strip() != cur:
            return None
        return int(fields["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def log(msg):
    sys.stderr.write("[bench] %s\n" % msg)
    sys.stderr.flush()


# zones of the stepwise refined cylinder workload (finest first): spacing h, 2h, 4h, and 8h outside
REFINED_ZONES = [(-1.5, 6.0, -1.5, 1.5), (-3.0, 12.0, -3.0, 3.0), (-6.0, 18.0, -6.0, 6.0)]


def workload(h, kind="lattice"):
    if kind == "refined":
        # flow past the cylinder on a stepwise refined node set (finest spacing h near the body,
        # doubling in three steps): every row takes the general sliced-ELL path
        return [ns.refined_cylinder_channel(h, REFINED_ZONES, n_surface=256)]
    cyl = ns.cylinder_channel(h, box=(-10.0, 20.0, -10.0, 10.0), shape="circle", n_surface=256)
    tri = ns.triangle_cavity(h)
    return [cyl, tri]


def _initial(spec, dev):
    import torch
    inflow = (1.0, 0.0) if spec.name.startswith(("cyl", "refined")) else (0.0, 0.0)
    u, v, p = ns.boundary_initial(spec, inflow)
    return [torch.tensor(a, device=dev) for a in (u, v, p)]


PATHS = {
    "learned": dict(precision="P_MIXED", warmstart="WS_LEARNED"),
    "mixed": dict(precision="P_MIXED", warmstart="WS_PREV"),
    "extrap": dict(precision="P_MIXED", warmstart="WS_EXTRAP"),
    "fp64": dict(precision="P_FP64", warmstart="WS_PREV"),
    "fp64x": dict(precision="P_FP64", warmstart="WS_EXTRAP"),
    "fp64zero": dict(precision="P_FP64", warmstart="WS_ZERO"),
    # plain FP64 Krylov: Jacobi preconditioner, previous increment as the start, no learned part
    # (opt-in: on the cylinder at h = D/128 Jacobi-BiCGStab does not converge)
    "plain": dict(precision="P_FP64", warmstart="WS_PREV", preconditioner="PC_JACOBI"),
}


# kernels timed with HIP events inside the library besides the pressure SpMV (vip_kernel_timing)
TIMED = {2: "pred_spmv", 3: "pred_t", 4: "pred_x", 5: "sweep0", 6: "pred_rhs"}
KERNEL_NAMES = {
    "pres_spmv": "k_bicg_v<%s,%s,1> (pressure SpMV)",
    "pred_spmv": "k_bicg_v<float,float,2> (predictor SpMV, both velocity systems)",
    "pred_spmv1": "k_bicg_v<float,float,1> x 2 (predictor SpMV, one launch per velocity system; per iteration)",
    "pred_t": "k_bicg_t<float,float,1,*,true> (predictor t = A s with s = r - alpha v formed inside, per system)",
    "pred_ts": "k_bicg_ts<float> (predictor t = A s with s = r - alpha v formed inside and the five sums, per system)",
    "pred_e": "k_bicg_e<float,2> (predictor: the last iteration's x and r update with the new p, both systems)",
    "pred_x": "k_bicg_x<float,2> (predictor iterate and residual update, both systems)",
    "sweep0": "k_sweep<float,0> (finest-level damped Jacobi post-smoothing sweep, LDS tiles)",
    "pred_rhs": "k_predictor_rhs (VIP convection, AB2 and the predictor right-hand side, FP64)",
}


def kernel_bytes(ctx, spec, fp32):
    """Algorithmic HBM bytes of one launch of each timed kernel on the first domain.  Vectors are
    read or written once (ideal reuse of gathered entries); canonical (tile) rows read no column
    or value stream; irregular rows read their values, their columns (int16 row-relative or
    int32) and, in FP32, their row sums; tiled launches read the irregular-row list and one
    256-byte record per 64 x 16 lattice tile."""
    n, _, nnz = ctx.vip_operator_shape("poisson")
    counts, taps = ctx.vip_canonical_rows()
    ne, ne16 = ctx.vip_column_bytes()[:2]
    cb = (2.0 * ne16 + 4.0 * (ne - ne16)) / max(ne, 1)   # mean bytes per stored column
    K = taps
    vb = 4 if fp32 else 8
    W = int(np.floor((spec.xy[:, 0].max() - spec.xy[:, 0].min()) / spec.h + 0.5)) + 1
    H = int(np.floor((spec.xy[:, 1].max() - spec.xy[:, 1].min()) / spec.h + 0.5)) + 1
    tiled = counts[4] > 0
    rec = 256 * (-(-W // 64) * -(-H // 16)) if tiled else 0

    def irregular(ncan, val_b, extra_b):
        # values + columns of the irregular rows, their per-row extras, the irregular-row list
        return (val_b + cb) * (nnz - K * ncan) + extra_b * (n - ncan) + (4 * (n - ncan) if tiled else 0)

    nc = {k: int(counts[k]) for k in range(7)}
    out = {}
    out["pres_spmv"] = 3 * vb * n + irregular(nc[4] if fp32 else nc[0], vb, 4 if fp32 else 0) + rec
    # predictor (FP32 matrices H D^-1 with their row sums), systems u and v
    out["pred_spmv"] = 2 * 3 * 4 * n + irregular(nc[5], 4, 4) + irregular(nc[6], 4, 4) + rec
    out["pred_t"] = 4 * 4 * n + (irregular(nc[5], 4, 4) + irregular(nc[6], 4, 4)) / 2 + rec
    out["pred_x"] = 2 * 7 * 4 * n
    # the update pass of the predictor's iteration (both systems): reads x, r, p, v, t and writes
    # x, r, p; its t kernel reads r, v (s formed inside) and r-hat and writes t
    out["pred_e"] = 2 * 8 * 4 * n
    out["pred_ts"] = out["pred_t"]
    out["pred_spmv1"] = out["pred_spmv"]
    # finest level: y, b in, out written; irregular rows add values, columns, row sum, damped diagonal
    out["sweep0"] = 3 * 4 * n + irregular(nc[4], 4, 8) + rec
    # u, v in; the AB2 history in and out (2 vectors each way); r_u, r_v out; VIP spacings d_ew,
    # d_ns; the canonical-node pixel; the lattice map once; general nodes read their four VIP rows
    # and the node rows (D^[0,0] and Laplacian values, shared columns) from the ELL
    vip_nnz = sum(ctx.vip_operator_shape(o)[2] for o in ("vip_e", "vip_w", "vip_n", "vip_s"))
    node_nnz = ctx.vip_operator_shape("identity")[2]
    frac_gen = (n - nc[3]) / max(n, 1)
    out["pred_rhs"] = (10 * 8 * n + 4 * n + (4 * W * H if nc[3] > 0 else 0)
                       + frac_gen * (vip_nnz * 12 + node_nnz * 20))
    return out


def configure(vip, ctxs, specs, path, tol, inner_tol, helmholtz_tol=None, learned_precond=False):
    """Options of a path on every domain's context, and a fresh step history."""
    cfg = PATHS[path]
    for ctx, spec in zip(ctxs, specs):
        opt = vip.default_options(period=spec.period, poisson_tol=tol, inner_tol=inner_tol,
                                  precision=getattr(vip, cfg["precision"]),
                                  warmstart=getattr(vip, cfg["warmstart"]),
                                  preconditioner=getattr(vip, cfg.get("preconditioner", "PC_AMG")),
                                  learned_precond=1 if (learned_precond and path == "learned") else 0)
        if helmholtz_tol is not None:
            opt.helmholtz_tol = helmholtz_tol
        ctx.vip_set_options(opt)
        ctx.vip_reset_history()


def spin_up(vip, ctxs, specs, dt, re, nsteps, tol, inner_tol, pool):
    """The flow after `nsteps` untimed fractional steps from the impulsive start (FP32 inner
    solves, extrapolated start vectors), as the initial state of every timed path: the timed
    steps then stand for the bulk of a long run rather than its first steps."""
    import torch
    dev = torch.device("cuda", 0)
    configure(vip, ctxs, specs, "extrap", tol, inner_tol)
    state = [_initial(s, dev) for s in specs]

    def one(j):
        u, v, p = state[j]
        for k in range(nsteps):
            ctxs[j].vip_step(u, v, p, dt, re)
            if j == 0 and (k + 1) % 100 == 0:
                log("spin-up step %d of %d" % (k + 1, nsteps))
    if pool is not None:
        list(pool.map(one, range(len(ctxs))))
    else:
        for j in range(len(ctxs)):
            one(j)
    torch.cuda.synchronize()
    out = [[t.clone() for t in st] for st in state]
    torch.cuda.synchronize()
    return out


def run_path(vip, ctxs, specs, path, dt, re, warmup, steps, tol, time_spmv, inner_tol, pool=None,
             helmholtz_tol=None, learned_precond=False, init=None):
    """Run `steps` timed steps of every domain (domains in parallel host threads, one HIP stream
    each, when a pool is given) from `init` (else the impulsive start); returns wall seconds,
    stats, SpMV timing, fields and the summed seconds of each domain's own steps."""
    import torch
    dev = torch.device("cuda", 0)
    configure(vip, ctxs, specs, path, tol, inner_tol, helmholtz_tol, learned_precond)
    state = [[t.clone() for t in st] for st in init] if init else [_initial(s, dev) for s in specs]
    # the copies run on torch's current stream and the domains step on streams of their own
    torch.cuda.synchronize()
    for w in range(warmup):
        for ctx, (u, v, p) in zip(ctxs, state):
            ctx.vip_step(u, v, p, dt, re)
        log("%s warmup step %d done" % (path, w + 1))
    torch.cuda.synchronize()
    if time_spmv:
        for w in [0, 1] + list(TIMED):
            ctxs[0].vip_kernel_timing(enable=True, reset=True, which=w)
    stats = []
    dom_s = [0.0] * len(ctxs)

    def one(j):
        u, v, p = state[j]
        t = time.perf_counter()
        st = ctxs[j].vip_step(u, v, p, dt, re)
        dom_s[j] += time.perf_counter() - t
        return st

    t0 = time.perf_counter()
    for k in range(steps):
        if pool is not None:
            row = list(pool.map(one, range(len(ctxs))))
        else:
            row = [one(j) for j in range(len(ctxs))]
        stats.append(row)
        log("%s step %d: poisson iters %s, residual %s, start %s ratio %s" % (
            path, k + 1, [s["poisson_iters"] for s in row],
            ["%.1e" % s["poisson_residual"] for s in row], [s["warm_start"] for s in row],
            ["%.3g" % s["warm_ratio"] for s in row]))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    spmv = conv = None
    kt = {}
    if time_spmv:
        spmv = ctxs[0].vip_kernel_timing(enable=False)
        conv = ctxs[0].vip_kernel_timing(enable=False, which=1)
        kt = {name: ctxs[0].vip_kernel_timing(enable=False, which=w) for w, name in TIMED.items()}
    fields = [[t.cpu().numpy() for t in st] for st in state]
    return (t1 - t0), stats, (spmv, conv, kt), fields, dom_s


def cpu_baseline(h, dt, re, budget_s):
    """FP64 oracle in Krylov mode on a window of the cylinder workload (same h, dt, Re): the
    window [-half, 2 half] x [-half, half] around the body, half = 1 (about 1% of the nodes);
    the impulsive first step is untimed, then whole steps are timed until budget_s is spent
    (at least one)."""
    from oracle import operators, step
    half = 1.0
    spec = ns.cylinder_channel(h, box=(-half, 2.0 * half, -half, half), n_surface=256)
    log("CPU oracle: window with %d nodes, building operators" % spec.n)
    prob = operators.Problem(**spec.as_kwargs())
    ops = operators.Operators(prob)
    st = step.Stepper(ops, dt, re, solver="krylov", tol=1e-8)
    u, v, p = ns.boundary_initial(spec, (1.0, 0.0))
    u, v, p = st.step(u, v, p)
    log("CPU oracle: first step done")
    from threadpoolctl import threadpool_limits
    n_steps = 0
    with threadpool_limits(limits=1):     # one core: BLAS/LAPACK pools held to one thread
        t0 = time.perf_counter()
        while True:
            u, v, p = st.step(u, v, p)
            n_steps += 1
            el = time.perf_counter() - t0
            log("CPU oracle: timed step %d, %.2f s" % (n_steps, el))
            if el > budget_s or n_steps >= 5:
                break
    per = el / n_steps
    return {"value": spec.n / per, "unit": "node-updates/s", "cores": 1, "nproc": os.cpu_count(),
            "kind": "oracle",
            "sample": "FP64 oracle (NumPy/SciPy, BiCGStab to 1e-8, zero start) on the window "
                      "[%g,%g]x[%g,%g] of the cylinder workload at h=1/%d (%d nodes), %d timed steps "
                      "after the impulsive first one; single-threaded SciPy sparse kernels" % (
                          -half, 2 * half, -half, half, round(1.0 / h), spec.n, n_steps),
            "ms_per_step": per * 1e3, "poisson_iters": st.last_iters.get("P")}


# ---- summaries of this script's rocprofv3 output (CSV), as committed under profiles/ ----------------

def _prof_csv(d, suffix):
    import csv
    import glob
    f = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not f:
        sys.exit("no %s under %s" % (suffix, d))
    return list(csv.DictReader(open(f[0])))


def _prof_col(row, *names):
    for want in (lambda k, n: k.lower() == n.lower(), lambda k, n: n.lower() in k.lower()):
        for k in row:
            if any(want(k, n) for n in names):
                return row[k]
    raise KeyError(names)


def _short_kernel(name):
    """Kernel name without 'void', namespaces and the argument list."""
    n = name.replace("(anonymous namespace)::", "").replace("void ", "").strip()
    return (n[:n.index("(")] if "(" in n else n).replace("vip::", "")


def summarize_trace(d, skip):
    """Per-step kernel tables of a --kernel-trace run: every dispatch from the (skip+1)-th
    k_predictor_rhs over at least 1e6 work items on (one per step of the large domain), divided
    by the number of steps after the skipped ones; first over all streams, then for the stream
    of the large domain alone."""
    rows = _prof_csv(d, "kernel_trace.csv")
    recs = sorted((int(_prof_col(r, "Start_Timestamp")), int(_prof_col(r, "End_Timestamp")),
                   _short_kernel(_prof_col(r, "Kernel_Name")), int(_prof_col(r, "Grid_Size", "Grid_Size_X")),
                   r.get("Stream_Id", "")) for r in rows)
    marks = [t0 for (t0, _, name, g, _s) in recs if name.startswith("k_predictor_rhs") and g >= 1000000]
    big = [s for (t0, _, name, g, s) in recs if name.startswith("k_predictor_rhs") and g >= 1000000]
    start = marks[skip] if len(marks) > skip else 0
    nsteps = max(1, len(marks) - skip)
    _trace_table(recs, start, nsteps, None, "all streams")
    if big and big[-1]:
        print("")
        _trace_table(recs, start, nsteps, big[-1], "the large domain's stream (%s) alone" % big[-1])
        _gap_table(recs, start, nsteps, big[-1])


def _gap_table(recs, start, nsteps, stream):
    """Idle time on one stream between the end of a dispatch and the start of the next, per
    step, by the kernel that ends before the gap (host round trips show as long gaps)."""
    prev = None
    gaps = {}
    for (t0, t1, name, g, sid) in recs:
        if t0 < start or sid != stream:
            continue
        if prev is not None and t0 > prev[0]:
            a = gaps.setdefault(prev[1], [0, 0.0, 0, 0.0])
            d = (t0 - prev[0]) / 1e3
            a[0] += 1
            a[1] += d
            if d >= 20.0:
                a[2] += 1
                a[3] += d
        prev = (t1, name) if prev is None or t1 > prev[0] else prev
    tot = sum(a[1] for a in gaps.values())
    out = ["", "idle time on that stream: %.3f ms per step; gaps of 20 us or more: %.1f per step, %.3f ms" % (
        tot / 1e3 / nsteps, sum(a[2] for a in gaps.values()) / nsteps, sum(a[3] for a in gaps.values()) / 1e3 / nsteps),
        "", "| kernel before the gap | gaps/step | idle ms/step | gaps >= 20 us per step, their ms/step |",
        "|---|---:|---:|---:|"]
    for k, (n, us, nb, usb) in sorted(gaps.items(), key=lambda kv: -kv[1][1])[:15]:
        out.append("| `%s` | %.1f | %.3f | %.1f, %.3f |" % (k, n / nsteps, us / 1e3 / nsteps, nb / nsteps, usb / 1e3 / nsteps))
    print("\n".join(out))


def _trace_table(recs, start, nsteps, stream, title):
    agg = {}
    short = 0
    t_first = t_last = None
    for (t0, t1, name, g, sid) in recs:
        if t0 < start or (stream is not None and sid != stream):
            continue
        a = agg.setdefault(name, [0, 0.0, 0, 0.0])
        a[0] += 1
        a[1] += (t1 - t0) / 1e3
        if g >= 1000000:
            a[2] += 1
            a[3] += (t1 - t0) / 1e3
        short += (t1 - t0) < 10000
        t_first = t0 if t_first is None else min(t_first, t0)
        t_last = t1 if t_last is None else max(t_last, t1)
    tot = sum(a[1] for a in agg.values())
    out = ["%s: steps summarized: %d; kernel time %.3f ms per step; first-to-last dispatch span %.3f ms "
           "per step; launches per step %.0f (%.0f under 10 us)" % (
               title, nsteps, tot / 1e3 / nsteps, (t_last - t_first) / 1e6 / nsteps,
               sum(a[0] for a in agg.values()) / nsteps, short / nsteps), "",
           "| kernel | calls/step | mean us | ms/step | share | grid >= 1e6: calls/step, mean us |",
           "|---|---:|---:|---:|---:|---:|"]
    for k, (n, us, nb, usb) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:40]:
        out.append("| `%s` | %.1f | %.1f | %.3f | %.1f%% | %s |" % (
            k, n / nsteps, us / n, us / 1e3 / nsteps, 100 * us / tot,
            "%.1f, %.1f" % (nb / nsteps, usb / nb) if nb else "-"))
    print("\n".join(out))


def summarize_counter(d, counter):
    """Mean of one PMC counter per kernel and grid size, over dispatches of >= 1e5 work items: over
    all of them, and over the working ones (at least a quarter of the largest value), since the
    Krylov launches issued after a solve stopped on the device return at once; and the largest
    (a two-system launch with both systems still iterating)."""
    agg = {}
    for r in _prof_csv(d, "counter_collection.csv"):
        g = int(_prof_col(r, "Grid_Size", "Grid_Size_X"))
        if _prof_col(r, "Counter_Name") != counter or g < 100000:
            continue
        agg.setdefault((_short_kernel(_prof_col(r, "Kernel_Name")), g), []).append(
            float(_prof_col(r, "Counter_Value")))
    unit = " (KiB)" if counter.endswith("_SIZE") else ""
    out = ["| kernel | grid | dispatches | mean %s%s | working dispatches | their mean%s | max%s |" % (
        counter, unit, unit, unit), "|---|---:|---:|---:|---:|---:|---:|"]
    for (k, g), v in sorted(agg.items()):
        w = [x for x in v if x >= 0.25 * max(v)]
        out.append("| `%s` | %d | %d | %.0f | %d | %.0f | %.0f |" % (k, g, len(v), sum(v) / len(v), len(w),
                                                                 sum(w) / len(w), max(v)))
    print("\n".join(out))


def network_bench(args):
    """The fused 4-layer network launch alone, on a synthetic input image of the cylinder
    lattice at the given h (2561 x 3841 pixels at h = D/128): scaled residual and right-hand
    side N(0, 1) on the lattice, 0 inside the body, plus the lattice mask."""
    import torch
    from paper_1401_6513_amd import vip
    torch.zeros(1, device="cuda")
    h = args.h
    W, H = int(round(30.0 / h)) + 1, int(round(20.0 / h)) + 1
    xs = -10.0 + h * np.arange(W)
    ys = -10.0 + h * np.arange(H)
    mask = (xs[None, :] ** 2 + ys[:, None] ** 2 >= 0.25).astype(np.float64)
    rng = np.random.default_rng(5)
    x = np.empty((1, H, W, 3))
    x[0, :, :, 0] = rng.standard_normal((H, W)) * mask
    x[0, :, :, 1] = rng.standard_normal((H, W)) * mask
    x[0, :, :, 2] = mask
    ctx = vip.Context(0)
    try:
        ctx.vip_learn_init(11)
        ctx.vip_kernel_timing(True, True, 1)
        for _ in range(args.warmup):
            ctx.vip_learn_infer(x)
        ctx.vip_kernel_timing(True, True, 1)
        for _ in range(args.steps):
            ctx.vip_learn_infer(x)
        avg_ms, count = ctx.vip_kernel_timing(True, False, 1)
    finally:
        ctx.close()
    per_px = 2 * 9 * (3 * 32 + 32 * 32 + 32 * 32 + 32 * 1)
    flops = float(per_px) * W * H
    tf = flops / (avg_ms * 1e-3) / 1e12
    print(json.dumps({"metric": "network inference pixels/s", "value": W * H / (avg_ms * 1e-3),
                      "unit": "pixels/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                      "ms_per_step": avg_ms, "higher_is_better": True, "dtype": "bf16+f32",
                      "data": "synthetic", "config": {"workload": "fused network inference",
                                                      "image": [H, W]},
                      "roofline": {"bound": "mfma", "achieved": tf, "peak": 2500.0, "unit": "TFLOP/s",
                                   "frac": tf / 2500.0, "traffic": None, "kernel": "k_cnn_fused",
                                   "flops_per_launch": flops, "launches": count}}))


def main():
    if len(sys.argv) > 1 and sys.argv[1] in ("--summarize-trace", "--summarize-counter"):
        # python bench.py --summarize-trace DIR [SKIP] | --summarize-counter DIR COUNTER
        if sys.argv[1] == "--summarize-trace":
            summarize_trace(sys.argv[2], int(sys.argv[3]) if len(sys.argv) > 3 else 3)
        else:
            summarize_counter(sys.argv[2], sys.argv[3])
        return
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=3,
                    help="untimed steps per path (the start-vector corrections need two)")
    ap.add_argument("--spinup", type=int, default=500,
                    help="untimed fractional steps from the impulsive start whose flow is the initial "
                         "state of every timed path (0: the timed paths start impulsively)")
    ap.add_argument("--transient-steps", type=int, default=10,
                    help="also time this many steps of the first path (and of fp64) from the "
                         "impulsive start, reported under 'transient' (0: skip)")
    ap.add_argument("--h", type=float, default=1.0 / 128)
    ap.add_argument("--re", type=float, default=200.0)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--helmholtz-tol", type=float, default=None,
                    help="tolerance of the predictor solves (default: the library's)")
    ap.add_argument("--inner-tol", type=float, default=1e-5,
                    help="relative tolerance of the FP32 inner solves (mixed paths; the library's "
                         "default)")
    ap.add_argument("--paths", default="learned,mixed,extrap,fp64,fp64x")
    ap.add_argument("--workload", default="lattice", choices=["lattice", "refined"],
                    help="lattice: cylinder + triangle on uniform lattices (the headline workload); "
                         "refined: the cylinder on a stepwise refined node set (general rows only; "
                         "the learned path needs a lattice and is skipped)")
    ap.add_argument("--no-delta", action="store_true",
                    help="general rows read int32 columns instead of int16 row-relative ones")
    ap.add_argument("--plain-steps", type=int, default=2,
                    help="timed steps of the plain path (slow: hundreds of Krylov iterations a step)")
    ap.add_argument("--train-iters", type=int, default=1000)
    ap.add_argument("--train-set", default="small", choices=["small", "config4"],
                    help="small: 4 short runs on a 129^2 cavity and an h=1/16 cylinder box (40 "
                         "snapshots each); config4: the bumpy-cylinder case's specification, 10 runs "
                         "of the 257^2 cavity and the h=D/40 cylinder, Re ~ U[60,200], 200 snapshots "
                         "each, one every 5 steps after 200 steps")
    ap.add_argument("--learned-precond", action="store_true",
                    help="the learned path also preconditions every refinement pass with the network")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--serial", action="store_true",
                    help="step the domains one after the other on one stream (default: each domain "
                         "on its own HIP stream, stepped from its own host thread)")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="before the timed region, copy a 1 GiB buffer once (reference dispatch "
                         "for the HBM byte counters of a profiler run)")
    ap.add_argument("--network-only", action="store_true",
                    help="time the fused network inference launch alone (synthetic image)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU only: the VIP hot path is built and measured on a single "
              "MI355X (multi-GPU sharding is a design note, not built); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    if args.network_only:
        network_bench(args)
        return
    import torch
    from paper_1401_6513_amd import vip
    h = args.h
    dt = h / 10.0
    re = args.re
    log("generating node sets (h = %g, %s)" % (h, args.workload))
    specs = workload(h, args.workload)
    if args.no_delta:
        os.environ["VIP_NO_DELTA"] = "1"      # read once by each context at creation
    n_total = sum(s.n for s in specs)
    log("nodes: %s (total %d)" % ([s.n for s in specs], n_total))
    ctxs = []
    streams = []
    t0 = time.perf_counter()
    for s in specs:
        if args.serial:
            c = vip.Context(0)
        else:
            streams.append(torch.cuda.Stream(device=0))
            c = vip.Context(0, stream=streams[-1].cuda_stream)
        c.build_from_spec(s)
        ctxs.append(c)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    log("stencils built in %.2f s" % build_s)

    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: %d bytes read, %d bytes written" % (src.numel() * 4, dst.numel() * 4))
        del src, dst

    paths = [p for p in args.paths.split(",") if p]
    if args.workload == "refined":
        paths = [p for p in paths if p != "learned"]
    for p in paths:
        if p not in PATHS:
            sys.exit("unknown path %r (known: %s)" % (p, ", ".join(PATHS)))
    train_info = None
    if "learned" in paths:
        from paper_1401_6513_amd import training
        t0 = time.perf_counter()
        if args.train_set == "config4":
            theta, nsnap, loss = training.trained_parameters(runs=training.config4_runs(),
                                                             iters=args.train_iters, transient=200,
                                                             per_run=200, every=5)
            data = ("10 runs alternating cavity 257x257 and cylinder h=1/40 in [-10,20]x[-10,10], "
                    "Re~U[60,200] (seeds 0-9), dt=h/10, 200 snapshots per run, one every 5 steps "
                    "after 200 steps")
        else:
            theta, nsnap, loss = training.trained_parameters(iters=args.train_iters)
            data = ("cavity 129x129 Re~U[100,1000] and cylinder h=1/16 in [-4,8]x[-4,4] "
                    "Re~U[60,200], dt=h/10, 40 snapshots per run after 40 steps, 4 runs")
        torch.cuda.synchronize()
        train_info = {"snapshots": nsnap, "iters": args.train_iters, "last_loss": loss,
                      "seconds": time.perf_counter() - t0, "data": data}
        log("network trained: %d snapshots, loss %.3e, %.1f s" % (nsnap, loss, train_info["seconds"]))
        for c in ctxs:
            c.vip_learn_set_params(theta)
    results = {}
    pool = None
    if not args.serial:
        from concurrent.futures import ThreadPoolExecutor
        pool = ThreadPoolExecutor(max_workers=len(ctxs))
    transient = {}
    if args.transient_steps > 0:
        # the first path (and fp64) timed from the impulsive start, for comparison
        for path in [paths[0]] + (["fp64"] if "fp64" in paths and paths[0] != "fp64" else []):
            el, stats, _, _, _ = run_path(vip, ctxs, specs, path, dt, re, args.warmup, args.transient_steps,
                                          args.tol, False, args.inner_tol, pool, args.helmholtz_tol,
                                          args.learned_precond)
            transient[path] = {"ms_per_step": el / args.transient_steps * 1e3,
                               "value": n_total * args.transient_steps / el,
                               "poisson_iters": [[s["poisson_iters"] for s in row] for row in stats],
                               "helmholtz_iters": [[s["helmholtz_iters"] for s in row] for row in stats]}
            log("%s from the impulsive start: %.2f ms per step" % (path, transient[path]["ms_per_step"]))
    init = None
    if args.spinup > 0:
        t0 = time.perf_counter()
        init = spin_up(vip, ctxs, specs, dt, re, args.spinup, args.tol, args.inner_tol, pool)
        log("spin-up: %d steps in %.1f s" % (args.spinup, time.perf_counter() - t0))
    for path in paths:
        nsteps = args.plain_steps if path == "plain" else args.steps
        el, stats, (spmv, conv, kt), fields, dom_s = run_path(vip, ctxs, specs, path, dt, re, args.warmup,
                                                  nsteps, args.tol, path == paths[0],
                                                  args.inner_tol, pool, args.helmholtz_tol,
                                                  args.learned_precond, init)
        results[path] = dict(seconds=el, stats=stats, spmv=spmv, conv=conv, kt=kt, fields=fields, dom_s=dom_s,
                             steps=nsteps)
        log("%s: %.3f s for %d steps" % (path, el, nsteps))

    main_path = paths[0]
    r = results[main_path]
    ms = r["seconds"] / args.steps * 1e3
    value = n_total * args.steps / r["seconds"]

    roof = None
    if r["spmv"] is not None and r["spmv"][1] > 0:
        n0, _, nnz0 = ctxs[0].vip_operator_shape("poisson")
        fp32 = PATHS[main_path]["precision"] != "P_FP64"
        counts, taps = ctxs[0].vip_canonical_rows()
        ne, ne16 = ctxs[0].vip_column_bytes()[:2]
        # mean bytes per stored column: int16 row-relative slices and int32 slices
        cb = (2.0 * ne16 + 4.0 * (ne - ne16)) / max(ne, 1)
        vs = 4 if fp32 else 0
        nc = int(counts[vs])
        vb = 4 if fp32 else 8            # bytes of one vector entry / value
        sp = specs[0]
        if nc > 0:
            W = int(np.floor((sp.xy[:, 0].max() - sp.xy[:, 0].min()) / sp.h + 0.5)) + 1
            H = int(np.floor((sp.xy[:, 1].max() - sp.xy[:, 1].min()) / sp.h + 0.5)) + 1
            ntiles = -(-W // 64) * -(-H // 16)
        else:
            ntiles = 0
        # algorithmic bytes of one launch: x read once, r-hat read, v written (3 vectors); stored
        # values + columns (int16 row-relative or int32) of the irregular rows (and, in FP32, their
        # row sums); with tiles, the irregular-row list and per 64 x 16 tile its 256-byte record
        # (position, 20 row starts, 16 row masks), counted for every lattice tile.  Canonical
        # (tile) rows read no column or value stream.
        bytes_per_launch = int(3 * vb * n0 + (vb + cb) * (nnz0 - taps * nc) + (4 if fp32 else 0) * (n0 - nc)
                               + (4 * (n0 - nc) + 256 * ntiles if ntiles else 0))
        avg_ms, count = r["spmv"]
        achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
        tiled = ntiles > 0
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS,
                "traffic": measured_traffic() if (abs(h - 1.0 / 128) < 1e-12 and tiled) else None,
                "kernel": "k_bicg_v<%s,%s,1> (pressure SpMV, %s)" % (
                    ("float", "float", "LDS-tiled canonical rows" if tiled else "general sliced-ELL rows")
                    if fp32 else
                    ("double", "double", "LDS-tiled canonical rows" if tiled else "general sliced-ELL rows")),
                "bytes_per_launch": bytes_per_launch, "avg_ms": avg_ms, "launches": count,
                "rows": n0, "nnz": nnz0, "canonical_rows": nc, "tiles": ntiles, "taps": taps,
                "column_bytes": cb,
                "ell_bytes_per_launch": (vb + 4) * nnz0 + 3 * vb * n0}

    # every timed kernel against the HBM roofline, and the one that takes the most time per step
    rooflines = {}
    if roof is not None:
        kb = kernel_bytes(ctxs[0], specs[0], PATHS[main_path]["precision"] != "P_FP64")
        timed = dict(r["kt"])
        timed["pres_spmv"] = r["spmv"]
        if os.environ.get("VIP_NO_FUSE") != "1" and args.workload == "lattice" and fp32:
            # the predictor's iteration on lattice tiles: one update pass (x, r and p) and the
            # t kernel with five sums instead of the separate p, s and x passes
            timed["pred_e"] = timed.pop("pred_x")
            timed["pred_ts"] = timed.pop("pred_t")
            if "pred_spmv" in timed:
                timed["pred_spmv1"] = timed.pop("pred_spmv")
        for name, (avg_ms, count) in timed.items():
            if count <= 0 or avg_ms <= 0:
                continue
            gbs = kb[name] / (avg_ms * 1e-3) / 1e9
            label = KERNEL_NAMES[name] % (("float", "float") if fp32 else ("double", "double")) \
                if name == "pres_spmv" else KERNEL_NAMES[name]
            rooflines[name] = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": gbs / HBM_PEAK_GBS, "kernel": label,
                               "bytes_per_launch": int(kb[name]), "avg_ms": avg_ms, "launches": count,
                               "ms_per_step": avg_ms * count / args.steps,
                               "traffic": measured_traffic(name) if abs(h - 1.0 / 128) < 1e-12 else None}
    if rooflines:
        dom = max(rooflines, key=lambda k: rooflines[k]["ms_per_step"])
        dominant = dict(rooflines[dom])
        dominant["name"] = dom
    else:
        dominant = roof

    roof_mfma = None
    if r.get("conv") is not None and r["conv"][1] > 0:
        sp = specs[0]
        W = int(np.floor((sp.xy[:, 0].max() - sp.xy[:, 0].min()) / sp.h + 0.5)) + 1
        H = int(np.floor((sp.xy[:, 1].max() - sp.xy[:, 1].min()) / sp.h + 0.5)) + 1
        # useful FLOPs of the four 3x3 layers per pixel: 3->32, 32->32 twice, 32->1
        per_px = 2 * 9 * (3 * 32 + 32 * 32 + 32 * 32 + 32 * 1)
        flops = float(per_px) * W * H
        avg_ms, count = r["conv"]
        tf = flops / (avg_ms * 1e-3) / 1e12
        roof_mfma = {"bound": "mfma", "achieved": tf, "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": tf / 2500.0, "traffic": None,
                     "kernel": "k_cnn_fused (the learned start vector's 4-layer BF16 network in one launch, "
                               "58-column strips walked row by row, v_mfma_f32_16x16x32_bf16)",
                     "flops_per_launch": flops, "flops_per_pixel": per_px, "avg_ms": avg_ms,
                     "launches": count, "image": [H, W]}

    if args.workload == "refined":
        wl = ("cylinder D=1 in [-10,20]x[-10,10] on a stepwise refined node set (spacing h=D/%d "
              "near the body, doubling in 3 steps), Re=%g, dt=%g, Poisson rel. residual %g" % (
                  round(1 / h), re, dt, args.tol))
    else:
        wl = ("cylinder D=1 in [-10,20]x[-10,10] + equilateral lid cavity, h=D/%d, Re=%g, dt=%g, "
              "Poisson rel. residual %g" % (round(1 / h), re, dt, args.tol))
    out = {"metric": METRIC, "value": value, "unit": "node-updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if PATHS[main_path]["precision"] == "P_FP64" else "f32+f64+bf16"
           if main_path == "learned" else "f32+f64", "data": "synthetic",
           "config": {"workload": wl,
                      "nodes": n_total, "nodes_per_domain": [s.n for s in specs],
                      "path": main_path, "build_s": build_s,
                      "domains_concurrent": not args.serial,
                      "initial_state": ("the flow after %d untimed fractional steps from the impulsive "
                                        "start (FP32 inner solves, extrapolated start vectors); then "
                                        "%d warm-up and %d timed steps per path" % (
                                            args.spinup, args.warmup, args.steps)) if args.spinup > 0
                      else "impulsive start; %d warm-up and %d timed steps per path" % (
                          args.warmup, args.steps)}}
    for path, rr in results.items():
        it = [[s["poisson_iters"] for s in row] for row in rr["stats"]]
        out["path_" + path] = {"value": n_total * rr["steps"] / rr["seconds"],
                               "ms_per_step": rr["seconds"] / rr["steps"] * 1e3,
                               "steps": rr["steps"],
                               "ms_per_step_by_domain": [d / rr["steps"] * 1e3 for d in rr["dom_s"]],
                               "poisson_iters": it,
                               "helmholtz_iters": [[s["helmholtz_iters"] for s in row] for row in rr["stats"]],
                               "poisson_residual": max(s["poisson_residual"] for row in rr["stats"]
                                                       for s in row)}
    per_step = {p: rr["seconds"] / rr["steps"] for p, rr in results.items()}
    if "plain" in results and main_path != "plain":
        # the plain FP64 GPU path: FP64 Krylov with the Jacobi preconditioner, no learned part
        out["speedup_vs_plain_fp64"] = per_step["plain"] / per_step[main_path]
    ref_path = "fp64" if "fp64" in results else None
    if ref_path and main_path != ref_path:
        # FP64 Krylov with the same multigrid preconditioner and start vector as the mixed path
        out["speedup_vs_fp64"] = per_step[ref_path] / per_step[main_path]
        out["fp64_comparator"] = ("fp64 path: FP64 BiCGStab (predictor and pressure) with the same "
                                  "aggregation-multigrid preconditioner and previous-increment start "
                                  "vector; plain Jacobi FP64 (path 'plain') does not converge on the "
                                  "cylinder at h=D/128; fp64x: the same with the extrapolated start "
                                  "vectors of the learned path (speedup_vs_fp64x isolates precision)")
        if "fp64x" in results:
            out["speedup_vs_fp64x"] = per_step["fp64x"] / per_step[main_path]
        # difference of the paths' fields after the same steps (all solve to 1e-8)
        out["rel_l2_vs_fp64"] = {}
        for path in results:
            if path == ref_path or results[path]["steps"] != results[ref_path]["steps"]:
                continue   # fields are compared after the same number of steps only
            diffs = []
            for a, b in zip(results[path]["fields"], results[ref_path]["fields"]):
                for k, (x, y) in enumerate(zip(a, b)):
                    if k == 2:
                        x, y = x - x.mean(), y - y.mean()
                    diffs.append(float(np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-300)))
            out["rel_l2_vs_fp64"][path] = {"u": max(diffs[0::3]), "v": max(diffs[1::3]),
                                           "p": max(diffs[2::3])}
    if "learned" in results and "mixed" in results:
        a = sum(sum(s["poisson_iters"] for s in row) for row in results["learned"]["stats"])
        b = sum(sum(s["poisson_iters"] for s in row) for row in results["mixed"]["stats"])
        out["learned_poisson_iters_vs_mixed"] = [a, b]
    if train_info:
        out["training"] = train_info
    if transient:
        tr = dict(transient)
        tr["window"] = "steps %d..%d from the impulsive start" % (args.warmup + 1,
                                                                 args.warmup + args.transient_steps)
        if main_path in transient and "fp64" in transient:
            tr["speedup_vs_fp64"] = transient["fp64"]["ms_per_step"] / transient[main_path]["ms_per_step"]
        out["transient"] = tr
    out["roofline"] = dominant
    out["roofline_pressure_spmv"] = roof
    out["rooflines"] = rooflines
    if rooflines:
        timed_ms = sum(v["ms_per_step"] for v in rooflines.values())
        timed_bytes = sum(v["bytes_per_launch"] * v["launches"] for v in rooflines.values()) / args.steps
        # the timed kernels' share of the step, and their combined bytes over their combined time
        out["timed_kernels_per_step"] = {"ms": timed_ms, "share_of_step": timed_ms / ms,
                                         "GB_per_step": timed_bytes / 1e9,
                                         "GBs_over_their_time": timed_bytes / (timed_ms * 1e-3) / 1e9}
    out["roofline_mfma"] = roof_mfma
    if not args.no_cpu:
        log("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(h, dt, re, args.cpu_budget)
    else:
        out["cpu_baseline"] = None
    if pool is not None:
        pool.shutdown()
    for c in ctxs:
        c.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
