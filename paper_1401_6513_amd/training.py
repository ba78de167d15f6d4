"""Training data and training of the learned Poisson start vector (library calls only).

Snapshots come from the solver itself: short runs of the lid-driven square
cavity and of the flow past a cylinder (a small box around the body) at seeded
Reynolds numbers, captured by vip_step once the run has passed its impulsive
start; the network is then trained by the library's own forward, backward and
Adam kernels (vip_learn_train).  Every step runs on the GPU; this module only
sequences the calls.
"""
import numpy as np

from . import nodesets, vip


def _state(spec, inflow):
    import torch
    u, v, p = nodesets.boundary_initial(spec, inflow)
    return [torch.tensor(a, device="cuda") for a in (u, v, p)]


def training_runs(h_cyl=1.0 / 16, n_cavity=129, runs=4, seed=0):
    """(spec, inflow, dt, Re) of the data-generation runs: cavities at Re ~ U[100, 1000] and
    cylinders at Re ~ U[60, 200], alternating, dt = h/10."""
    rng = np.random.default_rng(seed)
    cav = nodesets.lid_cavity(n_cavity)
    cyl = nodesets.cylinder_channel(h_cyl, box=(-4.0, 8.0, -4.0, 4.0))
    out = []
    for k in range(runs):
        if k % 2 == 0:
            out.append((cav, (0.0, 0.0), cav.h / 10.0, float(rng.uniform(100.0, 1000.0))))
        else:
            out.append((cyl, (1.0, 0.0), cyl.h / 10.0, float(rng.uniform(60.0, 200.0))))
    return out


def config4_runs(seed=0, n_cavity=257, h_cyl=1.0 / 40):
    """The training specification of the bumpy-cylinder case: 10 runs of the lid-driven cavity
    (257 x 257) and cylinder (h = D/40 in [-10, 20] x [-10, 10]) geometries, alternating, with
    Re ~ U[60, 200] drawn from seeds seed .. seed + 9 (one per run), dt = h/10."""
    cav = nodesets.lid_cavity(n_cavity)
    cyl = nodesets.cylinder_channel(h_cyl)
    out = []
    for k in range(10):
        re = float(np.random.default_rng(seed + k).uniform(60.0, 200.0))
        if k % 2 == 0:
            out.append((cav, (0.0, 0.0), cav.h / 10.0, re))
        else:
            out.append((cyl, (1.0, 0.0), cyl.h / 10.0, re))
    return out


def capture(ctx, runs, transient=40, per_run=40, precision=vip.P_MIXED, every=1):
    """Run each case, skip `transient` steps, then capture `per_run` snapshots, one every
    `every` steps."""
    for spec, inflow, dt, re in runs:
        ctx.build_from_spec(spec, precision=precision, warmstart=vip.WS_PREV)
        u, v, p = _state(spec, inflow)
        ctx.vip_learn_capture(0)
        for _ in range(transient):
            ctx.vip_step(u, v, p, dt, re)
        target = ctx.vip_learn_snapshot_count() + per_run
        k = 0
        while ctx.vip_learn_snapshot_count() < target:
            # capture is armed for the step that completes a block of `every`; a step stores a
            # snapshot only once the previous change of the increment is known
            on = (k + 1) % every == 0
            ctx.vip_learn_capture(ctx.vip_learn_snapshot_count() + 1 if on else 0)
            ctx.vip_step(u, v, p, dt, re)
            k += 1
            if k > 4 * every * per_run + 8:
                break
    ctx.vip_learn_capture(0)
    return ctx.vip_learn_snapshot_count()


def train(ctx, iters=1000, batch=16, crop=64, lr=1e-3, seed=0, init_seed=0):
    """Fresh He-uniform weights, then Adam; returns the last batch loss."""
    ctx.vip_learn_init(init_seed)
    loss = None
    done = 0
    while done < iters:
        k = min(250, iters - done)
        rate = lr if done < 0.75 * iters else 0.3 * lr
        loss = ctx.vip_learn_train(k, batch, crop, rate, seed + done)
        done += k
    return loss


def trained_parameters(runs=None, iters=1000, seed=0, device=0, transient=40, per_run=40, every=1,
                       batch=16, crop=64):
    """Generate snapshots, train, and return (parameters, snapshot count, last loss)."""
    ctx = vip.Context(device)
    try:
        n = capture(ctx, runs if runs is not None else training_runs(seed=seed), transient=transient,
                    per_run=per_run, every=every)
        loss = train(ctx, iters=iters, seed=seed, batch=batch, crop=crop)
        theta = ctx.vip_learn_get_params()
    finally:
        ctx.close()
    return theta, n, loss
