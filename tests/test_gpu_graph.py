"""The multigrid V-cycle below the finest level replayed as a captured graph against the same
launches issued one by one (VIP_NO_GRAPH=1 at context creation).  The graph holds the same
kernels in the same order on the same buffers, so the two runs give the same bits; both are
held to the FP64 oracle (eqs. 12-15) as well.  Covered: FP32 and FP64 cycles, a singular
(bordered) pressure system, a hierarchy of two levels (the graph is the coarsest solve alone),
one level (no graph), and a context rebuilt on another node set (the graph is captured again
for the new hierarchy).
"""
import os

import numpy as np
import pytest

from oracle import operators, step
from paper_1401_6513_amd import nodesets as ns

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _ctx(no_graph):
    from paper_1401_6513_amd import vip
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if no_graph:
        os.environ["VIP_NO_GRAPH"] = "1"
    try:
        return vip.Context(0)
    finally:
        os.environ.pop("VIP_NO_GRAPH", None)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


CASES = {
    # name: node set, inflow, dt, Re, steps, singular pressure system
    "cylinder": (lambda: ns.cylinder_channel(1.0 / 16, box=(-3.0, 6.0, -3.0, 3.0), n_surface=64),
                 (1.0, 0.0), 1.0 / 160, 100.0, 6, False),
    "cavity65": (lambda: ns.lid_cavity(65), (0.0, 0.0), 2e-3, 400.0, 6, True),
    "cavity33": (lambda: ns.lid_cavity(33), (0.0, 0.0), 2e-3, 100.0, 6, True),
    "cavity17": (lambda: ns.lid_cavity(17), (0.0, 0.0), 2e-3, 100.0, 4, True),
}


def _run(ctx, spec, inflow, dt, re, steps, precision):
    from paper_1401_6513_amd import vip
    ctx.build_from_spec(spec, precision=precision, warmstart=vip.WS_PREV, poisson_tol=1e-10)
    st = [torch.tensor(a, device="cuda") for a in ns.boundary_initial(spec, inflow)]
    its = []
    for _ in range(steps):
        s = ctx.vip_step(*st, dt, re)
        assert s["poisson_residual"] <= 1e-10
        its.append(s["poisson_iters"])
    return [t.cpu().numpy() for t in st], its


def _oracle(spec, inflow, dt, re, steps):
    stp = step.Stepper(operators.Operators(operators.Problem(**spec.as_kwargs())), dt, re)
    u, v, p = ns.boundary_initial(spec, inflow)
    for _ in range(steps):
        u, v, p = stp.step(u, v, p)
    return [u, v, p]


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("name", list(CASES))
def test_graph_cycle_same_bits_as_launches(name, precision):
    from paper_1401_6513_amd import vip
    make, inflow, dt, re, steps, singular = CASES[name]
    spec = make()
    prec = vip.P_MIXED if precision == "mixed" else vip.P_FP64
    out = {}
    for no_graph in (False, True):
        ctx = _ctx(no_graph)
        try:
            out[no_graph] = _run(ctx, spec, inflow, dt, re, steps, prec)
        finally:
            ctx.close()
    (fg, ig), (fl, il) = out[False], out[True]
    ref = _oracle(spec, inflow, dt, re, steps)
    errs = []
    for k in range(3):
        got, want = fg[k], ref[k]
        if singular and k == 2:
            got, want = got - got.mean(), want - want.mean()
        errs.append(_rel(got, want))
    print("%s %s: Poisson iterations graph %s launches %s; vs oracle u %.1e v %.1e p %.1e"
          % (name, precision, ig, il, *errs))
    assert ig == il
    for a, b in zip(fg, fl):
        assert np.array_equal(a, b)
    assert max(errs) <= 1e-7, errs


def test_graph_recaptured_after_rebuild():
    """One context built on a cavity, stepped, then rebuilt on a cylinder channel: the second
    hierarchy's graph must be captured anew (the first one's buffers are freed)."""
    from paper_1401_6513_amd import vip
    cav = CASES["cavity65"]
    cyl = CASES["cylinder"]
    ctx = _ctx(False)
    try:
        _run(ctx, cav[0](), *cav[1:5], vip.P_MIXED)
        got, its = _run(ctx, cyl[0](), *cyl[1:5], vip.P_MIXED)
    finally:
        ctx.close()
    ctx = _ctx(True)
    try:
        want, its_l = _run(ctx, cyl[0](), *cyl[1:5], vip.P_MIXED)
    finally:
        ctx.close()
    assert its == its_l
    for a, b in zip(got, want):
        assert np.array_equal(a, b)
