"""The FP32 predictor BiCGStab with its x, r and p updates in one pass (the update of the last
iteration and the new p, possible because the t kernel's five sums give omega, |r|^2 and
rhat . r before r is formed) against the same solve with separate p, s and x passes
(VIP_NO_FUSE=1 at context creation).  The two take the same iterations
in exact arithmetic; in FP32 they differ by rounding, so after the same steps the fields must
agree to the solve tolerances, and both must match the FP64 oracle (eqs. 12-15).
"""
import os

import numpy as np
import pytest

from oracle import operators, step
from paper_1401_6513_amd import nodesets as ns

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _ctx(no_fuse):
    from paper_1401_6513_amd import vip
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if no_fuse:
        os.environ["VIP_NO_FUSE"] = "1"
    try:
        return vip.Context(0)
    finally:
        os.environ.pop("VIP_NO_FUSE", None)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


CASES = {
    "cylinder": (lambda: ns.cylinder_channel(1.0 / 16, box=(-3.0, 6.0, -3.0, 3.0), n_surface=64),
                 (1.0, 0.0), 1.0 / 160, 100.0, 8, False),
    "bumpy": (lambda: ns.cylinder_channel(1.0 / 32, box=(-2.0, 4.0, -2.0, 2.0), shape=(0.05, 12),
                                          n_surface=128), (1.0, 0.0), 1.0 / 320, 100.0, 6, False),
    "cavity": (lambda: ns.lid_cavity(65), (0.0, 0.0), 2e-3, 400.0, 8, True),
}


@pytest.mark.parametrize("name", list(CASES))
def test_fused_predictor_matches_separate_passes_and_oracle(name):
    from paper_1401_6513_amd import vip
    make, inflow, dt, re, steps, singular = CASES[name]
    spec = make()
    fields, iters = {}, {}
    for no_fuse in (False, True):
        ctx = _ctx(no_fuse)
        try:
            ctx.build_from_spec(spec, precision=vip.P_MIXED, warmstart=vip.WS_EXTRAP, poisson_tol=1e-10,
                                helmholtz_tol=1e-12)
            st = [torch.tensor(a, device="cuda") for a in ns.boundary_initial(spec, inflow)]
            its = []
            for _ in range(steps):
                s = ctx.vip_step(*st, dt, re)
                assert s["helmholtz_residual"] <= 1e-12
                its.append(s["helmholtz_iters"])
            fields[no_fuse] = [t.cpu().numpy() for t in st]
            iters[no_fuse] = its
        finally:
            ctx.close()
    ops = operators.Operators(operators.Problem(**spec.as_kwargs()))
    stp = step.Stepper(ops, dt, re)
    uo, vo, po = ns.boundary_initial(spec, inflow)
    for _ in range(steps):
        uo, vo, po = stp.step(uo, vo, po)
    ref = [uo, vo, po]
    report = {}
    for key, label in ((False, "fused"), (True, "separate")):
        got = list(fields[key])
        want = list(ref)
        if singular:
            got[2], want[2] = got[2] - got[2].mean(), want[2] - want[2].mean()
        report[label] = [_rel(g, w) for g, w in zip(got, want)]
    between = [_rel(a, b) for a, b in zip(fields[False][:2], fields[True][:2])]
    print("%s predictor iterations fused %s separate %s; u, v between the two %.2e %.2e; vs oracle "
          "fused %s separate %s" % (name, iters[False], iters[True], between[0], between[1],
                                    ["%.1e" % e for e in report["fused"]],
                                    ["%.1e" % e for e in report["separate"]]))
    assert max(between) <= 1e-9, between
    for label, errs in report.items():
        assert max(errs) <= 1e-7, (label, errs)
    # the same method: iteration counts within one or two a step
    assert all(abs(a - b) <= 2 for a, b in zip(iters[False], iters[True])), iters
