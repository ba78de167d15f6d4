"""Pins of the oracle's fractional step (eqs. 12-15 of the paper) against closed
forms and properties that hold whatever the implementation: Taylor decaying
vortices (Section 5.1), convergence orders in space and time, a steady exact
Navier-Stokes solution with Dirichlet walls, linear stability of the step, and
agreement of the Krylov timing mode with the direct solve."""
import numpy as np
import pytest

from oracle import exact, operators, step
from paper_1401_6513_amd import nodesets as ns


def _tg_run(n, steps, dt, Re=10.0, solver="direct"):
    spec = ns.periodic_lattice(n)
    ops = operators.Operators(operators.Problem(**spec.as_kwargs()))
    st = step.Stepper(ops, dt, Re, solver=solver, tol=1e-12)
    u, v, p = ns.taylor_green_initial(spec.xy)
    for _ in range(steps):
        u, v, p = st.step(u, v, p)
    return spec, ops, st, u, v, p


def _tg_err(spec, u, v, p, t, Re=10.0):
    ue, ve, pe = exact.taylor_green(spec.xy, t, Re)
    return (np.abs(u - ue).max(), np.abs(v - ve).max(),
            np.abs((p - p.mean()) - (pe - pe.mean())).max())


def test_taylor_green_32_against_closed_form():
    spec, ops, st, u, v, p = _tg_run(32, 100, 1e-3)
    eu, ev, ep = _tg_err(spec, u, v, p, 0.1)
    assert eu < 5e-4 and ev < 5e-4 and ep < 2e-3, (eu, ev, ep)
    # the solution decays like exp(-2t/Re): check the kinetic-energy ratio
    ke0 = np.sum(np.square(ns.taylor_green_initial(spec.xy)[:2]))
    ke1 = np.sum(u * u + v * v)
    assert abs(ke1 / ke0 - np.exp(-4.0 * 0.1 / 10.0)) < 1e-3


def test_taylor_green_spatial_order():
    errs = []
    divs = []
    for n in (16, 32, 64):
        spec, ops, st, u, v, p = _tg_run(n, 50, 1e-3)
        errs.append(_tg_err(spec, u, v, p, 0.05))
        divs.append(np.abs(ops.divergence(u, v)).max())
    errs = np.array(errs)
    order_u = np.log2(errs[:-1, 0] / errs[1:, 0])
    order_p = np.log2(errs[1, 2] / errs[2, 2])
    assert np.all((order_u > 1.8) & (order_u < 2.2)), order_u
    assert 1.5 < order_p < 3.5, order_p
    # approximate projection: the discrete divergence left after eq. 14 falls with h
    assert np.all(np.log2(np.array(divs[:-1]) / np.array(divs[1:])) > 1.5), divs


def test_temporal_order_without_pressure():
    """u = 1, v = sin(x - t) exp(-t/Re), p = 0 solves eqs. 1-2 on the periodic box.

    Its pressure is constant, so the discrete projection does nothing and the
    time error is that of AB2 convection with Crank-Nicolson diffusion alone:
    second order, measured by self-convergence at fixed h.  (With a pressure, the
    approximate projection adds an O(dt h^2) term that dominates at coarse h.)
    """
    Re = 10.0
    spec = ns.periodic_lattice(32)
    ops = operators.Operators(operators.Problem(**spec.as_kwargs()))
    T = 0.8
    sols = []
    for dt in (0.08, 0.04, 0.02):
        st = step.Stepper(ops, dt, Re)
        u = np.ones(spec.n)
        v = np.sin(spec.xy[:, 0])
        p = np.zeros(spec.n)
        for _ in range(int(round(T / dt))):
            u, v, p = st.step(u, v, p)
        assert np.abs(u - 1.0).max() < 1e-12 and np.abs(p).max() < 1e-10
        sols.append(v)
    e1 = np.abs(sols[0] - sols[1]).max()
    e2 = np.abs(sols[1] - sols[2]).max()
    assert 1.8 < np.log2(e1 / e2) < 2.3, (e1, e2)
    # and the solution tracks the closed form (spatial error only)
    v_exact = np.sin(spec.xy[:, 0] - T) * np.exp(-T / Re)
    assert np.abs(sols[2] - v_exact).max() < 5e-3


def test_uniform_flow_is_preserved():
    spec = ns.periodic_lattice(16)
    ops = operators.Operators(operators.Problem(**spec.as_kwargs()))
    st = step.Stepper(ops, 0.01, 100.0)
    u = np.full(spec.n, 0.8)
    v = np.full(spec.n, -0.3)
    p = np.zeros(spec.n)
    for _ in range(5):
        u, v, p = st.step(u, v, p)
    assert np.abs(u - 0.8).max() < 1e-13 and np.abs(v + 0.3).max() < 1e-13
    assert np.abs(p).max() < 1e-11


def _kovasznay_spec(n, Re):
    def gval(x, y):
        uu, vv, _ = exact.kovasznay(np.array([[x, y]]), Re)
        return (uu[0], vv[0])
    sides = {s: ns.DIRICHLET for s in ("left", "right", "bottom", "top")}
    return ns.box_lattice(n, (n - 1) * 4 // 3 + 1, -0.5, 1.0, -0.5, 1.5, sides,
                          {s: gval for s in sides})


def test_kovasznay_steady_state_converges():
    Re = 40.0
    errs = []
    for n in (13, 25):
        spec = _kovasznay_spec(n, Re)
        ops = operators.Operators(operators.Problem(**spec.as_kwargs()))
        st = step.Stepper(ops, 0.002, Re)
        u, v, p = exact.kovasznay(spec.xy, Re)
        for _ in range(1500):
            u, v, p = st.step(u, v, p)
        ue, ve, pe = exact.kovasznay(spec.xy, Re)
        errs.append((np.abs(u - ue).max(), np.abs(v - ve).max(),
                     np.abs((p - p.mean()) - (pe - pe.mean())).max()))
    errs = np.array(errs)
    order = np.log2(errs[0] / errs[1])
    assert errs[1, 0] < 5e-2 and order[0] > 1.5 and order[1] > 1.0 and order[2] > 1.0, (errs, order)


def _linear_step_radius(spec, dt, Re):
    prob = operators.Problem(**spec.as_kwargs())
    prob.bnd_value[:] = 0.0
    ops = operators.Operators(prob)
    st = step.Stepper(ops, dt, Re)
    n = spec.n
    ops.convection = lambda u, v: (np.zeros(n), np.zeros(n))   # Stokes part of the step
    cols = []
    for k in range(3 * n):
        x = np.zeros(3 * n)
        x[k] = 1.0
        st.n_prev = None
        cols.append(np.concatenate(st.step(x[:n], x[n:2 * n], x[2 * n:])))
    return np.abs(np.linalg.eigvals(np.array(cols).T)).max()


@pytest.mark.parametrize("dt", [1e-3, 1e-1])
def test_linear_stability_of_the_step(dt):
    assert _linear_step_radius(ns.lid_cavity(9), dt, 40.0) <= 1.0 + 1e-9
    cyl = ns.cylinder_channel(0.25, box=(-2.0, 3.0, -2.0, 2.0), n_surface=16)
    assert _linear_step_radius(cyl, dt, 100.0) <= 1.0 + 1e-9


def test_krylov_mode_matches_direct():
    spec = ns.cylinder_channel(0.125, box=(-2.0, 4.0, -2.0, 2.0), n_surface=40)
    ops = operators.Operators(operators.Problem(**spec.as_kwargs()))
    a = step.Stepper(ops, 0.01, 100.0)
    b = step.Stepper(ops, 0.01, 100.0, solver="krylov", tol=1e-12)
    u0, v0, p0 = ns.boundary_initial(spec, (1.0, 0.0))
    ua, va, pa = u0, v0, p0
    ub, vb, pb = u0, v0, p0
    for _ in range(3):
        ua, va, pa = a.step(ua, va, pa)
        ub, vb, pb = b.step(ub, vb, pb)
    for x, y in ((ua, ub), (va, vb), (pa, pb)):
        assert np.abs(x - y).max() < 1e-8 * max(1.0, np.abs(x).max())
