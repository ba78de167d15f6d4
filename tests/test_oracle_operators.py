"""Pins of the oracle's VIP operators (Section 4 of the paper): exactness on
polynomials, the convection flux on linear fields, the placement of virtual
interpolation points, and the bordered pressure solve against dense algebra."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import operators, step
from paper_1401_6513_amd import nodesets as ns


def _problem(spec):
    return operators.Problem(**spec.as_kwargs())


@pytest.fixture(scope="module")
def cyl_ops():
    spec = ns.cylinder_channel(0.1, box=(-1.5, 2.5, -1.5, 1.5), n_surface=48)
    return spec, operators.Operators(_problem(spec))


@pytest.fixture(scope="module")
def jit_ops():
    spec = ns.jittered(ns.lid_cavity(19), 0.25, seed=11)
    return spec, operators.Operators(_problem(spec))


QUADS = [lambda x, y: np.ones_like(x), lambda x, y: x, lambda x, y: y,
         lambda x, y: x * x, lambda x, y: x * y, lambda x, y: y * y]
LAPS = [0.0, 0.0, 0.0, 2.0, 0.0, 2.0]


@pytest.mark.parametrize("which", ["cyl", "jit"])
def test_identity_and_laplacian_exact_on_quadratics(which, cyl_ops, jit_ops):
    spec, ops = cyl_ops if which == "cyl" else jit_ops
    x, y = spec.xy[:, 0], spec.xy[:, 1]
    for q, lap in zip(QUADS, LAPS):
        f = q(x, y)
        assert np.abs(ops.M00 @ f - f).max() < 1e-11
        assert np.abs(ops.L @ f - lap).max() < 1e-9 / spec.h ** 0


@pytest.mark.parametrize("which", ["cyl", "jit"])
def test_vip_interpolation_and_differences(which, cyl_ops, jit_ops):
    spec, ops = cyl_ops if which == "cyl" else jit_ops
    prob = ops.prob
    x, y = spec.xy[:, 0], spec.xy[:, 1]
    vxy = ops.vip_xy
    o = prob.vip_offset * prob.h
    clipped = np.any(np.abs(np.linalg.norm(vxy - spec.xy[prob.interior][:, None, :], axis=2) - o)
                     > 1e-12, axis=1)
    for q in QUADS:
        f = q(x, y)
        vals = ops.vip_values(f)[:, prob.interior]
        for k in range(4):
            assert np.allclose(vals[k], q(vxy[:, k, 0], vxy[:, k, 1]), atol=1e-11)
    # direct differences: exact derivative for quadratics at unclipped nodes ...
    xi, yi = x[prob.interior], y[prob.interior]
    for q, dqx, dqy in ((lambda x, y: x * x, lambda x, y: 2 * x, lambda x, y: 0 * x),
                        (lambda x, y: x * y, lambda x, y: y, lambda x, y: x),
                        (lambda x, y: y * y, lambda x, y: 0 * x, lambda x, y: 2 * y)):
        f = q(x, y)
        gx = ops.ddx(f)[prob.interior]
        gy = ops.ddy(f)[prob.interior]
        ok = ~clipped
        assert np.allclose(gx[ok], dqx(xi, yi)[ok], atol=1e-9)
        assert np.allclose(gy[ok], dqy(xi, yi)[ok], atol=1e-9)
    # ... and for linear functions everywhere
    for a, b in ((1.3, -0.4), (0.0, 2.0)):
        f = 0.7 + a * x + b * y
        assert np.allclose(ops.ddx(f)[prob.interior], a, atol=1e-9)
        assert np.allclose(ops.ddy(f)[prob.interior], b, atol=1e-9)
    # boundary rows of the difference operators are empty
    assert np.all(ops.ddx(x)[prob.bnd_idx] == 0.0)


def test_vips_stay_inside_body_fitted_domain(cyl_ops):
    spec, ops = cyl_ops
    prob = ops.prob
    vxy = ops.vip_xy
    xi = spec.xy[prob.interior]
    o = prob.vip_offset * prob.h
    r = np.hypot(vxy[..., 0], vxy[..., 1])
    assert r.min() >= 0.5 - 2e-3 * prob.h   # on or outside the circle (tangent-line chord)
    # every VIP moved only along its own axis, towards x_i, never past it
    disp = vxy - xi[:, None, :]
    for k, (dx, dy) in enumerate(operators.VIP_DIRS):
        t = disp[:, k, 0] * dx + disp[:, k, 1] * dy
        perp = disp[:, k, 0] * (-dy) + disp[:, k, 1] * dx
        assert np.all(np.abs(perp) < 1e-14) and np.all((t >= 0.0) & (t <= o + 1e-15))
    assert (np.abs(np.linalg.norm(disp, axis=2) - o) > 1e-9).any()   # some were clipped


def test_convection_exact_for_linear_velocity(jit_ops):
    spec, ops = jit_ops
    prob = ops.prob
    x, y = spec.xy[:, 0], spec.xy[:, 1]
    u = 0.3 + 1.1 * x - 0.6 * y
    v = -0.2 + 0.5 * x + 0.9 * y
    nx, ny = ops.convection(u, v)
    # d(u^2)/dx + d(uv)/dy and d(uv)/dx + d(v^2)/dy for linear u, v
    ux, uy, vx, vy = 1.1, -0.6, 0.5, 0.9
    ex = 2 * u * ux + (uy * v + u * vy)
    ey = (ux * v + u * vx) + 2 * v * vy
    i = prob.interior
    assert np.allclose(nx[i], ex[i], atol=1e-9)
    assert np.allclose(ny[i], ey[i], atol=1e-9)


def test_neumann_rows_exact_on_quadratics(cyl_ops):
    spec, ops = cyl_ops
    prob = ops.prob
    B = ops.neumann_rows()
    x, y = spec.xy[:, 0], spec.xy[:, 1]
    bx, by = x[prob.bnd_idx], y[prob.bnd_idx]
    nx, ny = prob.bnd_normal[:, 0], prob.bnd_normal[:, 1]
    d2 = 2.0 * prob.vip_offset * prob.h
    for f, fx, fy in ((lambda x, y: 2.0 + 0.4 * x - 1.7 * y, lambda x, y: 0.4 + 0 * x,
                       lambda x, y: -1.7 + 0 * x),
                      (lambda x, y: x * x - 0.5 * x * y, lambda x, y: 2 * x - 0.5 * y,
                       lambda x, y: -0.5 * x),
                      (lambda x, y: y * y + 3 * x * y, lambda x, y: 3 * y, lambda x, y: 2 * y + 3 * x)):
        want = d2 * (nx * fx(bx, by) + ny * fy(bx, by))
        assert np.allclose((B @ f(x, y))[prob.bnd_idx], want, atol=1e-10)
    assert np.all((B @ np.ones(spec.n)) == 0.0) or np.abs(B @ np.ones(spec.n)).max() < 1e-12


def _dense_bordered_solve(P, b):
    n = P.shape[0]
    A = np.zeros((n + 1, n + 1))
    A[:n, :n] = P.toarray()
    A[:n, n] = 1.0
    A[n, :n] = 1.0
    return np.linalg.solve(A, np.concatenate([b, [0.0]]))


@pytest.mark.parametrize("case", ["periodic", "cavity", "cylinder"])
def test_pressure_solve_matches_dense(case):
    spec = {"periodic": ns.periodic_lattice(8),
            "cavity": ns.lid_cavity(9),
            "cylinder": ns.cylinder_channel(0.25, box=(-2.0, 3.0, -2.0, 2.0), n_surface=16)}[case]
    ops = operators.Operators(_problem(spec))
    st = step.Stepper(ops, 0.01, 50.0)
    b = ns.random_field(spec.n, seed=4)
    b[spec.bnd_idx] = 0.0
    phi = st.poisson_solve(b)
    if st.bordered:
        ref = _dense_bordered_solve(st.P, b)
        assert abs(st.lam - ref[-1]) < 1e-9 * max(1.0, abs(ref[-1]))
        ref = ref[:-1]
        assert abs(phi.sum()) < 1e-9 * np.abs(phi).max() * spec.n
    else:
        ref = np.linalg.solve(st.P.toarray(), b)
    assert np.allclose(phi, ref, rtol=0, atol=1e-10 * np.abs(ref).max())
    # constants are in the null space of the bordered operator's block
    if st.bordered:
        assert np.abs(st.P @ np.ones(spec.n)).max() < 1e-9 / spec.h ** 2


def test_manufactured_neumann_poisson_converges():
    """cos(pi x) cos(pi y) on the unit square: dphi/dn = 0 on every side."""
    errs = []
    for n in (17, 33, 65):
        spec = ns.lid_cavity(n)
        ops = operators.Operators(_problem(spec))
        st = step.Stepper(ops, 0.01, 50.0)
        x, y = spec.xy[:, 0], spec.xy[:, 1]
        exact = np.cos(np.pi * x) * np.cos(np.pi * y)
        b = -2.0 * np.pi ** 2 * exact
        b[spec.bnd_idx] = 0.0
        phi = st.poisson_solve(b)
        errs.append(np.abs((phi - phi.mean()) - (exact - exact.mean())).max())
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert errs[-1] < 2e-3 and np.all(order > 1.4), (errs, order)
