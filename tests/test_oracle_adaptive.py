"""Pins of the oracle on stepwise refined node sets with a support radius that follows the
local spacing, rho(xbar) (Section 3; Section 5.5 refines its nodes in steps around the body):
support radii against brute force, exactness of every operator on quadratics across the
spacing jumps, uniform flow kept through a refined channel, and second-order convergence of
a manufactured pressure problem as the spacing is halved everywhere."""
import numpy as np
import pytest

from oracle import mls, operators, step
from paper_1401_6513_amd import nodesets as ns

ZONES = [(-1.5, 3.0, -1.5, 1.5), (-2.5, 5.0, -2.5, 2.5)]


def _refined(h=1.0 / 16, shape="circle"):
    return ns.refined_cylinder_channel(h, ZONES, box=(-4.0, 8.0, -4.0, 4.0), shape=shape, n_surface=64)


def _ops(spec):
    return operators.Operators(operators.Problem(**spec.as_kwargs()))


def test_support_radius_follows_the_local_spacing():
    spec = _refined()
    ops = _ops(spec)
    base = 2.5 * spec.h_node
    grown = ops.rho_node / base
    # every node keeps its base radius or a grown one (x1.25, x1.5625)
    assert np.all(np.isclose(grown, 1.0) | np.isclose(grown, 1.25) | np.isclose(grown, 1.5625))
    assert np.mean(np.isclose(grown, 1.0)) > 0.9
    # brute force: neighbours of a sample of nodes within their radius
    rng = np.random.default_rng(0)
    for i in rng.choice(spec.n, 60, replace=False):
        d = np.hypot(*(spec.xy - spec.xy[i]).T)
        want = np.flatnonzero(d < ops.rho_node[i])
        assert np.array_equal(np.sort(ops.node_nbrs[i]), want)
    # the three spacings are all present
    assert len(np.unique(spec.h_node)) == 3


def test_operators_exact_on_quadratics_across_spacing_jumps():
    spec = _refined()
    ops = _ops(spec)
    x, y = spec.xy[:, 0], spec.xy[:, 1]
    a, b, c, d, e, f = 0.3, -0.7, 0.2, 0.45, -0.15, 0.25
    q = a + b * x + c * y + d * x * x + e * x * y + f * y * y
    lap = 2 * d + 2 * f
    assert np.abs(ops.M00 @ q - q).max() < 1e-11
    assert np.abs(ops.L @ q - lap).max() < 1e-8
    for k, V in enumerate(ops.VIP):
        pts = ops.vip_xy[:, k, :]
        qv = a + b * pts[:, 0] + c * pts[:, 1] + d * pts[:, 0] ** 2 + e * pts[:, 0] * pts[:, 1] + f * pts[:, 1] ** 2
        assert np.abs((V @ q)[spec.n_lattice * 0 + ops.prob.interior] - qv).max() < 1e-11
    # VIP spacing follows the node spacing away from the body
    far = ops.prob.interior[np.hypot(x, y)[ops.prob.interior] > 1.5]
    assert np.allclose(ops.d_ew[far], spec.h_node[far]) and np.allclose(ops.d_ns[far], spec.h_node[far])
    # Neumann rows: 2 d_b dq/dn at every boundary node
    bi = spec.bnd_idx
    gx = b + 2 * d * x[bi] + e * y[bi]
    gy = c + e * x[bi] + 2 * f * y[bi]
    dqdn = spec.bnd_normal[:, 0] * gx + spec.bnd_normal[:, 1] * gy
    got = (ops.neumann_rows() @ q)[bi]
    assert np.abs(got - 2 * 0.5 * spec.h_node[bi] * dqdn).max() < 1e-10


def test_uniform_flow_through_a_refined_channel():
    spec = _refined(shape=None)
    st = step.Stepper(_ops(spec), 0.01, 100.0)
    u, v, p = np.ones(spec.n), np.zeros(spec.n), np.zeros(spec.n)
    for _ in range(3):
        u, v, p = st.step(u, v, p)
    assert np.abs(u - 1).max() < 1e-11 and np.abs(v).max() < 1e-11 and np.abs(p).max() < 1e-9


def test_manufactured_pressure_problem_converges_at_second_order():
    """phi = sin(pi (x - 8) / 24) cos(pi y / 4) has phi = 0 on the outlet x = 8 and zero
    normal derivative on the inlet and the slip walls; b = Delta phi at interior rows."""
    errs = []
    for h in (1.0 / 8, 1.0 / 16, 1.0 / 32):
        spec = _refined(h, shape=None)
        ops = _ops(spec)
        st = step.Stepper(ops, 0.01, 100.0)
        x, y = spec.xy[:, 0], spec.xy[:, 1]
        kx, ky = np.pi / 24, np.pi / 4
        phi = np.sin(kx * (x - 8.0)) * np.cos(ky * y)
        b = -(kx * kx + ky * ky) * phi
        b[spec.bnd_idx] = 0.0
        got = st.poisson_solve(b)
        errs.append(np.abs(got - phi).max())
    errs = np.array(errs)
    order = np.log2(errs[:-1] / errs[1:])
    assert np.all(order > 1.7), (errs, order)
