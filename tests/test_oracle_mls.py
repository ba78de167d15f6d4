"""Pins of the oracle's MLS shape functions (Section 3 of the paper) against facts
that do not come from the oracle itself: polynomial reproduction, an independent
least-squares route, a library B-spline, invariances and brute-force counts."""
import math

import numpy as np
import pytest
from scipy.interpolate import BSpline

from oracle import mls
from paper_1401_6513_amd import nodesets as ns

DERIVS = [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2)]
MONOMIALS = [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2)]


def _mono(a, b, x, y):
    return x ** a * y ** b


def _mono_deriv(a, b, da, db, x, y):
    """d^da/dx^da d^db/dy^db of x^a y^b."""
    if da > a or db > b:
        return np.zeros_like(x)
    ca = math.factorial(a) / math.factorial(a - da)
    cb = math.factorial(b) / math.factorial(b - db)
    return ca * cb * x ** (a - da) * y ** (b - db)


def test_cubic_spline_is_cardinal_bspline():
    # the cubic-spline weight is the cardinal cubic B-spline N(t) at t = 2r
    N = BSpline.basis_element([-2.0, -1.0, 0.0, 1.0, 2.0], extrapolate=False)
    r = np.linspace(0.0, 0.999, 500)
    assert np.allclose(mls.weight(r, mls.CUBIC_SPLINE), N(2.0 * r), atol=1e-14, rtol=0)
    assert np.all(mls.weight(np.array([1.0, 1.5, 7.0]), mls.CUBIC_SPLINE) == 0.0)


def test_paper_weight_limits():
    r = np.linspace(0.0, 0.9999, 2000)
    w = mls.weight(r, mls.PAPER)
    assert w[0] == 1.0
    assert np.all(np.diff(w) <= 0.0)           # non-increasing on [0, 1)
    assert w[-1] < 1e-30                        # tends to 0 at the support edge
    assert np.all(mls.weight(np.array([1.0, 2.0]), mls.PAPER) == 0.0)


def _sets():
    per = ns.periodic_lattice(24)
    cav = ns.lid_cavity(21)
    cyl = ns.cylinder_channel(0.125, box=(-2.0, 3.0, -2.0, 2.0), n_surface=40)
    jit = ns.jittered(ns.lid_cavity(21), 0.25, seed=0)
    return {"periodic": per, "cavity": cav, "cylinder": cyl, "jittered": jit}


@pytest.mark.parametrize("name", ["periodic", "cavity", "cylinder", "jittered"])
@pytest.mark.parametrize("kind", [mls.CUBIC_SPLINE, mls.PAPER])
def test_reproduces_quadratics(name, kind):
    spec = _sets()[name]
    nodes = mls.NodeSet(spec.xy, spec.period)
    rng = np.random.default_rng(1)
    # evaluation points: nodes themselves plus random off-node points inside
    pts = np.concatenate([spec.xy[rng.choice(spec.n, 60, replace=False)],
                          spec.xy[rng.choice(spec.n, 60, replace=False)]
                          + rng.uniform(-0.5, 0.5, (60, 2)) * spec.h])
    if name == "cylinder":   # keep evaluation points out of the body
        keep = np.hypot(pts[:, 0], pts[:, 1]) > 0.5
        pts = pts[keep]
    nb, rho, psi = mls.shape_functions(nodes, pts, spec.rho, DERIVS, weight_kind=kind)
    for i, p in enumerate(pts):
        # rounding bound: a small multiple of cond(M) * eps (cond ~ 2e2 cubic, up to ~1e9 paper)
        cond = mls.moment_condition(nodes, p, rho[i], kind)
        tol = max(1e-12, 100.0 * cond * np.finfo(float).eps)
        d = mls.min_image(spec.xy[nb[i]] - p, spec.period)
        for (a, b) in MONOMIALS:
            vals = _mono(a, b, d[:, 0], d[:, 1])          # q centred at p
            for (da, db) in DERIVS:
                got = psi[(da, db)][i] @ vals
                want = _mono_deriv(a, b, da, db, np.zeros(1), np.zeros(1))[0]
                scale = spec.h ** (a + b - da - db)
                assert abs(got - want) <= tol * max(scale, 1.0), (name, i, (a, b), (da, db))


def test_matches_independent_least_squares():
    spec = ns.jittered(ns.lid_cavity(17), 0.25, seed=3)
    nodes = mls.NodeSet(spec.xy, spec.period)
    rng = np.random.default_rng(7)
    pts = spec.xy[rng.choice(spec.n, 40, replace=False)] + rng.uniform(-0.4, 0.4, (40, 2)) * spec.h
    nb, rho, psi = mls.shape_functions(nodes, pts, spec.rho, DERIVS)
    u = rng.standard_normal(spec.n)
    for i, p in enumerate(pts):
        d = (spec.xy[nb[i]] - p) / rho[i]
        P = np.stack([np.ones(len(d)), d[:, 0], d[:, 1], d[:, 0] ** 2, d[:, 0] * d[:, 1],
                      d[:, 1] ** 2], axis=1)
        # weighted least squares by SVD-based lstsq on sqrt(W) P c = sqrt(W) u
        BN = BSpline.basis_element([-2.0, -1.0, 0.0, 1.0, 2.0], extrapolate=False)
        w = np.nan_to_num(BN(2.0 * np.hypot(d[:, 0], d[:, 1])))
        sw = np.sqrt(w)
        c = np.linalg.lstsq(sw[:, None] * P, sw * u[nb[i]], rcond=None)[0]
        for k, (a, b) in enumerate(DERIVS):
            want = c[k] * math.factorial(a) * math.factorial(b) / rho[i] ** (a + b)
            got = psi[(a, b)][i] @ u[nb[i]]
            assert abs(got - want) <= 1e-10 * max(1.0, abs(want)) * (1.0 / spec.h) ** (a + b)


def test_weight_scale_invariance():
    spec = ns.jittered(ns.lid_cavity(13), 0.2, seed=5)
    nodes = mls.NodeSet(spec.xy, spec.period)
    pts = spec.xy[::7]
    _, _, a = mls.shape_functions(nodes, pts, spec.rho, DERIVS)
    _, _, b = mls.shape_functions(nodes, pts, spec.rho, DERIVS,
                                  weight_fn=lambda r: 3.7 * mls.weight(r, mls.CUBIC_SPLINE))
    for d in DERIVS:
        for x, y in zip(a[d], b[d]):
            assert np.allclose(x, y, rtol=1e-12, atol=1e-12 * np.abs(x).max())


def test_coordinate_scaling():
    spec = ns.jittered(ns.lid_cavity(13), 0.2, seed=6)
    s = 7.25
    nodes1 = mls.NodeSet(spec.xy, spec.period)
    nodes2 = mls.NodeSet(spec.xy * s, spec.period)
    pts = spec.xy[::5] + 0.3 * spec.h
    _, _, a = mls.shape_functions(nodes1, pts, spec.rho, DERIVS)
    _, _, b = mls.shape_functions(nodes2, pts * s, spec.rho * s, DERIVS)
    for (da, db) in DERIVS:
        for x, y in zip(a[(da, db)], b[(da, db)]):
            assert np.allclose(y, x * s ** (-(da + db)), rtol=1e-11,
                               atol=1e-11 * np.abs(x).max() * s ** (-(da + db)))


def test_lattice_symmetry_and_stencil_sizes():
    spec = ns.periodic_lattice(16)
    nodes = mls.NodeSet(spec.xy, spec.period)
    i0 = 5 * 16 + 7
    x0 = spec.xy[i0]
    nb, _, psi = mls.shape_functions(nodes, x0[None], spec.rho, [(0, 0), (2, 0), (0, 2)])
    # brute-force neighbour count
    d = mls.min_image(spec.xy - x0, spec.period)
    brute = np.flatnonzero(d[:, 0] ** 2 + d[:, 1] ** 2 < spec.rho ** 2)
    assert len(brute) == 21 and np.array_equal(np.sort(brute), nb[0])
    off = np.rint(mls.min_image(spec.xy[nb[0]] - x0, spec.period) / spec.h).astype(int)
    m00 = dict(zip(map(tuple, off), psi[(0, 0)][0]))
    lap = dict(zip(map(tuple, off), psi[(2, 0)][0] + psi[(0, 2)][0]))
    for (i, j) in m00:    # dihedral symmetry of the lattice stencil
        for (a, b) in ((-i, j), (i, -j), (j, i), (-j, -i)):
            assert abs(m00[(a, b)] - m00[(i, j)]) < 1e-14
            assert abs(lap[(a, b)] - lap[(i, j)]) < 1e-9 / spec.h ** 2
    # VIP at x0 + h/2: 16 neighbours strictly inside, 6 more exactly on the support
    # circle (membership of those is decided by rounding; their weight is Phi(1) = 0)
    xv = x0 + np.array([0.5 * spec.h, 0.0])
    d = mls.min_image(spec.xy - xv, spec.period)
    d2 = d[:, 0] ** 2 + d[:, 1] ** 2
    assert np.count_nonzero(d2 < spec.rho ** 2 * (1.0 - 1e-9)) == 16
    assert np.count_nonzero(np.abs(d2 - spec.rho ** 2) <= 1e-9 * spec.rho ** 2) == 6
    nbv, _, pv = mls.shape_functions(nodes, xv[None], spec.rho, [(0, 0)])
    dv = mls.min_image(spec.xy[nbv[0]] - xv, spec.period)
    on_edge = np.abs(dv[:, 0] ** 2 + dv[:, 1] ** 2 - spec.rho ** 2) <= 1e-9 * spec.rho ** 2
    assert np.all(np.abs(pv[(0, 0)][0][on_edge]) < 1e-30)


def test_support_growth_and_failure():
    rng = np.random.default_rng(0)
    xy = rng.uniform(0.0, 1.0, (400, 2))
    nodes = mls.NodeSet(xy)
    # radius holding ~9 points on average: some points must grow
    r = math.sqrt(9.0 / (400 * math.pi))
    inner = xy[np.all((xy > 0.25) & (xy < 0.75), axis=1)]

    def brute(p, rad):
        d = xy - p
        return int(np.count_nonzero(d[:, 0] ** 2 + d[:, 1] ** 2 < rad * rad))

    # keep points that reach 12 neighbours within the largest grown radius
    inner = np.array([p for p in inner if brute(p, 1.5625 * r) >= 12])[:50]
    nb, rho, _ = mls.shape_functions(nodes, inner, r, [(0, 0)], min_neighbours=12)
    for p, n, rr in zip(inner, nb, rho):
        # the smallest radius in {r, 1.25 r, 1.5625 r} holding 12 neighbours is chosen
        first = next(s for s in (1.0, 1.25, 1.5625) if brute(p, s * r) >= 12)
        assert abs(rr - first * r) < 1e-15 and len(n) == brute(p, first * r)
    assert (rho > r).any()
    with pytest.raises(mls.SingularStencil):
        mls.shape_functions(nodes, xy[:5], 0.2 * r, [(0, 0)], min_neighbours=12)
