"""Further pins of the oracle, each against something other than the oracle itself:

* the weight function printed in Section 3, against values worked out in 50-digit
  decimal arithmetic (tests/golden/paper_weight.txt);
* the velocity boundary rows of eq. 12 (SLIP component selection, the OUTLET
  traction row with a nonzero pressure), against a manufactured quadratic solution
  that the discrete operators reproduce exactly;
* uniform flow through a channel with an inlet, slip walls and an outlet, which the
  scheme must keep exactly;
* one and two fractional steps (eqs. 12-15) against a dense-matrix formulation written
  here from the paper, with its own brute-force MLS by weighted least squares;
* the projection identity D u^(n+1) = dt (L phi + lambda - D G phi) at interior nodes,
  which holds to roundoff because eq. 13 uses the MLS Laplacian rather than D G.
"""
import math
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla
from scipy.interpolate import BSpline

from oracle import mls, operators, step
from paper_1401_6513_amd import nodesets as ns

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
EPS = np.finfo(float).eps


# ---- weight printed in Section 3 ---------------------------------------------------------------

def _golden_paper_weight():
    rows = []
    with open(os.path.join(GOLDEN, "paper_weight.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            r, w = line.split()
            rows.append((float(r), float(w)))
    return np.array(rows)


def test_paper_weight_values():
    """Phi(r) = (1 - r^((1-r)^2))^4 (Section 3) at worked values.  Near r = 1 the difference
    1 - r^e cancels, so the FP64 bound grows like eps / (1 - r^e)."""
    tab = _golden_paper_weight()
    got = mls.weight(tab[:, 0], mls.PAPER)
    for r, want, g in zip(tab[:, 0], tab[:, 1], got):
        q = 1.0 - r ** ((1.0 - r) ** 2) if r > 0 else 1.0
        tol = 1e-14 + 16.0 * EPS / q
        assert abs(g - want) <= tol * want, (r, g, want)
    # zero at and beyond the support edge
    assert np.all(mls.weight(np.array([1.0, 1.2]), mls.PAPER) == 0.0)


# ---- velocity boundary rows (eq. 12 with the boundary readings) ----------------------------------

def _channel(n, orient, wall_decoy=5.0):
    """Channel on [0,2]x[0,1] (orient 'x': inlet left, outlet right, SLIP bottom/top) or its
    transpose (orient 'y': inlet bottom, outlet top, SLIP left/right).  The SLIP walls carry a
    decoy in the tangential slot of their value: only the normal component may be held."""
    if orient == "x":
        kinds = {"left": ns.DIRICHLET, "right": ns.OUTLET, "bottom": ns.SLIP, "top": ns.SLIP}
        vals = {"left": (1.0, 0.0), "right": (0.0, 0.0),
                "bottom": (wall_decoy, 0.0), "top": (wall_decoy, 0.0)}
        return ns.box_lattice(2 * n - 1, n, 0.0, 2.0, 0.0, 1.0, kinds, vals, name="channel")
    kinds = {"bottom": ns.DIRICHLET, "top": ns.OUTLET, "left": ns.SLIP, "right": ns.SLIP}
    vals = {"bottom": (0.0, 1.0), "top": (0.0, 0.0),
            "left": (0.0, wall_decoy), "right": (0.0, wall_decoy)}
    spec = ns.box_lattice(n, 2 * n - 1, 0.0, 1.0, 0.0, 2.0, kinds, vals, name="channel_t")
    return spec


def _fix_corners(spec, orient):
    """box_lattice gives corners to the left/right sides; in the transposed channel the inlet
    and outlet are bottom/top, so give the four corners to those."""
    if orient == "x":
        return spec
    xy = spec.xy[spec.bnd_idx]
    y0, y1 = spec.xy[:, 1].min(), spec.xy[:, 1].max()
    bot = xy[:, 1] == y0
    top = xy[:, 1] == y1
    spec.bnd_kind[bot] = ns.DIRICHLET
    spec.bnd_value[bot] = (0.0, 1.0)
    spec.bnd_normal[bot] = (0.0, -1.0)
    spec.bnd_kind[top] = ns.OUTLET
    spec.bnd_value[top] = (0.0, 0.0)
    spec.bnd_normal[top] = (0.0, 1.0)
    return spec


@pytest.mark.parametrize("orient", ["x", "y"])
def test_uniform_channel_flow_is_kept(orient):
    """Uniform flow along the channel with p = 0 solves eqs. 1-2 with these boundary
    conditions; the scheme reproduces constants exactly, so it must stay put."""
    spec = _fix_corners(_channel(9, orient), orient)
    ops = operators.Operators(operators.Problem(**spec.as_kwargs()))
    st = step.Stepper(ops, 0.01, 50.0)
    ax = 0 if orient == "x" else 1
    u = np.zeros(spec.n) + (1.0 if ax == 0 else 0.0)
    v = np.zeros(spec.n) + (1.0 if ax == 1 else 0.0)
    p = np.zeros(spec.n)
    for _ in range(4):
        u, v, p = st.step(u, v, p)
    want_u = 1.0 if ax == 0 else 0.0
    want_v = 1.0 - want_u
    assert np.abs(u - want_u).max() < 1e-12 and np.abs(v - want_v).max() < 1e-12
    assert np.abs(p).max() < 1e-10


@pytest.mark.parametrize("orient", ["x", "y"])
def test_outlet_and_slip_rows_on_a_manufactured_predictor(orient):
    """Predictor of eq. 12 (convection off) for u^n = q(s), a quadratic in the stream-wise
    coordinate s, with the outlet pressure set to q'(s_out)/Re (nonzero):
    (M00 - cL) u* = (M00 + cL) q has the exact solution u* = q + 4 a c (c = dt/2Re, q'' = 2a),
    since D^[0,0] and the Laplacian reproduce quadratics.  That u* also satisfies the slip
    walls (zero normal derivative of the stream-wise component; the cross component is held
    at 0, whatever decoy sits in the other slot), the outlet row du/dn = Re p n and the inlet
    value q(s_in) + 4ac.  A wrong sign or factor in the outlet row, or the wrong component
    held on a slip wall, moves u* off this solution."""
    a, b, c0 = 0.3, -0.2, 0.7
    Re, dt = 50.0, 0.02
    cc = dt / (2.0 * Re)
    spec = _fix_corners(_channel(9, orient), orient)
    ax = 0 if orient == "x" else 1
    s = spec.xy[:, ax]
    q = a * s * s + b * s + c0
    want = q + 4.0 * a * cc
    # inlet value consistent with the manufactured solution
    inlet = spec.bnd_kind == ns.DIRICHLET
    spec.bnd_value[inlet, ax] = want[spec.bnd_idx[inlet]]
    prob = operators.Problem(**spec.as_kwargs())
    ops = operators.Operators(prob)
    st = step.Stepper(ops, dt, Re)
    p = np.zeros(spec.n)
    out = spec.bnd_idx[spec.bnd_kind == ns.OUTLET]
    s_out = s[out][0]
    p[out] = (2.0 * a * s_out + b) / Re          # q'(s_out) = Re p n_s, n_s = 1
    assert abs(p[out][0]) > 1e-3
    zero = np.zeros(spec.n)
    vel = (q, zero) if ax == 0 else (zero, q)
    ru, rv = st.predictor_rhs(vel[0], vel[1], p, zero, zero)
    us = spla.spsolve(st.Hu.tocsc(), ru)
    vs = spla.spsolve(st.Hv.tocsc(), rv)
    along, cross = (us, vs) if ax == 0 else (vs, us)
    assert np.abs(along - want).max() < 1e-11, np.abs(along - want).max()
    assert np.abs(cross).max() < 1e-11


# ---- dense-matrix formulation of one step (eqs. 12-15) ------------------------------------------

def _cubic_spline_weight(r):
    """Cubic-spline weight as the cardinal cubic B-spline at 2r (the same function the oracle
    uses, taken here from SciPy's B-spline basis instead)."""
    N = BSpline.basis_element([-2.0, -1.0, 0.0, 1.0, 2.0], extrapolate=False)
    w = N(2.0 * np.asarray(r, dtype=float))
    return np.nan_to_num(w, nan=0.0)


def _dense_mls_rows(xy, period, pts, rho, derivs):
    """Brute-force MLS rows: for each point, every node within rho (minimum image), the
    weighted least-squares fit of the scaled quadratic basis by QR (lstsq on W^(1/2) P), and
    the derivative of the local polynomial at the point (Section 3)."""
    n = len(xy)
    out = {d: np.zeros((len(pts), n)) for d in derivs}
    col = {(0, 0): 0, (1, 0): 1, (0, 1): 2, (2, 0): 3, (1, 1): 4, (0, 2): 5}
    for i, x in enumerate(pts):
        d = xy - x
        for k in range(2):
            d[:, k] -= period[k] * np.round(d[:, k] / period[k])
        dist = np.hypot(d[:, 0], d[:, 1])
        J = np.flatnonzero(dist < rho)
        z = d[J] / rho
        P = np.stack([np.ones(len(J)), z[:, 0], z[:, 1], z[:, 0] ** 2, z[:, 0] * z[:, 1],
                      z[:, 1] ** 2], axis=1)
        sw = np.sqrt(_cubic_spline_weight(dist[J] / rho))
        # coefficients c = pinv(W^1/2 P) W^1/2 u: column j of C is the fit of the unit vector e_j
        C = np.linalg.lstsq(sw[:, None] * P, np.diag(sw), rcond=None)[0]     # 6 x |J|
        for (a, b) in derivs:
            out[(a, b)][i, J] = math.factorial(a) * math.factorial(b) / rho ** (a + b) * C[col[(a, b)]]
    return out


class _DenseScheme:
    """Eqs. 12-15 on a periodic lattice with dense matrices, written from the paper:
    VIPs at x_i +- h/2 along each axis, I = D^[0,0] and Delta = D^[2,0] + D^[0,2] at the node,
    convection by direct VIP differences of products of interpolated values, AB2 with
    N^(-1) = N^0, Crank-Nicolson, the bordered pressure system (constants are in the null space
    of the periodic Laplacian), projection by the VIP gradient and p = phi - (dt/2Re) Delta phi."""

    def __init__(self, spec, dt, Re):
        xy, h, rho, per = spec.xy, spec.h, spec.rho, spec.period
        node = _dense_mls_rows(xy, per, xy, rho, [(0, 0), (2, 0), (0, 2)])
        self.I = node[(0, 0)]
        self.L = node[(2, 0)] + node[(0, 2)]
        o = 0.5 * h
        self.V = [_dense_mls_rows(xy, per, xy + sh, rho, [(0, 0)])[(0, 0)]
                  for sh in (np.array([o, 0.0]), np.array([-o, 0.0]), np.array([0.0, o]),
                             np.array([0.0, -o]))]
        self.h, self.dt, self.Re = h, dt, Re
        self.c = dt / (2.0 * Re)
        self.Nprev = None

    def convection(self, u, v):
        ue, uw, un, us = (V @ u for V in self.V)
        ve, vw, vn, vs = (V @ v for V in self.V)
        d = 2.0 * 0.5 * self.h          # |x_e - x_w| = |x_n - x_s| = h
        return ((ue ** 2 - uw ** 2) / d + (un * vn - us * vs) / d,
                (ue * ve - uw * vw) / d + (vn ** 2 - vs ** 2) / d)

    def step(self, u, v, p):
        n = len(u)
        N = self.convection(u, v)
        if self.Nprev is None:
            self.Nprev = N
        C = [1.5 * N[k] - 0.5 * self.Nprev[k] for k in range(2)]
        self.Nprev = N
        A = self.I - self.c * self.L
        R = self.I + self.c * self.L
        us = np.linalg.solve(A, R @ u - self.dt * C[0])
        vs = np.linalg.solve(A, R @ v - self.dt * C[1])
        Dx = (self.V[0] - self.V[1]) / self.h
        Dy = (self.V[2] - self.V[3]) / self.h
        rhs = (Dx @ us + Dy @ vs) / self.dt
        B = np.zeros((n + 1, n + 1))
        B[:n, :n] = self.L
        B[:n, n] = 1.0
        B[n, :n] = 1.0
        sol = np.linalg.solve(B, np.concatenate([rhs, [0.0]]))
        phi = sol[:n]
        return us - self.dt * Dx @ phi, vs - self.dt * Dy @ phi, phi - self.c * self.L @ phi


def test_dense_formulation_of_two_steps():
    """Oracle steps vs the dense formulation on an 8 x 8 periodic lattice (the smallest whose
    box is wider than twice the largest grown support, which minimum-image neighbour search
    needs), from a Taylor-Green state plus a seeded perturbation, two steps (AB2 with a real
    N^(n-1) on the second)."""
    spec = ns.periodic_lattice(8)
    dt, Re = 0.05, 10.0
    u0, v0, p0 = ns.taylor_green_initial(spec.xy)
    rng = np.random.default_rng(4)
    u0 = u0 + 0.1 * rng.standard_normal(spec.n)
    v0 = v0 + 0.1 * rng.standard_normal(spec.n)
    ops = operators.Operators(operators.Problem(**spec.as_kwargs()))
    st = step.Stepper(ops, dt, Re)
    dense = _DenseScheme(spec, dt, Re)
    a = (u0, v0, p0)
    b = (u0, v0, p0)
    for _ in range(2):
        a = st.step(*a)
        b = dense.step(*b)
        for x, y in zip(a, b):
            err = np.abs(x - y).max() / np.abs(y).max()
            assert err < 1e-12, err


# ---- projection identity (eqs. 13-14 with the MLS Laplacian) -------------------------------------

@pytest.mark.parametrize("case", ["periodic", "cavity", "cylinder"])
def test_projection_identity(case):
    if case == "periodic":
        spec = ns.periodic_lattice(16)
        u, v, p = ns.taylor_green_initial(spec.xy)
        dt, Re = 0.01, 10.0
    elif case == "cavity":
        spec = ns.lid_cavity(17)
        u, v, p = ns.boundary_initial(spec, (0.0, 0.0))
        dt, Re = 0.01, 100.0
    else:
        spec = ns.cylinder_channel(0.25, box=(-2.0, 4.0, -2.0, 2.0), n_surface=24)
        u, v, p = ns.boundary_initial(spec, (1.0, 0.0))
        dt, Re = 0.02, 100.0
    ops = operators.Operators(operators.Problem(**spec.as_kwargs()))
    st = step.Stepper(ops, dt, Re)
    for _ in range(2):
        u, v, p = st.step(u, v, p)
    phi = st.last["phi"]
    inner = ops.interior_mask
    lhs = ops.divergence(u, v)[inner]
    rhs = dt * (ops.L @ phi + st.lam - ops.divergence(ops.ddx(phi), ops.ddy(phi)))[inner]
    scale = np.abs(ops.divergence(st.last["us"], st.last["vs"])).max()
    assert np.abs(lhs - rhs).max() <= 1e-10 * scale, (np.abs(lhs - rhs).max(), scale)
    # and the identity is not trivial: D G differs from the Laplacian (approximate projection)
    assert np.abs(lhs).max() > 1e-6 * scale
