"""Moving-least-squares shape functions, plain FP64 (oracle; test infrastructure only).

This package is the CPU oracle that the HIP path is checked against. Only the
test suite, the smoke entry point and the CPU-baseline leg of the benchmark may
import it; the product library never does.

What is computed (Section 3 of the paper, "Moving Least-Squares Approximation"):

* local polynomial u_m(x, xbar) = sum_k c_k p_k((x - xbar)/rho), with the shifted
  and scaled quadratic basis p = [1, xi, eta, xi^2, xi*eta, eta^2];
* the coefficients minimise J(c) = sum_i Phi((x_i - xbar)/rho) |u_m(x_i, xbar) - u(x_i)|^2
  (the paper prints x where x_i is meant inside Phi);
* derivative approximants D^[a,b] u(xbar) = d^(a,b)_x u_m(x, xbar) at x = xbar,
  i.e. a! b! rho^-(a+b) c_k(a,b)  (the derivative of the local polynomial only,
  no derivative of the weights or of the moment matrix), giving the representation
  D^[a,b] u(xbar) = sum_i u(x_i) Psi_i^[a,b](xbar)  (eq. fmlsrk:2).

Readings of the paper taken here (shared with the HIP path by specification only):
* Phi: the default is the cubic spline; the printed weight (1 - r^((1-r)^2))^4 is
  the alternative.
* Support: x_i belongs to the stencil of xbar iff |x_i - xbar|^2 < rho^2 in FP64.
* Growth: if fewer than `min_neighbours` points fall inside rho, rho is multiplied
  by 1.25, at most twice; still too few is an error.
* Periodic boxes use the minimum image d - L*rint(d/L) per axis.
* Neighbours of an evaluation point are ordered by node index.
"""
import math

import numpy as np
from scipy.spatial import cKDTree

CUBIC_SPLINE = 0
PAPER = 1

# multi-index (a, b) -> position in the basis [1, xi, eta, xi^2, xi*eta, eta^2]
BASIS_INDEX = {(0, 0): 0, (1, 0): 1, (0, 1): 2, (2, 0): 3, (1, 1): 4, (0, 2): 5}

RHO_GROWTH = 1.25
MAX_GROWTH_STEPS = 2


class SingularStencil(RuntimeError):
    """Raised when an evaluation point cannot get a usable local fit."""

    def __init__(self, point_index, message):
        super().__init__(message)
        self.point_index = point_index


def weight(r, kind=CUBIC_SPLINE):
    """Weight Phi as a function of r = |y| (Section 3; cubic spline by default).

    Cubic spline: 2/3 - 4r^2 + 4r^3 for r <= 1/2, 4/3 - 4r + 4r^2 - 4r^3/3 for
    1/2 < r < 1 (evaluated as 4/3 (1 - r)^3, the same polynomial without the
    cancellation near r = 1), else 0.  Paper weight: (1 - r^((1-r)^2))^4 for
    r < 1, else 0.
    """
    r = np.asarray(r, dtype=np.float64)
    out = np.zeros_like(r)
    if kind == CUBIC_SPLINE:
        a = r <= 0.5
        b = (r > 0.5) & (r < 1.0)
        ra, rb = r[a], r[b]
        out[a] = 2.0 / 3.0 - 4.0 * ra ** 2 + 4.0 * ra ** 3
        out[b] = (4.0 / 3.0) * (1.0 - rb) ** 3
    elif kind == PAPER:
        a = r < 1.0
        ra = r[a]
        out[a] = (1.0 - ra ** ((1.0 - ra) ** 2)) ** 4
    else:
        raise ValueError("unknown weight kind %r" % (kind,))
    return out


def basis(xi, eta):
    """Quadratic basis p(xi, eta) = [1, xi, eta, xi^2, xi*eta, eta^2], last axis."""
    xi = np.asarray(xi, dtype=np.float64)
    eta = np.asarray(eta, dtype=np.float64)
    return np.stack([np.ones_like(xi), xi, eta, xi * xi, xi * eta, eta * eta], axis=-1)


def min_image(d, period):
    """Minimum-image displacement per axis; period entries of 0 mean not periodic."""
    d = np.array(d, dtype=np.float64, copy=True)
    for ax in range(2):
        L = period[ax] if period is not None else 0.0
        if L > 0.0:
            d[..., ax] = d[..., ax] - L * np.rint(d[..., ax] / L)
    return d


class NodeSet:
    """Node coordinates plus a candidate-neighbour search structure."""

    def __init__(self, xy, period=(0.0, 0.0)):
        self.xy = np.ascontiguousarray(np.asarray(xy, dtype=np.float64))
        self.period = tuple(float(p) for p in period)
        self.periodic = any(p > 0.0 for p in self.period)
        if self.periodic:
            if not all(p > 0.0 for p in self.period):
                raise ValueError("periodicity must be set on both axes")
            box = np.array(self.period)
            self._tree = cKDTree(np.mod(self.xy, box), boxsize=box)
        else:
            self._tree = cKDTree(self.xy)

    def _query_pts(self, pts):
        if self.periodic:
            return np.mod(pts, np.array(self.period))
        return pts

    def neighbours(self, xbar, radius):
        """Indices j (ascending) with |x_j - xbar|^2 < radius^2 (minimum image).

        `radius` is a scalar or one value per point.
        """
        xbar = np.atleast_2d(np.asarray(xbar, dtype=np.float64))
        radius = np.broadcast_to(np.asarray(radius, dtype=np.float64), (len(xbar),))
        cand = self._tree.query_ball_point(self._query_pts(xbar), radius * (1.0 + 1e-9),
                                           return_sorted=True)
        counts = np.fromiter((len(c) for c in cand), dtype=np.int64, count=len(cand))
        flat = np.fromiter((j for c in cand for j in c), dtype=np.int64, count=int(counts.sum()))
        owner = np.repeat(np.arange(len(xbar)), counts)
        d = min_image(self.xy[flat] - xbar[owner], self.period)
        keep = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] < radius[owner] * radius[owner]
        kept_counts = np.bincount(owner[keep], minlength=len(xbar))
        return np.split(flat[keep], np.cumsum(kept_counts)[:-1])


def stencils(nodes, xbar, rho0, min_neighbours=12):
    """Neighbour lists and support radii for each evaluation point (growth rule); rho0 is one
    radius or one per point (rho(xbar) of Section 3)."""
    xbar = np.asarray(xbar, dtype=np.float64).reshape(-1, 2)
    rho = np.array(np.broadcast_to(np.asarray(rho0, dtype=np.float64), (len(xbar),)))
    if len(xbar) == 0:
        return [], rho
    nb = nodes.neighbours(xbar, rho)
    for _ in range(MAX_GROWTH_STEPS):
        short = np.array([i for i, n in enumerate(nb) if len(n) < min_neighbours], dtype=np.int64)
        if len(short) == 0:
            break
        rho[short] *= RHO_GROWTH
        for i, n in zip(short, nodes.neighbours(xbar[short], rho[short])):
            nb[i] = n
    for i, n in enumerate(nb):
        if len(n) < min_neighbours:
            raise SingularStencil(i, "evaluation point %d has %d < %d neighbours after growth"
                                  % (i, len(n), min_neighbours))
    return nb, rho


def shape_functions(nodes, xbar, rho0, derivs, weight_kind=CUBIC_SPLINE, min_neighbours=12,
                    weight_fn=None, batch=16384):
    """Psi^[a,b]_j(xbar) for every evaluation point in `xbar`.

    Returns (neighbour index lists, rho per point, {(a,b): list of weight arrays}).
    The coefficients are c = M^-1 P^T W u with M = P^T W P (normal equations of
    J), solved per point with numpy.linalg.solve.  Points are processed in
    batches with their neighbour lists padded by zero-weight entries, which add
    nothing to M and receive no weight.  `weight_fn`, if given, replaces Phi
    (used by invariance tests).
    """
    xbar = np.asarray(xbar, dtype=np.float64).reshape(-1, 2)
    nb, rho = stencils(nodes, xbar, rho0, min_neighbours)
    wfun = weight_fn if weight_fn is not None else (lambda r: weight(r, weight_kind))
    out = {d: [None] * len(xbar) for d in derivs}
    for s0 in range(0, len(xbar), batch):
        ids = range(s0, min(s0 + batch, len(xbar)))
        kmax = max(len(nb[i]) for i in ids)
        B = len(ids)
        idx = np.zeros((B, kmax), dtype=np.int64)
        valid = np.zeros((B, kmax), dtype=bool)
        for b, i in enumerate(ids):
            idx[b, :len(nb[i])] = nb[i]
            valid[b, :len(nb[i])] = True
        r = rho[s0:s0 + B]
        d = min_image(nodes.xy[idx] - xbar[s0:s0 + B, None, :], nodes.period) / r[:, None, None]
        P = basis(d[..., 0], d[..., 1])                                   # B x K x 6
        w = np.where(valid, wfun(np.sqrt(d[..., 0] ** 2 + d[..., 1] ** 2)), 0.0)
        M = np.einsum('bki,bk,bkj->bij', P, w, P)                         # B x 6 x 6
        try:
            C = np.linalg.solve(M, np.transpose(P * w[..., None], (0, 2, 1)))  # B x 6 x K
        except np.linalg.LinAlgError:
            bad = next(b for b in range(B) if np.linalg.matrix_rank(M[b]) < 6)
            raise SingularStencil(s0 + bad, "moment matrix singular at evaluation point %d"
                                  % (s0 + bad))
        for (a, bb) in derivs:
            k = BASIS_INDEX[(a, bb)]
            scale = math.factorial(a) * math.factorial(bb) / r ** (a + bb)
            vals = C[:, k, :] * scale[:, None]
            for b, i in enumerate(ids):
                out[(a, bb)][i] = vals[b, :len(nb[i])].copy()
    return nb, rho, out


def moment_condition(nodes, xbar, rho, weight_kind=CUBIC_SPLINE):
    """2-norm condition number of the scaled moment matrix at one point (diagnostic)."""
    idx = nodes.neighbours(np.atleast_2d(xbar), rho)[0]
    d = min_image(nodes.xy[idx] - xbar, nodes.period) / rho
    P = basis(d[:, 0], d[:, 1])
    w = weight(np.hypot(d[:, 0], d[:, 1]), weight_kind)
    return np.linalg.cond(P.T @ (w[:, None] * P))
