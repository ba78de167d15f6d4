"""Discrete VIP operators as SciPy CSR matrices, plain FP64 (oracle; test infrastructure only).

Builds, from a node set and its boundary table, every linear operator the
fractional step uses (Section 4 of the paper, "Implementation using Virtual
Interpolation Point"):

* identity and Laplacian at each node, I = D^[0,0] and Delta = D^[2,0] + D^[0,2]
  (eq. vip:1), both evaluated at the node itself;
* Neumann rows at boundary nodes (the paper states no boundary rows): the
  normal derivative is taken, in the manner of the VIP direct differences, from
  values interpolated by Psi^[0,0] at two virtual points on the inward normal,
  df/dn(x_b) = (3 f(x_b) - 4 f(x_b - d n_b) + f(x_b - 2 d n_b)) / (2 d) with
  d = vip_offset * h (exact for quadratics).  (The diffuse derivative
  n . (D^[1,0], D^[0,1]) at the node itself gave Poisson matrices with
  eigenvalues of both signs of real part on body-fitted node sets, on which the
  Krylov methods broke down; a two-point difference was only first order.)
* for each interior node its four virtual interpolation points e, w, n, s and the
  interpolation rows u(x_vip) = sum_j Psi_j^[0,0](x_vip) u_j (Section 4.1), with
  the spacings |x_e - x_w| and |x_n - x_s| used by the direct differences.

Readings of the paper taken here:
* VIPs sit at x_i +- (o, 0) and x_i +- (0, o) with o = vip_offset * h_i (Fig. 1 is
  missing from the text; half the node's spacing by default).
* The support radius rho(xbar) of Section 3 depends on the evaluation point: on stepwise
  adaptive node sets it is rho h_i / h for a point belonging to node i (the node, its VIPs,
  or the inner Neumann points of a boundary node), with h_i that node's local spacing.
* Near the boundary (the paper only says a "technical problem" can arise there):
  for each VIP, take the boundary node nearest to the VIP among the boundary
  nodes within rho of x_i (ties: lowest index); if the VIP lies strictly on the
  outer side of that node's tangent line, n_b . (x_vip - x_b) > 0, move it along
  its axis onto the tangent line, never past x_i.
* Boundary kinds: DIRICHLET (velocity given; dphi/dn = 0), SLIP (the velocity
  component along the dominant axis of the normal is given, the other has zero
  normal derivative; dphi/dn = 0), OUTLET (traction free: du/dn = Re p n_x,
  dv/dn = Re p n_y with p lagged; phi = 0).
"""
import numpy as np
import scipy.sparse as sp
from scipy.spatial import cKDTree

from . import mls

DIRICHLET = 0
SLIP = 1
OUTLET = 2

# order of the four virtual interpolation points
VIP_NAMES = ("e", "w", "n", "s")
VIP_DIRS = np.array([[1.0, 0.0], [-1.0, 0.0], [0.0, 1.0], [0.0, -1.0]])


class Problem:
    """Node set, boundary table and discretisation parameters (inputs only)."""

    def __init__(self, xy, bnd_idx=(), bnd_normal=(), bnd_kind=(), bnd_value=(), rho=None, h=None,
                 period=(0.0, 0.0), vip_offset=0.5, weight_kind=mls.CUBIC_SPLINE,
                 min_neighbours=12, h_node=None):
        self.xy = np.ascontiguousarray(np.asarray(xy, dtype=np.float64))
        self.n = len(self.xy)
        self.bnd_idx = np.asarray(bnd_idx, dtype=np.int64).reshape(-1)
        nb = len(self.bnd_idx)
        self.bnd_normal = np.asarray(bnd_normal, dtype=np.float64).reshape(nb, 2)
        self.bnd_kind = np.asarray(bnd_kind, dtype=np.int32).reshape(nb)
        self.bnd_value = np.asarray(bnd_value, dtype=np.float64).reshape(nb, 2)
        self.rho = float(rho)
        self.h = float(h)
        # local spacing of each node (stepwise adaptive sets); the support radius of an
        # evaluation point is rho h_i / h with i the node it belongs to (the node itself, the
        # owner of a VIP, or the boundary node of a Neumann point), its VIP offset
        # vip_offset h_i and its Neumann distance vip_offset h_b
        self.h_node = (np.full(self.n, self.h) if h_node is None
                       else np.asarray(h_node, dtype=np.float64).reshape(self.n).copy())
        self.h_scale = np.ones(self.n) if h_node is None else self.h_node / self.h
        self.rho_node0 = self.rho * self.h_scale
        self.period = tuple(float(p) for p in period)
        self.vip_offset = float(vip_offset)
        self.weight_kind = int(weight_kind)
        self.min_neighbours = int(min_neighbours)
        self.is_boundary = np.zeros(self.n, dtype=bool)
        self.is_boundary[self.bnd_idx] = True
        self.interior = np.flatnonzero(~self.is_boundary)
        self.periodic = any(p > 0 for p in self.period)

    def singular_pressure(self):
        """Pressure rows all of Neumann type (no outlet) or periodic: constants in the null space."""
        return self.periodic or not np.any(self.bnd_kind == OUTLET)


def vip_points(prob):
    """VIP coordinates [n_interior, 4, 2] (order e, w, n, s) after boundary clipping."""
    oi = (prob.vip_offset * prob.h) * prob.h_scale[prob.interior]
    ri = prob.rho_node0[prob.interior]
    xi = prob.xy[prob.interior]
    pts = xi[:, None, :] + oi[:, None, None] * VIP_DIRS[None, :, :]
    if len(prob.bnd_idx) == 0:
        return pts
    bxy = prob.xy[prob.bnd_idx]
    tree = cKDTree(bxy)
    cand = tree.query_ball_point(xi, ri * (1.0 + 1e-9), return_sorted=True)
    for r, c in enumerate(cand):
        if not c:
            continue
        o = oi[r]
        c = np.asarray(c, dtype=np.int64)
        d0 = bxy[c] - xi[r]
        c = c[d0[:, 0] * d0[:, 0] + d0[:, 1] * d0[:, 1] < ri[r] * ri[r]]
        if len(c) == 0:
            continue
        # nearest boundary node by bnd_idx order (ties -> lowest boundary-table index)
        for k in range(4):
            dv = bxy[c] - pts[r, k]
            d2 = dv[:, 0] * dv[:, 0] + dv[:, 1] * dv[:, 1]
            b = c[int(np.argmin(d2))]   # argmin returns the first (lowest-index) minimum
            nrm = prob.bnd_normal[b]
            side = nrm[0] * (pts[r, k, 0] - bxy[b, 0]) + nrm[1] * (pts[r, k, 1] - bxy[b, 1])
            if side > 0.0:
                ndir = nrm[0] * VIP_DIRS[k, 0] + nrm[1] * VIP_DIRS[k, 1]
                t = (nrm[0] * (bxy[b, 0] - xi[r, 0]) + nrm[1] * (bxy[b, 1] - xi[r, 1])) / ndir
                t = min(max(t, 0.0), o)
                pts[r, k] = xi[r] + t * VIP_DIRS[k]
    return pts


def _csr(rows, nbrs, vals, n):
    if len(rows) == 0:
        return sp.csr_matrix((n, n))
    indptr = np.zeros(n + 1, dtype=np.int64)
    for r, nb in zip(rows, nbrs):
        indptr[r + 1] = len(nb)
    indptr = np.cumsum(indptr)
    order = np.argsort(np.asarray(rows), kind="stable")
    cols = np.concatenate([nbrs[i] for i in order]) if len(rows) else np.zeros(0, np.int64)
    data = np.concatenate([vals[i] for i in order]) if len(rows) else np.zeros(0)
    return sp.csr_matrix((data, cols, indptr), shape=(n, n))


class Operators:
    """All FP64 operators of one node set (built once)."""

    def __init__(self, prob):
        self.prob = prob
        n = prob.n
        nodes = mls.NodeSet(prob.xy, prob.period)
        if prob.periodic:
            assert 2.0 * prob.rho_node0.max() * mls.RHO_GROWTH ** mls.MAX_GROWTH_STEPS < min(prob.period)
        kw = dict(weight_kind=prob.weight_kind, min_neighbours=prob.min_neighbours)
        allrows = np.arange(n)
        nb, self.rho_node, psi = mls.shape_functions(
            nodes, prob.xy, prob.rho_node0, [(0, 0), (2, 0), (0, 2)], **kw)
        self.node_nbrs = nb
        self.M00 = _csr(allrows, nb, psi[(0, 0)], n)
        lap = [a + b for a, b in zip(psi[(2, 0)], psi[(0, 2)])]
        self.L = _csr(allrows, nb, lap, n)
        # inner points of the Neumann rows
        d = (prob.vip_offset * prob.h) * prob.h_scale[prob.bnd_idx]
        self.normal_xy = [prob.xy[prob.bnd_idx] - m * d[:, None] * prob.bnd_normal for m in (1.0, 2.0)]
        self.NB = []
        for pts in self.normal_xy:
            bnb, _, bpsi = mls.shape_functions(nodes, pts, prob.rho_node0[prob.bnd_idx], [(0, 0)],
                                               **kw)
            self.NB.append(_csr(prob.bnd_idx, bnb, bpsi[(0, 0)], n))
        # virtual interpolation points of interior nodes
        self.vip_xy = vip_points(prob)
        self.VIP = []
        self.rho_vip = []
        for k in range(4):
            vnb, vrho, vpsi = mls.shape_functions(nodes, self.vip_xy[:, k, :],
                                                  prob.rho_node0[prob.interior], [(0, 0)], **kw)
            self.VIP.append(_csr(prob.interior, vnb, vpsi[(0, 0)], n))
            self.rho_vip.append(vrho)
        self.d_ew = np.ones(n)
        self.d_ns = np.ones(n)
        dx = self.vip_xy[:, 0, :] - self.vip_xy[:, 1, :]
        dy = self.vip_xy[:, 2, :] - self.vip_xy[:, 3, :]
        self.d_ew[prob.interior] = np.sqrt(dx[:, 0] ** 2 + dx[:, 1] ** 2)
        self.d_ns[prob.interior] = np.sqrt(dy[:, 0] ** 2 + dy[:, 1] ** 2)
        self.interior_mask = ~prob.is_boundary

    # ---- VIP direct differences (Section 4.1, items 1-3) -------------------------
    def vip_values(self, f):
        """[4, n] values of a nodal field at the VIPs (zero on boundary rows)."""
        return np.stack([V @ f for V in self.VIP])

    def ddx(self, f):
        """(f(x_e) - f(x_w)) / |x_e - x_w| at interior nodes, 0 on boundary rows."""
        return (self.VIP[0] @ f - self.VIP[1] @ f) / self.d_ew

    def ddy(self, f):
        """(f(x_n) - f(x_s)) / |x_n - x_s| at interior nodes, 0 on boundary rows."""
        return (self.VIP[2] @ f - self.VIP[3] @ f) / self.d_ns

    def divergence(self, u, v):
        return self.ddx(u) + self.ddy(v)

    def convection(self, u, v):
        """VIP convection flux of Section 4.1 item 1, squares of interpolated values."""
        ue, uw, un, us = self.vip_values(u)
        ve, vw, vn, vs = self.vip_values(v)
        nx = (ue * ue - uw * uw) / self.d_ew + (un * vn - us * vs) / self.d_ns
        ny = (ue * ve - uw * vw) / self.d_ew + (vn * vn - vs * vs) / self.d_ns
        return nx, ny

    def neumann_rows(self):
        """Rows 3 e_b - 4 Psi^[0,0](x_b - d n_b) + Psi^[0,0](x_b - 2 d n_b) at boundary nodes.

        Row b applied to f gives 2 d_b times the normal derivative of f at x_b
        (d_b = vip_offset * h_b); rows of non-boundary nodes are empty.
        """
        n = self.prob.n
        ind = np.zeros(n)
        ind[self.prob.bnd_idx] = 3.0
        return (sp.diags(ind) - 4.0 * self.NB[0] + self.NB[1]).tocsr()
