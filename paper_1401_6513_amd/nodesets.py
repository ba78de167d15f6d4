"""Seeded synthetic node sets and initial fields shaped like the paper's test cases.

This module only produces input arrays (coordinates, boundary table, initial
fields); it holds none of the method's arithmetic, and both the HIP library and
the CPU checker consume what it returns.

Boundary table conventions (shared with the C ABI):
* `bnd_idx[k]`   node index of boundary entry k;
* `bnd_normal[k]` outward unit normal of the flow domain at that node;
* `bnd_kind[k]`  DIRICHLET (velocity given), SLIP (the velocity component along
  the dominant axis of the normal is given, the other has zero normal
  derivative) or OUTLET (traction free);
* `bnd_value[k]` the prescribed velocity (u, v) (only the held components are read).

Node order: lattice nodes row by row (y outer, x inner), body-surface nodes last.
"""
import math
from dataclasses import dataclass, field

import numpy as np

DIRICHLET = 0
SLIP = 1
OUTLET = 2


@dataclass
class NodeSetSpec:
    name: str
    xy: np.ndarray                      # [N, 2] float64
    h: float
    rho: float
    bnd_idx: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int64))
    bnd_normal: np.ndarray = field(default_factory=lambda: np.zeros((0, 2)))
    bnd_kind: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    bnd_value: np.ndarray = field(default_factory=lambda: np.zeros((0, 2)))
    period: tuple = (0.0, 0.0)
    lattice_shape: tuple = None         # (ny, nx) of the background lattice, if any
    lattice_origin: tuple = None        # (x0, y0)
    n_lattice: int = 0                  # first n_lattice nodes are lattice nodes
    surface: np.ndarray = None          # body surface nodes in order around the body, if any
    h_node: np.ndarray = None           # local node spacing of adaptive sets (None: uniform h)

    @property
    def n(self):
        return len(self.xy)

    def as_kwargs(self):
        """Arguments shared by the library's build call and the checker's problem."""
        kw = dict(xy=self.xy, bnd_idx=self.bnd_idx, bnd_normal=self.bnd_normal,
                  bnd_kind=self.bnd_kind, bnd_value=self.bnd_value, rho=self.rho, h=self.h,
                  period=self.period)
        if self.h_node is not None:
            kw["h_node"] = self.h_node
        return kw


def _lattice(x0, y0, nx, ny, h):
    """Row-major lattice coordinates x0 + i h, y0 + j h (y outer, x inner)."""
    i = np.arange(nx, dtype=np.float64)
    j = np.arange(ny, dtype=np.float64)
    X = x0 + i[None, :] * h
    Y = y0 + j[:, None] * h
    return np.stack([np.broadcast_to(X, (ny, nx)).ravel(), np.broadcast_to(Y, (ny, nx)).ravel()],
                    axis=1).copy()


def periodic_lattice(n, length=2.0 * math.pi, support=2.5):
    """n x n nodes on the periodic box [0, length)^2 (Taylor-Green case)."""
    h = length / n
    xy = _lattice(0.0, 0.0, n, n, h)
    return NodeSetSpec(name="periodic%d" % n, xy=xy, h=h, rho=support * h,
                       period=(length, length), lattice_shape=(n, n),
                       lattice_origin=(0.0, 0.0), n_lattice=n * n)


def box_lattice(nx, ny, x0, x1, y0, y1, side_kind, side_value, name="box", support=2.5):
    """Lattice on [x0,x1]x[y0,y1] with every side node a boundary node.

    side_kind / side_value: dicts keyed by 'left', 'right', 'bottom', 'top'.
    side_value[s] is either a constant (u, v) or a callable (x, y) -> (u, v).
    Corner nodes belong to the left and right sides.
    """
    h = (x1 - x0) / (nx - 1)
    hy = (y1 - y0) / (ny - 1)
    if abs(h - hy) > 1e-12 * h:
        raise ValueError("box_lattice needs equal spacing in x and y")
    xy = _lattice(x0, y0, nx, ny, h)
    I, J = np.meshgrid(np.arange(nx), np.arange(ny))
    I, J = I.ravel(), J.ravel()
    side = np.full(nx * ny, "", dtype=object)
    side[J == 0] = "bottom"
    side[J == ny - 1] = "top"
    side[I == 0] = "left"
    side[I == nx - 1] = "right"
    normals = {"left": (-1.0, 0.0), "right": (1.0, 0.0), "bottom": (0.0, -1.0), "top": (0.0, 1.0)}
    idx = np.flatnonzero(side != "")
    nrm = np.array([normals[s] for s in side[idx]])
    kind = np.array([side_kind[s] for s in side[idx]], dtype=np.int32)
    val = np.zeros((len(idx), 2))
    for k, g in enumerate(idx):
        sv = side_value[side[g]]
        val[k] = sv(xy[g, 0], xy[g, 1]) if callable(sv) else sv
    return NodeSetSpec(name=name, xy=xy, h=h, rho=support * h, bnd_idx=idx.astype(np.int64),
                       bnd_normal=nrm, bnd_kind=kind, bnd_value=val,
                       lattice_shape=(ny, nx), lattice_origin=(x0, y0), n_lattice=nx * ny)


def lid_cavity(n, lid=1.0):
    """Lid-driven unit square cavity with n x n nodes; lid y = 1 moves with u = lid."""
    sides = {s: DIRICHLET for s in ("left", "right", "bottom", "top")}
    vals = {"left": (0.0, 0.0), "right": (0.0, 0.0), "bottom": (0.0, 0.0), "top": (lid, 0.0)}
    return box_lattice(n, n, 0.0, 1.0, 0.0, 1.0, sides, vals, name="cavity%d" % n)


def body_radius_circle(theta):
    return np.full_like(np.asarray(theta, dtype=np.float64), 0.5)


def body_radius_bumpy(theta, amp=0.05, lobes=12):
    """r(theta) = 0.5 (1 + amp sin(lobes theta)) (bumpy cylinder)."""
    return 0.5 * (1.0 + amp * np.sin(lobes * np.asarray(theta, dtype=np.float64)))


def _body_radius_derivative(theta, shape):
    if shape in ("circle", None):
        return np.zeros_like(theta)
    amp, lobes = shape
    return 0.5 * amp * lobes * np.cos(lobes * theta)


def cylinder_channel(h, box=(-10.0, 20.0, -10.0, 10.0), shape="circle", n_surface=256,
                     u_inf=1.0, gap=0.25, support=2.5, name=None):
    """Flow past a body in a box: lattice nodes outside the body plus surface nodes.

    shape: "circle" (radius 0.5) or (amp, lobes) for r = 0.5 (1 + amp sin(lobes theta)).
    Lattice nodes closer than gap*h (radially) to the body surface are dropped.
    Inlet x = x0: DIRICHLET (u_inf, 0); outlet x = x1: OUTLET; y = y0, y1: SLIP
    with v = 0; corners belong to the inlet and outlet; the body: DIRICHLET (0, 0).
    """
    x0, x1, y0, y1 = box
    nx = int(round((x1 - x0) / h)) + 1
    ny = int(round((y1 - y0) / h)) + 1
    xy = _lattice(x0, y0, nx, ny, h)
    I = np.tile(np.arange(nx), ny)
    J = np.repeat(np.arange(ny), nx)
    rfun = body_radius_circle if shape == "circle" else (
        lambda t: body_radius_bumpy(t, amp=shape[0], lobes=shape[1]))
    r = np.hypot(xy[:, 0], xy[:, 1])
    th = np.arctan2(xy[:, 1], xy[:, 0])
    keep = r >= rfun(th) + gap * h
    xy, I, J = xy[keep], I[keep], J[keep]
    n_lat = len(xy)
    # box boundary (lattice nodes on the sides)
    side_inlet = I == 0
    side_outlet = I == nx - 1
    side_bottom = (J == 0) & ~side_inlet & ~side_outlet
    side_top = (J == ny - 1) & ~side_inlet & ~side_outlet
    b_idx, b_nrm, b_kind, b_val = [], [], [], []
    for mask, nrm, kind, val in ((side_inlet, (-1.0, 0.0), DIRICHLET, (u_inf, 0.0)),
                                 (side_outlet, (1.0, 0.0), OUTLET, (0.0, 0.0)),
                                 (side_bottom, (0.0, -1.0), SLIP, (0.0, 0.0)),
                                 (side_top, (0.0, 1.0), SLIP, (0.0, 0.0))):
        ids = np.flatnonzero(mask)
        b_idx.append(ids)
        b_nrm.append(np.tile(nrm, (len(ids), 1)))
        b_kind.append(np.full(len(ids), kind, np.int32))
        b_val.append(np.tile(val, (len(ids), 1)))
    # body surface nodes at equal angles
    theta = 2.0 * math.pi * np.arange(n_surface) / n_surface
    rs = rfun(theta)
    sxy = np.stack([rs * np.cos(theta), rs * np.sin(theta)], axis=1)
    drs = _body_radius_derivative(theta, shape)
    # gradient of F = |x| - r(theta) in polar components: e_r - r'(theta)/|x| e_theta
    er = np.stack([np.cos(theta), np.sin(theta)], axis=1)
    et = np.stack([-np.sin(theta), np.cos(theta)], axis=1)
    g = er - (drs / rs)[:, None] * et
    snrm = -g / np.linalg.norm(g, axis=1)[:, None]          # outward of the fluid domain
    s_ids = n_lat + np.arange(n_surface)
    b_idx.append(s_ids)
    b_nrm.append(snrm)
    b_kind.append(np.full(n_surface, DIRICHLET, np.int32))
    b_val.append(np.zeros((n_surface, 2)))
    xy = np.concatenate([xy, sxy])
    if name is None:
        name = "cylinder_h%g" % h if shape == "circle" else "bumpy_h%g" % h
    return NodeSetSpec(name=name, xy=xy, h=h, rho=support * h,
                       bnd_idx=np.concatenate(b_idx).astype(np.int64),
                       bnd_normal=np.concatenate(b_nrm), bnd_kind=np.concatenate(b_kind),
                       bnd_value=np.concatenate(b_val), lattice_shape=(ny, nx),
                       lattice_origin=(x0, y0), n_lattice=n_lat, surface=s_ids.astype(np.int64))


def taylor_green_initial(xy):
    """u = -cos x sin y, v = sin x cos y, p = -(cos 2x + cos 2y)/4 (Taylor-Green at t = 0)."""
    x, y = xy[:, 0], xy[:, 1]
    return (-np.cos(x) * np.sin(y), np.sin(x) * np.cos(y),
            -0.25 * (np.cos(2.0 * x) + np.cos(2.0 * y)))


def boundary_initial(spec, interior_u=(0.0, 0.0)):
    """Uniform interior velocity, boundary nodes at their prescribed values, p = 0."""
    n = spec.n
    u = np.full(n, float(interior_u[0]))
    v = np.full(n, float(interior_u[1]))
    held_u = (spec.bnd_kind == DIRICHLET) | ((spec.bnd_kind == SLIP) &
                                             (np.abs(spec.bnd_normal[:, 1]) < np.abs(spec.bnd_normal[:, 0])))
    held_v = (spec.bnd_kind == DIRICHLET) | ((spec.bnd_kind == SLIP) &
                                             (np.abs(spec.bnd_normal[:, 1]) >= np.abs(spec.bnd_normal[:, 0])))
    u[spec.bnd_idx[held_u]] = spec.bnd_value[held_u, 0]
    v[spec.bnd_idx[held_v]] = spec.bnd_value[held_v, 1]
    return u, v, np.zeros(n)


def random_field(n, seed, low=-1.0, high=1.0):
    """Seeded uniform test vector."""
    return np.random.default_rng(seed).uniform(low, high, n)


def jittered(spec, frac, seed):
    """Copy of a node set with interior nodes moved by up to frac*h per axis (seeded)."""
    rng = np.random.default_rng(seed)
    xy = spec.xy.copy()
    movable = np.ones(spec.n, bool)
    movable[spec.bnd_idx] = False
    xy[movable] += rng.uniform(-frac * spec.h, frac * spec.h, (int(movable.sum()), 2))
    out = NodeSetSpec(**{**spec.__dict__})
    out.xy = xy
    out.name = spec.name + "_jit"
    return out


def refined_cylinder_channel(h_fine, zones, box=(-10.0, 20.0, -10.0, 10.0), shape="circle",
                             n_surface=256, u_inf=1.0, gap=0.25, support=2.5, name=None):
    """Flow past a body on a stepwise refined node distribution (Section 5.5 places its nodes
    in nested regions of decreasing density around the bumpy cylinder).

    zones: nested boxes (x0, x1, y0, y1), finest first.  A point of the finest lattice
    (spacing h_fine) inside zone k but no finer zone has spacing h_fine 2^k and is kept when
    both its lattice indices are multiples of 2^k; points outside every zone have spacing
    h_fine 2^len(zones).  The box sides must lie on the coarsest lattice.  Boundary conditions,
    the body and its surface nodes are those of cylinder_channel (shape None: no body, a plain
    channel).  h_node holds each node's
    spacing (surface nodes: h_fine); the support radius of an evaluation point is
    `support` times the spacing of the node it belongs to.
    """
    x0, x1, y0, y1 = box
    L = len(zones)
    step = h_fine * 2 ** L
    for v, o in ((x1, x0), (y1, y0)):
        if abs((v - o) / step - round((v - o) / step)) > 1e-9:
            raise ValueError("box sides must lie on the coarsest lattice")
    nx = int(round((x1 - x0) / h_fine)) + 1
    ny = int(round((y1 - y0) / h_fine)) + 1
    i = np.arange(nx)
    j = np.arange(ny)
    I = np.tile(i, ny)
    J = np.repeat(j, nx)
    X = x0 + I * h_fine
    Y = y0 + J * h_fine
    level = np.full(len(X), L, dtype=np.int64)
    for k in range(L - 1, -1, -1):
        zx0, zx1, zy0, zy1 = zones[k]
        inside = (X >= zx0 - 1e-12) & (X <= zx1 + 1e-12) & (Y >= zy0 - 1e-12) & (Y <= zy1 + 1e-12)
        level[inside] = k
    m = 2 ** level
    keep = (I % m == 0) & (J % m == 0)
    if shape is None:
        n_surface = 0
    rfun = body_radius_circle if shape in ("circle", None) else (
        lambda t: body_radius_bumpy(t, amp=shape[0], lobes=shape[1]))
    if shape is not None:
        r = np.hypot(X, Y)
        th = np.arctan2(Y, X)
        keep &= r >= rfun(th) + gap * h_fine
    xy = np.stack([X[keep], Y[keep]], axis=1)
    I, J, hn = I[keep], J[keep], h_fine * m[keep].astype(np.float64)
    n_lat = len(xy)
    side_inlet = I == 0
    side_outlet = I == nx - 1
    side_bottom = (J == 0) & ~side_inlet & ~side_outlet
    side_top = (J == ny - 1) & ~side_inlet & ~side_outlet
    b_idx, b_nrm, b_kind, b_val = [], [], [], []
    for mask, nrm, kind, val in ((side_inlet, (-1.0, 0.0), DIRICHLET, (u_inf, 0.0)),
                                 (side_outlet, (1.0, 0.0), OUTLET, (0.0, 0.0)),
                                 (side_bottom, (0.0, -1.0), SLIP, (0.0, 0.0)),
                                 (side_top, (0.0, 1.0), SLIP, (0.0, 0.0))):
        ids = np.flatnonzero(mask)
        b_idx.append(ids)
        b_nrm.append(np.tile(nrm, (len(ids), 1)))
        b_kind.append(np.full(len(ids), kind, np.int32))
        b_val.append(np.tile(val, (len(ids), 1)))
    theta = 2.0 * math.pi * np.arange(n_surface) / n_surface
    rs = rfun(theta)
    sxy = np.stack([rs * np.cos(theta), rs * np.sin(theta)], axis=1)
    drs = _body_radius_derivative(theta, shape)
    er = np.stack([np.cos(theta), np.sin(theta)], axis=1)
    et = np.stack([-np.sin(theta), np.cos(theta)], axis=1)
    g = er - (drs / rs)[:, None] * et
    snrm = -g / np.linalg.norm(g, axis=1)[:, None]
    s_ids = n_lat + np.arange(n_surface)
    b_idx.append(s_ids)
    b_nrm.append(snrm)
    b_kind.append(np.full(n_surface, DIRICHLET, np.int32))
    b_val.append(np.zeros((n_surface, 2)))
    xy = np.concatenate([xy, sxy])
    hn = np.concatenate([hn, np.full(n_surface, h_fine)])
    if name is None:
        name = "refined_h%g_L%d" % (h_fine, L)
    return NodeSetSpec(name=name, xy=xy, h=h_fine, rho=support * h_fine,
                       bnd_idx=np.concatenate(b_idx).astype(np.int64),
                       bnd_normal=np.concatenate(b_nrm), bnd_kind=np.concatenate(b_kind),
                       bnd_value=np.concatenate(b_val), n_lattice=n_lat,
                       surface=s_ids.astype(np.int64), h_node=hn)


def triangle_cavity(h, lid=1.0, gap=0.25, support=2.5):
    """Equilateral triangle of side 1, horizontal lid on top, apex down.

    Vertices (0, H), (1, H), (0.5, 0) with H = sqrt(3)/2.  Boundary nodes sit
    on the edges at spacing close to h (vertices once each); lattice nodes
    x = i h, y = j h strictly inside and at least gap*h from every edge.  The
    lid (top edge, corners excluded) moves with u = lid; the other edges and
    the three corners are walls.
    """
    H = math.sqrt(3.0) / 2.0
    verts = np.array([[0.0, H], [1.0, H], [0.5, 0.0]])
    # edges (a, b, outward normal, kind value)
    edges = [(verts[0], verts[1], np.array([0.0, 1.0]), (lid, 0.0)),
             (verts[1], verts[2], np.array([H, -0.5]), (0.0, 0.0)),
             (verts[2], verts[0], np.array([-H, -0.5]), (0.0, 0.0))]
    nx = int(round(1.0 / h)) + 1
    ny = int(round(H / h)) + 1
    lat = _lattice(0.0, 0.0, nx, ny, h)
    inside = np.ones(len(lat), bool)
    for a, b, nrm, _ in edges:
        inside &= (lat - a) @ nrm <= -gap * h     # signed distance to the edge line
    lat = lat[inside]
    n_lat = len(lat)
    bxy, bn, bv = [], [], []
    m = int(round(1.0 / h))
    corner_normals = [np.array([-H, 0.5]), np.array([H, 0.5]), np.array([0.0, -1.0])]
    for k, (a, b, nrm, val) in enumerate(edges):
        # the corner at the start of each edge, then the edge interior
        bxy.append(a)
        cn = corner_normals[k]
        bn.append(cn / np.linalg.norm(cn))
        bv.append((0.0, 0.0))
        t = np.arange(1, m) / m
        pts = a[None, :] + t[:, None] * (b - a)[None, :]
        bxy.extend(pts)
        bn.extend([nrm] * len(pts))
        bv.extend([val] * len(pts))
    bxy = np.array(bxy)
    xy = np.concatenate([lat, bxy])
    nb = len(bxy)
    return NodeSetSpec(name="triangle_h%g" % h, xy=xy, h=h, rho=support * h,
                       bnd_idx=n_lat + np.arange(nb, dtype=np.int64), bnd_normal=np.array(bn),
                       bnd_kind=np.zeros(nb, np.int32), bnd_value=np.array(bv, dtype=np.float64),
                       n_lattice=n_lat)
