"""Fractional step of the VIP method, plain FP64 (oracle; test infrastructure only).

One step follows eqs. 12-15 of the paper (Section 2, Kim-Moin fractional step
with Adams-Bashforth convection and Crank-Nicolson viscous terms), with every
operator from Section 4 (identity and Laplacian by eq. vip:1, convection,
divergence and gradient by VIP direct differences):

  1. C = 3/2 N(u^n) - 1/2 N(u^(n-1))                      (AB2; first step N^(-1) = N^0)
  2. (I - c Delta) u* = (I + c Delta) u^n - dt C,  c = dt / (2 Re)     (eq. 12 times dt)
     with I -> D^[0,0] (MLS identity) by default, boundary rows replaced by
     the velocity boundary conditions
  3. Delta phi = (1/dt) div u*  with pressure boundary rows            (eq. 13)
  4. u^(n+1) = u* - dt grad phi at interior nodes, u^(n+1) = u* on boundary nodes (eq. 14)
  5. p^(n+1) = phi - c Delta phi                                       (eq. 15, see below)

Linear systems are solved exactly (sparse LU, factorised once per dt and Re),
or, in timing mode, by the plain FP64 Krylov methods of `oracle.krylov`.

Readings of the paper taken here (it states no boundary rows for eqs. 12-13):
* velocity rows: DIRICHLET u = g; SLIP the normal-axis component = g, the other
  has zero normal derivative; OUTLET du/dn = Re p^n n_x, dv/dn = Re p^n n_y
  (traction free with nu = 1/Re); normal derivatives as in `Operators.neumann_rows`;
* pressure rows: dphi/dn = 0 on DIRICHLET and SLIP nodes, phi = 0 on OUTLET nodes;
* singular pressure problems (periodic box, or no outlet so every pressure row
  is of Neumann type): Delta phi has the constants as null space, and the
  discrete right-hand side is in general not in its range.  The system is
  bordered, Delta phi + lambda 1 = b, sum(phi) = 0: lambda removes the part of b
  outside the range uniformly over all rows and phi has zero sum.  (Pinning one
  node instead puts that part at a single node; with the scheme below that made
  the step unstable on small lid-driven boxes.)
* identity "exact" variant: I is the identity matrix instead of D^[0,0].
* pressure update: eq. 12 as printed has no pressure term in r^n (the
  non-incremental Kim-Moin predictor, under which phi approximates the whole
  pressure), while eq. 15 adds p^n, which belongs to the incremental form.
  Together they make p grow by about p at every step.  The predictor is kept
  as printed and eq. 15 is read in the Kim-Moin form
  p^(n+1) = phi^(n+1) - (dt / 2 Re) Delta phi^(n+1).  (The other consistent
  reading, -grad p^n added to r^n with eq. 15 as printed, was weakly unstable
  with these boundary rows on small lid-driven boxes.)
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import krylov
from .operators import DIRICHLET, OUTLET, SLIP

IDENTITY_MLS = 0
IDENTITY_EXACT = 1


def _replace_rows(A, rows, B):
    """Copy of CSR A whose rows `rows` are taken from CSR B."""
    mask = np.zeros(A.shape[0])
    mask[rows] = 1.0
    keep = sp.diags(1.0 - mask)
    take = sp.diags(mask)
    return (keep @ A + take @ B).tocsr()


class Stepper:
    """Time-level state and per-(dt, Re) factorisations for one node set."""

    def __init__(self, ops, dt, Re, identity=IDENTITY_MLS, solver="direct", tol=1e-8,
                 maxiter=200000):
        self.ops = ops
        self.prob = ops.prob
        self.dt = float(dt)
        self.Re = float(Re)
        self.identity = identity
        self.solver = solver
        self.tol = tol
        self.maxiter = maxiter
        self.n_prev = None
        self.last_iters = {}
        self._assemble()

    # ---- matrices --------------------------------------------------------------
    def _assemble(self):
        prob, ops = self.prob, self.ops
        n = prob.n
        c = self.dt / (2.0 * self.Re)
        I_op = sp.identity(n, format="csr") if self.identity == IDENTITY_EXACT else ops.M00
        self.c = c
        self.H_int = (I_op - c * ops.L).tocsr()
        self.R_int = (I_op + c * ops.L).tocsr()
        eye = sp.identity(n, format="csr")
        dn = ops.neumann_rows()
        b, kind, nrm = prob.bnd_idx, prob.bnd_kind, prob.bnd_normal
        # which component is held by a Dirichlet row at each boundary node
        normal_is_y = np.abs(nrm[:, 1]) >= np.abs(nrm[:, 0])
        u_dir = (kind == DIRICHLET) | ((kind == SLIP) & ~normal_is_y)
        v_dir = (kind == DIRICHLET) | ((kind == SLIP) & normal_is_y)
        self.u_dir_rows, self.u_neu_rows = b[u_dir], b[~u_dir]
        self.v_dir_rows, self.v_neu_rows = b[v_dir], b[~v_dir]
        Hu = _replace_rows(self.H_int, self.u_dir_rows, eye)
        self.Hu = _replace_rows(Hu, self.u_neu_rows, dn)
        Hv = _replace_rows(self.H_int, self.v_dir_rows, eye)
        self.Hv = _replace_rows(Hv, self.v_neu_rows, dn)
        # Poisson matrix: Laplacian at interior nodes, boundary rows, optional pin
        out = b[kind == OUTLET]
        neu = b[kind != OUTLET]
        P = _replace_rows(ops.L, neu, dn)
        P = _replace_rows(P, out, eye)
        self.P = P.tocsr()
        self.P.eliminate_zeros()
        self.bordered = prob.singular_pressure()
        if self.bordered:
            one = sp.csr_matrix(np.ones((n, 1)))
            self.P_solve = sp.bmat([[self.P, one], [one.T, None]], format="csr")
        else:
            self.P_solve = self.P
        self._lu = {}

    def _solve(self, name, A, rhs, x0=None):
        if self.solver == "direct":
            if name not in self._lu:
                self._lu[name] = spla.splu(A.tocsc())
            return self._lu[name].solve(rhs)
        x, it, _ = krylov.solve(A, rhs, x0=x0, tol=self.tol, maxiter=self.maxiter)
        self.last_iters[name] = it
        return x

    # ---- pieces of a step ---------------------------------------------------------
    def predictor_rhs(self, u, v, p, cx, cy):
        """Right-hand sides of the two Helmholtz systems (eq. 12 times dt, BC rows)."""
        prob = self.prob
        ru = self.R_int @ u - self.dt * cx
        rv = self.R_int @ v - self.dt * cy
        pos = {int(g): k for k, g in enumerate(prob.bnd_idx)}
        for rows, vec, comp in ((self.u_dir_rows, ru, 0), (self.v_dir_rows, rv, 1)):
            for g in rows:
                vec[g] = prob.bnd_value[pos[int(g)], comp]
        for rows, vec, comp in ((self.u_neu_rows, ru, 0), (self.v_neu_rows, rv, 1)):
            for g in rows:
                k = pos[int(g)]
                if prob.bnd_kind[k] == OUTLET:
                    vec[g] = (2.0 * prob.vip_offset * prob.h * prob.h_scale[g] * self.Re * p[g]
                              * prob.bnd_normal[k, comp])
                else:
                    vec[g] = 0.0
        return ru, rv

    def poisson_rhs(self, us, vs):
        """(1/dt) div u* at interior nodes, 0 on boundary rows (eq. 13)."""
        b = self.ops.divergence(us, vs) / self.dt
        b[self.prob.bnd_idx] = 0.0
        return b

    def poisson_solve(self, b, x0=None):
        """phi of eq. 13; for singular problems also the border multiplier lambda."""
        if self.bordered:
            x0b = None if x0 is None else np.concatenate([x0, [0.0]])
            sol = self._solve("P", self.P_solve, np.concatenate([b, [0.0]]), x0b)
            self.lam = sol[-1]
            return sol[:-1]
        self.lam = 0.0
        return self._solve("P", self.P_solve, b, x0)

    def step(self, u, v, p):
        """Advance (u, v, p) by one step; returns new arrays and phi."""
        ops, prob = self.ops, self.prob
        nx, ny = ops.convection(u, v)
        if self.n_prev is None:
            self.n_prev = (nx, ny)
        cx = 1.5 * nx - 0.5 * self.n_prev[0]
        cy = 1.5 * ny - 0.5 * self.n_prev[1]
        self.n_prev = (nx, ny)
        ru, rv = self.predictor_rhs(u, v, p, cx, cy)
        us = self._solve("Hu", self.Hu, ru)
        vs = self._solve("Hv", self.Hv, rv)
        b = self.poisson_rhs(us, vs)
        phi = self.poisson_solve(b)
        inner = ops.interior_mask
        un = us.copy()
        vn = vs.copy()
        un[inner] = (us - self.dt * ops.ddx(phi))[inner]
        vn[inner] = (vs - self.dt * ops.ddy(phi))[inner]
        pn = phi - self.c * (ops.L @ phi)
        self.last = dict(us=us, vs=vs, b=b, phi=phi, nx=nx, ny=ny)
        return un, vn, pn
