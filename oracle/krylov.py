"""Plain FP64 Krylov solvers with a Jacobi preconditioner (oracle; test infrastructure only).

The paper names no linear solver for eqs. 12-13.  The oracle solves them
exactly (sparse LU) for parity; these textbook methods give the timing-mode
solve of the same systems and a second route for tests:

* preconditioned conjugate gradients (Hestenes-Stiefel with a diagonal
  preconditioner) for symmetric systems;
* preconditioned BiCGStab (van der Vorst) otherwise.

Convergence is judged on the true FP64 residual |b - A x|_2 / |b|_2 <= tol.
"""
import numpy as np


def _dinv(A):
    d = A.diagonal().astype(np.float64)
    return np.where(d != 0.0, 1.0 / np.where(d != 0.0, d, 1.0), 1.0)


def pcg(A, b, x0=None, tol=1e-8, maxiter=100000):
    dinv = _dinv(A)
    x = np.zeros_like(b) if x0 is None else x0.astype(np.float64).copy()
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return np.zeros_like(b), 0, 0.0
    r = b - A @ x
    z = dinv * r
    p = z.copy()
    rz = r @ z
    it = 0
    while it < maxiter:
        if np.linalg.norm(r) <= tol * bn:
            rt = np.linalg.norm(b - A @ x)
            if rt <= tol * bn:
                return x, it, rt / bn
            r = b - A @ x           # recurrence drifted: restart from the true residual
            z = dinv * r
            p = z.copy()
            rz = r @ z
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        z = dinv * r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
    return x, it, np.linalg.norm(b - A @ x) / bn


def bicgstab(A, b, x0=None, tol=1e-8, maxiter=100000):
    dinv = _dinv(A)
    x = np.zeros_like(b) if x0 is None else x0.astype(np.float64).copy()
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return np.zeros_like(b), 0, 0.0

    def restart():
        r = b - A @ x
        return r, r.copy(), 1.0, 1.0, 1.0, np.zeros_like(b), np.zeros_like(b)

    r, rhat, rho, alpha, omega, v, p = restart()
    it = 0
    while it < maxiter:
        if np.linalg.norm(r) <= tol * bn:
            rt = np.linalg.norm(b - A @ x)
            if rt <= tol * bn:
                return x, it, rt / bn
            r, rhat, rho, alpha, omega, v, p = restart()
        rho_new = rhat @ r
        if rho_new == 0.0 or omega == 0.0 or not np.isfinite(rho_new):
            # breakdown: restart from the true residual with a fresh shadow vector
            r, rhat, rho, alpha, omega, v, p = restart()
            rho_new = rhat @ r
        beta = (rho_new / rho) * (alpha / omega)
        p = r + beta * (p - omega * v)
        ph = dinv * p
        v = A @ ph
        rv = rhat @ v
        if rv == 0.0 or not np.isfinite(rv):
            r, rhat, rho, alpha, omega, v, p = restart()
            it += 1
            continue
        alpha = rho_new / rv
        s = r - alpha * v
        sh = dinv * s
        t = A @ sh
        tt = t @ t
        omega = (t @ s) / tt if tt > 0.0 else 0.0
        x += alpha * ph + omega * sh
        r = s - omega * t
        rho = rho_new
        it += 1
    return x, it, np.linalg.norm(b - A @ x) / bn


def solve(A, b, x0=None, tol=1e-8, maxiter=100000, symmetric=False):
    """PCG when the caller declares A symmetric positive or negative definite, BiCGStab otherwise."""
    if symmetric:
        return pcg(A, b, x0, tol, maxiter)
    return bicgstab(A, b, x0, tol, maxiter)
