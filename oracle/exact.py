"""Closed-form solutions of the incompressible Navier-Stokes equations (oracle; tests only).

* Taylor decaying vortices (Section 5.1 of the paper).  The paper prints
  p = -1/4 [cos 2x + cos y] e^{-4t} for nu = 1; substituting into eq. 1 fixes the
  second term to cos 2y (the convective term u du/dx = -1/2 sin 2x e^{-4t} must be
  balanced by -dp/dx, and symmetrically in y).  With nu = 1/Re the decay rates
  are e^{-2t/Re} for velocity and e^{-4t/Re} for pressure.
* Kovasznay flow (a steady exact solution used only to pin Dirichlet boundary
  handling): lambda = Re/2 - sqrt(Re^2/4 + 4 pi^2), u = 1 - e^{lambda x} cos 2 pi y,
  v = lambda/(2 pi) e^{lambda x} sin 2 pi y, p = (1 - e^{2 lambda x}) / 2.
"""
import numpy as np


def taylor_green(xy, t, Re):
    x, y = xy[:, 0], xy[:, 1]
    fu = np.exp(-2.0 * t / Re)
    fp = np.exp(-4.0 * t / Re)
    u = -np.cos(x) * np.sin(y) * fu
    v = np.sin(x) * np.cos(y) * fu
    p = -0.25 * (np.cos(2.0 * x) + np.cos(2.0 * y)) * fp
    return u, v, p


def kovasznay_lambda(Re):
    return Re / 2.0 - np.sqrt(Re * Re / 4.0 + 4.0 * np.pi * np.pi)


def kovasznay(xy, Re):
    lam = kovasznay_lambda(Re)
    x, y = xy[:, 0], xy[:, 1]
    e = np.exp(lam * x)
    u = 1.0 - e * np.cos(2.0 * np.pi * y)
    v = lam / (2.0 * np.pi) * e * np.sin(2.0 * np.pi * y)
    p = 0.5 * (1.0 - np.exp(2.0 * lam * x))
    return u, v, p
