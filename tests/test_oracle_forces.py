"""Pins of the oracle's body force (traction on the surface nodes; the drag and lift of the
cylinder cases, Section 5.4) and of its dominant-frequency estimate (Strouhal number), against
closed forms: a linear pressure field, whose force is minus the body area times the pressure
gradient; a quadratic velocity field vanishing on the circle, whose viscous force follows from
the traction t = -p n + nu du/dn that Section 5.4 defines; and pure sinusoids.  On a circle of N equally spaced surface nodes the chord
trapezoid rule gives these integrals exactly as R^2 N sin(pi/N) times the continuum factor
over pi, which is pinned to roundoff; the continuum value is approached as (pi/N)^2/6."""
import numpy as np
import pytest

from oracle import forces, operators
from paper_1401_6513_amd import nodesets as ns

R = 0.5


def _cyl(n_surface):
    spec = ns.cylinder_channel(1.0 / 16, box=(-2.0, 3.0, -2.0, 2.0), n_surface=n_surface)
    ops = operators.Operators(operators.Problem(**spec.as_kwargs()))
    return spec, ops


@pytest.mark.parametrize("nsurf", [48, 64])
def test_pressure_force_of_a_linear_field(nsurf):
    spec, ops = _cyl(nsurf)
    a, b, c = 0.4, -1.3, 0.7
    x, y = spec.xy[:, 0], spec.xy[:, 1]
    p = a + b * x + c * y
    z = np.zeros(spec.n)
    F = forces.body_force(ops, z, z, p, 100.0, spec.surface)
    quad = R * R * nsurf * np.sin(np.pi / nsurf)        # -> pi R^2
    want = -quad * np.array([b, c])
    assert np.abs(F - want).max() <= 1e-12 * np.abs(want).max(), (F, want)
    cont = -np.pi * R * R * np.array([b, c])
    assert np.abs(F - cont).max() <= 1.1 * (np.pi / nsurf) ** 2 / 6 * np.abs(cont).max()


@pytest.mark.parametrize("Re", [1.0, 40.0])
def test_viscous_force_of_a_quadratic_field(Re):
    """u = s (r^2 - R^2), v = q (r^2 - R^2) vanish on the circle; with n = -e_r,
    du/dn = -2 s R, and minus the viscous traction (1/Re) du/dn integrates to
    F = 4 pi R^2 (s, q) / Re.  A constant pressure adds nothing."""
    nsurf = 64
    spec, ops = _cyl(nsurf)
    s, q = 0.8, -0.35
    r2 = spec.xy[:, 0] ** 2 + spec.xy[:, 1] ** 2 - R * R
    F = forces.body_force(ops, s * r2, q * r2, np.full(spec.n, 2.5), Re, spec.surface)
    want = 4.0 * R * R * nsurf * np.sin(np.pi / nsurf) * np.array([s, q]) / Re
    assert np.abs(F - want).max() <= 1e-11 * np.abs(want).max(), (F, want)


def test_force_is_zero_for_uniform_pressure_on_a_bumpy_body():
    spec = ns.cylinder_channel(1.0 / 16, box=(-2.0, 3.0, -2.0, 2.0), shape=(0.05, 12), n_surface=96)
    ops = operators.Operators(operators.Problem(**spec.as_kwargs()))
    z = np.zeros(spec.n)
    F = forces.body_force(ops, z, z, np.full(spec.n, 3.0), 100.0, spec.surface)
    # the chord weights and the shape's normals do not close exactly; the residual is small
    assert np.abs(F).max() < 2e-3 * 3.0


@pytest.mark.parametrize("f0", [0.1637, 0.9, 2.345])
def test_spectral_peak_of_a_sinusoid(f0):
    dt = 0.02
    t = np.arange(5000) * dt
    sig = 0.31 * np.sin(2 * np.pi * f0 * t + 0.4) + 1.33
    f, amp = forces.spectral_peak(sig, dt)
    assert abs(f - f0) <= 1e-4 * f0, (f, f0)
    assert abs(amp - 0.31) <= 5e-3 * 0.31, amp
