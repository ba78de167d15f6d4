"""Body force by surface traction, and the dominant frequency of a signal, plain FP64
(oracle; test infrastructure only).

Force on a body (drag and lift of the cylinder cases, Section 5.4 of the paper).  Section 5.4
defines the traction t = -p n + nu du/dn with n the outward normal (of the flow domain: at a
surface node it points into the body) and nu = 1/Re; the fluid's force on the body is
F = -integral of t dS over the surface.  The paper gives no discrete formula; the reading taken
here: du/dn is the discrete normal derivative of the boundary rows (`Operators.neumann_rows`
divided by 2 d_b, exact for quadratics), and dS is the trapezoid weight of the closed chain of
surface nodes (half the chords to the two neighbours along the chain).

Dominant frequency (Strouhal number of the lift history): maximum of the periodogram of the
mean-removed, Hann-windowed signal, taken here from a 64-times zero-padded FFT with a
parabolic fit through the largest bin and its neighbours.
"""
import numpy as np


def body_force(ops, u, v, p, Re, surf):
    """(F_x, F_y) on the body whose surface nodes, in order around it, are `surf`."""
    prob = ops.prob
    surf = np.asarray(surf, dtype=np.int64)
    two_d = 2.0 * prob.vip_offset * prob.h * prob.h_scale[surf]
    rows = ops.neumann_rows()
    dudn = (rows @ u)[surf] / two_d
    dvdn = (rows @ v)[surf] / two_d
    entry = {int(g): k for k, g in enumerate(prob.bnd_idx)}
    nrm = prob.bnd_normal[[entry[int(i)] for i in surf]]
    xy = prob.xy[surf]
    chord_next = np.linalg.norm(np.roll(xy, -1, axis=0) - xy, axis=1)
    chord_prev = np.linalg.norm(xy - np.roll(xy, 1, axis=0), axis=1)
    w = 0.5 * (chord_next + chord_prev)
    tx = p[surf] * nrm[:, 0] - dudn / Re
    ty = p[surf] * nrm[:, 1] - dvdn / Re
    return np.array([np.sum(w * tx), np.sum(w * ty)])


def spectral_peak(signal, dt, pad=64):
    """(frequency, amplitude) at the periodogram maximum of a sampled signal."""
    s = np.asarray(signal, dtype=np.float64)
    n = len(s)
    k = np.arange(n)
    win = 0.5 * (1.0 - np.cos(2.0 * np.pi * k / (n - 1)))
    x = (s - s.mean()) * win
    m = pad * n
    X = np.fft.rfft(x, m)
    P = np.abs(X) ** 2
    j = 1 + int(np.argmax(P[1:-1]))
    a, b, c = np.log(P[j - 1]), np.log(P[j]), np.log(P[j + 1])
    shift = 0.5 * (a - c) / (a - 2.0 * b + c)
    f = (j + shift) / (m * dt)
    amp = 2.0 * np.abs(np.sum(x * np.exp(-2j * np.pi * f * k * dt))) / win.sum()
    return f, amp
