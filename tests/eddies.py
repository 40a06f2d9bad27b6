"""Eddy centres of a steady cavity flow, for comparison with Tables 1-3 of
arXiv:2306.07603 (Section 6.1).

The stream function psi (u = d psi / dy, v = -d psi / dx) is integrated up
each grid line of constant xi from psi = 0 on the bottom wall.  On the map of
Eq. (3.8.1), y = eta and x_eta = cot(theta) (2 xi - 1), so along such a line
d psi / d eta = u y_eta - v x_eta = u - v cot(theta) (2 xi - 1)
(trapezoid rule).  The primary eddy turns with the lid and is the minimum of
psi; the two bottom-corner eddies turn the other way and are local maxima in
the lower left and lower right parts of the cavity.  Each extremum is refined
by a quadratic fit over its 3 x 3 neighbourhood in (xi, eta) and mapped to
(x, y) by Eq. (3.8.1).
"""
from __future__ import annotations

import math

import numpy as np


def stream_function(u: np.ndarray, v: np.ndarray, theta_deg: float) -> np.ndarray:
    ny, nx = u.shape
    C = 0.0 if theta_deg == 90.0 else 1.0 / math.tan(math.radians(theta_deg))
    xi = np.arange(nx) / (nx - 1)
    deta = 1.0 / (ny - 1)
    integrand = u - v * (C * (2 * xi - 1))[None, :]
    psi = np.zeros_like(u)
    psi[1:] = np.cumsum(0.5 * (integrand[1:] + integrand[:-1]) * deta, axis=0)
    return psi


def to_xy(xi: float, eta: float, theta_deg: float):
    C = 0.0 if theta_deg == 90.0 else 1.0 / math.tan(math.radians(theta_deg))
    return 2 * C * xi * eta + xi - C * eta + C, eta


def _refine(psi: np.ndarray, j: int, i: int):
    ny, nx = psi.shape
    j = min(max(j, 1), ny - 2)
    i = min(max(i, 1), nx - 2)
    w = psi[j - 1:j + 2, i - 1:i + 2]
    # f = a + b x + c y + d x^2 + e y^2 + f xy on the 3x3 stencil (unit spacing)
    X, Y = np.meshgrid([-1.0, 0.0, 1.0], [-1.0, 0.0, 1.0])
    A = np.stack([np.ones(9), X.ravel(), Y.ravel(), X.ravel() ** 2, Y.ravel() ** 2, (X * Y).ravel()], axis=1)
    a, b, c, d, e, f = np.linalg.lstsq(A, w.ravel(), rcond=None)[0]
    H = np.array([[2 * d, f], [f, 2 * e]])
    try:
        dx, dy = np.linalg.solve(H, [-b, -c])
    except np.linalg.LinAlgError:
        dx, dy = 0.0, 0.0
    dx, dy = float(np.clip(dx, -1, 1)), float(np.clip(dy, -1, 1))
    return (i + dx) / (nx - 1), (j + dy) / (ny - 1)


def eddy_centres(u: np.ndarray, v: np.ndarray, theta_deg: float):
    """{'primary': (x, y), 'left': (x, y) or None, 'right': (x, y) or None}."""
    psi = stream_function(u, v, theta_deg)
    ny, nx = psi.shape
    out = {}
    j, i = np.unravel_index(np.argmin(psi[1:-1, 1:-1]), (ny - 2, nx - 2))
    out["primary"] = to_xy(*_refine(psi, j + 1, i + 1), theta_deg)
    low = slice(1, max(3, int(0.35 * (ny - 1))))
    for name, cols in (("left", slice(1, (nx - 1) // 2)), ("right", slice((nx - 1) // 2 + 1, nx - 1))):
        sub = psi[low, cols]
        if sub.size == 0 or sub.max() <= 0.0:
            out[name] = None
            continue
        jj, ii = np.unravel_index(np.argmax(sub), sub.shape)
        out[name] = to_xy(*_refine(psi, jj + low.start, ii + cols.start), theta_deg)
    return out
