"""Pins of the CPU oracle against what the paper and mathematics fix.

Each ``check_*`` function raises AssertionError when the oracle disagrees with
a value printed in the paper, a closed form, an invariant, or a textbook
special case.  ``test_oracle_pins.py`` runs them on the oracle as built;
``test_oracle_mutations.py`` runs them on copies of the oracle with a
plausible mistake planted, and requires that at least one of them fails.

Equation numbers are the labels of arXiv:2306.07603.
"""
from __future__ import annotations

import math
import os
from fractions import Fraction

import numpy as np

import oracle as O

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def golden_geometry():
    return {k: float(v) for k, v in _golden_rows("geometry.txt")}


def golden_eddies():
    out = []
    for r in _golden_rows("eddy_centres.txt"):
        vals = [None if x == "-" else float(x) for x in r]
        out.append({"theta": vals[0], "n": vals[1], "primary": (vals[2], vals[3]),
                    "left": None if vals[4] is None else (vals[4], vals[5]),
                    "right": None if vals[6] is None else (vals[6], vals[7])})
    return out


def _rng(seed=0):
    return np.random.default_rng(seed)


# ----------------------------------------------------------------- lattice

def check_lattice_matches_paper():
    """Eq. (2.9) as printed (golden file), and the isotropy that fixes c_s^2."""
    cx, cy, w, wb, cs2 = O.lattice()
    for r in _golden_rows("d2q9_lattice.txt"):
        k = int(r[0])
        assert cx[k] == float(r[1]) and cy[k] == float(r[2]), ("velocity", k)
        assert abs(w[k] - float(Fraction(r[3]))) < 1e-16, ("omega", k)
        assert abs(wb[k] - float(Fraction(r[4]))) < 1e-16, ("omegabar", k)
    # sum omega = 1, sum omega c = 0, sum omega c c = c_s^2 I (moment design A1)
    assert abs(w.sum() - 1.0) < 1e-15
    assert abs((w * cx).sum()) < 1e-16 and abs((w * cy).sum()) < 1e-16
    assert abs((w * cx * cx).sum() - cs2) < 1e-16 and abs((w * cy * cy).sum() - cs2) < 1e-16
    assert abs((w * cx * cy).sum()) < 1e-16
    assert abs(cs2 - 1.0 / 3.0) < 1e-16


# -------------------------------------------------------------- equilibrium

def check_equilibrium_moments():
    """Moment design (A1): sum f_eq = rho0, sum c f_eq = u, sum c c f_eq = (P + c_s^2 rho0) I + u u."""
    cx, cy, _, _, cs2 = O.lattice()
    rng = _rng(1)
    for _ in range(50):
        P, ux, uy = rng.normal(0, 0.02), rng.normal(0, 0.1), rng.normal(0, 0.1)
        rho0 = rng.uniform(0.5, 2.0)
        f = O.equilibrium(P, ux, uy, rho0)
        assert abs(f.sum() - rho0) < 1e-15
        assert abs((cx * f).sum() - ux) < 1e-16 and abs((cy * f).sum() - uy) < 1e-16
        assert abs((cx * cx * f).sum() - (P + cs2 * rho0 + ux * ux)) < 1e-15
        assert abs((cy * cy * f).sum() - (P + cs2 * rho0 + uy * uy)) < 1e-15
        assert abs((cx * cy * f).sum() - ux * uy) < 1e-16


def check_moments_round_trip():
    """Eqs. (2.10)-(2.11) invert Eq. (2.8): (P, u) -> f_eq -> (P, u)."""
    rng = _rng(2)
    for _ in range(50):
        P, ux, uy = rng.normal(0, 0.02), rng.normal(0, 0.1), rng.normal(0, 0.1)
        rho0 = rng.uniform(0.5, 2.0)
        P2, ux2, uy2 = O.moments(O.equilibrium(P, ux, uy, rho0), rho0)
        assert abs(P2 - P) < 1e-15 and abs(ux2 - ux) < 1e-16 and abs(uy2 - uy) < 1e-16


def _nonequilibrium(Q):
    """A population set with zero density, pressure and momentum moments whose
    second moment sum_k c c g_k is the symmetric traceless tensor Q (uses the
    fourth-order isotropy of the D2Q9 weights)."""
    cx, cy, w, _, cs2 = O.lattice()
    qc = Q[0][0] * cx * cx + 2 * Q[0][1] * cx * cy + Q[1][1] * cy * cy
    return w * (qc - cs2 * (Q[0][0] + Q[1][1])) / (2 * cs2 * cs2)


def _random_node(rng, rho0=1.0):
    P, ux, uy = rng.normal(0, 0.01), rng.normal(0, 0.05), rng.normal(0, 0.05)
    a, b = rng.normal(0, 1e-3), rng.normal(0, 1e-3)
    return O.equilibrium(P, ux, uy, rho0), np.array([[a, b], [b, -a]])


def check_conversions_follow_definitions():
    """Eqs. (2.15)-(2.18) against the definitions (2.3)-(2.4) with the BGK
    operator of Eq. (2.0): f-hat = f + dt/(2 lam) (f - f_eq), f-hat+ = f -
    dt/(2 lam)(f - f_eq), f-bar = f + dt/(4 lam)(f - f_eq), f-bar+ = f -
    dt/(4 lam)(f - f_eq)."""
    rng = _rng(3)
    for _ in range(30):
        feq, Q = _random_node(rng)
        f = feq + _nonequilibrium(Q)
        lam, dt = rng.uniform(1e-3, 1.0), rng.uniform(1e-3, 0.1)
        fne = f - feq
        fhat = f + dt / (2 * lam) * fne
        fbar = f + dt / (4 * lam) * fne
        # f_eq is the same whether computed from f, f-hat or f-bar (Eqs. 2.10-2.11)
        P, ux, uy = O.moments(fhat)
        assert np.abs(O.equilibrium(P, ux, uy) - feq).max() < 1e-15
        assert np.abs(O.f_from_fhat_node(fhat, feq, lam, dt) - f).max() < 1e-15
        assert np.abs(O.f_from_fbar(fbar, feq, lam, dt) - f).max() < 1e-15
        fhp, fbp = O.collide(fhat, feq, lam, dt)
        assert np.abs(fhp - (f - dt / (2 * lam) * fne)).max() < 1e-15
        assert np.abs(fbp - (f - dt / (4 * lam) * fne)).max() < 1e-15


def check_collision_invariants():
    """sum_{k != 0} X_k and sum_k c_k X_k are the same for X = f-hat, f-hat+,
    f-bar+ and f (the collision conserves the pressure moment and momentum)."""
    cx, cy, _, _, _ = O.lattice()
    rng = _rng(4)
    for _ in range(30):
        fhat = O.equilibrium(rng.normal(0, 0.01), rng.normal(0, 0.05), rng.normal(0, 0.05)) \
            + rng.normal(0, 1e-3, 9)        # an arbitrary population set
        feq = O.equilibrium(*O.moments(fhat))
        lam, dt = rng.uniform(1e-3, 1.0), rng.uniform(1e-3, 0.1)
        fhp, fbp = O.collide(fhat, feq, lam, dt)
        f = O.f_from_fhat_node(fhat, feq, lam, dt)
        for X in (fhp, fbp, f):
            assert abs(X[1:].sum() - fhat[1:].sum()) < 1e-15
            assert abs((cx * X).sum() - (cx * fhat).sum()) < 1e-16
            assert abs((cy * X).sum() - (cy * fhat).sum()) < 1e-16


def check_relaxation_time_power_law():
    """Step (2): for a node whose f carries the non-equilibrium part of a given
    traceless strain rate S = grad u + grad u^T, namely sum c c f^ne =
    -lam c_s^2 S (Eq. 2.12), the new lambda is the power-law value
    K (S:S/2)^((n-1)/2) / c_s^2 (Eqs. 1.3.1, 1.4, 2.14)."""
    _, _, _, _, cs2 = O.lattice()
    rng = _rng(5)
    for n in (0.5, 0.8, 1.0, 1.3, 1.5):
        for _ in range(10):
            feq, _ = _random_node(rng)
            a, b = rng.normal(0, 0.05), rng.normal(0, 0.05)
            S = np.array([[2 * a, b], [b, -2 * a]])
            lam, dt, K = rng.uniform(1e-3, 0.1), rng.uniform(1e-3, 0.05), rng.uniform(1e-4, 1e-2)
            f = feq + _nonequilibrium(-lam * cs2 * S)
            fhat = f + dt / (2 * lam) * (f - feq)
            gamma2 = 0.5 * (S * S).sum()                # 2 D:D with D = S/2
            want = K * gamma2 ** ((n - 1) / 2) / cs2
            got = O.relaxation_time(fhat, feq, lam, dt, K, n, 1e-9)
            assert abs(got - want) < 1e-9 * want, (n, got, want)
        # zero shear takes the floor gamma_min
        feq, _ = _random_node(rng)
        got = O.relaxation_time(feq, feq, 0.01, 0.01, 1e-3, n, 1e-3)
        assert abs(got - 1e-3 * (1e-6) ** ((n - 1) / 2) / cs2) < 1e-12 * got


def check_initial_lambda():
    """Step (1), reading R9: the initial relaxation time is the power-law value
    at the cavity's characteristic strain rate U / L.  Built here from the
    paper's definitions one at a time: K from Re = U^(2-n) L^n / K
    (Eq. 2.15.1, L = 1), mu = K gamma^(n-1) at gamma = U / L (Eq. 1.4),
    lambda = mu / c_s^2 (Eq. 2.14) with c_s^2 from the lattice isotropy."""
    _, _, _, _, cs2 = O.lattice()
    L = 1.0
    for re, n, U, th in ((100.0, 0.8, 0.1, 60.0), (2500.0, 1.5, 0.1, 45.0), (40.0, 0.5, -0.05, 90.0),
                         (400.0, 1.0, 0.2, 75.0)):
        p = O.Params(nx=9, ny=7, re=re, n=n, u_lid=U, theta_deg=th)
        K = abs(U) ** (2.0 - n) * L ** n / re
        gamma = abs(U) / L
        mu = K * gamma ** (n - 1.0)
        want = mu / cs2
        _, Lam = O.init(p)
        assert np.all(np.abs(Lam - want) <= 1e-14 * want), (re, n, U, Lam.ravel()[0], want)
        assert abs(O.derive(p)["K"] - K) <= 1e-15 * K


def check_implicit_lambda():
    """Implicit Step (2) (reading R20): (a) for a node whose f carries the
    non-equilibrium part of a strain rate S at the power-law lambda of S
    itself, the implicit lambda is that lambda (closed form, Eqs. 1.4, 2.12,
    2.14, 2.18); (b) on arbitrary nodes it is a fixed point of the lagged
    Step (2), an independent code path; (c) Newtonian: K / c_s^2 exactly."""
    _, _, _, _, cs2 = O.lattice()
    rng = _rng(17)
    for n in (0.5, 0.8, 1.3, 1.5):
        for _ in range(10):
            feq, _ = _random_node(rng)
            a, b = rng.normal(0, 0.05), rng.normal(0, 0.05)
            S = np.array([[2 * a, b], [b, -2 * a]])
            dt, K = rng.uniform(1e-3, 0.05), rng.uniform(1e-4, 1e-2)
            lam = K * (0.5 * (S * S).sum()) ** ((n - 1) / 2) / cs2
            f = feq + _nonequilibrium(-lam * cs2 * S)
            fhat = f + dt / (2 * lam) * (f - feq)
            got = O.relaxation_time_implicit(fhat, feq, dt, K, n, 1e-9)
            assert abs(got - lam) <= 1e-12 * lam, (n, got, lam)
            # arbitrary node: f-hat with a random non-equilibrium part
            fh = feq + rng.normal(0, 1e-3, 9)
            li = O.relaxation_time_implicit(fh, feq, dt, K, n, 1e-9)
            back = O.relaxation_time(fh, feq, li, dt, K, n, 1e-9)
            assert abs(back - li) <= 1e-12 * li, (n, back, li)
    feq, _ = _random_node(rng)
    fh = feq + rng.normal(0, 1e-3, 9)
    assert O.relaxation_time_implicit(fh, feq, 0.01, 2e-3, 1.0, 1e-6) == 2e-3 / cs2


def check_implicit_steady_state_equals_lagged():
    """At a steady state the lag of Step (2) vanishes (lambda_old = lambda):
    lagged and implicit runs of a slow power-law cavity reach the same state,
    while their transients differ."""
    base = dict(nx=17, ny=17, re=1.0, n=0.7, theta_deg=60.0, rho0=0.0)
    pl, pi = O.Params(**base), O.Params(**base, lambda_mode=O.LAMBDA_IMPLICIT)
    Fl, Ll = O.init(pl)
    Fi, Li = O.init(pi)
    O.run(pl, Fl, Ll, 40)
    O.run(pi, Fi, Li, 40)
    ul, ui = O.fields(pl, Fl)[0], O.fields(pi, Fi)[0]
    assert np.abs(ul - ui).max() > 1e-6 * np.abs(ul).max()
    O.run(pl, Fl, Ll, 3960)
    O.run(pi, Fi, Li, 3960)
    rl = O.run(pl, Fl, Ll, 1)
    O.run(pi, Fi, Li, 1)
    assert rl[0] < 1e-12, rl
    ul, ui = O.fields(pl, Fl)[0], O.fields(pi, Fi)[0]
    assert np.abs(ul - ui).max() <= 1e-9 * np.abs(ul).max()


# ---------------------------------------------------------------- geometry

def check_geometry_matches_paper():
    """Eq. (3.8.1) with the facts of Section 4 (unit bottom and height, top
    angle theta) and the centre probe point of Section 6.2."""
    g = golden_geometry()
    for th, t in ((75, g["tan75"]), (60, g["tan60"]), (45, g["tan45"])):
        p = O.Params(nx=17, ny=17, theta_deg=th)
        C = O.derive(p)["cot"]
        assert abs(C * t - 1.0) < 1e-14
        N = p.nx - 1
        bl, tl, br, tr = O.node_xy(p, 0, 0), O.node_xy(p, 0, N), O.node_xy(p, N, 0), O.node_xy(p, N, N)
        assert abs((br[0] - bl[0]) - g["bottom_length"]) < 1e-14
        assert abs((tl[1] - bl[1]) - g["height"]) < 1e-14 and bl[1] == 0.0 and br[1] == 0.0
        assert abs(tl[0]) < 1e-15          # the lid starts at x = 0
        # top interior angle between the lid (+x) and the left wall
        wall = np.array(bl) - np.array(tl)
        ang = math.degrees(math.acos(wall[0] / np.hypot(*wall)))
        assert abs(ang - th) < 1e-9
        # isosceles: mirror image about the centre line
        assert abs((bl[0] + br[0]) - (tl[0] + tr[0])) < 1e-14
    p = O.Params(nx=17, ny=17, theta_deg=60)
    cx_, cy_ = O.node_xy(p, 8, 8)
    assert abs(cx_ - g["probe60_x"]) < 5e-6 and abs(cy_ - g["probe60_y"]) < 1e-15
    p90 = O.Params(nx=9, ny=9, theta_deg=90)
    assert O.derive(p90)["cot"] == 0.0


def _linear_field(p, alpha, beta, gamma):
    Phi = np.zeros((9, p.ny, p.nx))
    for j in range(p.ny):
        for i in range(p.nx):
            x, y = O.node_xy(p, i, j)
            Phi[:, j, i] = alpha + beta * x + gamma * y
    return Phi


def check_metric_exact_on_linear_fields():
    """Eqs. (3.2)-(3.8.2) with Eqs. (2.5)-(2.7): for a field linear in the
    physical coordinates, the transformed transport term equals c_k . grad Phi
    exactly at every interior node (central, upwind and one-sided points)."""
    cx, cy, _, _, _ = O.lattice()
    for th in (40, 45, 60, 75, 90):
        for mix in (0.0, 0.5, 1.0):
            p = O.Params(nx=9, ny=7, theta_deg=th, mix=mix)
            beta, gamma = 0.37, -1.21
            Phi = _linear_field(p, 0.3, beta, gamma)
            for j in range(1, p.ny - 1):
                for i in range(1, p.nx - 1):
                    for k in range(9):
                        want = cx[k] * beta + cy[k] * gamma
                        got = O.stream_term(p, Phi, k, i, j)
                        assert abs(got - want) < 1e-12, (th, mix, k, i, j, got, want)


def check_stencils_on_quartics():
    """Eqs. (2.6)-(2.7) on Phi = xi^4 and Phi = eta^4, whose Taylor series end
    at the fourth derivative: central = Phi' + h^2 Phi'''/6; second-order
    upwind = Phi' - h^2 Phi'''/3 +/- h^3 Phi''''/4 (+ for c >= 0, using the
    points behind, - for c < 0); first-order one-sided = Phi' -/+ h Phi''/2 +
    h^2 Phi'''/6 -/+ h^3 Phi''''/24.  The upwind side follows the sign of the
    contravariant velocity at the node."""
    for th in (60, 40):
        mix = 0.3
        p = O.Params(nx=11, ny=9, theta_deg=th, mix=mix)
        d = O.derive(p)
        for axis in ("xi", "eta"):
            h = d["dxi"] if axis == "xi" else d["deta"]
            npts = p.nx if axis == "xi" else p.ny
            Phi = np.zeros((9, p.ny, p.nx))
            for j in range(p.ny):
                for i in range(p.nx):
                    s = (i * d["dxi"]) if axis == "xi" else (j * d["deta"])
                    Phi[:, j, i] = s ** 4
            signs_seen = set()
            for j in range(1, p.ny - 1):
                for i in range(1, p.nx - 1):
                    cxi, ceta, _ = O.contravariant(p, i, j)
                    pos = i if axis == "xi" else j
                    s = pos * h
                    d1, d2, d3, d4 = 4 * s ** 3, 12 * s ** 2, 24 * s, 24.0
                    for k in range(1, 9):
                        c = cxi[k] if axis == "xi" else ceta[k]
                        cen = d1 + h * h * d3 / 6
                        if c >= 0:
                            up = (d1 - h * d2 / 2 + h * h * d3 / 6 - h ** 3 * d4 / 24) if pos == 1 \
                                else (d1 - h * h * d3 / 3 + h ** 3 * d4 / 4)
                        else:
                            up = (d1 + h * d2 / 2 + h * h * d3 / 6 + h ** 3 * d4 / 24) if pos == npts - 2 \
                                else (d1 - h * h * d3 / 3 - h ** 3 * d4 / 4)
                        want = c * (mix * cen + (1 - mix) * up)
                        got = O.stream_term(p, Phi, k, i, j)
                        assert abs(got - want) < 1e-11 * max(1.0, abs(want)), (th, axis, k, i, j, got, want)
                        if c != 0:
                            signs_seen.add(c > 0)
            assert signs_seen == {True, False}


def check_kinetic_energy_weights():
    """Eq. (5.1): a uniform velocity field has E = |u|^2/2 times the cavity
    area (1 + cot theta for unit bottom and height); the trapezoid rule is
    exact because J is linear in eta."""
    for th in (45, 60, 90):
        p = O.Params(nx=9, ny=13, theta_deg=th)
        C = O.derive(p)["cot"]
        F = np.zeros((9, p.ny, p.nx))
        F[:] = O.equilibrium(0.0, 0.03, -0.02)[:, None, None]
        e = O.kinetic_energy(p, F)
        want = 0.5 * (0.03 ** 2 + 0.02 ** 2) * (1.0 + C)
        assert abs(e - want) < 1e-15, (th, e, want)


# --------------------------------------------------------------- dynamics

def _state_from(p, P, u, v, lam):
    F = np.zeros((9, p.ny, p.nx))
    for j in range(p.ny):
        for i in range(p.nx):
            F[:, j, i] = O.equilibrium(P[j, i], u[j, i], v[j, i], p.rho0)
    return F, np.full((p.ny, p.nx), lam)


def check_rest_state():
    """A fluid at rest with no moving boundary stays at rest (periodic box)."""
    p = O.Params(nx=8, ny=8, n=0.6, re=10.0, bc_mode=O.PERIODIC)
    _, _, w, _, _ = O.lattice()
    F, Lam = O.init(p)
    assert np.all(F == w[:, None, None] * p.rho0)
    O.run(p, F, Lam, 50)
    assert np.abs(F - w[:, None, None] * p.rho0).max() < 1e-15
    u, v, P = O.fields(p, F)
    assert np.abs(u).max() < 1e-16 and np.abs(v).max() < 1e-16 and np.abs(P).max() < 1e-15


def _random_smooth(p, rng, amp):
    x = np.arange(p.nx) / p.nx
    y = np.arange(p.ny) / p.ny
    X, Y = np.meshgrid(x, y)
    out = np.zeros((p.ny, p.nx))
    for _ in range(4):
        kx, ky = rng.integers(1, 3, 2)
        ph = rng.uniform(0, 2 * np.pi, 2)
        out += rng.normal(0, amp) * np.sin(2 * np.pi * kx * X + ph[0]) * np.cos(2 * np.pi * ky * Y + ph[1])
    return out


def check_exact_conservation_periodic():
    """In the periodic box the scheme conserves sum_x sum_{k != 0} f-hat_k (the
    pressure/mass moment of Eq. 2.11) and the momentum sum_x sum_k c_k f-hat_k
    to rounding, for a power-law fluid with spatially varying lambda: the
    collision keeps both moments at each node and every difference stencil
    telescopes."""
    cx, cy, _, _, _ = O.lattice()
    rng = _rng(7)
    p = O.Params(nx=16, ny=12, n=0.7, re=50.0, u_lid=0.05, bc_mode=O.PERIODIC)
    u, v, P = _random_smooth(p, rng, 0.03), _random_smooth(p, rng, 0.03), _random_smooth(p, rng, 0.005)
    F, Lam = _state_from(p, P, u, v, O.derive(p)["lam0"])
    M0 = F[1:].sum()
    jx0, jy0 = (cx[:, None, None] * F).sum(), (cy[:, None, None] * F).sum()
    O.run(p, F, Lam, 300)
    assert Lam.std() > 1e-3 * Lam.mean()   # the viscosity really varies
    assert abs(F[1:].sum() - M0) < 1e-12 * M0
    scale = np.abs(u).sum() + np.abs(v).sum()
    assert abs((cx[:, None, None] * F).sum() - jx0) < 1e-13 * scale
    assert abs((cy[:, None, None] * F).sum() - jy0) < 1e-13 * scale


def _taylor_green(N, T=2.0, U=0.01, re=10.0):
    p = O.Params(nx=N, ny=N, n=1.0, re=re, u_lid=U, bc_mode=O.PERIODIC)
    d = O.derive(p)
    x = np.arange(N) / N
    X, Y = np.meshgrid(x, x)
    k = 2 * np.pi
    u = -U * np.cos(k * X) * np.sin(k * Y)
    v = U * np.sin(k * X) * np.cos(k * Y)
    P = -U * U / 4 * (np.cos(2 * k * X) + np.cos(2 * k * Y))
    _, _, _, _, cs2 = O.lattice()
    F, Lam = _state_from(p, P, u, v, d["K"] / cs2)
    t1, t2 = 0.5, T
    s1, s2 = int(round(t1 / d["dt"])), int(round(t2 / d["dt"]))
    O.run(p, F, Lam, s1)
    e1 = O.kinetic_energy(p, F)
    O.run(p, F, Lam, s2 - s1)
    e2 = O.kinetic_energy(p, F)
    rate = -math.log(e2 / e1) / ((s2 - s1) * d["dt"])
    nu = d["K"]                      # mu = K at n = 1, lambda c_s^2 = mu (A12)
    return rate, 4 * nu * k * k      # |u|^2 decays as exp(-2 nu (kx^2 + ky^2) t)


def check_taylor_green_decay():
    """Newtonian recovery (n = 1): the Taylor-Green vortex decays at the
    closed-form rate 4 nu k^2 with nu = K (Eqs. 1.2, 1.4, 2.14 and A12); the
    rate error falls faster than second order with the grid (the leading
    error is the fourth-derivative dissipation of the upwind part of
    Eq. 2.7, third order in the spacing)."""
    errs = []
    for N in (32, 64):
        rate, want = _taylor_green(N)
        errs.append(abs(rate - want) / want)
    assert errs[-1] < 0.02, errs
    assert errs[0] / errs[1] > 4.0, errs


def _couette(n, U):
    _, _, _, _, cs2 = O.lattice()
    # Re = 10 U keeps the apparent viscosity K U^(n-1) at 0.1 for every U
    p = O.Params(nx=5, ny=17, n=n, re=10.0 * U, u_lid=U, bc_mode=O.COUETTE)
    d = O.derive(p)
    F, Lam = O.init(p)
    O.run(p, F, Lam, int(round(40.0 / d["dt"])))
    u, v, P = O.fields(p, F)
    y = np.arange(p.ny) * d["deta"]
    want = d["K"] * U ** (n - 1) / cs2
    return (np.abs(u - U * y[:, None]).max() / U, np.abs(v).max() / U,
            np.abs(Lam[1:-1] / want - 1).max())


def check_couette_power_law():
    """Plane Couette flow of a power-law fluid (periodic in x, walls at y = 0
    and y = 1, top wall at U): the steady velocity is U y and the relaxation
    time is lambda = K (U/H)^(n-1) / c_s^2 at every interior node
    (Eqs. 1.4, 2.12, 2.14).  The small remaining difference is the
    O((lambda U)^2) term that the Chapman-Enskog analysis drops as a
    low-Mach term (Appendix A), so it falls as U^2 at fixed viscosity."""
    for n in (0.5, 1.5):
        du, dv, dlam = _couette(n, 0.01)
        assert du < 1e-6 and dv < 1e-10, (n, du, dv)
        assert dlam < 1e-5, (n, dlam)
        _, _, dlam_fast = _couette(n, 0.1)
        assert 80.0 < dlam_fast / dlam < 120.0, (n, dlam_fast, dlam)


def check_mirror_symmetry():
    """The isosceles map of Eq. (3.8.1) is symmetric about xi = 1/2: mirroring
    the cavity and reversing the lid gives u -> -u(mirror), v, P -> mirror."""
    for th, n in ((60, 0.7), (90, 1.5)):
        p1 = O.Params(nx=17, ny=15, theta_deg=th, n=n, re=100.0, u_lid=0.1)
        p2 = O.Params(nx=17, ny=15, theta_deg=th, n=n, re=100.0, u_lid=-0.1)
        u1, v1, P1, _, _ = O.simulate(p1, 150)
        u2, v2, P2, _, _ = O.simulate(p2, 150)
        assert np.abs(u2 + u1[:, ::-1]).max() < 1e-12 * np.abs(u1).max()
        assert np.abs(v2 - v1[:, ::-1]).max() < 1e-12 * np.abs(v1).max()
        assert np.abs(P2 - P1[:, ::-1]).max() < 1e-12 * np.abs(P1).max()


def _stokes_asymmetry(re):
    p = O.Params(nx=17, ny=17, theta_deg=90, n=1.0, re=re, u_lid=0.001)
    u, v, _, _, _ = O.simulate(p, 3000)
    s = np.abs(u).max()
    return max(np.abs(u - u[:, ::-1]).max(), np.abs(v + v[:, ::-1]).max()) / s


def check_stokes_left_right_symmetry():
    """In the square (theta = 90) creeping flow is left-right symmetric (u even,
    v odd about x = 1/2); the asymmetry is the inertial effect and falls in
    proportion to Re (a low lid speed keeps the O(Ma^2) part of the
    boundary equilibria out of the way)."""
    a1, a2 = _stokes_asymmetry(0.1), _stokes_asymmetry(0.01)
    assert a2 < 1e-4, a2
    assert 4.0 < a1 / a2 < 15.0, (a1, a2)


def check_newtonian_limit_is_exact():
    """At n = 1 Eq. (1.4) gives mu = K for any strain, so lambda = K/c_s^2 at
    every node after one step and the shear-rate floor has no effect."""
    _, _, _, _, cs2 = O.lattice()
    pa = O.Params(nx=13, ny=13, theta_deg=60, n=1.0, re=200.0, gamma_min=1e-6)
    pb = O.Params(nx=13, ny=13, theta_deg=60, n=1.0, re=200.0, gamma_min=1e-1)
    ua, va, Pa, Fa, La = O.simulate(pa, 40)
    ub, vb, Pb, Fb, Lb = O.simulate(pb, 40)
    assert np.array_equal(Fa, Fb) and np.array_equal(La, Lb)
    assert np.all(La == O.derive(pa)["K"] / cs2)


def check_rho0_invariance():
    """u and P do not depend on the constant rho0 of Eq. (2.8) (it only offsets
    each population by omega_k rho0)."""
    p1 = O.Params(nx=13, ny=11, theta_deg=45, n=1.3, re=300.0, rho0=1.0)
    p2 = O.Params(nx=13, ny=11, theta_deg=45, n=1.3, re=300.0, rho0=2.0)
    u1, v1, P1, _, _ = O.simulate(p1, 100)
    u2, v2, P2, _, _ = O.simulate(p2, 100)
    assert np.abs(u1 - u2).max() < 1e-13 and np.abs(v1 - v2).max() < 1e-13
    assert np.abs(P1 - P2).max() < 1e-13


def check_cavity_grid_convergence():
    """Nested grids 17/33/65 at the same physical time: the differences shrink
    faster than first order away from the singular lid corners.  Taken with
    equal central and upwind weights in Eq. (2.5): on grids this coarse, shortly
    after the impulsive start, the more central mixtures still carry grid-scale
    dispersive error and show no clean order."""
    T = 1.0
    sols = {}
    for N in (17, 33, 65):
        p = O.Params(nx=N, ny=N, theta_deg=60, n=1.0, re=50.0, u_lid=0.1, mix=0.5)
        steps = int(round(T / O.derive(p)["dt"]))
        u, v, _, _, _ = O.simulate(p, steps)
        sols[N] = (u, v)

    def coarse(a, f):
        return a[::f, ::f]

    sel = (slice(1, 13), slice(1, 16))   # rows below the lid corners of the 17-grid
    e1 = np.sqrt(((sols[17][0] - coarse(sols[33][0], 2))[sel] ** 2).mean()
                 + ((sols[17][1] - coarse(sols[33][1], 2))[sel] ** 2).mean())
    e2 = np.sqrt(((coarse(sols[33][0], 2) - coarse(sols[65][0], 4))[sel] ** 2).mean()
                 + ((coarse(sols[33][1], 2) - coarse(sols[65][1], 4))[sel] ** 2).mean())
    order = math.log2(e1 / e2)
    assert order > 1.0, (e1, e2, order)


def check_steady_residual_decreases():
    """Eq. (2.19): the global relative errors fall as the cavity flow settles;
    the residual evaluated from two stored states agrees with the one of the
    time loop; at steady state E(u) and the mean-removed E(P) reach rounding
    level while the raw E(P) keeps the constant drift of the pressure level."""
    p = O.Params(nx=17, ny=17, theta_deg=75, n=0.8, re=20.0)
    F, Lam = O.init(p)
    r1 = O.run(p, F, Lam, 50)
    F0 = F.copy()
    r2 = O.run(p, F, Lam, 1)
    eu, ep, eg = O.residuals(p, F0, F)
    assert abs(eu - r2[0]) <= 1e-14 * eu and abs(ep - r2[1]) <= 1e-14 * ep
    O.run(p, F, Lam, 12000)
    F0 = F.copy()
    r3 = O.run(p, F, Lam, 1)
    eu, ep, eg = O.residuals(p, F0, F)
    assert r3[0] < 1e-12 and eg < 1e-11, (r3, eg)
    assert ep > 1e-7, ep


ALL_CHECKS = [
    check_lattice_matches_paper,
    check_equilibrium_moments,
    check_moments_round_trip,
    check_conversions_follow_definitions,
    check_collision_invariants,
    check_relaxation_time_power_law,
    check_initial_lambda,
    check_implicit_lambda,
    check_implicit_steady_state_equals_lagged,
    check_geometry_matches_paper,
    check_metric_exact_on_linear_fields,
    check_stencils_on_quartics,
    check_kinetic_energy_weights,
    check_rest_state,
    check_exact_conservation_periodic,
    check_taylor_green_decay,
    check_couette_power_law,
    check_mirror_symmetry,
    check_stokes_left_right_symmetry,
    check_newtonian_limit_is_exact,
    check_rho0_invariance,
    check_cavity_grid_convergence,
    check_steady_residual_decreases,
]
