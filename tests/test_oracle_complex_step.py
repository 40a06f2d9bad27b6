"""The complex-step build of the oracle (the same source in complex doubles) against what fixes its
derivatives independently of it: closed forms of the parameter rules, Richardson-extrapolated central
differences of the FP64 oracle, and the FP64 oracle's own values for its real part.  No GPU."""
import math

import numpy as np

import oracle as O
from oracle import complex_step as CS

H = 1e-20


def test_real_part_is_the_fp64_oracle():
    p = O.Params(nx=17, ny=13, re=80.0, n=1.3, theta_deg=50.0, u_lid=0.1, rho0=0.0)
    F, L = O.init(p)
    O.run(p, F, L, 60)
    J = O.kinetic_energy(p, F)
    Jc = CS.kinetic_energy(p, 60, {})
    assert Jc.imag == 0.0 and abs(Jc.real - J) <= 1e-13 * J


def test_parameter_rules_closed_forms():
    """Derivatives of the derived constants against their closed forms: K = U^(2-n) / Re (Eq. 2.15.1),
    lambda_0 = U / (Re c_s^2) (Step 1), cot(theta) with d cot / d theta = -(1 + cot^2), exactly 0 at
    90 degrees in the real build, and the contravariant time step dt = cfl dxi / (1 + cot theta)."""
    for re, n, th, u in ((100.0, 0.8, 60.0, 0.1), (400.0, 1.3, 90.0, -0.05), (2500.0, 0.5, 45.0, 0.2)):
        p = O.Params(nx=33, ny=33, re=re, n=n, theta_deg=th, u_lid=u)
        d0 = O.derive(p)
        K, U, C = d0["K"], abs(u), d0["cot"]
        dn = CS.derive(p, {"n": H})
        du = CS.derive(p, {"u_lid": H})
        dth = CS.derive(p, {"theta_deg": H * 180.0 / math.pi})
        assert abs(dn["K"].imag / H - (-K * math.log(U))) <= 1e-14 * abs(K * math.log(U))
        sgn = math.copysign(1.0, u)
        assert abs(du["K"].imag / H - (2.0 - n) * K / U * sgn) <= 1e-14 * abs((2.0 - n) * K / U)
        assert abs(du["lam0"].imag / H - 3.0 / re * sgn) <= 1e-14 * 3.0 / re
        assert abs(dth["cot"].imag / H - (-(1.0 + C * C))) <= 1e-14 * (1.0 + C * C)
        assert abs(dth["cot"].real - C) <= 4e-16 * max(C, 1.0)   # complex division: a few ulp
        dxi = 1.0 / 32
        # (1 + C) / dxi >= 1 / deta here, so dt = cfl dxi / (1 + C)
        want = -0.5 * dxi / (1.0 + C) ** 2 * (-(1.0 + C * C))
        assert abs(dth["dt"].imag / H - want) <= 1e-14 * abs(want)


def test_gradient_against_richardson_differences():
    """dJ/d(theta [rad], n, U) of Eq. (5.1) after 120 steps on 17 x 17 against Richardson extrapolation of
    central differences of the FP64 oracle (steps h and h/2, error O(h^4) plus rounding / h): the two
    agree to the accuracy of the differences, 1e-8 relative."""
    re, n, th, u, steps = 80.0, 1.3, 50.0, 0.1, 120
    p = O.Params(nx=17, ny=17, re=re, n=n, theta_deg=th, u_lid=u)

    def ke(theta_deg, nn, uu):
        q = O.Params(nx=17, ny=17, re=re, n=nn, theta_deg=theta_deg, u_lid=uu)
        F, L = O.init(q)
        O.run(q, F, L, steps)
        return O.kinetic_energy(q, F)

    def richardson(f, h):
        d1 = (f(h) - f(-h)) / (2 * h)
        d2 = (f(h / 2) - f(-h / 2)) / h
        return (4 * d2 - d1) / 3

    ref = [richardson(lambda d: ke(th + math.degrees(d), n, u), 1e-3),
           richardson(lambda d: ke(th, n + d, u), 1e-3),
           richardson(lambda d: ke(th, n, u + d), 1e-4)]
    J, g = CS.kinetic_energy_gradient(p, steps)
    for q in range(3):
        err = abs(g[q] - ref[q]) / abs(ref[q])
        print("param %d complex step %.14e Richardson %.14e rel %.2e" % (q, g[q], ref[q], err))
        assert err <= 1e-8
