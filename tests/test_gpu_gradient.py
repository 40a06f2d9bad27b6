"""dJ/d(theta, n, U) of the kinetic energy after a fixed number of steps: the
tangent-linear sweep and the checkpointed discrete adjoint of the library
against each other (both are the exact derivative of the same discrete map),
against central differences of the FP64 forward (h = 1e-4) and against the
complex-step derivative of the CPU oracle; and the torch.autograd.Function
over them."""
import math

import numpy as np
import pytest

import oracle as O
import paper_2306_07603_amd as M

pytestmark = pytest.mark.gpu


def ke_forward(n_xi, n_eta, re, n, theta_deg, u, steps):
    o = M.ifdlbm_default_options(precision="fp64")
    h = M.ifdlbm_create([M.Cavity(n_xi, n_eta, re, n, theta_deg, u)], o)
    M.ifdlbm_step(h, steps)
    e = M.ifdlbm_kinetic_energy(h, 0)
    h.close()
    return e


def test_gradient_against_central_differences():
    n_xi = n_eta = 33
    re, n, th, u, steps = 150.0, 0.7, 60.0, 0.1, 400
    J, g = M.ifdlbm_gradient(M.Cavity(n_xi, n_eta, re, n, th, u), M.ifdlbm_default_options(), steps)
    J0 = ke_forward(n_xi, n_eta, re, n, th, u, steps)
    assert abs(J - J0) <= 1e-11 * J0
    h = 1e-4
    fd = [
        (ke_forward(n_xi, n_eta, re, n, th + math.degrees(h), u, steps)
         - ke_forward(n_xi, n_eta, re, n, th - math.degrees(h), u, steps)) / (2 * h),
        (ke_forward(n_xi, n_eta, re, n + h, th, u, steps) - ke_forward(n_xi, n_eta, re, n - h, th, u, steps)) / (2 * h),
        (ke_forward(n_xi, n_eta, re, n, th, u + h * u, steps)
         - ke_forward(n_xi, n_eta, re, n, th, u - h * u, steps)) / (2 * h * u),
    ]
    for q in range(3):
        err = abs(g[q] - fd[q]) / abs(fd[q])
        print("param %d tangent %.10e central %.10e rel %.2e" % (q, g[q], fd[q], err), flush=True)
        assert err <= 1e-4


COMPLEX_STEP_CASES = [
    # (n_xi, n_eta, Re, n, theta, U, steps, options)
    (17, 17, 80.0, 1.3, 50.0, 0.1, 120, {}),
    (17, 17, 100.0, 0.8, 90.0, -0.1, 80, {}),                               # tie of the time-step rule, lid -x
    (21, 13, 200.0, 0.6, 60.0, 0.1, 60, {"dt_rule": 1, "mix": 0.5}),        # Cartesian time step
]


@pytest.mark.parametrize("method", ["tangent", "adjoint"])
@pytest.mark.parametrize("case", COMPLEX_STEP_CASES, ids=lambda c: "%dx%d_th%g_n%g" % (c[0], c[1], c[4], c[3]))
def test_gradient_against_oracle_complex_step(method, case):
    """dJ/d(theta [rad], n, U) of Eq. (5.1) against the complex-step derivative of the CPU oracle (the
    oracle's source in complex doubles, itself pinned to closed forms and to Richardson differences): both
    are the derivative of the same discrete map to rounding, 1e-9 relative."""
    from oracle import complex_step as CS
    n_xi, n_eta, re, n, th, u, steps, opt = case
    p = O.Params(nx=n_xi, ny=n_eta, re=re, n=n, theta_deg=th, u_lid=u, rho0=0.0,
                 dt_rule=opt.get("dt_rule", O.DT_CONTRAVARIANT), mix=opt.get("mix", 0.75))
    J_ref, g_ref = CS.kinetic_energy_gradient(p, steps)
    cav = M.Cavity(n_xi, n_eta, re, n, th, u)
    o = M.ifdlbm_default_options(rho0=0.0, **opt)
    if method == "tangent":
        J, g = M.ifdlbm_gradient(cav, o, steps)
    else:
        J, g = M.ifdlbm_adjoint(cav, o, steps, 25)
    assert abs(J - J_ref) <= 1e-12 * J_ref
    for q in range(3):
        err = abs(g[q] - g_ref[q]) / abs(g_ref[q])
        print("param %d %s %.14e complex step %.14e rel %.2e" % (q, method, g[q], g_ref[q], err), flush=True)
        assert err <= 1e-9


@pytest.mark.parametrize("method", ["tangent", "adjoint"])
def test_autograd_function(method):
    import torch
    from paper_2306_07603_amd.autograd import cavity_kinetic_energy
    theta = torch.tensor(math.radians(60.0), dtype=torch.float64, requires_grad=True)
    n = torch.tensor(0.7, dtype=torch.float64, requires_grad=True)
    u = torch.tensor(0.1, dtype=torch.float64, requires_grad=True)
    J = cavity_kinetic_energy(theta, n, u, 25, 25, 200.0, 100, None, 30, method)
    (2.0 * J).backward()
    _, g = M.ifdlbm_gradient(M.Cavity(25, 25, 200.0, 0.7, 60.0, 0.1), M.ifdlbm_default_options(), 100)
    assert np.allclose([theta.grad.item(), n.grad.item(), u.grad.item()], 2.0 * g, rtol=1e-9, atol=0)
    with torch.no_grad():
        J2 = cavity_kinetic_energy(theta, n, u, 25, 25, 200.0, 100)
    assert abs(J2.item() - J.item()) <= 1e-12 * J.item()


ADJ_CASES = [
    # n_xi, n_eta, Re, n, theta, U, steps, options
    (33, 33, 150.0, 0.7, 60.0, 0.1, 300, {}),
    (29, 37, 400.0, 1.3, 45.0, 0.08, 200, {"dt_rule": M.IFDLBM_DT_CARTESIAN, "mix": 0.7}),
    (25, 25, 100.0, 0.6, 90.0, 0.1, 150, {}),
    (21, 27, 250.0, 1.0, 70.0, -0.1, 150, {"cfl": 0.3}),
    (17, 17, 50.0, 0.5, 40.0, 0.1, 400, {"gamma_min": 1e-2}),
]


@pytest.mark.parametrize("kernel", ["staged", "fused"])
@pytest.mark.parametrize("case", ADJ_CASES, ids=lambda c: "%dx%d_n%g_th%g" % (c[0], c[1], c[3], c[4]))
def test_adjoint_equals_tangent(kernel, case):
    """Reverse and forward differentiation of one discrete map: equal up to
    FP64 rounding (1e-9 relative per component)."""
    nx, ny, re, n, th, u, steps, opt = case
    cav = M.Cavity(nx, ny, re, n, th, u)
    o = M.ifdlbm_default_options(kernel=kernel, **opt)
    Jt, gt = M.ifdlbm_gradient(cav, o, steps)
    Ja, ga = M.ifdlbm_adjoint(cav, o, steps, 64)
    print(case, kernel, "tangent", gt, "adjoint", ga, flush=True)
    assert abs(Ja - Jt) <= 1e-11 * abs(Jt)
    for q in range(3):
        assert abs(ga[q] - gt[q]) <= 1e-9 * abs(gt[q]) + 1e-13 * np.abs(gt).max(), q


def test_adjoint_does_not_depend_on_checkpoint_spacing():
    cav = M.Cavity(33, 29, 300.0, 0.8, 55.0, 0.1)
    o = M.ifdlbm_default_options(kernel="fused")
    res = [M.ifdlbm_adjoint(cav, o, 150, c) for c in (1, 7, 64, 150, 1000)]
    for J, g in res[1:]:
        assert J == res[0][0] and np.array_equal(g, res[0][1])


@pytest.mark.parametrize("precision", ["fp32sr", "fp64"])
def test_adjoint_129_20k_steps(precision):
    """129 x 129, Re 400, n 0.7, theta 60, 20k steps (FP32 storage with
    stochastic rounding, and FP64), checkpoints every 500 steps: within 1e-4 of central differences
    (h = 1e-4) of the FP64 forward."""
    nx = ny = 129
    re, n, th, u, steps = 400.0, 0.7, 60.0, 0.1, 20000

    def ke(theta_deg, nn, uu):
        return ke_forward(nx, ny, re, nn, theta_deg, uu, steps)

    h = 1e-4
    fd = [(ke(th + math.degrees(h), n, u) - ke(th - math.degrees(h), n, u)) / (2 * h),
          (ke(th, n + h, u) - ke(th, n - h, u)) / (2 * h),
          (ke(th, n, u + h * u) - ke(th, n, u - h * u)) / (2 * h * u)]
    J, g = M.ifdlbm_adjoint(M.Cavity(nx, ny, re, n, th, u),
                            M.ifdlbm_default_options(precision=precision, kernel="fused"), steps, 500)
    J64 = ke(th, n, u)
    print(precision, "J", J, J64, "adjoint", g, "central", fd, flush=True)
    assert abs(J - J64) <= 1e-4 * J64
    for q in range(3):
        err = abs(g[q] - fd[q]) / abs(fd[q])
        print("param %d rel %.2e" % (q, err), flush=True)
        assert err <= 1e-4
