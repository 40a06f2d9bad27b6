"""GPU library against the CPU oracle, element by element, through the C ABI.

Bars: FP64 max relative difference <= 1e-12 per field (max |a - b| / max |b|)
over fixed step counts; FP32 <= 1e-5 on the velocity; batched, graph-replayed
and rerun results bitwise equal to their plain counterparts.

The oracle runs with rho0 = 0.  u and P do not depend on rho0 (a pin of the
oracle), and the library stores f-hat as deviations from omega_k rho0; an
oracle run with rho0 = 1 carries, in P, the FP64 cancellation of recovering
an O(0.01) pressure from O(1) population sums (Eq. 2.11), about 1e-11
relative after 2000 steps, which test_oracle_at_rho0_one bounds separately.
"""
import numpy as np
import pytest

import oracle as O
import paper_2306_07603_amd as M
from paper_2306_07603_amd import workloads as W

pytestmark = pytest.mark.gpu

KERNELS = ["staged", "fused"]
FP64_TOL = 1e-12
FP32_TOL = 1e-5


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def oparams(spec, **kw):
    kw.setdefault("rho0", 0.0)
    return O.Params(nx=spec.n_xi, ny=spec.n_eta, re=spec.re, n=spec.n, theta_deg=spec.theta_deg, u_lid=spec.u_lid, **kw)


def cav(spec):
    return M.Cavity(spec.n_xi, spec.n_eta, spec.re, spec.n, spec.theta_deg, spec.u_lid)


def gpu(specs, steps, precision="fp64", kernel="staged", **opt):
    opt.setdefault("rho0", 0.0)
    o = M.ifdlbm_default_options(precision=precision, kernel=kernel, **opt)
    h = M.ifdlbm_create([cav(s) for s in specs], o)
    if steps:
        M.ifdlbm_step(h, steps)
    return h


W9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def compare_fp64(h, c, spec, steps, tol=FP64_TOL, p_tol=None, **okw):
    u, v, p = M.ifdlbm_get_fields(h, c)
    uo, vo, po, Fo, Lo = O.simulate(oparams(spec, **okw), steps)
    F, L = M.ifdlbm_get_state(h, c)
    F = F + (okw.get("rho0", 0.0) - h.options.rho0) * W9[:, None, None]
    errs = {"u": rel(u, uo), "v": rel(v, vo), "P": rel(p, po), "lambda": rel(L, Lo), "fhat": rel(F, Fo)}
    print(spec, steps, errs, flush=True)
    for k, e in errs.items():
        assert e <= (p_tol if (k == "P" and p_tol) else tol), (k, e)
    return errs


@pytest.mark.parametrize("kernel", KERNELS)
def test_oracle_at_rho0_one(kernel):
    """Against the oracle at rho0 = 1 (both sides): u, v, lambda, f-hat within
    1e-12; P within the oracle's own cancellation bound."""
    spec = W.single_small()
    h = gpu([spec], 2000, kernel=kernel, rho0=1.0)
    errs = compare_fp64(h, 0, spec, 2000, p_tol=3e-11, rho0=1.0)
    assert errs["P"] > 0


@pytest.mark.parametrize("kernel", KERNELS)
def test_single_small_fp64_2000_steps(kernel):
    spec = W.single_small()
    h = gpu([spec], 2000, kernel=kernel)
    compare_fp64(h, 0, spec, 2000)


TINY = [W.CavitySpec(17, 17, 100.0, n, th) for th in (40.0, 45.0, 60.0, 75.0, 90.0) for n in (0.5, 1.0, 1.5)] + [
    W.CavitySpec(13, 21, 300.0, 0.7, 60.0), W.CavitySpec(21, 13, 50.0, 1.3, 45.0),
    W.CavitySpec(5, 5, 10.0, 0.9, 70.0), W.CavitySpec(70, 9, 500.0, 1.0, 80.0)]


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("spec", TINY, ids=lambda s: "%dx%d_th%g_n%g" % (s.n_xi, s.n_eta, s.theta_deg, s.n))
def test_tiny_variants_fp64(kernel, spec):
    h = gpu([spec], 60, kernel=kernel)
    compare_fp64(h, 0, spec, 60)


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("opt", [{"mix": 0.25}, {"mix": 1.0}, {"mix": 0.7}, {"cfl": 0.25}, {"rho0": 2.0}, {"gamma_min": 1e-3},
                                 {"dt_rule": M.IFDLBM_DT_CARTESIAN}, {"dt_rule": M.IFDLBM_DT_CARTESIAN, "mix": 0.5}])
def test_options_fp64(kernel, opt):
    spec = W.CavitySpec(19, 17, 200.0, 0.6, 55.0)
    h = gpu([spec], 80, kernel=kernel, **opt)
    okw = {k: v for k, v in opt.items() if k != "rho0"}   # fields do not depend on rho0
    compare_fp64(h, 0, spec, 80, **okw)


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("spec", [W.CavitySpec(17, 17, 100.0, 0.5, 60.0), W.CavitySpec(21, 19, 400.0, 1.4, 45.0),
                                  W.CavitySpec(33, 33, 1000.0, 0.8, 90.0)],
                         ids=lambda s: "%dx%d_n%g" % (s.n_xi, s.n_eta, s.n))
def test_implicit_lambda_fp64(kernel, spec):
    """Step (2) solved for its own fixed point (lambda_mode IMPLICIT) against
    the oracle's bisection of the same equation."""
    h = gpu([spec], 300, kernel=kernel, lambda_mode=M.IFDLBM_LAMBDA_IMPLICIT)
    compare_fp64(h, 0, spec, 300, lambda_mode=O.LAMBDA_IMPLICIT)


@pytest.mark.parametrize("kernel", KERNELS)
def test_negative_lid(kernel):
    spec = W.CavitySpec(17, 15, 100.0, 0.7, 60.0, -0.1)
    h = gpu([spec], 100, kernel=kernel)
    compare_fp64(h, 0, spec, 100)


@pytest.mark.parametrize("kernel", KERNELS)
def test_full_size_grids_fp64(kernel):
    """Full-size sides of the uneven batch (257 and 513 nodes), short runs, whole fields."""
    for spec, steps in ((W.CavitySpec(257, 257, 1000.0, 0.5, 45.0), 12), (W.CavitySpec(513, 513, 3000.0, 1.5, 40.0), 4)):
        h = gpu([spec], steps, kernel=kernel)
        compare_fp64(h, 0, spec, steps)
        h.close()


@pytest.mark.parametrize("spec", [W.CavitySpec(4096, 4096, 1000.0, 1.0, 60.0),     # largest square: n_eta * pitch = 2^24
                                  W.CavitySpec(32767, 512, 400.0, 0.8, 90.0)])     # widest: 32767 columns, pitch 32768
def test_maximum_size_cavity_fp64(spec):
    """A cavity at the size limit of ifdlbm_create (nine FP64 planes of 1.125 GiB in all), one step with each
    kernel, whole fields against the oracle.  Stores that the step drops go past the end of these planes.
    u, v, lambda, f-hat within 1e-12; P within the cancellation bound of recovering a small pressure from the
    sums of the populations (3e-11, as at rho0 = 1)."""
    steps = 1
    uo, vo, po, Fo, Lo = O.simulate(oparams(spec), steps)
    # one step after the start, v exists only next to the lid corners and is orders of magnitude below u: both
    # components are measured against the velocity scale, so that an ulp of the lid speed does not count as a
    # relative error of v
    vs = max(np.abs(uo).max(), np.abs(vo).max())
    print("max |u|", np.abs(uo).max(), "max |v|", np.abs(vo).max(), "max |P|", np.abs(po).max(), flush=True)
    for kernel in KERNELS:
        print("maximum size", spec, kernel, flush=True)
        h = gpu([spec], steps, kernel=kernel)
        u, v, p = M.ifdlbm_get_fields(h, 0)
        F, L = M.ifdlbm_get_state(h, 0)
        h.close()
        errs = {"u": float(np.abs(u - uo).max() / vs), "v": float(np.abs(v - vo).max() / vs), "P": rel(p, po),
                "lambda": rel(L, Lo), "fhat": rel(F, Fo)}
        print(kernel, errs, flush=True)
        for k, e in errs.items():
            assert e <= (3e-11 if k == "P" else FP64_TOL), (kernel, k, e)
    # the benchmarked storage mode on the same planes (FP32: 0.56 GiB), fused kernel
    h = gpu([spec], steps, "fp32srf", "fused")
    u, v, _ = M.ifdlbm_get_fields(h, 0)
    h.close()
    errs = (float(np.abs(u - uo).max() / vs), float(np.abs(v - vo).max() / vs))
    print("fp32srf fused errors u v", errs, flush=True)
    assert errs[0] <= FP32_TOL and errs[1] <= FP32_TOL


@pytest.mark.parametrize("kernel", KERNELS)
def test_batched_equals_unbatched_bitwise(kernel):
    specs = [W.CavitySpec(17, 17, 100.0, 0.8, 60.0), W.CavitySpec(65, 65, 1000.0, 1.2, 45.0),
             W.CavitySpec(13, 29, 400.0, 0.5, 80.0), W.CavitySpec(129, 129, 2000.0, 1.0, 90.0)]
    hb = gpu(specs, 30, kernel=kernel, batched=1)
    hu = gpu(specs, 30, kernel=kernel, batched=0)
    for c in range(len(specs)):
        Fb, Lb = M.ifdlbm_get_state(hb, c)
        Fu, Lu = M.ifdlbm_get_state(hu, c)
        assert np.array_equal(Fb, Fu) and np.array_equal(Lb, Lu), c


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_graph_equals_eager_bitwise(kernel, precision):
    specs = [W.CavitySpec(33, 33, 100.0, 0.8, 60.0), W.CavitySpec(65, 65, 500.0, 1.3, 50.0)]
    he = gpu(specs, 0, precision, kernel, residual_every=5)
    hg = gpu(specs, 0, precision, kernel, residual_every=5, graph_steps=10)
    for n in (3, 25, 40):   # unaligned start, several replays, aligned tail
        M.ifdlbm_step(he, n)
        M.ifdlbm_step(hg, n)
    for c in range(2):
        Fe, Le = M.ifdlbm_get_state(he, c)
        Fg, Lg = M.ifdlbm_get_state(hg, c)
        assert np.array_equal(Fe, Fg) and np.array_equal(Le, Lg)
    re_, rg = M.ifdlbm_get_residuals(he), M.ifdlbm_get_residuals(hg)
    assert np.array_equal(re_[0], rg[0]) and np.array_equal(re_[1], rg[1])


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("precision", ["fp32", "fp32sr", "fp32srf"])
def test_rerun_bitwise(kernel, precision):
    specs = [W.CavitySpec(65, 65, 800.0, 0.6, 50.0)]
    a = M.ifdlbm_get_state(gpu(specs, 50, precision, kernel), 0)
    b = M.ifdlbm_get_state(gpu(specs, 50, precision, kernel), 0)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("precision", ["fp32sr", "fp32srf"])
def test_fp32sr_graph_replay_equals_eager_calls_bitwise(kernel, precision):
    """Stochastic rounding draws its random words from a counter bumped once
    per call (eager) or per replay (graph) and the step index within it: a
    replay of G steps and an eager call of G steps store the same values."""
    specs = [W.CavitySpec(33, 33, 100.0, 0.8, 60.0), W.CavitySpec(65, 65, 500.0, 1.3, 50.0)]
    he = gpu(specs, 0, precision, kernel, residual_every=5)
    hg = gpu(specs, 0, precision, kernel, residual_every=5, graph_steps=10)
    for _ in range(3):
        M.ifdlbm_step(he, 10)
        M.ifdlbm_step(hg, 10)
    for c in range(2):
        Fe, Le = M.ifdlbm_get_state(he, c)
        Fg, Lg = M.ifdlbm_get_state(hg, c)
        assert np.array_equal(Fe, Fg) and np.array_equal(Le, Lg)
    re_, rg = M.ifdlbm_get_residuals(he), M.ifdlbm_get_residuals(hg)
    assert np.array_equal(re_[0], rg[0]) and np.array_equal(re_[1], rg[1])


@pytest.mark.parametrize("kernel", KERNELS)
def test_fp32sr_rounding_is_unbiased(kernel):
    """Sixteen one-step updates from the same FP32 state with different random
    words: every stored value takes one of two adjacent FP32 numbers lo < hi
    around the pre-rounding value, and the frequency of hi matches the
    fraction (v - lo) / (hi - lo) of the FP64 update v.  The stochastic mode
    takes the relaxation coefficients in FP32, so its pre-rounding value can
    differ from v by a fraction of an ulp where the collision increment is
    large against the value: a Newtonian fluid (no FP32 power law) and the
    values above 1e-3 of the largest keep that below 2% of the values, which
    are excluded."""
    K = 16
    spec = W.CavitySpec(129, 129, 400.0, 1.0, 60.0)
    h32 = gpu([spec], 200, "fp32", kernel)
    F, L = M.ifdlbm_get_state(h32, 0)
    F = F.astype(np.float32).astype(np.float64)
    L = L.astype(np.float32).astype(np.float64)
    h64 = gpu([spec], 0, "fp64", kernel)
    M.ifdlbm_set_state(h64, 0, F, L)
    M.ifdlbm_step(h64, 1)
    v = M.ifdlbm_get_state(h64, 0)[0].ravel()
    big = np.abs(v) >= 1e-3 * np.abs(v).max()
    v = v[big]
    hsr = gpu([spec], 0, "fp32sr", kernel)
    draws = []
    for _ in range(K):   # each call advances the random-word counter
        M.ifdlbm_set_state(hsr, 0, F, L)
        M.ifdlbm_step(hsr, 1)
        draws.append(M.ifdlbm_get_state(hsr, 0)[0].ravel()[big].astype(np.float32))
    d = np.stack(draws)
    dmin, dmax = d.min(axis=0), d.max(axis=0)
    # at most two distinct values per element, and adjacent
    assert np.all((dmax == dmin) | (dmax == np.nextafter(dmin, np.float32(np.inf))))
    rn = v.astype(np.float32)
    lo = np.where(rn.astype(np.float64) <= v, rn, np.nextafter(rn, np.float32(-np.inf)))
    hi = np.where(rn.astype(np.float64) >= v, rn, np.nextafter(rn, np.float32(np.inf)))
    inside = (hi > lo) & np.all((d == lo) | (d == hi), axis=0)
    print("values %d, draws next to v: %.5f" % (v.size, inside.mean()), flush=True)
    assert inside.mean() >= 0.98 and inside.sum() > 20000
    lo64, hi64 = lo.astype(np.float64), hi.astype(np.float64)
    phi = (v[inside] - lo64[inside]) / (hi64[inside] - lo64[inside])
    up = (d[:, inside] == hi[inside]).mean(axis=0)
    for b in range(10):
        sel = (phi >= b / 10) & (phi < (b + 1) / 10)
        n = int(sel.sum()) * K
        p = float(phi[sel].mean())
        freq = float(up[sel].mean())
        sigma = np.sqrt(max(p * (1 - p), 1e-4) / n)
        print("bin %d: draws %d  P(up) expected %.4f observed %.4f" % (b, n, p, freq), flush=True)
        assert abs(freq - p) <= 5 * sigma + 0.005, b


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("precision", ["fp32", "fp32x", "fp32sr", "fp32srf"])
def test_fp32_against_oracle(kernel, precision):
    spec = W.single_small()
    h = gpu([spec], 2000, precision, kernel)
    u, v, p = M.ifdlbm_get_fields(h, 0)
    uo, vo, po, _, _ = O.simulate(oparams(spec), 2000)
    errs = (rel(u, uo), rel(v, vo), rel(p, po))
    print(precision, "errors u v P", errs, flush=True)
    assert errs[0] <= FP32_TOL and errs[1] <= FP32_TOL


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("precision", ["fp32sr", "fp32srf"])
def test_implicit_lambda_fp32_storage_against_oracle(kernel, precision):
    """Step (2) solved for its own fixed point in the FP32 storage modes with stochastic rounding, against the
    FP64 oracle's bisection of the same equation after 2000 steps of the 33 x 33 case (n = 0.8: the power law
    matters): the velocity within the FP32 bar of the explicit modes (1e-5)."""
    spec = W.CavitySpec(33, 33, 100.0, 0.8, 60.0)
    h = gpu([spec], 2000, precision, kernel, lambda_mode=M.IFDLBM_LAMBDA_IMPLICIT)
    u, v, p = M.ifdlbm_get_fields(h, 0)
    uo, vo, po, _, Lo = O.simulate(oparams(spec, lambda_mode=O.LAMBDA_IMPLICIT), 2000)
    L = M.ifdlbm_get_state(h, 0)[1]
    errs = (rel(u, uo), rel(v, vo), rel(p, po), rel(L, Lo))
    print(precision, kernel, "implicit lambda: errors u v P lambda", errs, flush=True)
    assert errs[0] <= FP32_TOL and errs[1] <= FP32_TOL


def fp16dev_noise_bound(spec, steps, weights_sq_sum, scale=1.0):
    """Largest error expected at a node of a sum of populations (scale times sum_k a_k g_k) stored as FP16 of
    g_k / omega_k with stochastic rounding.  Values |g/omega| < 1/2 have an FP16 ulp of at most 2^-12, and a
    rounding that keeps the upper neighbour with probability equal to the dropped fraction leaves a zero-mean
    error of variance p (1 - p) ulp^2, ulp^2 / 6 on average: per step the sum gets
    sigma = scale ulp sqrt(sum_k a_k^2 omega_k^2 / 6).  The noise is white in space; viscosity damps its
    grid-scale part within tau = 1 / (8 nu dt / dxi^2) steps (nu = U / Re, the viscosity of the initial
    lambda), and the ln(M) octaves of the M nodes' modes each hold about that share, so the accumulated
    standard deviation is at most sigma sqrt(tau ln M) (below sigma sqrt(steps), the undamped walk), and
    the largest of M nodes stays within 4.5 of it."""
    import math
    ulp = 2.0 ** -12
    sigma = scale * ulp * math.sqrt(weights_sq_sum / 6.0)
    p = oparams(spec)
    d = O.derive(p)
    nu = abs(spec.u_lid) / spec.re
    tau = 1.0 / (8.0 * nu * d["dt"] / d["dxi"] ** 2)
    m = spec.n_xi * spec.n_eta
    return 4.5 * sigma * math.sqrt(min(tau * math.log(m), steps))


@pytest.mark.parametrize("kernel", KERNELS)
def test_fp16dev_against_oracle(kernel):
    """FP16 storage of g_k / omega_k with stochastic rounding against the FP64 oracle after 2000 steps of
    the 33 x 33 case: the velocity within the accumulated rounding noise of its populations, the pressure
    likewise (both bounds from fp16dev_noise_bound)."""
    spec = W.single_small()
    steps = 2000
    h = gpu([spec], steps, "fp16dev", kernel)
    u, v, p = M.ifdlbm_get_fields(h, 0)
    uo, vo, po, _, _ = O.simulate(oparams(spec), steps)
    w = W9
    # u = sum c_kx g_k: weights c_kx^2 omega_k^2; P = 0.6 sum_{k>0} g_k - 0.4 |u|^2: weights omega_k^2 (k > 0)
    bu = fp16dev_noise_bound(spec, steps, float((np.array([0, 1, 0, 1, 0, 1, 1, 1, 1]) * w * w).sum()))
    bp = fp16dev_noise_bound(spec, steps, float((w[1:] * w[1:]).sum()), 0.6)
    errs = {"u": float(np.abs(u - uo).max()), "v": float(np.abs(v - vo).max()), "P": float(np.abs(p - po).max())}
    print("fp16dev absolute errors", errs, "bounds u, v %.3e, P %.3e" % (bu, bp),
          "relative to max |u| %.3e, max |P| %.3e" % (errs["u"] / np.abs(uo).max(), errs["P"] / np.abs(po).max()),
          flush=True)
    assert errs["u"] <= bu and errs["v"] <= bu and errs["P"] <= bp


@pytest.mark.parametrize("kernel", KERNELS)
def test_divergence_is_isolated(kernel):
    specs = [W.CavitySpec(17, 17, 100.0, 0.8, 60.0), W.CavitySpec(17, 17, 100.0, 1.0, 45.0),
             W.CavitySpec(33, 33, 500.0, 1.2, 75.0)]
    h = gpu(specs, 0, kernel=kernel)
    ref = gpu([specs[0], specs[2]], 0, kernel=kernel)
    F, L = M.ifdlbm_get_state(h, 1)
    F[3, 8, 8] = np.nan
    M.ifdlbm_set_state(h, 1, F, L)
    rc, steps, ru, rp = M.ifdlbm_run_to_steady(h, 1e-14, 40)
    assert rc == M.IFDLBM_EDIVERGED
    assert M.ifdlbm_status(h, 1) == M.IFDLBM_STATUS_DIVERGED and steps[1] == 1
    assert M.ifdlbm_status(h, 0) == M.IFDLBM_STATUS_NOT_CONVERGED and steps[0] == 40
    M.ifdlbm_step(ref, 40)
    for c, rc_ in ((0, 0), (2, 1)):
        a = M.ifdlbm_get_state(h, c)
        b = M.ifdlbm_get_state(ref, rc_)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("kernel", KERNELS)
def test_divergence_found_by_get_residuals(kernel):
    """Fixed-count stepping: reading the residuals marks a non-finite cavity
    DIVERGED and stops it; the others continue bitwise as without it."""
    specs = [W.CavitySpec(17, 17, 100.0, 0.8, 60.0), W.CavitySpec(17, 17, 100.0, 1.0, 45.0),
             W.CavitySpec(33, 33, 500.0, 1.2, 75.0)]
    h = gpu(specs, 0, kernel=kernel, residual_every=5)
    ref = gpu([specs[0], specs[2]], 0, kernel=kernel, residual_every=5)
    F, L = M.ifdlbm_get_state(h, 1)
    F[3, 8, 8] = np.nan
    M.ifdlbm_set_state(h, 1, F, L)
    M.ifdlbm_step(h, 10)
    ru, rp = M.ifdlbm_get_residuals(h)
    assert np.isnan(ru[1]) and np.isfinite(ru[0]) and np.isfinite(ru[2])
    assert M.ifdlbm_status(h, 1) == M.IFDLBM_STATUS_DIVERGED
    assert M.ifdlbm_status(h, 0) == M.IFDLBM_STATUS_RUNNING and M.ifdlbm_status(h, 2) == M.IFDLBM_STATUS_RUNNING
    M.ifdlbm_step(h, 10)
    M.ifdlbm_step(ref, 20)
    for c, rc_ in ((0, 0), (2, 1)):
        a = M.ifdlbm_get_state(h, c)
        b = M.ifdlbm_get_state(ref, rc_)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("kernel", KERNELS)
def test_run_to_steady_and_fp32_round_to_nearest_misses_the_bar(kernel):
    """Converge FP64 to E <= 1e-10, run FP32 with round-to-nearest storage as many steps: its steady velocity
    misses the 1e-5 bar (about 2.9e-5 on this case), because the rounding of the stored state acts as a
    constant forcing at the fixed point; the storage modes with stochastic rounding meet it on the same case
    (test_fp32sr_steady_velocity).  Bounded above so that a regression of the FP32 arithmetic still fails."""
    spec = W.CavitySpec(65, 65, 100.0, 0.8, 60.0)
    h64 = gpu([spec], 0, "fp64", kernel, residual_every=50)
    rc, steps, ru, rp = M.ifdlbm_run_to_steady(h64, 1e-10, 200000)
    print("fp64 steady after", steps, ru, rp, flush=True)
    assert rc == M.IFDLBM_OK and M.ifdlbm_status(h64, 0) == M.IFDLBM_STATUS_CONVERGED
    h32 = gpu([spec], int(steps[0]), "fp32", kernel)
    u64, v64, _ = M.ifdlbm_get_fields(h64, 0)
    u32, v32, _ = M.ifdlbm_get_fields(h32, 0)
    err = max(rel(u32, u64), rel(v32, v64))
    print("fp32 steady velocity error", err, flush=True)
    assert FP32_TOL < err < 1e-4


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("precision", ["fp32sr", "fp32srf"])
def test_fp32sr_steady_velocity(kernel, precision):
    """Converge FP64 to E <= 1e-10, run FP32 storage with stochastic rounding as
    many steps: the steady velocity stays within 1e-5 of the FP64 one."""
    spec = W.CavitySpec(65, 65, 100.0, 0.8, 60.0)
    h64 = gpu([spec], 0, "fp64", kernel, residual_every=500, graph_steps=1000)
    rc, steps, ru, rp = M.ifdlbm_run_to_steady(h64, 1e-10, 400000)
    print("fp64 steady after", steps, ru, rp, flush=True)
    assert rc == M.IFDLBM_OK and M.ifdlbm_status(h64, 0) == M.IFDLBM_STATUS_CONVERGED
    hsr = gpu([spec], 0, precision, kernel, residual_every=500, graph_steps=1000)
    M.ifdlbm_step(hsr, int(steps[0]))
    u64, v64, _ = M.ifdlbm_get_fields(h64, 0)
    u32, v32, _ = M.ifdlbm_get_fields(hsr, 0)
    err = max(rel(u32, u64), rel(v32, v64))
    print(precision, "steady velocity error", err, flush=True)
    assert err <= FP32_TOL


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("precision", ["fp32sr", "fp32srf"])
def test_batch_fp32sr_bench_configuration_against_oracle(kernel, precision):
    """The 256-cavity batch exactly as the benchmark times it (FP32 storage with
    stochastic rounding, one launch per step, 100-step graph replays, residual
    sums every 100 steps): after 200 steps, one sampled cavity of every side
    against the FP64 oracle."""
    specs = W.batch_sweep()
    steps = 200
    h = gpu(specs, steps, precision, kernel, residual_every=100, graph_steps=100, batched=1)
    picks = []
    for side in (65, 129, 257, 513):
        picks += [i for i, s in enumerate(specs) if s.n_xi == side][:1]
    for c in picks:
        u, v, p = M.ifdlbm_get_fields(h, c)
        uo, vo, po, _, _ = O.simulate(oparams(specs[c]), steps)
        errs = (rel(u, uo), rel(v, vo), rel(p, po))
        print(c, specs[c], precision, "errors u v P", errs, flush=True)
        assert errs[0] <= FP32_TOL and errs[1] <= FP32_TOL, c


@pytest.mark.parametrize("kernel", KERNELS)
def test_batch_sweep_sampled_against_oracle(kernel):
    """The 256-cavity uneven batch in the benchmark's launch configuration
    (all cavities in one launch per step, graph-replayed, residual sums every
    10 steps) in FP64: sampled cavities of every side against the oracle."""
    specs = W.batch_sweep()
    steps = 20
    h = gpu(specs, steps, "fp64", kernel, residual_every=10, graph_steps=10)
    picks = []
    for side in (65, 129, 257, 513):
        picks += [i for i, s in enumerate(specs) if s.n_xi == side][:1]
    for c in picks:
        compare_fp64(h, c, specs[c], steps)


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_batch_equals_single_cavity_runs(kernel, precision):
    """Batched and graph-replayed: each sampled cavity is bitwise equal to the
    same cavity run alone with one launch per step (the two runs split the
    cavity into different row segments)."""
    specs = W.batch_sweep()
    steps = 20
    h = gpu(specs, steps, precision, kernel, residual_every=10, graph_steps=10)
    for c in (0, 5, 17, 255):
        F, L = M.ifdlbm_get_state(h, c)
        F1, L1 = M.ifdlbm_get_state(gpu([specs[c]], steps, precision, kernel, residual_every=10), 0)
        assert np.array_equal(F, F1) and np.array_equal(L, L1), c


@pytest.mark.parametrize("precision", ["fp32", "fp32srf", "fp16dev"])
@pytest.mark.parametrize("rows", [0, 8, 24, 64, 4096])
def test_fused_segmentation_does_not_change_results(rows, precision):
    """Fused kernel with other segment lengths (0: the automatic choice): bitwise
    equal to 16-row segments, in the storage modes with round-to-nearest, with
    the exact final update and with FP16 stochastic rounding."""
    specs = [W.CavitySpec(129, 129, 400.0, 0.8, 60.0), W.CavitySpec(65, 97, 1000.0, 1.3, 45.0)]
    ref = gpu(specs, 30, precision, "fused", segment_rows=16)
    h = gpu(specs, 30, precision, "fused", segment_rows=rows)
    for c in range(2):
        a, b = M.ifdlbm_get_state(ref, c), M.ifdlbm_get_state(h, c)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), c


@pytest.mark.parametrize("precision", ["fp32sr", "fp64"])
def test_autotune_keeps_state_and_results(precision):
    """The tile-shape autotuner restores the state, step count and random-word
    counter: stepping after it is bitwise equal to stepping without it."""
    specs = [W.CavitySpec(129, 129, 400.0, 0.8, 60.0), W.CavitySpec(65, 97, 1000.0, 1.3, 45.0)]
    ref = gpu(specs, 20, precision, "fused")
    M.ifdlbm_step(ref, 15)
    h = gpu(specs, 20, precision, "fused")
    rows, ms = M.ifdlbm_autotune(h, 5)
    print(precision, rows, ms, flush=True)
    assert rows in (8, 16, 24, 32, 40, 48, 56, 64, 72, 80, 96, 128) and ms > 0.0
    M.ifdlbm_step(h, 15)
    for c in range(2):
        a, b = M.ifdlbm_get_state(ref, c), M.ifdlbm_get_state(h, c)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), c


def test_autotune_staged_is_a_no_op():
    h = gpu([W.CavitySpec(33, 33, 100.0, 0.8, 60.0)], 3, "fp64", "staged")
    assert M.ifdlbm_autotune(h, 2) == (0, 0.0)
