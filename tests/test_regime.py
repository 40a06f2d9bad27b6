"""Host-side regime classifier of probe series (ifdlbm_classify) on signals
whose regime and frequencies are known in closed form."""
import numpy as np
import pytest

import paper_2306_07603_amd as M

DT = 0.5
T = np.arange(4000) * DT


def test_periodic_with_harmonic():
    f = 0.0137
    x = 0.3 + 0.01 * np.sin(2 * np.pi * f * T) + 0.003 * np.sin(2 * np.pi * 2 * f * T + 0.4)
    r = M.ifdlbm_classify(x, DT)
    assert r["name"] == "periodic", r
    assert abs(r["f_main"] - f) <= 2e-3 * f, r
    assert abs(r["mean"] - x.mean()) < 1e-12 and r["harmonic_fraction"] > 0.99


def test_quasi_periodic_two_incommensurate_frequencies():
    f1, f2 = 0.021, 0.021 * (1 + 5 ** 0.5) / 2
    x = np.sin(2 * np.pi * f1 * T) + 0.6 * np.sin(2 * np.pi * f2 * T + 1.0)
    r = M.ifdlbm_classify(x, DT)
    assert r["name"] == "quasi-periodic", r
    assert abs(r["f_main"] - f1) <= 2e-3 * f1 and abs(r["f_second"] - f2) <= 2e-3 * f2, r


def test_steady_below_tolerance():
    rng = np.random.default_rng(5)
    x = 0.02 + 1e-10 * rng.standard_normal(T.size)
    r = M.ifdlbm_classify(x, DT, steady_tol=1e-6)
    assert r["name"] == "steady" and r["f_main"] == 0.0, r


def test_white_noise_is_aperiodic():
    rng = np.random.default_rng(6)
    r = M.ifdlbm_classify(rng.standard_normal(T.size), DT)
    assert r["name"] == "aperiodic", r


def test_frequency_units_follow_sample_spacing():
    f = 0.05
    x = np.cos(2 * np.pi * f * T)
    a = M.ifdlbm_classify(x, DT)
    b = M.ifdlbm_classify(x, DT * 2)   # same samples, twice the spacing: half the frequency
    assert abs(a["f_main"] - f) <= 1e-3 * f and abs(b["f_main"] - f / 2) <= 1e-3 * f


@pytest.mark.parametrize("x,dt", [(np.zeros(8), 1.0), (np.r_[np.zeros(31), np.nan], 1.0), (np.zeros(64), 0.0)])
def test_classify_rejects_bad_input(x, dt):
    with pytest.raises(M.IfdlbmError) as e:
        M.ifdlbm_classify(x, dt)
    assert e.value.code == M.IFDLBM_EINVAL


def test_periodic_on_a_drift_is_periodic():
    f = 0.0137
    x = 0.3 + 2e-5 * T + 0.01 * np.sin(2 * np.pi * f * T)
    r = M.ifdlbm_classify(x, DT)
    assert r["name"] == "periodic", r
    assert abs(r["f_main"] - f) <= 2e-3 * f, r


def test_decaying_transient_is_not_periodic():
    """A relaxation still under way (slow exponential plus a period longer
    than the record) has no spectral peak above 1.5 cycles per record."""
    x = 0.02 + 0.005 * np.exp(-T / 700.0) + 0.002 * np.sin(2 * np.pi * T / 2600.0)
    r = M.ifdlbm_classify(x, DT)
    assert r["name"] == "aperiodic", r
