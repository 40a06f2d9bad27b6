"""The C ABI library loads and exports every call include/ifdlbm.h declares;
argument validation rejects bad input before any device work (no GPU)."""
import ctypes
import os
import re

import pytest

import paper_2306_07603_amd as M

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_calls():
    text = open(os.path.join(ROOT, "include", "ifdlbm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ifdlbm_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_call():
    L = M.lib()
    names = declared_calls()
    assert len(names) >= 16
    for n in names:
        assert hasattr(L, n), n


def test_binding_has_same_names():
    for n in declared_calls():
        assert hasattr(M, n), n


def test_default_options():
    o = M.ifdlbm_default_options()
    assert o.precision == M.IFDLBM_FP64 and o.cfl == 0.5 and o.mix == 0.75 and o.rho0 == 1.0
    assert o.gamma_min == 1e-6 and o.residual_every == 1 and o.batched == 1 and o.graph_steps == 0
    assert o.segment_rows == 0 and o.dt_rule == M.IFDLBM_DT_CONTRAVARIANT


def test_unknown_option_name_is_an_error():
    with pytest.raises(TypeError):
        M.ifdlbm_default_options(segment_row=64)


BAD_CAVITIES = [
    M.Cavity(4, 17, 100.0, 1.0, 60.0),     # too few nodes
    M.Cavity(17, 17, 100.0, 1.0, 0.0),     # theta out of (0, 90]
    M.Cavity(17, 17, 100.0, 1.0, 95.0),
    M.Cavity(17, 17, 100.0, 0.0, 60.0),    # n <= 0
    M.Cavity(17, 17, -1.0, 1.0, 60.0),     # Re <= 0
    M.Cavity(17, 17, 100.0, 1.0, 60.0, 0.0),   # lid at rest: Re of Eq. (2.15.1) undefined
    M.Cavity(17, 17, float("nan"), 1.0, 60.0),
    M.Cavity(5793, 5793, 100.0, 1.0, 60.0),   # nine FP64 planes would span 4 GiB or more
    M.Cavity(4097, 4097, 100.0, 1.0, 60.0),   # n_eta * pitch above 2^24: FP64 planes past the 2 GiB drop offset
    M.Cavity(32768, 5, 100.0, 1.0, 60.0),     # n_xi beyond 16-bit column indices
]


@pytest.mark.parametrize("cav", BAD_CAVITIES)
def test_create_rejects_bad_cavity(cav):
    with pytest.raises(M.IfdlbmError) as e:
        M.ifdlbm_create([cav])
    assert e.value.code == M.IFDLBM_EINVAL


@pytest.mark.parametrize("field,value", [("cfl", 0.0), ("mix", 1.5), ("gamma_min", 0.0), ("residual_every", 0),
                                         ("precision", 7), ("kernel", 9), ("graph_steps", 3),
                                         ("segment_rows", 7), ("segment_rows", 5000), ("dt_rule", 2),
                                         ("lambda_mode", 2)])
def test_create_rejects_bad_options(field, value):
    o = M.ifdlbm_default_options(**{field: value})
    with pytest.raises(M.IfdlbmError) as e:
        M.ifdlbm_create([M.Cavity(17, 17, 100.0, 1.0, 60.0)], o)
    assert e.value.code == M.IFDLBM_EINVAL


def test_strerror_texts():
    L = M.lib()
    for code in (0, -1, -2, -3, -4, -5):
        assert L.ifdlbm_strerror(code)
    assert L.ifdlbm_strerror(-99) == b"unknown error code"


def test_batch_recipe_is_seeded_and_in_range():
    a, b = M.workloads.batch_sweep(), M.workloads.batch_sweep()
    assert a == b and len(a) == 256
    for c in a:
        assert c.n_xi in (65, 129, 257, 513) and c.n_xi == c.n_eta
        assert 100.0 <= c.re <= 5000.0 and 0.5 <= c.n <= 1.5 and 40.0 <= c.theta_deg <= 90.0
    # SplitMix64 of the published definition: first output for seed 0
    assert M.workloads.splitmix64(0)[1] == 0xE220A8397B1DCDAF


def test_gradient_calls_reject_bad_arguments():
    cav = M.Cavity(17, 17, 100.0, 0.8, 60.0, 0.1)
    o = M.ifdlbm_default_options()
    calls = [
        lambda: M.ifdlbm_adjoint(cav, o, 0, 10),
        lambda: M.ifdlbm_adjoint(cav, o, 10, 0),
        lambda: M.ifdlbm_adjoint(cav, o, 1 << 40, 1),   # more than 2^24 checkpoints
        lambda: M.ifdlbm_adjoint(cav, o, 10, 5, objective=3),
        lambda: M.ifdlbm_adjoint(cav, M.ifdlbm_default_options(lambda_mode=M.IFDLBM_LAMBDA_IMPLICIT), 10, 5),
        lambda: M.ifdlbm_adjoint(M.Cavity(4, 17, 100.0, 0.8, 60.0), o, 10, 5),
        lambda: M.ifdlbm_adjoint(cav, M.ifdlbm_default_options(cfl=0.0), 10, 5),
        lambda: M.ifdlbm_gradient(cav, o, 0),
        lambda: M.ifdlbm_gradient(cav, M.ifdlbm_default_options(lambda_mode=M.IFDLBM_LAMBDA_IMPLICIT), 10),
    ]
    for call in calls:
        with pytest.raises(M.IfdlbmError) as e:
            call()
        assert e.value.code == M.IFDLBM_EINVAL


def test_autotune_rejects_bad_arguments():
    L = M.lib()
    assert L.ifdlbm_autotune(None, 5, None, None) == M.IFDLBM_EINVAL


def test_stale_library_is_refused(monkeypatch):
    """The library carries the digest of the sources it was built from; the binding refuses a library whose
    digest differs from that of the sources beside it."""
    from paper_2306_07603_amd import _build
    L = M.ifdlbm.lib()
    assert M.ifdlbm_build_digest() == _build.source_digest()
    monkeypatch.setattr(_build, "source_digest", lambda: "0" * 64)
    with pytest.raises(ImportError, match="rebuild"):
        M.ifdlbm.verify_build(L)
