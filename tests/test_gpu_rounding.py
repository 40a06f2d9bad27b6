"""The stochastic rounding of the FP32SR / FP32SRF storage modes, checked exactly
through ifdlbm_round_stochastic_device: the random bits are inputs here, so
every output is fixed by the definition (add 16 random bits at the top of the
29 significand bits FP32 drops, then truncate them), and over all 2^16 random
numbers the count of values rounded away from zero is floor(2^16 x the dropped
fraction) exactly.  The step's statistical check of the same rounding is
test_fp32sr_rounding_is_unbiased."""
import numpy as np
import pytest
import torch

import paper_2306_07603_amd as M

pytestmark = pytest.mark.gpu

DROP = np.uint64(0x1FFFFFFF)   # the 29 low significand bits of an FP64 value that FP32 does not keep


def definition(v, r16):
    """The rounding written out on the bit patterns (FP64 sign-magnitude: adding to the magnitude bits rounds
    away from zero; a carry out of the dropped bits moves to the next FP32 value, exponent included)."""
    b = v.view(np.uint64)
    b = (b + ((r16.astype(np.uint64) & np.uint64(0xFFFF)) << np.uint64(13))) & ~DROP
    return b.view(np.float64).astype(np.float32)   # exact: the low 29 bits are zero (normal range)


def on_device(v, r16):
    vd = torch.from_numpy(v).cuda()
    rd = torch.from_numpy(r16.astype(np.int32)).cuda()
    out = torch.empty(v.size, dtype=torch.float32, device="cuda")
    M.ifdlbm_round_stochastic_device(vd, rd, out)
    return out.cpu().numpy()


def sample_values(rng, n):
    mag = 10.0 ** rng.uniform(-6.0, 3.0, n)
    v = np.where(rng.random(n) < 0.5, -mag, mag)
    exact = v[: n // 8].astype(np.float32).astype(np.float64)                 # FP32 values: unchanged by any bits
    a = v[n // 8: n // 4].astype(np.float32)
    mid = (a.astype(np.float64) + np.nextafter(a, np.float32(np.inf)).astype(np.float64)) / 2   # half-way points
    below = np.ldexp(1.0, rng.integers(-20, 10, n // 8)) * (1.0 - 2.0 ** -40)  # a carry into the exponent
    return np.concatenate([v[n // 4 + n // 8:], exact, mid, below, -below])


def test_rounding_matches_its_definition_bitwise():
    rng = np.random.default_rng(2306)
    v = sample_values(rng, 1 << 20)
    r16 = rng.integers(0, 1 << 32, v.size, dtype=np.uint64).astype(np.uint32)   # high bits must be ignored
    got, want = on_device(v, r16), definition(v, r16)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    # the FP32 values themselves never move
    ex = v == v.astype(np.float32).astype(np.float64)
    assert ex.sum() > 1000 and np.array_equal(got[ex], v[ex].astype(np.float32))
    # every output is one of the two FP32 neighbours of v
    t = (v.view(np.uint64) & ~DROP).view(np.float64).astype(np.float32)          # truncation toward zero
    away = np.nextafter(t, np.where(v > 0, np.float32(np.inf), np.float32(-np.inf)))
    assert np.all((got == t) | (got == away))


def test_probability_of_rounding_away_is_exact():
    """All 65 536 random numbers for each of 36 values (random, FP32, half-way and carrying ones): the number
    that round away from zero equals the top 16 of the 29 dropped bits, floor(2^16 x dropped fraction)."""
    rng = np.random.default_rng(75)
    vals = sample_values(rng, 32)
    assert vals.size == 36
    r16 = np.arange(1 << 16, dtype=np.uint32)
    v = np.repeat(vals, r16.size)
    got = on_device(v, np.tile(r16, vals.size)).reshape(vals.size, r16.size)
    for q, x in enumerate(vals):
        bits = np.array([x]).view(np.uint64)[0]
        t = np.array([bits & ~DROP], dtype=np.uint64).view(np.float64).astype(np.float32)[0]
        n_away = int(np.count_nonzero(got[q] != t))
        assert n_away == int((bits & DROP) >> np.uint64(13)), (x, n_away)
        # the rounded-away results are all the same neighbour
        assert np.unique(got[q][got[q] != t]).size <= 1


def test_rejects_bad_arguments():
    x = torch.zeros(4, dtype=torch.float64, device="cuda")
    r = torch.zeros(4, dtype=torch.int32, device="cuda")
    o = torch.zeros(4, dtype=torch.float32, device="cuda")
    lib = M.ifdlbm.lib()
    import ctypes
    assert lib.ifdlbm_round_stochastic_device(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(r.data_ptr()),
                                              ctypes.c_void_p(o.data_ptr()), -1, None) == M.IFDLBM_EINVAL
    assert lib.ifdlbm_round_stochastic_device(None, ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(o.data_ptr()), 4,
                                              None) == M.IFDLBM_EINVAL
    assert lib.ifdlbm_round_stochastic_device(None, None, None, 0, None) == M.IFDLBM_OK
