"""ifdlbm_gradient_noalloc through the C ABI against ifdlbm_gradient, the
entry point it is a variant of: the same kernels in a per-GPU scratch array
instead of a fresh allocation, so J and the three derivatives must agree
bitwise.  Two calls in a row, the second on a smaller grid (the scratch
array keeps the first call's contents), then a grid beyond the array's
capacity, which is refused before any device work."""
import numpy as np
import pytest

import paper_2306_07603_amd as M

pytestmark = pytest.mark.gpu

CASES = [
    # (cavity, steps, options): a larger grid first, then a smaller one over its leftovers
    (M.Cavity(33, 29, 400.0, 0.7, 60.0, 0.1), 60, {}),
    (M.Cavity(17, 13, 100.0, 1.3, 75.0, -0.1), 40, {"dt_rule": M.IFDLBM_DT_CARTESIAN, "mix": 0.5}),
]


def test_noalloc_gradient_equals_allocating_gradient():
    for cav, steps, kw in CASES:
        opt = M.ifdlbm_default_options(**kw)
        J0, g0 = M.ifdlbm_gradient(cav, opt, steps)
        J1, g1 = M.ifdlbm_gradient_noalloc(cav, opt, steps)
        print(cav, steps, kw, J0, g0, J1, g1, flush=True)
        assert np.isfinite(J0) and J0 > 0 and np.all(np.isfinite(g0))
        assert J1 == J0 and np.array_equal(g1, g0)


def test_noalloc_gradient_on_a_torch_stream():
    import torch
    s = torch.cuda.Stream()
    cav, steps, kw = CASES[1]
    J0, g0 = M.ifdlbm_gradient(cav, M.ifdlbm_default_options(**kw), steps)
    J1, g1 = M.ifdlbm_gradient_noalloc(cav, M.ifdlbm_default_options(hip_stream=s.cuda_stream, **kw), steps)
    assert J1 == J0 and np.array_equal(g1, g0)


def test_noalloc_gradient_rejects_grids_beyond_the_scratch_array():
    # 148 x 148 needs 48 * 21904 + 296 + 86 = 1 051 774 work values, more than the 2^20 the array holds
    with pytest.raises(M.IfdlbmError) as e:
        M.ifdlbm_gradient_noalloc(M.Cavity(148, 148, 100.0, 1.0, 60.0), M.ifdlbm_default_options(), 1)
    assert e.value.code == M.IFDLBM_EINVAL and "too large" in str(e.value)
    # the largest square that fits (147 x 147: 1 037 611 values) runs the full array, here for five steps
    J, g = M.ifdlbm_gradient_noalloc(M.Cavity(147, 147, 100.0, 1.0, 60.0), M.ifdlbm_default_options(), 5)
    J0, g0 = M.ifdlbm_gradient(M.Cavity(147, 147, 100.0, 1.0, 60.0), M.ifdlbm_default_options(), 5)
    assert J == J0 and np.array_equal(g, g0)
