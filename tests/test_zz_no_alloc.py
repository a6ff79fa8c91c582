"""mc_thermo_static, the reduced reweighting for callers that cannot allocate
device memory, through the C ABI: bit for bit the results of mc_thermo on the
same weight and inverse temperatures, on two calls in a row (the second with
fewer inverse temperatures, so stale results of the first stay in the shared
array), and refusals beyond the array's capacity."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _static(mc, ctx, betas, i=0):
    b = np.ascontiguousarray(np.asarray(betas, dtype=np.float64))
    out = np.full(4 * b.size, np.nan)
    st = mc.lib().mc_thermo_static(ctx._h, i, b.ctypes.data_as(ctypes.c_void_p), int(b.size),
                                   out.ctypes.data_as(ctypes.c_void_p))
    return st, out.reshape(4, b.size)


def test_thermo_static_equals_thermo_on_two_calls():
    import paper_0812_2964_amd as mc

    cap = 8192
    rng = np.random.default_rng(7)
    sizes = [(32, 2, 1, 1), (256, 2, 1, 1)]
    ctx = mc.Context(sizes)
    for i, (L, _, _, bs) in enumerate(sizes):
        nb = ((L * L) >> bs) + 1
        x = (np.arange(nb) - nb / 2) / nb
        ctx.init_weights(-0.6 * L * L * x * x + np.cumsum(rng.normal(0, 0.05, nb)), i)
    calls = [(1, np.linspace(0.05, 2.0, cap)), (0, np.sort(rng.uniform(0.1, 1.5, 300)))]
    for i, betas in calls:
        st, got = _static(mc, ctx, betas, i)
        assert st == mc.MC_OK, mc.lib().mc_last_error()
        want = np.array(ctx.thermo(betas, i))
        assert np.isfinite(got).all()
        assert np.array_equal(got.view(np.uint64), want.view(np.uint64)), i
    # beyond the static array's capacity, and bad inverse temperatures
    st, _ = _static(mc, ctx, np.full(cap + 1, 0.5))
    assert st == mc.MC_EINVAL
    st, _ = _static(mc, ctx, [0.5, -1.0])
    assert st == mc.MC_EINVAL
    ctx.close()
