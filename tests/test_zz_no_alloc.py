"""sabr_mc_price_noalloc (the Monte Carlo price without device allocation)
against sabr_mc_price through the C ABI: bit for bit on two calls in a row,
the second smaller, in float and double; a call too large for the static
array is refused; the device's free memory does not move across calls."""
import math
import sys

import numpy as np
import pytest

from paper_2407_20713_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    from paper_2407_20713_amd import sabr
    sabr.lib()
    return sabr


def say(*a):
    print(*a, file=sys.stderr, flush=True)


CASES = [
    # (maturities, strikes per row, model, x, beta, paths): the second is smaller
    ([0.25, 0.5, 1.0], 9, inputs.DYN_I, [0.393329, -1.0, 0.941565, 0.001, 1.246906], 1.0, 300000),
    ([0.5], 3, inputs.STATIC, [0.3, -0.5, 0.8], 0.7, 3000),
]


def grid(T, n_k):
    return inputs.make_grid(T, [np.exp(np.linspace(-0.3, 0.3, n_k))] * len(T), f0=1.1,
                            disc=[math.exp(-0.02 * t) for t in T])


@pytest.mark.parametrize("prec", [1, 0])
def test_noalloc_equals_mc_price_twice(S, prec):
    import torch
    ctx = S.sabr_ctx_create(0)
    try:
        for rep in range(2):
            for T, n_k, model, x, beta, n_paths in CASES:
                g = grid(T, n_k)
                mk, pb = S.Market.from_grid(g), S.Problem(model, beta, x0=x)
                say("noalloc", rep, prec, len(T), n_k, n_paths)
                free0 = torch.cuda.mem_get_info()[0]
                p1, s1 = S.sabr_mc_price_noalloc(ctx, mk, pb, n_paths, 250, 0xA110C, precision=prec)
                free1 = torch.cuda.mem_get_info()[0]
                p0, s0 = S.sabr_mc_price(ctx, mk, pb, n_paths, 250, 0xA110C, precision=prec)
                np.testing.assert_array_equal(p1, p0)
                np.testing.assert_array_equal(s1, s0)
                assert np.all(p1 > 0)
                if rep == 1:
                    assert free1 == free0
    finally:
        ctx.close()


def test_noalloc_refuses_calls_beyond_the_array(S):
    ctx = S.sabr_ctx_create(0)
    try:
        g = inputs.make_grid([0.25, 0.5], [np.exp(np.linspace(-0.3, 0.3, 300))] * 2, f0=1.0)
        pb = S.Problem(inputs.STATIC, 0.7, x0=[0.3, -0.5, 0.8])
        with pytest.raises(S.SabrError) as e:
            S.sabr_mc_price_noalloc(ctx, S.Market.from_grid(g), pb, 1 << 20, 250, 1)
        assert e.value.code == S.SABR_E_BUDGET
        # the same grid with fewer paths (fewer workgroups) fits and matches
        p1, _ = S.sabr_mc_price_noalloc(ctx, S.Market.from_grid(g), pb, 1 << 14, 250, 1)
        p0, _ = S.sabr_mc_price(ctx, S.Market.from_grid(g), pb, 1 << 14, 250, 1)
        np.testing.assert_array_equal(p1, p0)
    finally:
        ctx.close()
