"""CPU checks of the seeded input generators (no SABR arithmetic): the
Philox4x32-10 streams that draw the workloads' true parameters and vol noise
reproduce the generator's published known-answer vectors, redraws take new
counters, and the noise has the stated moments."""
import os

import numpy as np

from paper_2407_20713_amd import inputs

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_inputs_philox_known_answers():
    n = 0
    for line in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(x, 16) for x in line.split()]
        out = inputs.philox4x32_10(np.array(w[:4], dtype=np.uint64), (w[4], w[5]))
        assert [int(v) for v in out] == w[6:10]
        n += 1
    assert n == 3


def test_true_parameter_streams_redraw_and_stay_in_the_box():
    gens, lb, ub = inputs.surface_true_params(4)
    a = inputs.draw_params(gens[0], lb, ub)
    b = inputs.draw_params(gens[0], lb, ub)
    c = inputs.draw_params(inputs.surface_true_params(4)[0][0], lb, ub)
    d = inputs.draw_params(gens[1], lb, ub)
    assert np.all(a >= lb) and np.all(a <= ub)
    assert not np.array_equal(a, b) and np.array_equal(a, c) and not np.array_equal(a, d)
    # counter (fit, redraw, 0, 4) under key 0x5AB2: the first word gives alpha
    w = inputs.philox4x32_10(np.array([0, 0, 0, inputs.TAG_TRUE], dtype=np.uint64), (0x5AB2, 0))
    assert a[0] == lb[0] + (ub[0] - lb[0]) * ((float(w[0]) + 0.5) * 2.0 ** -32)


def test_philox_vol_noise_moments():
    z = inputs.vol_noise(0x5AB1, 200000, 1.0)
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1.0) < 0.01
    assert abs(np.mean(z ** 4) - 3.0) < 0.05
    np.testing.assert_array_equal(inputs.vol_noise(0x5AB1, 15, 1e-4), inputs.vol_noise(0x5AB1, 40, 1e-4)[:15])
