"""The Sweepline inputs (Sec. 5.1): the uniform draw, reordered along the
first axis, stably."""
import numpy as np

import synth


def test_sweepline_is_the_uniform_draw_sorted_on_x():
    for dim, bits in ((2, 30), (3, 21), (3, 3)):
        u = synth.uniform(5000, dim, bits, seed=8)
        s = synth.sweepline(5000, dim, bits, seed=8)
        assert (np.diff(s[:, 0].astype(np.int64)) >= 0).all()
        # a permutation of the same rows, equal x kept in draw order
        order = np.lexsort((np.arange(len(u)), u[:, 0]))
        np.testing.assert_array_equal(s, u[order])
    assert synth.sweepline(0, 2, 30, seed=1).shape == (0, 2)
    np.testing.assert_array_equal(synth.points("sweepline", 100, 2, 30, 3), synth.sweepline(100, 2, 30, 3))
