"""Divergence measure D (Sec. 3.1): the oracle's definition pinned by closed
forms, and the library's argument checks on the CPU."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1309_2710_amd import rkc


def test_equal_work_gives_one():
    assert np.all(O.divergence([7] * 96, 32) == 1.0)


def test_one_busy_cell_gives_one_over_width():
    d = [0] * 64
    d[5] = 40
    d[40] = 3
    assert np.allclose(O.divergence(d, 32), [1 / 32, 1 / 32], rtol=0, atol=0)


def test_hand_computed_runs_and_short_tail():
    # runs [1 2 3 4] [5 5] -> 10 / (4 * 4), 10 / (2 * 5)
    assert list(O.divergence([1, 2, 3, 4, 5, 5], 4)) == [0.625, 1.0]
    # all-zero run counts as converged
    assert list(O.divergence([0, 0, 0, 2], 2)) == [1.0, 0.5]


def test_bounds():
    rng = np.random.default_rng(3)
    d = rng.integers(0, 1000, 32 * 50)
    D = O.divergence(d, 32)
    assert np.all(D >= 1 / 32) and np.all(D <= 1.0)


def test_library_rejects_bad_arguments_before_the_device():
    L = rkc.lib()
    w = np.ones(10, np.int32)
    D = np.zeros(10)
    assert L.rkc_divergence(10, rkc._np_ptr(w), 1, 0, rkc._np_ptr(D), None) == rkc.EINVAL
    assert L.rkc_divergence(10, rkc._np_ptr(w), 0, 32, rkc._np_ptr(D), None) == rkc.EINVAL
    assert L.rkc_divergence(10, None, 1, 32, rkc._np_ptr(D), None) == rkc.EINVAL
    assert L.rkc_divergence(0, None, 1, 32, None, None) == rkc.OK
