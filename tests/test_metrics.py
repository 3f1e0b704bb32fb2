"""Eq. 3 (bad-pixel percentage), worked by hand on the host."""
import numpy as np

from paper_2001_07809_amd import pipeline


def test_bad_pixel_percent_counts_errors_above_delta():
    computed = np.array([[0, 2, 5], [7, 9, 9]], np.uint8)
    truth = np.array([[1, 2, 3], [9, 5, 9]], np.uint8)
    # errors 1 0 2 / 2 4 0: above delta = 1 are 2, 2 and 4 (an error of exactly delta is not bad)
    assert pipeline.bad_pixel_percent(computed, truth) == 50.0
    # delta 0: every nonzero error
    assert abs(pipeline.bad_pixel_percent(computed, truth, delta=0) - 100.0 * 4 / 6) < 1e-12
    # the mask picks the compared pixels: errors 1, 0, 4, 0 -> one of four
    mask = np.array([[1, 1, 0], [0, 1, 1]], bool)
    assert pipeline.bad_pixel_percent(computed, truth, mask) == 25.0
    # nothing compared
    assert pipeline.bad_pixel_percent(computed, truth, np.zeros((2, 3), bool)) == 0.0
