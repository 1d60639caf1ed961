"""CPU checks of the host-side measures of the Couette steady-state study
(paper_2412_16843_amd.couette_steady)."""
import numpy as np

from paper_2412_16843_amd import couette_steady as CS


def test_crossings_of_a_periodic_slab_profile():
    """A linear ramp up through 1/2 at x = 2.3 and down at x = 7.1 on a
    periodic row of cell centres (i + 1/2) h, h = 0.1: exact crossings."""
    h, n = 0.1, 100
    x = (np.arange(n) + 0.5) * h
    w = np.clip(0.5 + np.minimum(x - 2.3, 7.1 - x) / (4 * h), 0.0, 1.0)
    up, down = CS.crossings(w, h)
    assert len(up) == 1 and len(down) == 1
    assert abs(up[0] - 2.3) < 1e-12 and abs(down[0] - 7.1) < 1e-12


def test_crossing_across_the_periodic_seam():
    h, n = 0.5, 8
    w = np.array([0.9, 0.9, 0.9, 0.1, 0.1, 0.1, 0.1, 0.3])   # rises between cells 7 and 0
    up, down = CS.crossings(w, h)
    assert len(up) == 1 and len(down) == 1
    # rising: between x = 3.75 (cell 7, 0.3) and 4.25 = 0.25 (cell 0, 0.9)
    assert abs(up[0] - ((7.5 + (0.3 - 0.5) / (0.3 - 0.9)) * h) % 4.0) < 1e-12
    assert abs(down[0] - (2.5 + 0.4 / 0.8) * h) < 1e-12


def test_sample_interpolates_corner_values_periodically():
    f = np.array([0.0, 1.0, 4.0, 9.0])
    assert CS.sample(0.25, f, 0.5) == 0.5          # halfway between corners 0 and 1
    assert CS.sample(1.75, f, 0.5) == 4.5          # between corner 3 and corner 0 (wrap)
