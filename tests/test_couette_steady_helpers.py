"""CPU check of the host-side interpolation of the Couette steady-state study
(paper_2412_16843_amd.couette_steady); the contact-line positions come from
the device diagnostics (tests/test_gpu_diagnostics.py)."""
import numpy as np

from paper_2412_16843_amd import couette_steady as CS


def test_sample_interpolates_corner_values_periodically():
    f = np.array([0.0, 1.0, 4.0, 9.0])
    assert CS.sample(0.25, f, 0.5) == 0.5          # halfway between corners 0 and 1
    assert CS.sample(1.75, f, 0.5) == 4.5          # between corner 3 and corner 0 (wrap)
