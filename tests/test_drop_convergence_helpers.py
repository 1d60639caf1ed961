"""CPU checks of the drop convergence campaign set-up
(paper_2412_16843_amd.drop_convergence): the exact wetted length and the
interface thickness rule; the measured wetted length comes from the device
diagnostics (tests/test_gpu_diagnostics.py)."""
import math

import numpy as np

import workloads as W
from paper_2412_16843_amd import drop_convergence as D


def test_exact_wetted_length_closed_forms():
    # 90 degrees: the semicircle itself, chord 2 r0
    assert abs(D.exact_wetted_length(0.15, math.pi / 2) - 0.3) < 1e-15
    # 60 degrees: cap of area pi r0^2 / 2, chord 2 R sin 60
    a0 = math.pi * 0.15 ** 2 / 2
    R = math.sqrt(a0 / (math.pi / 3 - math.sqrt(3) / 4))
    assert abs(D.exact_wetted_length() - R * math.sqrt(3)) < 1e-15


def test_case_eps_follows_h_to_the_two_thirds():
    """eps = 0.175 h^(2/3): eps / h = 0.7 at Nx = 64 and 1.4 at Nx = 512, the
    range of Sec. 5.1; the initial field is the 90-degree prescribed drop."""
    p, phi0 = D.case(256)
    assert abs(p.eps / p.h - 0.175 * 256 ** (1 / 3)) < 1e-12
    assert abs(D.case(64)[0].eps / (1 / 64) - 0.7) < 1e-12
    assert abs(D.case(512)[0].eps / (1 / 512) - 1.4) < 1e-12
    assert phi0.shape == (128, 256)
