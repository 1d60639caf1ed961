"""CPU checks of the host-side measures of the drop convergence campaign
(paper_2412_16843_amd.drop_convergence): the exact wetted length and the
wall-crossing measure applied to a phase field whose answer is known."""
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


def test_wetted_length_of_a_step_profile_is_exact():
    """phi linear across the crossing: the interpolated crossings are exact."""
    nx, h = 64, 1.0 / 64
    x = (np.arange(nx) + 0.5) * h
    prof = np.clip(0.5 + (0.2 - np.abs(x - 0.5)) / (4 * h), 0.0, 1.0)
    phi = np.vstack([prof, prof])          # equal rows: the wall value is prof
    assert abs(D.wetted_length(phi, h) - 0.4) < 1e-12


def test_wetted_length_of_the_initial_drop_is_its_diameter():
    """The prescribed 90-degree drop at eps/h = 0.7: its phi = 1/2 base
    chord is the diameter 0.3 up to the profile's discretisation."""
    p, phi0 = D.case(256)
    L = D.wetted_length(phi0, p.h)
    assert abs(L - 0.3) < 2 * p.h, L
    assert abs(p.eps / p.h - 0.175 * 256 ** (1 / 3)) < 1e-12
