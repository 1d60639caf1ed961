"""Accuracy of the device logarithm cdi_log (csrc/cdi_math.h), built here by
the host compiler from the same header: within 2 ulp of the exact logarithm
(60-digit decimal reference) over the phase-field argument range of psi =
eps ln((phi + d)/(1 - phi + d)) and across the normal doubles."""
import math
import os
import random
import shutil
import struct
import subprocess
from decimal import Decimal, getcontext

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER_DIR = os.path.join(ROOT, "paper_2412_16843_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <cstdint>
#include <cstring>
#include "cdi_math.h"
int main() {
  unsigned long long b;
  while (std::scanf("%llx", &b) == 1) {
    double x;
    std::memcpy(&x, &b, 8);
    const double y = cdi::cdi_log(x);
    unsigned long long o;
    std::memcpy(&o, &y, 8);
    std::printf("%016llx\n", o);
  }
  return 0;
}
"""


def _bits(x: float) -> str:
    return "%016x" % struct.unpack("<Q", struct.pack("<d", x))[0]


def _from_bits(h: str) -> float:
    return struct.unpack("<d", struct.pack("<Q", int(h, 16)))[0]


@pytest.fixture(scope="module")
def cdi_log_exe(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    d = tmp_path_factory.mktemp("cdi_log")
    src = d / "drv.cpp"
    src.write_text(DRIVER)
    exe = d / "drv"
    subprocess.run([cxx, "-O2", "-std=c++17", "-ffp-contract=off", "-I", HEADER_DIR, str(src),
                    "-o", str(exe)], check=True)
    return str(exe)


def _run(exe, xs):
    out = subprocess.run([exe], input="\n".join(_bits(x) for x in xs), capture_output=True,
                         text=True, check=True).stdout.split()
    return [_from_bits(h) for h in out]


def _ulp_errors(xs, ys):
    getcontext().prec = 60
    errs = []
    for x, y in zip(xs, ys):
        ref = Decimal(x).ln()
        r = float(ref)
        errs.append(float(abs(Decimal(y) - ref)) / math.ulp(r) if r != 0.0 else abs(y))
    return errs


def test_psi_argument_range(cdi_log_exe):
    rng = random.Random(20241216)
    d = 1e-12
    phis = [0.0, 1.0, 0.5, 1e-15, 1.0 - 1e-15, 0.25, 0.75, 1e-6, 1.0 - 1e-6]
    phis += [rng.random() for _ in range(3000)]
    phis += [10.0 ** rng.uniform(-14, -1) for _ in range(500)]
    phis += [1.0 - 10.0 ** rng.uniform(-14, -1) for _ in range(500)]
    xs = [(p + d) / (1.0 - p + d) for p in phis]
    errs = _ulp_errors(xs, _run(cdi_log_exe, xs))
    assert max(errs) <= 2.0, max(errs)


def test_normal_range_and_reduction_boundaries(cdi_log_exe):
    rng = random.Random(7)
    xs = [2.0 ** rng.uniform(-1020, 1020) for _ in range(3000)]
    # around 1 (e = 0, s -> 0), the powers of two and the sqrt(1/2) switch
    for k in range(-40, 41):
        xs.append(1.0 + k * 2.0 ** -52)
    for e in (-1000, -52, -1, 0, 1, 52, 1000):
        for k in (-3, -1, 0, 1, 3):
            xs.append(math.ldexp(1.0 + k * 2.0 ** -52, e))
    h = math.sqrt(0.5)
    for k in range(-20, 21):
        xs.append(h + k * 2.0 ** -53)
        xs.append(2.0 * h + k * 2.0 ** -52)
    xs = [x for x in xs if x > 0.0]
    ys = _run(cdi_log_exe, xs)
    errs = _ulp_errors(xs, ys)
    assert max(errs) <= 2.0, max(errs)
    assert _run(cdi_log_exe, [1.0]) == [0.0]
