"""Host check of the binary64 coupled kernels' own elementary functions
(csrc/phase64.hpp, compiled for the host from the same source the kernels
use) against long double: the -2 ln U1 and the cos / sin of 2 pi U2 of the
Box-Muller pair on every one of the 2^24 values each 24-bit uniform can take,
and the sine of a phase difference on a dense grid of [-2 pi, 2 pi] and next
to the multiples of pi.  Bounds: 2 ulp of the result (the logarithm, the
sine) and 2 x 2^-53 absolute (cos / sin of a turn, whose values cross
zero)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1908_03869_amd", "csrc")


@pytest.fixture(scope="module")
def phase64_errors(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the host check")
    exe = str(tmp_path_factory.mktemp("xcheck") / "phase64_check")
    src = os.path.join(HERE, "xcheck", "phase64_check.cpp")
    subprocess.check_call([hipcc, "-O2", "-x", "hip", "--offload-arch=gfx950", "-I" + CSRC, "-o", exe, src],
                          stderr=subprocess.DEVNULL)
    out = subprocess.run([exe], capture_output=True, text=True, check=True, timeout=300).stdout
    res = {}
    for line in out.strip().splitlines():
        name, worst, worst_abs, count = line.split()
        res[name] = (float(worst), float(worst_abs), int(count))
    print(res)
    return res


def test_minus_two_ln_every_u1(phase64_errors):
    worst, _, count = phase64_errors["minus_two_ln_u24"]
    assert count == 2**24
    assert worst <= 2.0


def test_cos_sin_of_a_turn_every_u2(phase64_errors):
    worst_half_ulps, worst_abs, count = phase64_errors["cos_sin_turn_u24"]
    assert count == 2**24
    assert worst_half_ulps <= 2.0 and worst_abs <= 2.0 * 2.0**-53


def test_sin_of_phase_differences(phase64_errors):
    worst, _, count = phase64_errors["sin_phase64"]
    assert count > 2 * 10**7
    assert worst <= 2.0
