"""Accuracy of the device elementary functions of the noise transform and the
spin normalisation (paper_2605_26016_amd/csrc/spx_math.hpp), compiled for the
CPU with g++ with the hardware estimates replaced by values carrying their
stated 2^-23 relative error, against long-double libm over the Box-Muller
arguments of ~4M Philox words (random, both ends of the u32 range, and the
reduction boundaries) and 2M squared norms.  Bounds: log within 2 ulp, sqrt
and 1/sqrt within 1 ulp (+ rounding slack), sin(pi t) and cos(pi t) within
2^-52 absolute.  Together these keep the normals within a few ulp of the
libm-based oracle (whose own 2 pi u rounding is of the same size).

The GNEB passes' functions are checked the same way: the quotient (half an
ulp), the angle between two unit vectors from (|a x b|, a.b) over random,
nearly parallel and nearly opposite pairs and the reduction's octant
boundaries (3 ulp), and cos r, sin(r)/r of the exponential map from r^2
(1.5 ulp up to r = 1, a few 2^-53 absolute up to r = 4).

The Monte Carlo moves' functions (spx_mc_math.hpp): e^y - 1 and e^y for
y <= 0 over random magnitudes and both sides of every reduction boundary
(1.5 ulp), ln(1 + w) for -1 < w <= 0 over random magnitudes down to 2^-60
and around w = -1/2 (2.5 ulp)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_device_math_accuracy(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "math_check"
    subprocess.run([gxx, "-O2", "-std=c++17", "-ffp-contract=off", "-o", str(exe),
                    os.path.join(HERE, "host", "math_check.cpp")], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    res = {ln.split()[0]: float(ln.split()[1]) for ln in out.strip().splitlines()}
    print(res)
    assert res["log"] <= 2.0
    assert res["sqrt"] <= 1.01
    assert res["rsqrt"] <= 1.01
    assert res["sinpi_abs"] <= 2.0
    assert res["cospi_abs"] <= 2.0
    # GNEB: image distances and the exponential-map retraction
    assert res["div"] <= 0.51
    assert res["atan2"] <= 3.0
    assert res["expmap_cos_abs"] <= 1.5
    assert res["expmap_sinc"] <= 1.5
    # beyond |u| = 1 (up to 4 rad) the angle goes through u / pi in one rounding
    assert res["expmap_far_cos_abs"] <= 8.0
    assert res["expmap_far_sin_abs"] <= 8.0
    # Monte Carlo: heat-bath inverse distribution function, Metropolis test
    assert res["expm1_nonpos"] <= 1.5
    assert res["exp_nonpos"] <= 1.5
    assert res["log1p_neg"] <= 2.5
