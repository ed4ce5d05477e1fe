"""The straggling normal quantile of the transport kernels: its 18 constants
in vpmc_kernels.hip are the ones gen_quantile.py fits, and that FP32
evaluation stays within 3e-7 relative of sqrt(2) erfinv(2u - 1) (scipy, FP64)
over the uniform grid the kernels draw from."""
import importlib.util
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2307_01416_amd", "csrc")


def _gen():
    spec = importlib.util.spec_from_file_location("gen_quantile", os.path.join(CSRC, "gen_quantile.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def _kernel_constants():
    src = open(os.path.join(CSRC, "vpmc_kernels.hip")).read()
    body = src[src.index("float normal_quantile(float u)"):]
    body = body[:body.index("return 1.41421356237f")]
    nums = [float(x) for x in re.findall(r"([-+]?\d\.\d+e[-+]\d+)f", body)]
    assert len(nums) == 18
    # the central polynomial's nine coefficients, then the tail's
    return np.array(nums[:9]), np.array(nums[9:])


def test_kernel_constants_are_the_fit():
    g = _gen()
    central = g.fit(1e-12, 5.0, lambda w: w - 2.5)
    tail = g.fit(5.0, g.W_MAX, lambda w: np.sqrt(w) - 3.0)
    a, b = _kernel_constants()
    np.testing.assert_allclose(a, central, rtol=1e-8, atol=1e-15)
    np.testing.assert_allclose(b, tail, rtol=1e-8, atol=1e-15)


def test_fp32_quantile_error_bound():
    from scipy.special import erfinv
    a, b = _kernel_constants()
    f32 = np.float32
    k = np.concatenate([np.arange(0, 2 ** 23, 61), np.arange(4096), 2 ** 23 - 1 - np.arange(4096)])
    u = ((k + 0.5) * 2.0 ** -23).astype(f32)
    t = f32(2) * u - f32(1)
    w = -np.log(f32(4) * u * (f32(1) - u)).astype(f32)
    s1, s2 = w - f32(2.5), np.sqrt(w) - f32(3)
    pa, pb = np.full_like(w, f32(a[0])), np.full_like(w, f32(b[0]))
    for ca, cb in zip(a[1:], b[1:]):
        pa = (pa * s1 + f32(ca)).astype(f32)
        pb = (pb * s2 + f32(cb)).astype(f32)
    z = (f32(np.sqrt(2)) * np.where(w < 5, pa, pb) * t).astype(np.float64)
    ref = np.sqrt(2) * erfinv(2 * u.astype(np.float64) - 1)
    assert np.max(np.abs(z - ref) / np.abs(ref)) < 3e-7
    # odd symmetry about the median, exactly: u -> 1 - u is exact on the grid
    lo, hi = z[np.arange(4096) + len(k) - 8192], z[np.arange(4096) + len(k) - 4096]
    assert np.array_equal(lo, -hi)
