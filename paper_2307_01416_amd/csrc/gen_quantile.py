"""Coefficients of the FP32 standard-normal quantile used by the transport
kernels for straggling (normal_quantile in vpmc_kernels.hip).

z(u) = sqrt(2) erfinv(t), t = 2u - 1, with g(t) = erfinv(t) / t written as
a function of w = -log(1 - t^2) = -log(4 u (1 - u)) as in M. Giles'
single-precision erfinv (GPU Computing Gems Jade Edition, 2011): a degree-8
polynomial in w - 2.5 for w < 5 and in sqrt(w) - 3 for w >= 5, fitted by weighted least
squares (relative error) to the FP64 function on Chebyshev nodes.  Prints
the coefficients (highest power first) and the largest relative error of the
FP32 evaluation over the uniform grid the kernels draw from,
u = (k + 1/2) 2^-23."""
import numpy as np
from scipy.special import erfinv

W_MAX = -np.log(4 * 2.0 ** -24 * (1 - 2.0 ** -24)) + 0.1


def fit(lo, hi, to_s, deg=8, n=4000):
    k = np.arange(n)
    w = 0.5 * (lo + hi) + 0.5 * (hi - lo) * np.cos(np.pi * (k + 0.5) / n)
    t = np.sqrt(-np.expm1(-w))
    g = erfinv(t) / t
    V = np.vander(to_s(w), deg + 1)
    c, *_ = np.linalg.lstsq(V / np.abs(g)[:, None], np.ones_like(g), rcond=None)
    return c


def main():
    central = fit(1e-12, 5.0, lambda w: w - 2.5)
    tail = fit(5.0, W_MAX, lambda w: np.sqrt(w) - 3.0)
    f32 = np.float32
    k = np.concatenate([np.arange(0, 2 ** 23, 97), np.arange(4096), 2 ** 23 - 1 - np.arange(4096)])
    u = ((k + 0.5) * 2.0 ** -23).astype(f32)
    t = f32(2) * u - f32(1)
    w = -np.log(f32(4) * u * (f32(1) - u)).astype(f32)

    def horner(c, s):
        p = f32(c[0])
        for cc in c[1:]:
            p = (p * s + f32(cc)).astype(f32)
        return p

    p = np.where(w < 5, horner(central, w - f32(2.5)), horner(tail, np.sqrt(w) - f32(3)))
    z = (f32(np.sqrt(2)) * p * t).astype(np.float64)
    ref = np.sqrt(2) * erfinv(2 * u.astype(np.float64) - 1)
    print("central", ", ".join(f"{x:.9e}f" for x in central))
    print("tail", ", ".join(f"{x:.9e}f" for x in tail))
    print("max relative error", float(np.max(np.abs(z - ref) / np.abs(ref))))


if __name__ == "__main__":
    main()
