"""Fits the polynomials of the library's single-precision inverse normal CDF.

The device computes z = Phi^-1(u) for the single-precision uniforms
u = (k + 1/2) 2^-23 (so 2^-24 <= u <= 1 - 2^-24) as

    w = -ln(4 u (1 - u)),   x = 2u - 1,   z = x * g(w)

where g(w) = Phi^-1(u) / (2u - 1) is smooth in w.  This is the change of
variable of Giles, "Approximating the erfinv function" (GPU Computing Gems,
2011): one logarithm per draw, a polynomial in w - c0 on the central range
w < W_SPLIT, and a polynomial in sqrt(w) - c1 on the rare tail (entered by a
wave only when one of its lanes needs it).  The coefficients are our own
least-squares fits, relative-error weighted on Chebyshev nodes, against
scipy's double-precision ndtri.

Run it to print the C++ constants:  python -m paper_2108_03076_amd.fit_normal
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import chebyshev as C
from numpy.polynomial import polynomial as Pm
from scipy.special import ndtri

W_SPLIT = 5.0
U_MIN = 2.0 ** -24                   # smallest single-precision uniform
W_MAX = -np.log(4 * U_MIN * (1 - U_MIN))
CENTRAL = (0.0, W_SPLIT, 8)          # domain and degree in w
TAIL = (np.sqrt(W_SPLIT), np.sqrt(W_MAX) + 1e-3, 8)   # domain and degree in s = sqrt(w)


def g_of_w(w):
    """Phi^-1(u) / (2u - 1) for the u < 1/2 that gives w (the function is even in x)."""
    w = np.asarray(w, np.float64)
    e = np.exp(-w)
    x = np.sqrt(-np.expm1(-w))                 # 1 - 2u
    u = e / (2.0 * (1.0 + x))                  # stable (1 - x) / 2
    return -ndtri(u) / x


def fit(lo, hi, deg, f, n=4000):
    t = np.cos(np.pi * (np.arange(n) + 0.5) / n)          # Chebyshev nodes on [-1, 1]
    v = 0.5 * (hi + lo) + 0.5 * (hi - lo) * t
    y = f(v)
    c = C.chebfit(t, y, deg, w=1.0 / np.abs(y))
    # monomials in (v - mid) / 1: rescale the Chebyshev variable
    mono_t = C.cheb2poly(c)                                # in t
    half = 0.5 * (hi - lo)
    mono = mono_t / half ** np.arange(len(mono_t))         # in (v - mid)
    return 0.5 * (hi + lo), mono


def horner32(coef, d):
    """Single-precision Horner with fused multiply-add rounding."""
    d = np.float32(d)
    acc = np.float32(coef[-1])
    for k in coef[-2::-1]:
        acc = np.float32(np.float64(acc) * np.float64(d) + np.float64(np.float32(k)))
    return acc


def device_model(u):
    """The device's arithmetic, in numpy single precision (for the error report)."""
    u = np.asarray(u, np.float32)
    t = (u * (np.float32(1) - u)).astype(np.float32)
    w = (-np.log(np.float64(np.float32(4) * t))).astype(np.float32)
    x = (np.float32(2) * u - np.float32(1)).astype(np.float32)
    (c0, pc), (c1, pt) = CENTRAL_FIT, TAIL_FIT
    out = np.empty_like(u)
    m = w < W_SPLIT
    out[m] = x[m] * horner32(pc, w[m] - np.float32(c0))
    s = np.sqrt(w[~m]).astype(np.float32)
    out[~m] = x[~m] * horner32(pt, s - np.float32(c1))
    return out


CENTRAL_FIT = fit(CENTRAL[0], CENTRAL[1], CENTRAL[2], g_of_w)
TAIL_FIT = fit(TAIL[0], TAIL[1], TAIL[2], lambda s: g_of_w(s * s))


def report():
    k = np.arange(0, 1 << 23, 37, dtype=np.int64)
    u = ((k + 0.5) * 2.0 ** -23).astype(np.float32)
    ref = ndtri(u.astype(np.float64))
    z = device_model(u).astype(np.float64)
    rel = np.abs(z - ref) / np.maximum(1.0, np.abs(ref))
    return float(rel.max())


def main():
    for name, (mid, coef) in (("kCentral", CENTRAL_FIT), ("kTail", TAIL_FIT)):
        print(f"// {name}: centre {mid!r}")
        print(", ".join(f"{float(np.float32(c))!r}f" for c in coef))
    print(f"// max |z - Phi^-1(u)| / max(1, |z|) over a sample of single-precision uniforms: {report():.3e}")


if __name__ == "__main__":
    main()
