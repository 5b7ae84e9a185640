"""Coefficients of the lift's inverse standard normal CDF (csrc/coarse.hip).

The quiet start needs z = Phi^{-1}(b) for the Hammersley coordinate
b = (u + 1/2) 2^-32.  With p = min(b, 1 - b) and x = 1 - 2p,
Phi^{-1}(p) = -sqrt(2) erfinv(x), and erfinv(x) / x is a smooth function of
w = -log(4 p (1 - p)) = -log(1 - x^2) (the change of variable of M. Giles,
"Approximating the erfinv function", GPU Computing Gems, 2011): a polynomial in
w - 2.5 for w < 5 and one in sqrt(w) - 3 above (w reaches 21.5 at
b = 2^-33).  Both are fitted here by least squares on Chebyshev nodes against
scipy's erfinv, then checked in FP32 arithmetic against scipy's ndtri over
2 million random b, both ends of the range and the middle, with p and 1 - 2p formed
from the integers as the kernel does.  Run this file to print the coefficients
(lowest order first) and the check.
"""
import numpy as np
from numpy.polynomial import chebyshev as C
from scipy.special import erfinv, ndtri

DEGREE = 9
W_SPLIT = 5.0
W_MAX = -np.log(4 * 2.0 ** -33 * (1 - 2.0 ** -33))


def ratio(w):
    x = np.sqrt(-np.expm1(-w))
    return erfinv(x) / x


def fit(lo, hi, arg_of_w, w_of_arg, n=4000):
    t = (lo + hi) / 2 + (hi - lo) / 2 * np.cos(np.pi * (np.arange(n) + 0.5) / n)
    w = np.clip(w_of_arg(t), 1e-12, None)
    cheb = C.Chebyshev.fit(t, ratio(w), DEGREE, domain=[lo, hi])
    return cheb.convert(kind=np.polynomial.Polynomial).coef.astype(np.float32)


def coefficients():
    central = fit(-2.5, W_SPLIT - 2.5, None, lambda t: t + 2.5)
    tail = fit(np.sqrt(W_SPLIT) - 3.0, np.sqrt(W_MAX) - 3.0, None, lambda t: (t + 3.0) ** 2)
    return central, tail


def evaluate(u, central, tail):
    """The kernel's arithmetic for the Hammersley integers u (b = (u + 1/2) 2^-32):
    p = (min(u, ~u) + 1/2) 2^-32 and x = |u - ~u| 2^-32 from the integers, the rest
    in FP32."""
    f32 = np.float32
    u = np.asarray(u, dtype=np.uint32)
    nu = ~u
    lower = u < nu
    lo = np.where(lower, u, nu)
    p = ((lo.astype(f32) + f32(0.5)) * f32(2.0 ** -32)).astype(f32)
    x = (np.where(lower, nu - u, u - nu).astype(f32) * f32(2.0 ** -32)).astype(f32)
    w = (f32(-np.log(2.0)) * np.log2((f32(4.0) * p * (f32(1.0) - p)).astype(f32))).astype(f32)

    def horner(c, t):
        r = np.float32(c[-1]) * np.ones_like(t)
        for k in c[-2::-1]:
            r = (r * t + np.float32(k)).astype(f32)
        return r

    rc = horner(central, (w - f32(2.5)).astype(f32))
    rt = horner(tail, (np.sqrt(w) - f32(3.0)).astype(f32))
    z = (f32(-np.sqrt(2.0)) * x * np.where(w < W_SPLIT, rc, rt)).astype(f32)
    return np.where(lower, z, -z)


if __name__ == "__main__":
    central, tail = coefficients()
    fmt = lambda c: ", ".join(f"{float(v):.9e}f" for v in c)
    print(f"central (w - 2.5): {{{fmt(central)}}}")
    print(f"tail (sqrt(w) - 3): {{{fmt(tail)}}}")
    u = np.random.default_rng(0).integers(0, 2 ** 32, 2_000_000, dtype=np.uint64)
    u = np.concatenate([u, np.arange(2000, dtype=np.uint64),
                        2 ** 32 - 1 - np.arange(2000, dtype=np.uint64),
                        np.arange(2 ** 31 - 1000, 2 ** 31 + 1000, dtype=np.uint64)])
    b = (u.astype(np.float64) + 0.5) / 2.0 ** 32
    z, ref = evaluate(u, central, tail), ndtri(b)
    print("max |z - ndtri(b)|:", np.max(np.abs(z - ref)),
          " max relative:", np.max(np.abs(z - ref) / np.abs(ref)))
