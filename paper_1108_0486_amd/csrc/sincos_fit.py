"""Coefficients of the sine and cosine kernels in xg_normal.h.

sin(pi f) ~ f (pi + t (S3 + t (S5 + t S7))) and cos(pi f) ~ 1 + t (C2 + t (C4 +
t (C6 + t C8))), t = f^2, |f| <= 1/4: the polynomials in t of least maximum
relative error on a grid of 20000 points, by Lawson's iteratively reweighted
least squares (a weighted least-squares fit repeated with each point's weight
scaled by its last error, which converges to the minimax fit).  Prints the
coefficients as C float literals and the maximum relative errors.
Run: python3 sincos_fit.py
"""
import numpy as np


def lawson(A, g, w, iters=300):
    wt = np.ones(A.shape[0])
    for _ in range(iters):
        W = np.sqrt(wt) * w
        c, *_ = np.linalg.lstsq(A * W[:, None], g * w * np.sqrt(wt), rcond=None)
        err = np.abs((A @ c - g) * w)
        wt = wt * err
        wt /= wt.sum()
    return c, err.max()


def c_float(v):
    """v rounded to float, as a C hexadecimal float literal."""
    h = float(np.float32(v)).hex()            # e.g. -0x1.4abbbe0000000p+2
    mant, exp = h.split("p")
    return "%sp%sf" % (mant.rstrip("0").rstrip("."), exp)


def main():
    n = 20000
    f = (np.arange(1, n + 1, dtype=np.longdouble) / n) * np.longdouble(0.25)
    t = f * f
    pi = np.longdouble("3.14159265358979323846264338327950288")
    sin_pf, cos_pf = np.sin(pi * f), np.cos(pi * f)
    g_sin = ((sin_pf / f - pi) / t).astype(np.float64)   # sin: f (pi + t P(t))
    w_sin = (f * t / sin_pf).astype(np.float64)          # relative error per unit of P
    g_cos = ((cos_pf - 1) / t).astype(np.float64)        # cos: 1 + t Q(t)
    w_cos = (t / cos_pf).astype(np.float64)
    tt = t.astype(np.float64)
    s, es = lawson(np.stack([tt ** k for k in range(3)], axis=1), g_sin, w_sin)
    c, ec = lawson(np.stack([tt ** k for k in range(4)], axis=1), g_cos, w_cos)
    for name, v in zip(("kS3", "kS5", "kS7"), s):
        print("constexpr float %s = %s;" % (name, c_float(v)))
    for name, v in zip(("kC2", "kC4", "kC6", "kC8"), c):
        print("constexpr float %s = %s;" % (name, c_float(v)))
    print("max relative error: sin %.3e, cos %.3e" % (es, ec))


if __name__ == "__main__":
    main()
