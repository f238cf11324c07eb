"""Least-squares polynomial approximations used by the ray kernels.

    python paper_2606_30620_amd/csrc/gen_poly.py

atan(x) = x P(x^2) on [0, 1] (the kernels use atan(x) = pi/2 - atan(1/x)
beyond 1) and atanh(x) = x Q(x^2) on [0, 1/2] (the kernels use
atanh(x) = ln((1+x)/(1-x))/2 beyond 1/2).  Coefficients are fitted in FP64 by
least squares on Chebyshev points of x^2 with relative weighting, then the
maximum relative error of the FP32 Horner evaluation is measured on a dense
grid.  Printed as C initialisers for rtu_device.h.
"""
import numpy as np


def fit(fun, lo, hi, deg):
    k = np.arange(4000)
    t = 0.5 * (lo + hi) + 0.5 * (hi - lo) * np.cos((2 * k + 1) * np.pi / (2 * k.size))  # x^2
    x = np.sqrt(t)
    target = np.where(x > 0, fun(x) / np.where(x > 0, x, 1), 1.0)
    A = np.vander(t, deg + 1, increasing=True)
    c, *_ = np.linalg.lstsq(A, target, rcond=None)
    return c


def horner32(c, x):
    x = x.astype(np.float32)
    t = x * x
    r = np.float32(c[-1])
    for a in c[-2::-1]:
        r = np.float32(r * t + np.float32(a))
    return r * x


def report(name, fun, c, lo, hi):
    x = np.linspace(np.sqrt(lo), np.sqrt(hi), 200001)[1:]
    ref = fun(x.astype(np.float32).astype(np.float64))
    got = horner32(c, x).astype(np.float64)
    err = np.max(np.abs(got - ref) / np.abs(ref))
    print(f"// {name}: degree {len(c) - 1} in x^2, max relative error (FP32 Horner) {err:.2e}")
    print("{" + ", ".join(f"{np.float32(a)!r}f".replace("np.float32(", "").replace(")", "") for a in c) + "}")


if __name__ == "__main__":
    ca = fit(np.arctan, 0.0, 1.0, 8)
    report("atan(x)/x on [0, 1]", np.arctan, ca, 0.0, 1.0)
    ch = fit(np.arctanh, 0.0, 0.25, 6)
    report("atanh(x)/x on [0, 1/2]", np.arctanh, ch, 0.0, 0.25)
