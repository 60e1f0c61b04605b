"""Coefficients of phi_lower_f32() in psf_gauss.h: weighted least-squares
fits (float64, then rounded to float32) of

  centre, 0 <= x < 1:   Phi(-x) = 1/2 - x Q(x^2),  Q a degree-5 polynomial
  tail,   x >= 1:       Phi(-x) = exp(-x^2 / 2) S(t),  t = 1 / (1 + 0.35 x),
                        S a degree-9 polynomial, fitted in relative error on
                        1 <= x <= 9

where Phi is the standard normal CDF.  Prints the coefficients (constant
term first) and the largest absolute error of a float32 evaluation (each
step rounded to float32, fused multiply-adds rounded once) over [0, 9].
Needs numpy and scipy; run by hand, not at build time.
"""
import numpy as np
from scipy.special import erfc

P = np.polynomial.polynomial
X0, DEG_C, A, DEG_T = 1.0, 5, 0.35, 9


def phi_lower(x):
    return 0.5 * erfc(x / np.sqrt(2.0))


def fit():
    u = np.linspace(0.0, X0 * X0, 20001)[1:]
    xq = np.sqrt(u)
    cq = P.polyfit(u, (0.5 - phi_lower(xq)) / xq, DEG_C).astype(np.float32)
    x = np.linspace(X0, 9.0, 40001)
    s = phi_lower(x) * np.exp(0.5 * x * x)
    cs = P.polyfit(1.0 / (1.0 + A * x), s, DEG_T, w=1.0 / s).astype(np.float32)
    return cq, cs


def eval_f32(x, cq, cs):
    f32 = np.float32

    def fma(a, b, c):
        return f32(np.float64(a) * np.float64(b) + np.float64(c))

    x = f32(x)
    u = f32(x * x)
    q = cq[-1]
    for c in cq[-2::-1]:
        q = fma(q, u, c)
    if x < X0:
        return fma(-x, q, f32(0.5))
    t = f32(f32(1.0) / fma(f32(A), x, f32(1.0)))
    s = cs[-1]
    for c in cs[-2::-1]:
        s = fma(s, t, c)
    e = f32(np.exp2(np.float64(f32(u * f32(-0.5 / np.log(2.0))))))
    return f32(e * s)


if __name__ == "__main__":
    cq, cs = fit()
    print("centre Q:", ", ".join(f"{float(c):.9e}f" for c in cq))
    print("tail S:  ", ", ".join(f"{float(c):.9e}f" for c in cs))
    xs = np.linspace(0.0, 9.0, 90001)
    got = np.array([eval_f32(x, cq, cs) for x in xs], dtype=np.float64)
    ref = phi_lower(xs.astype(np.float32).astype(np.float64))
    print(f"max abs error over [0, 9]: {np.max(np.abs(got - ref)):.3e}")
