"""CPU: the fitted FP32 normal CDF used by the separable MFMA staging
(phi_lower_f32 in csrc/psf_gauss.h).  Its coefficients are read from the
header and the function is evaluated in float32 arithmetic (fused
multiply-adds rounded once) against scipy's erfc: the absolute error stays
below 1e-7 (about one FP32 ulp of 1/2) on [0, 12], and the two forms meet at
|z| = 1 without a step larger than that."""
import os
import re

import numpy as np
from scipy.special import erfc

HDR = os.path.join(os.path.dirname(__file__), "..", "paper_2008_05858_amd", "csrc", "psf_gauss.h")


def _coeffs():
    src = open(HDR).read()
    body = src[src.index("float phi_lower_f32(float z)"):]
    body = body[:body.index("\n}\n")]
    num = r"(-?\d+\.\d+e[+-]\d+)f"
    q = [float(re.search(r"float q = " + num, body).group(1))]
    q += [float(v) for v in re.findall(r"q = fmaf\(q, u, " + num + r"\)", body)]
    p = [float(re.search(r"float p = " + num, body).group(1))]
    p += [float(v) for v in re.findall(r"p = fmaf\(p, t, " + num + r"\)", body)]
    a = float(re.search(r"fmaf\((\d+\.\d+)f, x, 1\.0f\)", body).group(1))
    k = float(re.search(r"u \* (-\d+\.\d+)f", body).group(1))
    return q, p, a, k


def _eval(z, q, p, a, k):
    f32 = np.float32

    def fma(x, y, c):
        return f32(np.float64(x) * np.float64(y) + np.float64(c))

    x = f32(abs(f32(z)))
    u = f32(x * x)
    qq = f32(q[0])
    for c in q[1:]:
        qq = fma(qq, u, f32(c))
    centre = fma(-x, qq, f32(0.5))
    t = f32(f32(1.0) / fma(f32(a), x, f32(1.0)))
    pp = f32(p[0])
    for c in p[1:]:
        pp = fma(pp, t, f32(c))
    tail = f32(f32(np.exp2(np.float64(f32(u * f32(k))))) * pp)
    return centre if x < 1.0 else tail


def test_fitted_normal_cdf_within_one_ulp_of_half():
    q, p, a, k = _coeffs()
    assert len(q) == 6 and len(p) == 10
    zs = np.concatenate([np.linspace(-12.0, 12.0, 24001), [-1.0, 1.0, np.nextafter(1.0, 0.0)]])
    got = np.array([_eval(z, q, p, a, k) for z in zs], dtype=np.float64)
    ref = 0.5 * erfc(np.abs(zs.astype(np.float32).astype(np.float64)) / np.sqrt(2.0))
    err = np.abs(got - ref)
    assert err.max() < 1e-7, (err.max(), zs[np.argmax(err)])
    # non-increasing in |z| up to the float32 rounding of the values
    order = np.argsort(np.abs(zs))
    assert np.all(np.diff(got[order]) <= 1e-7)
