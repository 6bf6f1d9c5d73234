"""Coefficients of the FP32 erfc used by the Ewald real-space pair kernels.

    erfc(x) = exp(-x^2) * erfcx(x),   erfcx(x) ~= sum_k a_k t^k,   t = 1 / (1 + x / 2)

on 0 <= x <= 6 (beta r_cut <= 6 covers erfc(beta r_cut) down to 2e-17).  exp(-x^2) is
also the factor of the derivative term 2 beta / sqrt(pi) exp(-beta^2 r^2), so a pair
costs one exponential, one reciprocal and eight fused multiply-adds for both.

The a_k minimise the largest relative error of erfcx over a dense grid (least squares
reweighted towards the largest errors), against scipy's erfcx.  Run this file to
regenerate them and print the error of the FP64 fit and of its FP32 evaluation.
"""
import numpy as np

C, DEG, XMAX = 0.5, 8, 6.0


def fit():
    from scipy.special import erfcx
    x = np.linspace(0.0, XMAX, 20001)
    y = erfcx(x)
    t = 1.0 / (1.0 + C * x)
    A = np.vstack([t ** k for k in range(DEG + 1)]).T / y[:, None]
    w = np.ones_like(x)
    for _ in range(30):
        coef, *_ = np.linalg.lstsq(A * w[:, None], w, rcond=None)
        err = np.abs(A @ coef - 1.0)
        w = w * (1.0 + err / err.max())
        w /= w.mean()
    return x, y, coef


def eval_f32(coef, x):
    t = (np.float32(1.0) / (np.float32(1.0) + np.float32(C) * x.astype(np.float32)))
    p = np.float32(coef[-1])
    for k in range(DEG - 1, -1, -1):
        p = (p * t + np.float32(coef[k])).astype(np.float32)
    return p


if __name__ == "__main__":
    x, y, coef = fit()
    e64 = np.max(np.abs(np.polyval(coef[::-1], 1.0 / (1.0 + C * x)) - y) / y)
    e32 = np.max(np.abs(eval_f32(coef, x).astype(np.float64) - y) / y)
    print("a_k:", ", ".join(f"{c:.9e}f" for c in coef))
    print(f"max relative error: FP64 fit {e64:.2e}, FP32 evaluation {e32:.2e}")
