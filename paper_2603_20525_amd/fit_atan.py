"""Coefficients of the slip angle's arctangent (csrc/rollout_step.h, atan_mm).

atan(x) on [0, 1] is approximated by x + x^3 P(x^2) with P of degree 5; the
six coefficients minimise the largest absolute error over 4001 equispaced
points, a discrete minimax problem solved as a linear program (minimise e
subject to |x^3 P(x^2) - (atan x - x)| <= e at every point). Beyond 1 the
kernel uses pi/2 - atan(1/|x|) with the sign of x. Run this module to print
the float32 coefficients and the largest error of their float32 evaluation
(fused multiply-adds, as on the GPU) over 200 001 points of [0, 1].
"""
import numpy as np

DEGREE = 5
POINTS = 4001


def fit(degree=DEGREE, points=POINTS):
    from scipy.optimize import linprog
    x = np.linspace(0.0, 1.0, points)
    A = np.stack([x ** 3 * x ** (2 * j) for j in range(degree + 1)], 1)
    b = np.arctan(x) - x
    n = degree + 1
    cost = np.zeros(n + 1)
    cost[-1] = 1.0
    ones = np.ones((points, 1))
    A_ub = np.vstack([np.hstack([A, -ones]), np.hstack([-A, -ones])])
    b_ub = np.concatenate([b, -b])
    r = linprog(cost, A_ub=A_ub, b_ub=b_ub, bounds=[(None, None)] * n + [(0, None)],
                method="highs")
    assert r.success, r.message
    return r.x[:n].astype(np.float32), float(r.x[-1])


def eval_f32(coef, x):
    """The kernel's evaluation in float32: Horner in t = x^2 with fused
    multiply-adds (a float64 product and sum rounded once to float32)."""
    x = np.asarray(x, dtype=np.float32)
    t = (x * x).astype(np.float32)

    def fma(a, b, c):
        return (np.float64(a) * np.float64(b) + np.float64(c)).astype(np.float32)

    p = np.full_like(x, coef[-1])
    for c in coef[-2::-1]:
        p = fma(p, t, np.float32(c))
    x3 = (x * t).astype(np.float32)
    return fma(x3, p, x)


if __name__ == "__main__":
    coef, e = fit()
    xs = np.linspace(0.0, 1.0, 200001).astype(np.float32)
    err = np.abs(eval_f32(coef, xs).astype(np.float64) - np.arctan(xs.astype(np.float64)))
    print("coefficients c0..c5:", ", ".join(f"{c:.9e}f" for c in coef))
    print(f"minimax error {e:.3e}; float32 evaluation max abs error {err.max():.3e}")
