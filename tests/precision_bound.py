"""Per-query error bound of the exact KDE computed by the GEMM form with FP32,
BF16 or FP16 operands and FP32 accumulation (first-order in the unit
roundoffs, worst case over summation orders):
  * operand rounding: x~ = fl_p(fl_32(x - c)) moves every point by at most
    e_x = (u_p + u_32) ||x - c||, so |d~ - d| <= E = e_x + e_y and
    |d~^2 - d^2| <= 2 d E + E^2;
  * dot product: FP32 accumulation of d_p products, at most
    2 gamma(d_p + 2) ||x~|| ||y~|| of d^2 (gamma(k) = k u / (1 - k u));
  * epilogue: 1.5 u_32 (||x~||^2 + ||y~||^2) of d^2 (norm term, add, FMA);
  * the kernel constant rounded to FP32 (and the square root of the
    exponential kernel): u_32 d^2 resp. 2 u_32 d in the exponent's units;
  * exp2 and the FP32 tile partial sums: 1e-6 relative.
The float32-split form (fp32_split) splits every prepared float32 value into
three bfloat16 parts exactly (v = h + m + l) and accumulates six products per
element (h h, h m, m h, h l, m m, l h; exact in FP32) with FP32 additions:
no operand rounding beyond FP32, 6 d_p + 2 accumulated terms in gamma, and the
three dropped products below 2^-26 |x~||y~| (2^-25 of d^2 after the factor 2).
With D the sum of the d^2 terms, a Gaussian term is off by at most a factor
exp((D + u_32 d^2) / (2 h^2)), an exponential one by
exp((min(sqrt(D), D / d) + 2 u_32 d) / h).  The bound of a query is the
kernel-weighted mean of those factors minus one, plus the 1e-6.  In the
near/far form the terms of the neighbours are exact (FP64) and leave the mean.
"""
import numpy as np

import oracle
from oracle import GAUSSIAN

U32 = 2.0 ** -24
UNIT = {"fp32": 0.0, "bf16": 2.0 ** -8, "fp16": 2.0 ** -11,   # operand rounding beyond FP32
        "fp32_split": 0.0}
ELEMS_PER_CHUNK = {"fp32": 32, "bf16": 64, "fp16": 64,        # rows are padded to these
                   "fp32_split": 64}
TERMS_PER_ELEM = {"fp32": 1, "bf16": 1, "fp16": 1, "fp32_split": 6}
DROPPED = {"fp32": 0.0, "bf16": 0.0, "fp16": 0.0, "fp32_split": 2.0 ** -26}


def geometry(X, Y):
    """(||x - c||, ||y - c||, exact squared distances [q, n]) with c the column mean of X."""
    c = X.astype(np.float64).mean(axis=0)
    xn = np.sqrt(((X - c) ** 2).sum(1))
    yn = np.sqrt(((Y - c) ** 2).sum(1))
    d2 = np.stack([oracle.sq_dists(X, Y[j]) for j in range(Y.shape[0])])
    return xn, yn, d2


def exact_kde_bound(geo, dim, h, kern, prec, near=None):
    """Per-query relative error bound (see the module docstring); geo from geometry().

    near: [q, k] rows of each query whose kernel values are exact (the near
    part of the near/far form, FP64 from the float32 rows); their terms drop
    out of the bound, and the 1e-6 applies to the far share of the sum only.
    """
    xn, yn, d2 = geo
    up = UNIT[prec] + U32
    per = ELEMS_PER_CHUNK[prec]
    dp = (dim + per - 1) // per * per
    terms = TERMS_PER_ELEM[prec] * dp + 2
    gam = terms * U32 / (1 - terms * U32)
    xt, yt = xn * (1 + up), yn * (1 + up)              # bounds on ||x~||, ||y~||
    E = up * (xn[None, :] + yn[:, None])
    d = np.sqrt(d2)
    D = (2 * d * E + E * E + 2 * (gam + DROPPED[prec]) * xt[None, :] * yt[:, None]
         + 1.5 * U32 * (xt[None, :] ** 2 + yt[:, None] ** 2))
    if kern == GAUSSIAN:
        K = np.exp(-d2 / (2 * h * h))
        f = np.expm1((D + U32 * d2) / (2 * h * h))
    else:
        K = np.exp(-d / h)
        f = np.expm1((np.minimum(np.sqrt(D), D / np.maximum(d, 1e-300)) + 2 * U32 * d) / h)
    w = K.sum(1)
    far = np.ones_like(K, dtype=bool)
    if near is not None:
        for j, rows in enumerate(near):
            far[j, np.asarray(rows, dtype=np.int64)] = False
    with np.errstate(invalid="ignore", divide="ignore"):
        b = (K * f * far).sum(1) / w
        share = (K * far).sum(1) / w
    return b + 1e-6 * share + 1e-12
