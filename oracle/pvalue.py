"""Two-sided Student-t p-values on the -log10 scale, in FP64.

Test infrastructure only (see the package docstring).

The paper converts its t-statistics "directly to P values" (Methods, 2.2
Association kernel, after Eq. 3) without naming the distribution or the
sidedness; the reading used here is the two-sided Student t with the test's
residual degrees of freedom.  With x = df / (df + t^2),

    p = I_x(df/2, 1/2)

where I is the regularized incomplete beta function.  In the bulk the value
comes from scipy's Student-t log survival function.  Where that underflows
(p below about 1e-308) or leaves less than full relative precision, ln p is
evaluated directly in log space:

    ln I_x(a, b) = a ln x + b ln(1 - x) - ln a - ln B(a, b) + ln F(x; a, b)

with F the continued fraction of the incomplete beta function (Abramowitz &
Stegun 26.5.8; DLMF 8.17.22) evaluated by the modified Lentz method
(Lentz 1976; Thompson & Barnett 1986).  The fraction converges quickly for
x < (a + 1)/(a + b + 2); otherwise the symmetry I_x(a, b) = 1 - I_{1-x}(b, a)
is used.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special, stats

LN10 = math.log(10.0)
_TINY = 1e-300
_EPS = 1e-16


def _beta_cf(x: float, a: float, b: float, max_iter: int = 100000) -> float:
    """Continued fraction F(x; a, b) of I_x(a, b), modified Lentz method.

    F = 1 / (1 + d1 / (1 + d2 / (1 + ...))) with
      d_{2m+1} = -(a + m)(a + b + m) x / ((a + 2m)(a + 2m + 1))
      d_{2m}   =  m (b - m) x / ((a + 2m - 1)(a + 2m)).
    """
    f = _TINY
    c = f
    d = 0.0
    for j in range(0, max_iter):
        if j == 0:
            num = 1.0
        else:
            m = j // 2
            if j % 2 == 1:
                num = -(a + m) * (a + b + m) * x / ((a + 2 * m) * (a + 2 * m + 1))
            else:
                num = m * (b - m) * x / ((a + 2 * m - 1) * (a + 2 * m))
        d = 1.0 + num * d
        if abs(d) < _TINY:
            d = _TINY
        c = 1.0 + num / c
        if abs(c) < _TINY:
            c = _TINY
        d = 1.0 / d
        delta = c * d
        f *= delta
        if j > 0 and abs(delta - 1.0) < _EPS:
            return f
    raise RuntimeError("incomplete beta continued fraction did not converge")


def _ln_betai_cf(x: float, a: float, b: float) -> float:
    """ln I_x(a, b) by the continued fraction; requires x < (a+1)/(a+b+2)."""
    lbeta = special.betaln(a, b)
    front = a * math.log(x) + b * math.log1p(-x) - math.log(a) - lbeta
    # the fraction as defined above carries the leading 1/(1 + d1 ...) with
    # num = 1 at j = 0, i.e. it returns 1 / (1 + d1 / (1 + ...))
    return front + math.log(_beta_cf(x, a, b))


def ln_p_two_sided_cf(t: float, df: float) -> float:
    """ln p for one statistic, entirely through the continued fraction."""
    t = abs(float(t))
    if math.isinf(t):
        return -math.inf
    if t == 0.0:
        return 0.0
    a, b = 0.5 * df, 0.5
    x = df / (df + t * t)
    one_minus_x = t * t / (df + t * t)
    if x < (a + 1.0) / (a + b + 2.0):
        return _ln_betai_cf(x, a, b)
    # p = 1 - I_{1-x}(b, a)
    q = math.exp(_ln_betai_cf(one_minus_x, b, a))
    return math.log1p(-q)


def nlog10p_two_sided(t, df) -> np.ndarray:
    """-log10 of the two-sided Student-t p-value, elementwise.

    NaN in gives NaN out; |t| = inf gives +inf.
    """
    t = np.abs(np.asarray(t, dtype=np.float64))
    df_arr = np.broadcast_to(np.asarray(df, dtype=np.float64), t.shape)
    out = np.full(t.shape, np.nan)
    fin = np.isfinite(t)
    out[np.isinf(t)] = np.inf
    if fin.any():
        lsf = stats.t.logsf(t[fin], df_arr[fin])
        val = -(lsf + math.log(2.0)) / LN10
        out[fin] = val
    # log-space continued fraction where the bulk path loses precision
    redo = fin & (~np.isfinite(out) | (out > 300.0))
    for idx in zip(*np.nonzero(redo)):
        out[idx] = -ln_p_two_sided_cf(t[idx], df_arr[idx]) / LN10
    return out
