"""The oracle's binary128 build against the printed rows of the linear
convergence test that lie below the FP64 floor (Sec. 4.1, Tables
1DAdvectionConvergence9th, 1DAdvectionConvergence13th17th): the paper computed
these in quadruple precision (Sec. 4 preamble).  The test runs start to finish
in binary128: lam sin^alpha(pi x) on [-1, 1], linear SSP-RK(order+1, order)
with dt = h to t = 2, errors over the n+1 points (the periodic end point
counted twice).  No GPU."""
from fractions import Fraction

import pytest

import oracle
from test_oracle_pins import _golden_rows

# printed L_inf below 1e-13 (out of FP64's reach), n^2 (order + 1) <= 4.2e6
# (a few seconds each); the scale-invariance rows (lam = 1e6) for the cheaper ones
QUAD_CASES = [(9, 3, Fraction(1, 200), (1.0, 1e6)), (9, 4, Fraction(1, 200), (1.0,)),
              (13, 3, Fraction(1, 100), (1.0, 1e6)), (13, 4, Fraction(1, 100), (1.0,)),
              (13, 3, Fraction(1, 200), (1.0,)), (13, 4, Fraction(1, 200), (1.0,)),
              (17, 3, Fraction(1, 60), (1.0, 1e6)), (17, 4, Fraction(1, 60), (1.0,)),
              (17, 3, Fraction(1, 120), (1.0,)), (17, 4, Fraction(1, 120), (1.0,)),
              (17, 4, Fraction(1, 240), (1.0,))]


@pytest.mark.parametrize("order,alpha,h,lams", QUAD_CASES)
def test_quad_rows_below_the_fp64_floor(order, alpha, h, lams):
    rows = {(o, lam, a, hh): (l1, li) for (o, lam, a, hh, l1, li) in _golden_rows("advection")}
    n = int(2 / h)
    for lam in lams:
        p1, pinf = rows[(order, lam, alpha, h)]
        l1, linf = oracle.quad_advection_errors(order, alpha, lam, n)
        assert float("%.2e" % l1) == pytest.approx(p1, rel=1e-9), (l1, p1)
        assert float("%.2e" % linf) == pytest.approx(pinf, rel=1e-9), (linf, pinf)


def test_quad_and_fp64_agree_above_the_floor():
    # Where FP64 reaches the printed digits the two precisions agree closely.
    import numpy as np
    import workloads
    order, alpha, n = 9, 3, 100
    x, h, u0 = workloads.sin_power(alpha, 1.0, n)
    u = oracle.scalar_lssp_run(order, u0, h, h, n, order + 1)
    e = np.abs(u - u0)
    l1d = np.concatenate([e, e[:1]]).mean()
    l1q, _ = oracle.quad_advection_errors(order, alpha, 1.0, n)
    assert abs(l1d - l1q) <= 1e-3 * l1q
