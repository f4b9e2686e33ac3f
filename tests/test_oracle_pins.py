"""Pins of the CPU oracle to what the paper prints and to exact mathematics.

Nothing here needs a GPU.  Each test names the passage it checks.
"""
import os
from fractions import Fraction
from math import comb

import numpy as np
import pytest

import oracle
from oracle import coeffs
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_table(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            m, n, l, num, den, _ = line.split()
            rows.append((int(m), int(n), int(l), Fraction(int(num), int(den))))
    return rows


# ---------------------------------------------------------------------------
# Coefficient tables (Sec. 3.1 Eq. Candidates, Tables Flux_reconstruction1/2,
# Sec. 3.2 Tables ISCoe1/2)
# ---------------------------------------------------------------------------

def test_candidate_pool_matches_paper_listing():
    # 29 stencils; one each of 1, 3, 5, 7 and 17 points, two of every other size.
    sizes = [m + n + 1 for (m, n) in coeffs.CANDIDATES_17]
    assert len(sizes) == 29
    for s in range(1, 18):
        expect = 1 if s in (1, 3, 5, 7, 17) else 2
        assert sizes.count(s) == expect, s
    assert sizes == sorted(sizes, reverse=True)
    # The restriction to lower orders keeps the list order (nested pools).
    assert [len(coeffs.candidates(p)) for p in (5, 9, 13, 17)] == [7, 13, 21, 29]


def test_a_coefficients_equal_printed_tables():
    printed = _read_table("a_coefficients.txt")
    assert len(printed) == 273
    got = {(m, n): a for (m, n, a, _) in coeffs.exact_table(17)}
    seen = set()
    for m, n, l, val in printed:
        assert got[(m, n)][l + m] == val, (m, n, l)
        seen.add((m, n, l))
    # every coefficient of every candidate is printed exactly once
    assert seen == {(m, n, l) for (m, n) in coeffs.CANDIDATES_17 for l in range(-m, n + 1)}


# Two printed b_l entries read 3423 where the binomial closed form (and the
# requirement sum b_l = 0, IS(constant) = 0) gives 3432 = C(14, 7): stencils
# S_{j-8}^{j+6} at l = -1 and S_{j-7}^{j+7} at l = 0 in Table ISCoe1.
B_TYPOS = {(8, 6, -1): (-3423, -3432), (7, 7, 0): (-3423, -3432)}


def test_b_coefficients_equal_printed_tables_up_to_two_typos():
    printed = _read_table("b_coefficients.txt")
    got = {(m, n): b for (m, n, _, b) in coeffs.exact_table(17)}
    assert len(printed) == 272      # S_j^j has no indicator
    for m, n, l, val in printed:
        if (m, n, l) in B_TYPOS:
            pr, true = B_TYPOS[(m, n, l)]
            assert val == pr and got[(m, n)][l + m] == true
        else:
            assert got[(m, n)][l + m] == val, (m, n, l)


def test_b_is_the_undivided_difference_and_a_sums_to_one():
    for (m, n, a, b) in coeffs.exact_table(17):
        k = m + n
        for l in range(-m, n + 1):
            assert b[l + m] == (-1) ** (k - (l + m)) * comb(k, l + m)
        assert sum(a) == 1
        if k > 0:
            assert sum(b) == 0


def test_a_reproduces_polynomials_exactly():
    # Cell averages of x^d (d <= m+n) reconstruct the point value of x^d at
    # x_{j+1/2} = 1/2 exactly (the defining property, Eq. Polynomial_Construction).
    half = Fraction(1, 2)
    for (m, n, a, _) in coeffs.exact_table(17):
        for d in range(m + n + 1):
            avg = [((l + half) ** (d + 1) - (l - half) ** (d + 1)) / (d + 1) for l in range(-m, n + 1)]
            # the flux approximates H, whose cell averages are f: with f = x^d
            # averaged, H = x^d, so f-hat must be (1/2)^d
            assert sum(x * y for x, y in zip(a, avg)) == half ** d


def test_double_table_is_correctly_rounded():
    for order in coeffs.ORDERS:
        ex = coeffs.exact_table(order)
        db = coeffs.double_table(order)
        for (m, n, a, b), (_, _, ad, bd) in zip(ex, db):
            for x, y in zip(a, ad):
                # nearest double: |x - y| <= half an ulp of y
                assert abs(Fraction(y) - x) <= Fraction(np.spacing(abs(y))) / 2


# ---------------------------------------------------------------------------
# Linear SSP-RK coefficients (Sec. 2.3, Eq. lSSPRK_Coe)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("m", [2, 3, 6, 10, 14, 18])
def test_lssp_is_order_m_minus_1_and_nonnegative(m):
    a = oracle.lssp_coefficients(m)
    assert all(x >= 0 for x in a) and sum(a) == 1
    # stability polynomial of the scheme applied to u' = z u (dt = 1):
    # u^(k) = (1 + z/2)^k; u^{n+1} = sum_{k<m-1} a_k (1+z/2)^k + a_{m-1} (1+z/2)^{m-1} (1 + z/2)
    # must agree with e^z through z^{m-1}.
    def poly_pow(k):
        # coefficients of (1 + z/2)^k
        return [Fraction(comb(k, i), 2 ** i) for i in range(k + 1)]
    R = [Fraction(0)] * (m + 1)
    for k in range(m - 1):
        for i, c in enumerate(poly_pow(k)):
            R[i] += a[k] * c
    for i, c in enumerate(poly_pow(m)):
        R[i] += a[m - 1] * c
    fact = 1
    for i in range(m):
        if i > 0:
            fact *= i
        assert R[i] == Fraction(1, fact), (m, i)


# ---------------------------------------------------------------------------
# Convergence rows (Sec. 4.1 Tables 1DAdvectionConvergence*, Sec. 4.2 Table
# 1DBurgersConvergence)
# ---------------------------------------------------------------------------

def _golden_rows(problem):
    rows = []
    with open(os.path.join(GOLDEN, "convergence_rows.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            kind, scheme, lam, alpha, h, l1, linf, _ = line.split()
            if kind != problem:
                continue
            rows.append((int(scheme[6:]), float(lam), None if alpha == "-" else int(alpha),
                         Fraction(h), float(l1), float(linf)))
    return rows


def _errors(u, ue):
    e = np.abs(u - ue)
    # L1 is the mean over the N+1 grid points x_1..x_{N+1} (periodic end
    # point counted twice); Linf the maximum.
    return np.concatenate([e, e[:1]]).mean(), e.max()


# FP64 reaches the printed three digits wherever the error is above ~1e-12.
ADVECTION_CASES = [(5, 3, Fraction(1, 100)), (5, 3, Fraction(1, 200)), (5, 4, Fraction(1, 100)),
                   (5, 4, Fraction(1, 200)), (9, 3, Fraction(1, 50)), (9, 4, Fraction(1, 50)),
                   (9, 3, Fraction(1, 100)), (13, 4, Fraction(1, 50)), (17, 3, Fraction(1, 15)),
                   (17, 4, Fraction(1, 15)), (17, 4, Fraction(1, 30))]


@pytest.mark.parametrize("order,alpha,h", ADVECTION_CASES)
def test_advection_rows_reproduced(order, alpha, h):
    rows = {(o, lam, a, hh): (l1, li) for (o, lam, a, hh, l1, li) in _golden_rows("advection")}
    n = int(2 / h)
    for lam in (1.0, 1e6):
        x, hh, u0 = workloads.sin_power(alpha, lam, n)
        # linear SSP-RK(m, m-1) with m - 1 = order and dt = h (Sec. 4 preamble), t = 2
        u = oracle.scalar_lssp_run(order, u0, hh, hh, n, order + 1)
        l1, linf = _errors(u, u0)
        p1, pinf = rows[(order, lam, alpha, h)]
        assert float("%.2e" % l1) == pytest.approx(p1, rel=1e-9), (l1, p1)
        assert float("%.2e" % linf) == pytest.approx(pinf, rel=1e-9), (linf, pinf)


def _burgers_exact(x, t, lam):
    u0 = lambda s: lam * (1 + 0.5 * np.sin(np.pi * s) ** 3)
    du0 = lambda s: lam * 1.5 * np.pi * np.sin(np.pi * s) ** 2 * np.cos(np.pi * s)
    s = x - u0(x) * t
    for _ in range(60):                       # Newton on s + u0(s) t = x
        s = s - (s + u0(s) * t - x) / (1 + du0(s) * t)
    return u0(s)


BURGERS_DT = {5: (1.0, Fraction(5, 3)), 9: (100.0, Fraction(3)), 13: (1e4, Fraction(13, 3)),
              17: (1e6, Fraction(17, 3))}


@pytest.mark.parametrize("order", [5, 9, 13, 17])
@pytest.mark.parametrize("lam", [1.0, 1e3])
def test_burgers_rows_reproduced(order, lam):
    h = Fraction(1, 128) if order == 5 else Fraction(1, 64)
    rows = {(o, la, hh): (l1, li) for (o, la, _, hh, l1, li) in _golden_rows("burgers")}
    p1, pinf = rows[(order, lam, h)]
    x, hh, u0 = workloads.burgers_sin3(lam, int(2 / h))
    C, e = BURGERS_DT[order]
    dt = C * hh ** float(e) / lam
    T = 0.1 / lam
    u = oracle.scalar_ssprk3_run(order, u0, hh, dt, t_end=T, flux=oracle.BURGERS, split=oracle.SPLIT_NONE)
    l1, linf = _errors(u, _burgers_exact(x, T, lam))
    # The printed rows come from a quad-precision code with an unstated
    # end-of-run rule; these resolutions agree to within 2.5 percent.
    assert l1 == pytest.approx(p1, rel=0.025)
    assert linf == pytest.approx(pinf, rel=0.025)


# ---------------------------------------------------------------------------
# Properties of the selection (Sec. 3.3)
# ---------------------------------------------------------------------------

def _window(order, f_cells, sign):
    return oracle.recon_faces(order, sign, f_cells)


@pytest.mark.parametrize("order", coeffs.ORDERS)
def test_full_stencil_on_smooth_data(order):
    # Smooth data with critical points of order <= 2r-4 and small h: the
    # global stencil is chosen at every face (Sec. 3.3, first property).
    r = (order + 1) // 2
    for seed in range(5):
        for n in (100, 400):
            x = np.arange(-(r - 1), n + r) * (1.0 / n)
            f = workloads.smooth_sines(seed, x, 1.0)
            for sign in (1, -1):
                _, idx = oracle.recon_faces(order, sign, f)
                assert np.all(idx == 0), (seed, n, sign, np.flatnonzero(idx))


@pytest.mark.parametrize("order", [5, 9, 13, 17])
def test_stencils_never_cross_an_isolated_jump(order):
    # One discontinuity inside smooth data: every selected stencil stays on one
    # side of it (Sec. 3.3, second property).
    r = (order + 1) // 2
    rng = np.random.default_rng(order)
    cands = coeffs.candidates(order)
    for trial in range(60):
        n = 200
        x = np.arange(-(r - 1), n + r) * (1.0 / n)
        f = 0.3 * workloads.smooth_sines(trial, x, 1.0)
        pos = int(rng.integers(20, n - 20))          # jump between cells pos-1 and pos
        f = f + np.where(np.arange(f.size) >= pos, rng.uniform(1.0, 3.0) * rng.choice([-1, 1]), 0.0)
        for sign in (1, -1):
            _, idx = oracle.recon_faces(order, sign, f)
            for i, k in enumerate(idx):
                m, nn = cands[k]
                c = i + r - 1 if sign > 0 else i + r
                lo, hi = (c - m, c + nn) if sign > 0 else (c - nn, c + m)
                assert not (lo < pos <= hi), (trial, sign, i, (m, nn), pos)


@pytest.mark.parametrize("order", [5, 9, 13, 17])
def test_scale_invariance_is_bitwise_for_powers_of_two(order):
    # IS(lambda f) = |lambda| IS(f) (Sec. 3.3, third property); with
    # lambda = +-2^k every operation scales exactly.
    rng = np.random.default_rng(7)
    f = np.cumsum(rng.standard_normal(300)) + np.where(np.arange(300) > 150, 2.0, 0.0)
    for sign in (1, -1):
        base, idx0 = oracle.recon_faces(order, sign, f)
        for lam in (2.0 ** 20, 2.0 ** -30, -8.0):
            got, idx = oracle.recon_faces(order, sign, lam * f)
            assert np.array_equal(idx, idx0)
            assert np.array_equal(got, lam * base)


def _exact_select(order, f, c, s):
    """Steps 1-3.2 of Sec. 3.2 in exact rationals at one face; returns (idx, fhat, margin)."""
    F = lambda l: f[c + s * l]
    is_l = max(abs(F(0) - F(-1)), abs(F(0) - 2 * F(-1) + F(-2)))
    is_r = max(abs(F(0) - F(1)), abs(F(0) - 2 * F(1) + F(2)))
    is0 = min(is_l, is_r)
    margin = None
    for k, (m, n, a, b) in enumerate(coeffs.exact_table(order)):
        if m < 1 or n < 1:
            continue
        isc = abs(sum(b[l + m] * F(l) for l in range(-m, n + 1)))
        scale = max(sum(abs(b[l + m] * F(l)) for l in range(-m, n + 1)), abs(F(0)) + 2 * abs(F(-1)) + abs(F(-2)))
        mu = abs(isc - is0) / scale if scale else Fraction(1)
        margin = mu if margin is None else min(margin, mu)
        if isc < is0:
            return k, sum(a[l + m] * F(l) for l in range(-m, n + 1)), margin
    da, db = F(1) - F(0), F(0) - F(-1)
    if da * db > 0:
        mm = da if abs(da) <= abs(db) else db
    else:
        mm = 0
    cands = coeffs.candidates(order)
    pick = (0, 1) if (da * db > 0 and abs(da) <= abs(db)) else ((1, 0) if da * db > 0 else (0, 0))
    return cands.index(pick), F(0) + mm / 2, margin


@pytest.mark.parametrize("order", [5, 9, 17])
def test_fp64_selection_matches_exact_rational_selection(order):
    # Brute force on small inputs: the FP64 oracle takes the same decisions as
    # the exact-rational evaluation wherever no comparison is a near-tie.
    r = (order + 1) // 2
    rng = np.random.default_rng(100 + order)
    checked = 0
    for trial in range(40):
        n = 12
        vals = rng.integers(-40, 41, size=n + 2 * r - 1) / 8.0      # exact in binary
        if trial % 3 == 0:
            vals = np.round(np.sin(np.arange(vals.size) * 0.3 + trial) * 64) / 64.0
        fx = [Fraction(float(v)) for v in vals]
        for sign in (1, -1):
            got, idx = oracle.recon_faces(order, sign, vals)
            for i in range(n):
                c = i + r - 1 if sign > 0 else i + r
                k, fh, margin = _exact_select(order, fx, c, sign)
                if margin is not None and margin < Fraction(1, 10 ** 12):
                    continue
                assert idx[i] == k, (trial, sign, i)
                assert abs(Fraction(float(got[i])) - fh) <= Fraction(1, 10 ** 12) * (1 + abs(fh))
                checked += 1
    assert checked > 500


def test_recon_faces_minus_is_mirror_of_plus():
    # f^- at x_{j+1/2} is the mirror image of f^+ (Sec. 3.1): reversing the
    # array turns one into the other, face for face.
    rng = np.random.default_rng(3)
    f = np.cumsum(rng.standard_normal(120))
    for order in (5, 9, 17):
        p, ip = oracle.recon_faces(order, 1, f)
        m, im = oracle.recon_faces(order, -1, f[::-1].copy())
        assert np.array_equal(ip, im[::-1])
        # sums run in opposite cell order, so values agree to rounding
        np.testing.assert_allclose(p, m[::-1], rtol=1e-13, atol=1e-13)


# ---------------------------------------------------------------------------
# Scalar laws: conservation and no new extrema at a step
# ---------------------------------------------------------------------------

def test_scalar_operator_is_conservative():
    _, h, u = workloads.advection_sines_step(0, 200)
    for order in (5, 9, 17):
        L = oracle.scalar_rhs(order, u, h)
        assert abs(L.sum()) < 1e-11 * np.abs(L).sum()


@pytest.mark.parametrize("order", [5, 9, 13, 17])
def test_advected_square_wave_has_no_new_extrema(order):
    n = 200
    x, h = workloads.nodes(-1.0, 1.0, n)
    u0 = np.where((x >= -0.4) & (x < 0.3), 1.0, 0.0)
    u = oracle.scalar_ssprk3_run(order, u0, h, 0.5 * h, nsteps=200)
    # ENO: overshoots only at the level of rounding and a tiny fraction of the jump
    assert u.max() < 1.0 + 2e-3 and u.min() > -2e-3, (u.min(), u.max())
    assert abs(u.sum() - u0.sum()) < 1e-10
