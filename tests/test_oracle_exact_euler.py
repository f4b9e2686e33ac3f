"""The oracle's characteristic Euler path against an exact-rational
evaluation of the same steps (no GPU).

Given the split fluxes G+- (Eq. LF_Flux_Split) and the face's eigenvector
matrices L, R as the oracle forms them in FP64 (every double is an exact
rational), the steps after them are done here in exact arithmetic
(fractions.Fraction): each window cell projected onto each characteristic
field (Sec. 4 preamble), IS0 (Eq. Baseline_IS), the candidates' indicators
|sum_l b_l w| in list order with the first one below IS0 accepted (Sec. 3.2,
Step 3.1, Eq. ISCoe), minmod otherwise (Step 3.2), the flux sum_l a_l w
(Eq. ReconstructedFlux), F-hat = R w-hat and the conservative difference
(Eq. 1DWENOFD).  On grids with jumps, smooth parts and flat parts:

  * every (face, field, sign) choice of the FP64 oracle equals the exact one
    unless the exact margin of the deciding comparison is below 1e-12;
  * L(U) agrees within 1e-12 relative per variable, the exact evaluation
    taking the oracle's choice at those near-ties.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads
from oracle import coeffs

TIE = Fraction(1, 10 ** 12)
GAMMA = 1.4


def _split(U, alpha, gamma=GAMMA):
    """G+- per cell in FP64, the formulas of the LF split with the plain
    primitive variables (Python floats are IEEE doubles)."""
    nv, n = U.shape
    Gp = np.empty((n, nv))
    Gm = np.empty((n, nv))
    for i in range(n):
        rho, mn, E = U[0, i], U[1, i], U[nv - 1, i]
        mt = U[2, i] if nv == 4 else 0.0
        un = mn / rho
        ut = mt / rho if nv == 4 else 0.0
        ke = 0.5 * (mn * un + mt * ut) if nv == 4 else 0.5 * (mn * un)
        p = (gamma - 1.0) * (E - ke)
        F = [mn, mn * un + p] + ([mt * un] if nv == 4 else []) + [(E + p) * un]
        for v in range(nv):
            t = alpha * U[v, i]
            Gp[i, v] = 0.5 * (F[v] + t)
            Gm[i, v] = 0.5 * (F[v] - t)
    return Gp, Gm


def _exact_recon(order, w, a, c, s):
    """Steps 1-3.2 at one face in exact arithmetic: w, a map a cell index to
    its value and rounding magnitude.  Returns (choice, value, margin)."""
    table = coeffs.exact_table(order)
    nc = len(table)
    F = lambda l: w[c + s * l]
    A = lambda l: a[c + s * l]
    is_l = max(abs(F(0) - F(-1)), abs(F(0) - 2 * F(-1) + F(-2)))
    is_r = max(abs(F(0) - F(1)), abs(F(0) - 2 * F(1) + F(2)))
    is0 = min(is_l, is_r)
    s0 = max(A(0) + 2 * A(-1) + A(-2), A(0) + 2 * A(1) + A(2))
    margin = None
    for k, (m, n, al, bl) in enumerate(table[:nc - 3]):
        isc = abs(sum(bl[l + m] * F(l) for l in range(-m, n + 1)))
        scale = max(sum(abs(bl[l + m]) * A(l) for l in range(-m, n + 1)), s0)
        mu = abs(isc - is0) / scale if scale else Fraction(0)
        margin = mu if margin is None else min(margin, mu)
        if isc < is0:
            return k, sum(al[l + m] * F(l) for l in range(-m, n + 1)), margin
    da, db = F(1) - F(0), F(0) - F(-1)
    S = A(1) + 2 * A(0) + A(-1)
    if S:
        margin = min(margin, min(abs(da), abs(db)) / S, abs(abs(da) - abs(db)) / S)
    if da * db > 0:
        k, mm = (nc - 3, da) if abs(da) <= abs(db) else (nc - 2, db)
    else:
        k, mm = nc - 1, 0
    return k, F(0) + Fraction(mm) / 2, margin


def _exact_value(order, w, c, s, k):
    table = coeffs.exact_table(order)
    nc = len(table)
    F = lambda l: w[c + s * l]
    if k < nc - 3:
        m, n, al, _ = table[k]
        return sum(al[l + m] * F(l) for l in range(-m, n + 1))
    if k == nc - 3:
        return F(0) + (F(1) - F(0)) / 2
    if k == nc - 2:
        return F(0) + (F(0) - F(-1)) / 2
    return F(0)


def _exact_line(order, U, h, bc, idx_fp64, gamma=GAMMA):
    """Exact L of one line in its face-normal frame (U [nv][n], FP64) with the
    FP64 oracle's stencil log idx_fp64 [n+1][nv][2].  Returns (L exact as
    floats, number of choices compared, number of near-ties)."""
    nv, n = U.shape
    r = (order + 1) // 2
    g = r + 1
    cells = [(i - g) % n if bc == oracle.PERIODIC else min(max(i - g, 0), n - 1) for i in range(n + 2 * g)]
    Ug = U[:, cells]
    alpha = oracle.euler_maxspeed_1d(U, gamma)      # max |u_n| + c over the line
    Gp, Gm = _split(Ug, alpha, gamma)
    Fh = []
    compared = ties = 0
    for f in range(n + 1):
        j = f - 1 + g
        Lm, Rm = oracle.roe_eigen(Ug[:, j], Ug[:, j + 1], gamma)
        Lq = [[Fraction(float(x)) for x in row] for row in Lm]
        Rq = [[Fraction(float(x)) for x in row] for row in Rm]
        what = []
        for k in range(nv):
            val = []
            for sg, G, s, c in ((0, Gp, 1, j), (1, Gm, -1, j + 1)):
                win = range(j - r + 1, j + r + 1)
                w = {i: sum(Lq[k][v] * Fraction(float(G[i, v])) for v in range(nv)) for i in win}
                a = {i: sum(abs(Lq[k][v]) * abs(Fraction(float(G[i, v]))) for v in range(nv)) for i in win}
                ke, ve, mu = _exact_recon(order, w, a, c, s)
                got = int(idx_fp64[f, k, sg])
                compared += 1
                if got != ke:
                    assert mu < TIE, ("choice differs off a near-tie", f, k, sg, got, ke, float(mu))
                    ties += 1
                    ve = _exact_value(order, w, c, s, got)
                val.append(ve)
            what.append(val[0] + val[1])
        Fh.append([sum(Rq[v][k] * what[k] for k in range(nv)) for v in range(nv)])
    ih = Fraction(1.0 / h)
    L = np.array([[float(-(Fh[i + 1][v] - Fh[i][v]) * ih) for i in range(n)] for v in range(nv)])
    return L, compared, ties


def _assert_close(L, Lx):
    for v in range(L.shape[0]):
        scale = np.abs(Lx[v]).max()
        assert np.abs(L[v] - Lx[v]).max() <= 1e-12 * scale, (v, np.abs(L[v] - Lx[v]).max(), scale)


@pytest.mark.parametrize("order", [5, 9, 17])
@pytest.mark.parametrize("case", ["lax", "riemann"])
def test_euler1d_selection_and_operator_match_exact_rationals(order, case):
    if case == "lax":
        # the Lax shock tube (Sec. 4.3) after 12 oracle steps: rarefaction,
        # contact and shock, with flat states between them
        _, h, U = workloads.euler1d_lax(48)
        U, _ = oracle.euler1d_run(5, U, h, 12, cfl=0.5)
        bc = oracle.OUTFLOW
    else:
        _, h, U = workloads.euler1d_riemann_perturbed(order, 44)
        U = U.copy()
        U[:, 34:] = U[:, 34:35]               # a flat tail after the smooth wave right of the jump
        bc = oracle.PERIODIC
    L, idx, _ = oracle.euler1d_rhs(order, U, h, bc=bc, with_idx=True)
    Lx, compared, ties = _exact_line(order, U, h, bc, idx)
    assert compared == (U.shape[1] + 1) * 6 and ties <= compared // 4   # rounding-level flat states
    assert len(set(idx.reshape(-1).tolist())) >= 3               # jumps exercise the candidates
    _assert_close(L, Lx)


def test_euler2d_lines_match_exact_rationals():
    # The 2D operator is the sum of its x and y sweeps; each sweep's lines are
    # 1D characteristic problems with four fields (the y lines on the
    # permuted state).  Quadrant states give jumps across both axes.
    order = 9
    nx, ny = 14, 12
    (x, y, hx, hy), U = workloads.euler2d_quadrants_vortices(4, nx, ny, nvort=1)
    L, ix, iy, _, _ = oracle.euler2d_rhs(order, U, hx, hy, bcx=oracle.PERIODIC, bcy=oracle.OUTFLOW, with_idx=True)
    Lx = np.zeros_like(U)
    for yy in range(ny):
        lx, _, _ = _exact_line(order, np.ascontiguousarray(U[:, yy, :]), hx, oracle.PERIODIC, ix[yy])
        Lx[:, yy, :] += lx
    perm = [0, 2, 1, 3]
    for xx in range(nx):
        line = np.ascontiguousarray(U[perm, :, xx])
        ly, _, _ = _exact_line(order, line, hy, oracle.OUTFLOW, iy[:, xx])
        Lx[perm, :, xx] += ly
    _assert_close(L, Lx)
