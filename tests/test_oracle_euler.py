"""Derived checks of the oracle's Euler path (Sec. 4 preamble, 4.3, 4.4).

The paper prints no numbers for its Euler runs (their results are figures), so
these checks pin the characteristic path by identities: eigenvectors are
inverse to each other, a uniform state has no residual, the operator is
conservative and symmetric, a 2D run invariant in y is the 1D run, and the
operator reaches its designed order on smooth data.
"""
import numpy as np
import pytest

import oracle
import workloads

G = 1.4


def _rand_state(rng, nv):
    rho = rng.uniform(0.2, 2.0)
    u = rng.uniform(-1.5, 1.5)
    v = rng.uniform(-1.5, 1.5)
    p = rng.uniform(0.2, 2.0)
    if nv == 3:
        return workloads.conserved_1d([rho], [u], [p])[:, 0]
    return workloads.conserved_2d(np.array([rho]), np.array([u]), np.array([v]), np.array([p]))[:, 0]


@pytest.mark.parametrize("nv", [3, 4])
def test_roe_eigenvectors_are_inverse_and_diagonalise(nv):
    rng = np.random.default_rng(nv)
    for _ in range(50):
        UL, UR = _rand_state(rng, nv), _rand_state(rng, nv)
        Lm, Rm = oracle.roe_eigen(UL, UR, G)
        np.testing.assert_allclose(Lm @ Rm, np.eye(nv), atol=1e-12)
        # Columns of R are eigenvectors of the flux Jacobian at the Roe state:
        # check A r = lambda r with A from a finite difference of the flux at the
        # Roe-averaged state (Roe property: F(UR) - F(UL) = A (UR - UL)).
        def flux(U):
            rho, m = U[0], U[1]
            mt = U[2] if nv == 4 else 0.0
            E = U[-1]
            u = m / rho
            p = (G - 1) * (E - 0.5 * (m * u + mt * mt / rho))
            F = [m, m * u + p] + ([mt * u] if nv == 4 else []) + [(E + p) * u]
            return np.array(F)
        # Roe matrix property: (F(UR) - F(UL)) lies in span and equals R diag(lam) L (UR - UL)
        sL, sR = np.sqrt(UL[0]), np.sqrt(UR[0])
        u = (sL * UL[1] / UL[0] + sR * UR[1] / UR[0]) / (sL + sR)
        lam_idx = [0, 1, 2, 3] if nv == 4 else [0, 1, 2]
        # eigenvalues from R's second row: u - c, u, (u), u + c
        c = (Rm[1, -1] - Rm[1, 0]) / 2.0
        lam = np.array([u - c, u] + ([u] if nv == 4 else []) + [u + c])
        A = Rm @ np.diag(lam) @ Lm
        dF = flux(UR) - flux(UL)
        np.testing.assert_allclose(A @ (UR - UL), dF, rtol=1e-11, atol=1e-11)


def test_uniform_state_has_zero_residual():
    U = workloads.conserved_1d(np.full(64, 0.7), np.full(64, 0.3), np.full(64, 1.2))
    for order in (5, 9, 17):
        L = oracle.euler1d_rhs(order, U, 0.01, G, oracle.PERIODIC)
        assert np.all(L == 0.0)
    U2 = workloads.conserved_2d(np.full((40, 48), 0.7), np.full((40, 48), 0.3), np.full((40, 48), -0.2),
                                np.full((40, 48), 1.2))
    L2 = oracle.euler2d_rhs(9, U2, 0.02, 0.03, G, oracle.PERIODIC, oracle.OUTFLOW)
    assert np.all(L2 == 0.0)


def test_euler_operator_is_conservative():
    _, h, U = workloads.euler1d_riemann_perturbed(1, 256)
    for order in (5, 9, 13, 17):
        L = oracle.euler1d_rhs(order, U, h, G, oracle.PERIODIC)
        for v in range(3):
            assert abs(L[v].sum()) < 1e-12 * np.abs(L[v]).sum() + 1e-13
    _, U2 = workloads.euler2d_quadrants_vortices(3, 40, 36, nvort=2)
    L2 = oracle.euler2d_rhs(9, U2, 0.05, 0.05, G, oracle.PERIODIC, oracle.PERIODIC)
    for v in range(4):
        assert abs(L2[v].sum()) < 1e-12 * np.abs(L2[v]).sum()


def test_y_invariant_2d_equals_1d_bitwise():
    _, h, U1 = workloads.euler1d_riemann_perturbed(5, 96)
    ny = 20
    U2 = np.zeros((4, ny, 96))
    U2[0] = U1[0]
    U2[1] = U1[1]
    U2[3] = U1[2]
    for order in (5, 13, 17):
        L1 = oracle.euler1d_rhs(order, U1, h, G, oracle.OUTFLOW)
        L2 = oracle.euler2d_rhs(order, U2, h, 0.1, G, oracle.OUTFLOW, oracle.PERIODIC)
        for y in range(ny):
            assert np.array_equal(L2[0, y], L1[0])
            assert np.array_equal(L2[1, y], L1[1])
            assert np.array_equal(L2[3, y], L1[2])
            assert np.all(L2[2, y] == 0.0)


@pytest.mark.parametrize("lam", [4.0, 1.0 / 16.0, 2.0 ** 40])
def test_mass_scaling_by_powers_of_four_is_bitwise(lam):
    # Scaling rho, the momenta and E by lam = 4^k keeps u, v, p/rho, c, H
    # and alpha exactly, scales p, F, G+- and every projected value by lam
    # exactly, and scales the Roe weights sqrt(rho) by 2^k exactly, so the
    # Roe state and eigenvectors are unchanged.  Every IS and IS0 scales by
    # lam, so every stencil choice is the same and L(lam U) = lam L(U) bit
    # for bit (Sec. 4.2: the selection is invariant under scaling of the
    # data).  Any term of the wrong degree in the scaled variables breaks it:
    # a sound speed from p instead of p/rho, an additive constant in a
    # weight, an unscaled threshold in a comparison.
    _, h, U1 = workloads.euler1d_riemann_perturbed(3, 120)
    _, U2 = workloads.euler2d_quadrants_vortices(4, 40, 36, nvort=3)
    for order in (5, 9, 17):
        L, idx, a = oracle.euler1d_rhs(order, U1, h, G, oracle.OUTFLOW, with_idx=True)
        Ls, idxs, a_s = oracle.euler1d_rhs(order, lam * U1, h, G, oracle.OUTFLOW, with_idx=True)
        assert np.array_equal(Ls, lam * L)
        assert np.array_equal(idxs, idx) and a_s == a
        L = oracle.euler2d_rhs(order, U2, 0.05, 0.055, G, oracle.PERIODIC, oracle.OUTFLOW)
        Ls = oracle.euler2d_rhs(order, lam * U2, 0.05, 0.055, G, oracle.PERIODIC, oracle.OUTFLOW)
        assert np.array_equal(Ls, lam * L)
    # An odd power of two rounds the Roe weights differently, and choices at
    # rounding-level ties (flat fields) flip: there it is not an identity.
    L = oracle.euler2d_rhs(17, U2, 0.05, 0.055, G, oracle.PERIODIC, oracle.OUTFLOW)
    Ls = oracle.euler2d_rhs(17, 2.0 * U2, 0.05, 0.055, G, oracle.PERIODIC, oracle.OUTFLOW)
    assert not np.array_equal(Ls, 2.0 * L)


def test_transposed_problem_gives_transposed_residual_bitwise():
    _, U = workloads.euler2d_quadrants_vortices(11, 36, 36, nvort=3)
    UT = np.stack([U[0].T, U[2].T, U[1].T, U[3].T]).copy()
    for order in (7, 17):
        L = oracle.euler2d_rhs(order, U, 0.05, 0.05, G, oracle.OUTFLOW, oracle.OUTFLOW)
        LT = oracle.euler2d_rhs(order, UT, 0.05, 0.05, G, oracle.OUTFLOW, oracle.OUTFLOW)
        assert np.array_equal(LT[0], L[0].T)
        assert np.array_equal(LT[1], L[2].T)
        assert np.array_equal(LT[2], L[1].T)
        assert np.array_equal(LT[3], L[3].T)


def test_mirror_symmetry_1d():
    _, h, U = workloads.euler1d_riemann_perturbed(2, 128)
    U[1] = 0.3 * U[0] * np.sin(np.arange(128) * 0.2)
    UR = U[:, ::-1].copy()
    UR[1] = -UR[1]
    for order in (5, 9, 17):
        L = oracle.euler1d_rhs(order, U, h, G, oracle.OUTFLOW)
        LR = oracle.euler1d_rhs(order, UR, h, G, oracle.OUTFLOW)
        np.testing.assert_allclose(LR[0], L[0, ::-1], rtol=1e-12, atol=1e-12 * np.abs(L[0]).max())
        np.testing.assert_allclose(LR[1], -L[1, ::-1], rtol=1e-12, atol=1e-12 * np.abs(L[1]).max())
        np.testing.assert_allclose(LR[2], L[2, ::-1], rtol=1e-12, atol=1e-12 * np.abs(L[2]).max())


def _entropy_wave_1d(n):
    x, h = workloads.nodes(0.0, 1.0, n)
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * x)
    U = workloads.conserved_1d(rho, np.ones(n), np.ones(n))
    drho = -0.2 * 2 * np.pi * np.cos(2 * np.pi * x)         # rho_t = -u rho_x, u = 1, p = 1
    exact = np.stack([drho, drho, 0.5 * drho])
    return h, U, exact


@pytest.mark.parametrize("order,n0", [(5, 32), (7, 24), (9, 16), (13, 12)])
def test_operator_reaches_design_order_on_entropy_wave(order, n0):
    errs = []
    for n in (n0, 2 * n0):
        h, U, exact = _entropy_wave_1d(n)
        L = oracle.euler1d_rhs(order, U, h, G, oracle.PERIODIC)
        errs.append(np.abs(L - exact).max())
    rate = np.log2(errs[0] / errs[1])
    assert rate > order - 0.5, (errs, rate)


@pytest.mark.parametrize("order,n0", [(5, 24), (9, 12)])
def test_2d_operator_reaches_design_order_on_diagonal_wave(order, n0):
    errs = []
    for n in (n0, 2 * n0):
        x, h = workloads.nodes(0.0, 1.0, n)
        X, Y = np.meshgrid(x, x)
        rho = 1.0 + 0.2 * np.sin(2 * np.pi * (X + Y))
        one = np.ones_like(X)
        U = workloads.conserved_2d(rho, one, one, one)
        drho = -2 * 0.2 * 2 * np.pi * np.cos(2 * np.pi * (X + Y))   # -(u rho_x + v rho_y)
        exact = np.stack([drho, drho, drho, drho])                 # E_t = 1/2 |u|^2 rho_t = rho_t
        L = oracle.euler2d_rhs(order, U, h, h, G, oracle.PERIODIC, oracle.PERIODIC)
        errs.append(np.abs(L - exact).max())
    rate = np.log2(errs[0] / errs[1])
    assert rate > order - 0.5, (errs, rate)


def test_lax_shock_tube_runs_and_stays_physical():
    x, h, U0 = workloads.euler1d_lax(200)
    for order in (5, 17):
        U, dts = oracle.euler1d_run(order, U0, h, 60, cfl=0.5, bc=oracle.OUTFLOW)
        rho = U[0]
        # the exact solution's density lies in [0.345, 1.31] (rarefaction on the
        # left, shocked plateau on the right); allow small ENO wiggles only
        assert rho.min() > 0.33 and rho.max() < 1.32
