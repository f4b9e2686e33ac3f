"""Pins of the oracle's Euler operator variants.

Variants: component-wise reconstruction (no characteristic projection),
per-field alphas (alpha_k = max over the line of the field's |lambda_k|, a
field-wise reading of the maximum in Eq. LF_Flux_Split), and the gravity
source g [0, 0, rho, rho v] of the Rayleigh-Taylor problem (Sec. 4.4).

The paper prints no numbers for these, so they are pinned by reductions and
invariants that hold whatever the evaluation order:
  - on a contact (u, p constant) every split flux component is an affine map
    of rho, and ENO-MR commutes with affine maps (its indicators are
    differences and its selection compares magnitudes), so the component-wise
    fluxes are affine maps of the bare scalar reconstruction of rho;
  - the per-field alphas equal a brute-force maximum over the cells, and where
    a field's alpha equals the line's alpha (u+c with u >= 0, u-c with
    u <= 0) that field chooses the same stencils as the characteristic
    operator with one alpha;
  - every variant reaches the design order on smooth periodic data, against
    a spectral derivative of the exact flux;
  - a uniform state's residual is exactly the source; a hydrostatic state
    (dp/dy = g rho, u = v = 0) is balanced to the design order.
"""
import numpy as np
import pytest

import oracle
import workloads

G = 1.4


def _primitives(U):
    rho = U[0]
    if U.shape[0] == 3:
        u = U[1] / rho
        p = (G - 1) * (U[2] - 0.5 * rho * u * u)
        return rho, u, None, p
    u, v = U[1] / rho, U[2] / rho
    p = (G - 1) * (U[3] - 0.5 * rho * (u * u + v * v))
    return rho, u, v, p


def _flux_1d(U):
    rho, u, _, p = _primitives(U)
    return np.stack([rho * u, rho * u * u + p, (U[2] + p) * u])


def _spectral_dx(f, h):
    n = f.shape[-1]
    k = np.fft.fftfreq(n, d=h) * 2 * np.pi
    return np.real(np.fft.ifft(1j * k * np.fft.fft(f, axis=-1), axis=-1))


def _smooth_periodic_1d(n):
    x, h = workloads.nodes(0.0, 1.0, n)
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * x)
    u = 0.4 + 0.15 * np.cos(2 * np.pi * x + 0.3)
    p = 1.0 + 0.1 * np.sin(2 * np.pi * x + 1.1)
    return h, workloads.conserved_1d(rho, u, p)


def _halo_periodic(f, r):
    n = f.size
    return f[(np.arange(n + 2 * r) - r) % n]


@pytest.mark.parametrize("order", [5, 9, 17])
def test_componentwise_contact_is_affine_in_scalar_reconstruction(order):
    r = (order + 1) // 2
    n = 96
    rng = np.random.default_rng(order)
    x, h = workloads.nodes(0.0, 1.0, n)
    rho = 1.0 + 0.3 * np.sin(2 * np.pi * x + rng.uniform(0, 6)) + 0.5 * ((x > 0.3) & (x < 0.6))
    u0, p0 = 0.7, 1.3
    U = workloads.conserved_1d(rho, np.full(n, u0), np.full(n, p0))
    L, idx, alpha = oracle.euler1d_rhs_var(order, U, h, G, oracle.PERIODIC, componentwise=True)
    a = alpha[0]
    rho_, u_, _, p_ = _primitives(U)
    assert a == np.max(np.abs(u_) + np.sqrt(G * p_ / rho_))
    f = _halo_periodic(rho, r)            # faces 0..n: n+1 faces, n + 2r values
    Rp, ip = oracle.recon_faces(order, +1, f)
    Rm, im = oracle.recon_faces(order, -1, f)
    # G+- = c+- rho + d+- per component (F and U are affine in rho on a contact)
    gm1 = G - 1.0
    cF = [u0, u0 * u0, 0.5 * u0 ** 3]
    dF = [0.0, p0, G * p0 * u0 / gm1]
    cU = [1.0, u0, 0.5 * u0 * u0]
    dU = [0.0, 0.0, p0 / gm1]
    for k in range(3):
        cp, dp = 0.5 * (cF[k] + a * cU[k]), 0.5 * (dF[k] + a * dU[k])
        cm, dm = 0.5 * (cF[k] - a * cU[k]), 0.5 * (dF[k] - a * dU[k])
        Fh = (cp * Rp + dp) + (cm * Rm + dm)
        ref = -(Fh[1:] - Fh[:-1]) / h
        scale = np.abs(ref).max() + np.abs(Fh).max() / h * 1e-3
        np.testing.assert_allclose(L[k], ref, rtol=0, atol=1e-11 * scale)
        # the same stencils as rho's (the negative scale of the - side included)
        assert np.array_equal(idx[:, k, 0], ip)
        assert np.array_equal(idx[:, k, 1], im)


@pytest.mark.parametrize("per_field", [False, True])
def test_per_field_alphas_are_brute_force_maxima(per_field):
    _, U = workloads.euler2d_quadrants_vortices(3, 24, 20, nvort=2)
    _, _, _, ax, ay = oracle.euler2d_rhs_var(7, U, 0.05, 0.05, G, oracle.PERIODIC, oracle.OUTFLOW,
                                             per_field=per_field)
    rho, u, v, p = _primitives(U)
    c = np.sqrt(G * p / rho)
    if per_field:
        want_x = np.stack([np.abs(u - c).max(1), np.abs(u).max(1), np.abs(u + c).max(1)])
        want_y = np.stack([np.abs(v - c).max(0), np.abs(v).max(0), np.abs(v + c).max(0)])
        np.testing.assert_allclose(ax, want_x, rtol=1e-15)
        np.testing.assert_allclose(ay, want_y, rtol=1e-15)
        # max over the three fields is the line's alpha, bit for bit
        _, _, _, bx, by = oracle.euler2d_rhs_var(7, U, 0.05, 0.05, G, oracle.PERIODIC, oracle.OUTFLOW)
        assert np.array_equal(ax.max(0), bx[0]) and np.array_equal(ay.max(0), by[0])
    else:
        np.testing.assert_allclose(ax[0], (np.abs(u) + c).max(1), rtol=1e-15)
        np.testing.assert_allclose(ay[0], (np.abs(v) + c).max(0), rtol=1e-15)


@pytest.mark.parametrize("sign", [+1, -1])
def test_per_field_matches_line_alpha_where_the_field_speed_is_the_line_speed(sign):
    # u of one sign everywhere: the u+c field (u >= 0) or the u-c field
    # (u <= 0) has the line's alpha, so it must choose the same stencils.
    order, n = 9, 160
    x, h = workloads.nodes(0.0, 1.0, n)
    rho = np.where(x < 0.5, 1.0, 0.4) + 0.1 * np.sin(6 * np.pi * x)
    u = sign * (0.3 + 0.2 * (x > 0.3) + 0.05 * np.cos(2 * np.pi * x))
    p = np.where(x < 0.7, 1.0, 0.3)
    U = workloads.conserved_1d(rho, u, p)
    _, ipf, apf = oracle.euler1d_rhs_var(order, U, h, G, oracle.OUTFLOW, per_field=True)
    _, iline, aline = oracle.euler1d_rhs_var(order, U, h, G, oracle.OUTFLOW)
    k = 2 if sign > 0 else 0
    assert apf[k] == aline[0]
    assert np.array_equal(ipf[:, k, :], iline[:, k, :])
    # the other acoustic field splits with a smaller alpha: its choices differ somewhere
    o = 2 - k
    assert apf[o] < aline[0]


# Per-field alphas at order 5 are left out: where a field's |lambda_k| reaches
# alpha_k, its f^- has a flat critical point, and on this data the order-5
# selection falls back to minmod next to that cell up to n = 256 (it takes
# the full stencil from n = 512 on).  Orders 7 and 9 take it at these sizes.
@pytest.mark.parametrize("variant,order,n0", [("componentwise", 5, 32), ("componentwise", 9, 16),
                                              ("per_field", 7, 32), ("per_field", 9, 24)])
def test_1d_variants_reach_design_order(variant, order, n0):
    errs = []
    for n in (n0, 2 * n0):
        h, U = _smooth_periodic_1d(n)
        exact = -_spectral_dx(_flux_1d(U), h)
        L, _, _ = oracle.euler1d_rhs_var(order, U, h, G, oracle.PERIODIC, **{variant: True})
        errs.append(np.abs(L - exact).max())
    rate = np.log2(errs[0] / errs[1])
    assert rate > order - 0.5, (errs, rate)


@pytest.mark.parametrize("variant,order", [("componentwise", 5), ("per_field", 7)])
def test_2d_variants_reach_design_order(variant, order):
    n0 = 24
    errs = []
    for n in (n0, 2 * n0):
        x, h = workloads.nodes(0.0, 1.0, n)
        X, Y = np.meshgrid(x, x)
        rho = 1.0 + 0.2 * np.sin(2 * np.pi * (X + 2 * Y))
        u = 0.3 + 0.1 * np.cos(2 * np.pi * Y)
        v = -0.2 + 0.1 * np.sin(2 * np.pi * X)
        p = 1.0 + 0.1 * np.cos(2 * np.pi * (X - Y))
        U = workloads.conserved_2d(rho, u, v, p)
        E = U[3]
        Fx = np.stack([rho * u, rho * u * u + p, rho * u * v, (E + p) * u])
        Fy = np.stack([rho * v, rho * u * v, rho * v * v + p, (E + p) * v])
        exact = -_spectral_dx(Fx, h) - np.swapaxes(_spectral_dx(np.swapaxes(Fy, 1, 2), h), 1, 2)
        L = oracle.euler2d_rhs_var(order, U, h, h, G, oracle.PERIODIC, oracle.PERIODIC, **{variant: True})[0]
        errs.append(np.abs(L - exact).max())
    rate = np.log2(errs[0] / errs[1])
    assert rate > order - 0.5, (errs, rate)


def test_uniform_state_residual_is_exactly_the_source():
    ny, nx, g = 20, 18, 0.75
    rho0, u0, v0, p0 = 1.7, 0.4, -0.9, 2.2
    one = np.ones((ny, nx))
    U = workloads.conserved_2d(rho0 * one, u0 * one, v0 * one, p0 * one)
    for cw, pf in [(False, False), (True, False), (False, True)]:
        L = oracle.euler2d_rhs_var(7, U, 0.1, 0.1, G, oracle.PERIODIC, oracle.OUTFLOW, cw, pf, gravity=g)[0]
        assert np.all(L[0] == 0) and np.all(L[1] == 0)
        assert np.all(L[2] == g * U[2 * 0][0, 0]) and np.all(L[3] == g * U[2][0, 0])


@pytest.mark.parametrize("order", [5, 9])
def test_hydrostatic_state_is_balanced_to_design_order(order):
    # rho(y) smooth, u = v = 0, p(y) = p0 + g * integral of rho: dp/dy = g rho
    g = 1.0
    errs = []
    r = (order + 1) // 2
    for ny in (32, 64):
        y, hy = workloads.nodes(0.0, 1.0, ny)
        nx, hx = 8, 0.125
        rho_y = 2.0 + 0.5 * np.sin(2 * np.pi * y)
        p_y = 3.0 + g * (2.0 * y - 0.5 * np.cos(2 * np.pi * y) / (2 * np.pi))
        rho = np.repeat(rho_y[:, None], nx, 1)
        p = np.repeat(p_y[:, None], nx, 1)
        z = np.zeros_like(rho)
        U = workloads.conserved_2d(rho, z, z, p)
        L = oracle.euler2d_rhs_var(order, U, hx, hy, G, oracle.PERIODIC, oracle.OUTFLOW, gravity=g)[0]
        inner = slice(r + 2, ny - r - 2)     # away from the outflow copies
        errs.append(np.abs(L[:, inner, :]).max())
    rate = np.log2(errs[0] / errs[1])
    assert rate > order - 1.0, (errs, rate)
    # with the source's sign flipped the residual is 2 g rho, not small
    L = oracle.euler2d_rhs_var(order, U, hx, hy, G, oracle.PERIODIC, oracle.OUTFLOW, gravity=-g)[0]
    assert np.abs(L[2, inner, :]).min() > 1.0


def test_variant_switches_reject_both():
    h, U = _smooth_periodic_1d(16)
    with pytest.raises(RuntimeError):
        oracle.euler1d_rhs_var(5, U, h, G, oracle.PERIODIC, componentwise=True, per_field=True)
