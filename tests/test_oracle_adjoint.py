"""The oracle's frozen-stencil operator and its tangent (the reference for the
GPU adjoint).  No GPU."""
import numpy as np
import pytest

import oracle
import workloads


@pytest.mark.parametrize("order", [5, 9, 17])
@pytest.mark.parametrize("bc", [oracle.OUTFLOW, oracle.PERIODIC])
def test_frozen_operator_equals_forward_and_tangent_equals_fd(order, bc):
    _, h, U = workloads.euler1d_riemann_perturbed(order + bc, 80)
    L, idx, alpha = oracle.euler1d_rhs(order, U, h, bc=bc, with_idx=True)
    assert len(set(idx.reshape(-1).tolist())) > 2          # shocks: several stencils chosen
    Lf = oracle.euler1d_rhs_frozen(order, U, h, idx, alpha, bc=bc)
    assert np.array_equal(L, Lf)
    rng = np.random.default_rng(order)
    for _ in range(3):
        d = rng.standard_normal(U.shape) * np.abs(U)
        _, dL = oracle.euler1d_rhs_frozen(order, U, h, idx, alpha, d, bc=bc)
        e = 1e-6
        fd = (oracle.euler1d_rhs_frozen(order, U + e * d, h, idx, alpha, bc=bc)
              - oracle.euler1d_rhs_frozen(order, U - e * d, h, idx, alpha, bc=bc)) / (2 * e)
        assert np.abs(fd - dL).max() <= 1e-7 * np.abs(dL).max()


def test_jacobian_is_linear_in_the_direction():
    _, h, U = workloads.euler1d_riemann_perturbed(1, 40)
    _, idx, alpha = oracle.euler1d_rhs(9, U, h, with_idx=True)
    J = oracle.euler1d_rhs_frozen_jacobian(9, U, h, idx, alpha)
    rng = np.random.default_rng(0)
    d = rng.standard_normal(U.shape)
    _, dL = oracle.euler1d_rhs_frozen(9, U, h, idx, alpha, d)
    np.testing.assert_allclose(J @ d.reshape(-1), dL.reshape(-1), rtol=1e-12, atol=1e-12 * np.abs(dL).max())
