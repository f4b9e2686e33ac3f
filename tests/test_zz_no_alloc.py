"""enomr_rhs_noalloc, the entry point that allocates nothing (its per-line
alphas live in a library-owned device array), against enomr_rhs through the
C ABI: two calls in a row, the second with a smaller input, for 2D and 1D
Euler (default operator and per-field alphas) and a scalar law.  Both entry
points run the same kernels, so results and stencil logs are bitwise equal;
each call is also checked against the oracle (tests/parity.py)."""
import numpy as np
import pytest

import oracle
import workloads
from parity import check_euler1d_operator, check_euler2d_operator, check_scalar_operator, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2311_15504_amd as enomr
    c = enomr.Context(0)
    yield c
    c.close()


def _both(ctx, prob, U):
    import torch
    a, ia = ctx.rhs_noalloc(prob, U, with_idx=True)
    ctx.check()
    b, ib = ctx.rhs(prob, U, with_idx=True)
    ctx.check()
    assert torch.equal(a, b) and torch.equal(ia, ib)
    return host(a), host(ia)


@pytest.mark.parametrize("per_field", [False, True])
def test_noalloc_2d_equals_rhs_twice_second_smaller(ctx, per_field):
    import paper_2311_15504_amd as enomr
    for (nx, ny, order, seed) in ((300, 260, 17, 1), (97, 41, 9, 2)):
        (x, y, hx, hy), U0 = workloads.euler2d_quadrants_vortices(seed, nx, ny)
        prob = enomr.Problem.euler2d(nx, ny, hx, hy, order, per_field=per_field)
        L, idx = _both(ctx, prob, dev(U0))
        check_euler2d_operator(order, U0, hx, hy, L, idx, what="rhs_noalloc", per_field=per_field)


def test_noalloc_1d_and_scalar_twice_second_smaller(ctx):
    import paper_2311_15504_amd as enomr
    for n, order in ((3000, 13), (200, 5)):
        _, h, U0 = workloads.euler1d_riemann_perturbed(order, n)
        L, idx = _both(ctx, enomr.Problem.euler1d(n, h, order), dev(U0))
        check_euler1d_operator(order, U0, h, L, idx, what="rhs_noalloc 1D")
    for n, order in ((20011, 17), (301, 7)):
        _, h, u = workloads.advection_sines_step(order, n)
        L, idx = _both(ctx, enomr.Problem.scalar(enomr.ADVECTION, n, h, order), dev(u[None]))
        check_scalar_operator(order, u, h, L, idx, what="rhs_noalloc scalar")


def test_noalloc_rejects_what_does_not_fit(ctx):
    # argument errors return before any work is enqueued: the per-field
    # alphas of a 30000 x 30000 grid need more than the scratch array holds,
    # and dUdt may not alias U
    import ctypes
    import torch
    import paper_2311_15504_amd as enomr
    small = dev(np.ones((4, 32, 32)))
    big = enomr.Problem.euler2d(30000, 30000, 1e-3, 1e-3, 9, per_field=True)
    with pytest.raises(enomr.EnomrError) as e:
        enomr._call("enomr_rhs_noalloc", ctx.handle, ctypes.byref(big), enomr._ptr(small), enomr._ptr(small.clone()),
                    None)
    assert e.value.status == 1 and "scratch" in str(e.value)
    (x, y, hx, hy), U0 = workloads.euler2d_quadrants_vortices(3, 40, 30)
    prob = enomr.Problem.euler2d(40, 30, hx, hy, 9)
    U = dev(U0)
    with pytest.raises(enomr.EnomrError) as e:
        enomr._call("enomr_rhs_noalloc", ctx.handle, ctypes.byref(prob), enomr._ptr(U), enomr._ptr(U), None)
    assert e.value.status == 1
    torch.cuda.synchronize()
