"""Parity of the Euler operator variants on the GPU with the oracle:
component-wise reconstruction, per-field alphas and the gravity source of the
Rayleigh-Taylor problem (Sec. 4.4), under the near-tie rule of
tests/parity.py."""
import numpy as np
import pytest

import oracle
import workloads
from parity import check_euler1d_operator, check_euler2d_operator, follow_run_2d

pytestmark = pytest.mark.gpu

VARIANTS = [dict(componentwise=True), dict(per_field=True)]


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2311_15504_amd as enomr
    c = enomr.Context(0)
    yield c
    c.close()


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _host(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("kw", VARIANTS, ids=["componentwise", "per_field"])
@pytest.mark.parametrize("order", [5, 9, 13, 17])
def test_euler1d_variant_operator(ctx, order, kw):
    import paper_2311_15504_amd as enomr
    n = 1000
    _, h, U = workloads.euler1d_riemann_perturbed(order + 100, n)
    for bc in (enomr.OUTFLOW, enomr.PERIODIC):
        got, gidx = ctx.rhs(enomr.Problem.euler1d(n, h, order, bc=bc, **kw), _dev(U), with_idx=True)
        ctx.check()
        check_euler1d_operator(order, U, h, _host(got), _host(gidx), what=str(kw), bc=bc, **kw)


@pytest.mark.parametrize("kw", VARIANTS + [dict(gravity=1.0), dict(per_field=True, gravity=-0.5)],
                         ids=["componentwise", "per_field", "gravity", "per_field_gravity"])
@pytest.mark.parametrize("order", [5, 9, 13, 17])
def test_euler2d_variant_operator(ctx, order, kw):
    import paper_2311_15504_amd as enomr
    nx, ny = 150, 70                                   # ragged against both tile shapes
    (x, y, hx, hy), U = workloads.euler2d_quadrants_vortices(order + 7, nx, ny)
    got, gidx = ctx.rhs(enomr.Problem.euler2d(nx, ny, hx, hy, order, **kw), _dev(U), with_idx=True)
    ctx.check()
    check_euler2d_operator(order, U, hx, hy, _host(got), _host(gidx), what=str(kw), **kw)


@pytest.mark.parametrize("kw", VARIANTS, ids=["componentwise", "per_field"])
def test_smallest_periodic_grid_variants(ctx, kw):
    import paper_2311_15504_amd as enomr
    order = 17
    n = order + 2
    (x, y, hx, hy), U = workloads.euler2d_quadrants_vortices(5, n, n)
    got, gidx = ctx.rhs(enomr.Problem.euler2d(n, n, hx, hy, order, enomr.PERIODIC, enomr.PERIODIC, **kw), _dev(U),
                        with_idx=True)
    ctx.check()
    check_euler2d_operator(order, U, hx, hy, _host(got), _host(gidx), what=str(kw), bcx=oracle.PERIODIC,
                           bcy=oracle.PERIODIC, **kw)


@pytest.mark.parametrize("order", [5, 9])
def test_rayleigh_taylor_run_matches_oracle(ctx, order):
    # The Rayleigh-Taylor data with its gravity source, x periodic (the
    # perturbation has period 1/4), y outflow; 6 SSP-RK3 steps.
    import paper_2311_15504_amd as enomr
    g53 = 5.0 / 3.0
    nx, ny = 32, 128
    (x, y, hx, hy), U0 = workloads.euler2d_rayleigh_taylor(nx, ny, g53)
    prob = enomr.Problem.euler2d(nx, ny, hx, hy, order, enomr.PERIODIC, enomr.OUTFLOW, gamma=g53, gravity=1.0)
    follow_run_2d(ctx, prob, U0, 6, what="Rayleigh-Taylor run", gamma=g53, gravity=1.0)


def test_per_field_run_and_dt_match_oracle(ctx):
    import paper_2311_15504_amd as enomr
    nx, ny = 48, 40
    (x, y, hx, hy), U0 = workloads.euler2d_quadrants_vortices(11, nx, ny)
    # the per-field maxima give the same step as the line maxima
    assert oracle.euler2d_run(13, U0, hx, hy, 1, cfl=0.5, per_field=True)[1] == \
        oracle.euler2d_run(13, U0, hx, hy, 1, cfl=0.5)[1]
    prob = enomr.Problem.euler2d(nx, ny, hx, hy, 13, per_field=True)
    follow_run_2d(ctx, prob, U0, 4, what="per-field run", per_field=True)


def test_variants_are_rejected_where_unsupported(ctx):
    import torch
    import paper_2311_15504_amd as enomr
    _, h, U = workloads.euler1d_riemann_perturbed(1, 64)
    p = enomr.Problem.euler1d(64, h, 9, per_field=True)
    with pytest.raises(enomr.EnomrError) as e:
        enomr.Batch(ctx, [p], [_dev(U)], autotune=False)
    assert e.value.status == 1
    with pytest.raises(ValueError):
        enomr.solve(ctx, p, _dev(U).requires_grad_(True), 0.5, 2)
    ib = p.idx_bytes()
    stages = torch.empty((2, 3, U.size), dtype=torch.float64, device="cuda")
    idx = torch.empty((2, 3 * ib), dtype=torch.uint8, device="cuda")
    alpha = torch.empty((2, 3), dtype=torch.float64, device="cuda")
    dts = torch.empty((2, 1), dtype=torch.float64, device="cuda")
    with pytest.raises(enomr.EnomrError) as e:
        ctx.record_steps(p, _dev(U), 0.5, 2, stages, idx, alpha, dts)
    assert e.value.status == 1


@pytest.mark.parametrize("dim,kw", [(1, dict()), (1, dict(componentwise=True)), (1, dict(per_field=True)),
                                    (2, dict()), (2, dict(componentwise=True)), (2, dict(per_field=True)),
                                    (2, dict(gravity=1.0))],
                         ids=["1d", "1d-componentwise", "1d-per_field", "2d", "2d-componentwise", "2d-per_field",
                              "2d-gravity"])
def test_advance_equals_single_steps(ctx, dim, kw):
    # enomr_advance alternates its stages between two alpha buffers, each
    # alpha pass zeroing the next stage's; single steps fill the one buffer
    # before every alpha pass.  Both give the same run bit for bit (dt of each
    # step from the CFL rule either way).
    import paper_2311_15504_amd as enomr
    order, nsteps = 9, 7
    if dim == 1:
        n = 700
        _, h, U0 = workloads.euler1d_riemann_perturbed(21, n)
        prob = enomr.Problem.euler1d(n, h, order, **kw)
    else:
        nx, ny = 130, 90
        (x, y, hx, hy), U0 = workloads.euler2d_quadrants_vortices(22, nx, ny)
        prob = enomr.Problem.euler2d(nx, ny, hx, hy, order, **kw)
    A = _dev(U0)
    ctx.advance(prob, A, 0.5, nsteps)
    B = _dev(U0)
    for _ in range(nsteps):
        dt = ctx.dt(prob, B, 0.5)
        ctx.ssprk3_step(prob, B, dt)
    ctx.check()
    assert np.array_equal(_host(A), _host(B))


def test_advance_to_an_end_time_equals_single_steps(ctx):
    # With an end time the run's step that would pass it is shortened and the
    # later steps do nothing (every kernel of the run checks the active flag,
    # the alternating alpha buffers included): the same states as single steps
    # with the logged step sizes.
    import torch
    import paper_2311_15504_amd as enomr
    nx, ny, order, nsteps = 120, 100, 13, 12
    (x, y, hx, hy), U0 = workloads.euler2d_quadrants_vortices(23, nx, ny)
    prob = enomr.Problem.euler2d(nx, ny, hx, hy, order)
    probe = _dev(U0)
    dt0 = float(_host(ctx.dt(prob, probe, 0.5))[0])
    t_end = 6.5 * dt0                               # ends inside a step, well before nsteps
    A = _dev(U0)
    log = torch.zeros(nsteps, dtype=torch.float64, device="cuda")
    ctx.advance(prob, A, 0.5, nsteps, t_end=t_end, dt_log=log)
    ctx.check()
    dts = _host(log)
    k = int(np.count_nonzero(dts))
    assert 6 <= k < nsteps and np.all(dts[k:] == 0.0)
    assert abs(dts[:k].sum() - t_end) <= 1e-13 * t_end
    B = _dev(U0)
    for j in range(k):
        ctx.ssprk3_step(prob, B, log[j:j + 1])
    ctx.check()
    assert np.array_equal(_host(A), _host(B))
