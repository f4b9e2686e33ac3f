"""Frozen-stencil adjoint on the GPU against the oracle's transposed Jacobians
and against central finite differences (h = 1e-6) of runs with the recorded
step sizes.  The reference adjoint runs along the GPU's recorded forward
run (its stage states, stencil choices, alphas and step sizes), whose
choices are checked against the oracle's under the near-tie rule."""
import numpy as np
import pytest

import oracle
import workloads
from adjoint_ref import adjoint as ref_adjoint
from adjoint_ref import frozen_run
from parity import DT_TOL, FINAL_TOL, assert_ties, check_euler1d_operator, rel_err_per_var

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


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.mark.parametrize("order,n", [(5, 70), (9, 70), (17, 70), (9, 200), (17, 19), (5, 7)])
@pytest.mark.parametrize("bc", [oracle.OUTFLOW, oracle.PERIODIC])
def test_rhs_adjoint_is_the_transposed_jacobian(ctx, order, n, bc):
    # n = 70: two workgroups, the second ragged; n = 200: interior workgroups
    # whose faces come only from their neighbours' cells; n = 2r + 1 (the
    # smallest grid accepted): the widest stencils of every face wrap
    # (periodic) or reach ghost images at both ends (outflow).
    import torch
    import paper_2311_15504_amd as enomr
    _, h, U = workloads.euler1d_riemann_perturbed(10 + order + bc, n)
    L, idx, alpha = oracle.euler1d_rhs(order, U, h, bc=bc, with_idx=True)
    J = oracle.euler1d_rhs_frozen_jacobian(order, U, h, idx, alpha, bc=bc)
    rng = np.random.default_rng(order)
    lam = rng.standard_normal(U.shape)
    ref = (J.T @ lam.reshape(-1)).reshape(U.shape)
    prob = enomr.Problem.euler1d(n, h, order, bc=bc)
    got = ctx.rhs_adjoint(prob, _dev(U), torch.from_numpy(idx.reshape(-1).copy()).cuda(),
                          torch.tensor([alpha], dtype=torch.float64, device="cuda"), _dev(lam))
    ctx.check()
    got2 = ctx.rhs_adjoint(prob, _dev(U), torch.from_numpy(idx.reshape(-1).copy()).cuda(),
                           torch.tensor([alpha], dtype=torch.float64, device="cuda"), _dev(lam))
    ctx.check()
    assert torch.equal(got, got2)   # no atomics: bitwise reproducible
    got = got.cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max(), np.abs(got - ref).max() / np.abs(ref).max()


def _gpu_record(ctx, prob, U0, nsteps, cfl=0.5):
    """The GPU's recorded run as the oracle-side reference takes it:
    [(dt, [(stage state, stencil log, alpha) x 3])], each stage's choices
    checked against the oracle on the same stage state."""
    import torch
    n = prob.nx
    ib = prob.idx_bytes()
    stages = torch.empty((nsteps, 3, 3 * n), dtype=torch.float64, device="cuda")
    idx = torch.empty((nsteps, 3 * ib), dtype=torch.uint8, device="cuda")
    alpha = torch.empty((nsteps, 3), dtype=torch.float64, device="cuda")
    dts = torch.empty((nsteps, 1), dtype=torch.float64, device="cuda")
    U = _dev(U0)
    ctx.record_steps(prob, U, cfl, nsteps, stages, idx, alpha, dts)
    ctx.check()
    S, I, A, D = stages.cpu().numpy(), idx.cpu().numpy(), alpha.cpu().numpy(), dts.cpu().numpy()
    rec = []
    for k in range(nsteps):
        st = []
        for s in range(3):
            us = S[k, s].reshape(3, n)
            log = I[k, s * ib:(s + 1) * ib].reshape(n + 1, 3, 2)
            _, _, oa, rep = oracle.euler1d_rhs_follow(prob.order, us, prob.hx, log, bc=prob.bc_x)
            assert_ties(rep, "recorded step %d stage %d" % (k, s + 1))
            assert abs(A[k, s] - oa[0]) <= 1e-14 * oa[0]
            st.append((us, log, float(A[k, s])))
        rec.append((float(D[k, 0]), st))
    return U.cpu().numpy(), rec


def test_recorded_step_equals_plain_step(ctx):
    import torch
    import paper_2311_15504_amd as enomr
    _, h, U0 = workloads.euler1d_riemann_perturbed(3, 300)
    prob = enomr.Problem.euler1d(300, h, 9)
    A = _dev(U0)
    B = _dev(U0)
    stages = torch.empty((3, 900), dtype=torch.float64, device="cuda")
    idx = torch.empty(3 * prob.idx_bytes(), dtype=torch.uint8, device="cuda")
    alpha = torch.empty(3, dtype=torch.float64, device="cuda")
    dt = torch.empty(1, dtype=torch.float64, device="cuda")
    ctx.step_record(prob, A, 0.5, stages, idx, alpha, dt)
    ctx.advance(prob, B, 0.5, 1)
    ctx.check()
    assert torch.equal(A, B)
    assert torch.equal(stages[0].view(3, 300), _dev(U0))
    assert abs(dt.item() - oracle.dt_1d(U0, h, 0.5)) <= DT_TOL * dt.item()
    ib = prob.idx_bytes()
    for s in range(3):
        us = stages[s].cpu().numpy().reshape(3, 300)
        got, _ = ctx.rhs(prob, _dev(us), with_idx=True)
        check_euler1d_operator(9, us, h, got.cpu().numpy(), idx[s * ib:(s + 1) * ib].cpu().numpy())
        assert abs(alpha[s].item() - oracle.euler_maxspeed_1d(us)) <= 1e-14 * alpha[s].item()


def _loss_grad_gpu(ctx, prob, U0, target, h, cfl, nsteps, every):
    import torch
    import paper_2311_15504_amd as enomr
    U = _dev(U0).requires_grad_(True)
    UT = enomr.solve(ctx, prob, U, cfl, nsteps, every)
    J = h * ((UT[0] - _dev(target)) ** 2).sum()
    J.backward()
    ctx.check()
    return J.item(), U.grad.cpu().numpy(), UT.detach().cpu().numpy()


@pytest.mark.parametrize("bc", [oracle.OUTFLOW, oracle.PERIODIC])
def test_gradient_matches_oracle_adjoint_and_fd(ctx, bc):
    import paper_2311_15504_amd as enomr
    n, order, nsteps, every = 48, 9, 12, 5
    if bc == oracle.PERIODIC:
        _, h, U0 = workloads.euler1d_smooth_periodic(4, n)
    else:
        _, h, U0 = workloads.euler1d_riemann_perturbed(4, n)
    target = workloads.density_target(4, n)
    prob = enomr.Problem.euler1d(n, h, order, bc=bc)
    Jv, g, UT = _loss_grad_gpu(ctx, prob, U0, target, h, 0.5, nsteps, every)
    UT_rec, rec = _gpu_record(ctx, prob, U0, nsteps)
    assert np.array_equal(UT, UT_rec)
    # the oracle's frozen run with the recorded choices reproduces the GPU run
    assert max(rel_err_per_var(frozen_run(order, U0, h, rec, bc=bc), UT, floor=1.0)) <= FINAL_TOL
    lamT = np.zeros_like(U0)
    lamT[0] = 2.0 * h * (UT[0] - target)
    g_ref = ref_adjoint(order, h, rec, lamT, bc=bc).reshape(U0.shape)
    assert np.abs(g - g_ref).max() <= 1e-10 * np.abs(g_ref).max()
    # central differences of the frozen run
    rng = np.random.default_rng(7)
    for _ in range(6):
        d = rng.standard_normal(U0.shape) * 0.1
        eps = 1e-6
        Jp = h * ((frozen_run(order, U0 + eps * d, h, rec, bc=bc)[0] - target) ** 2).sum()
        Jm = h * ((frozen_run(order, U0 - eps * d, h, rec, bc=bc)[0] - target) ** 2).sum()
        fd = (Jp - Jm) / (2 * eps)
        assert abs(fd - (g * d).sum()) <= 1e-6 * max(abs(fd), 1e-12), (fd, (g * d).sum())


def test_adjoint_workload_gradient_and_fd(ctx):
    # 1D Euler, N = 8192, 9th order, 400 steps checkpointed every 20, smooth
    # seeded data; central differences (h = 1e-6) of GPU runs that replay the
    # recorded step sizes, in random smooth directions.
    import torch
    import paper_2311_15504_amd as enomr
    n, order, nsteps, every = 8192, 9, 400, 20
    x, h, U0 = workloads.euler1d_smooth_periodic(0, n)
    target = workloads.density_target(0, n)
    prob = enomr.Problem.euler1d(n, h, order, bc=enomr.PERIODIC)
    Jv, g, UT = _loss_grad_gpu(ctx, prob, U0, target, h, 0.5, nsteps, every)
    assert np.all(np.isfinite(g)) and np.abs(g).max() > 0
    # the step sizes of the run
    dts = torch.empty(nsteps, dtype=torch.float64, device="cuda")
    U = _dev(U0)
    ctx.advance(prob, U, 0.5, nsteps, dt_log=dts)
    ctx.check()

    def loss(Ustart):
        V = _dev(Ustart)
        for s in range(nsteps):
            ctx.ssprk3_step(prob, V, dts[s:s + 1])
        ctx.check()
        return h * ((V[0].cpu().numpy() - target) ** 2).sum()

    rng = np.random.default_rng(1)
    for k in range(4):
        d = np.stack([workloads.smooth_sines(100 + 3 * k + v, x, 1.0) for v in range(3)]) * 0.01
        eps = 1e-6
        fd = (loss(U0 + eps * d) - loss(U0 - eps * d)) / (2 * eps)
        ad = (g * d).sum()
        assert abs(fd - ad) <= 1e-5 * abs(fd), (fd, ad)
