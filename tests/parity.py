"""Parity of the HIP path with the CPU oracle, under the near-tie rule.

Two FP64 implementations of ENO-MR that evaluate the same formulas in
different orders take the same stencil decisions, except where a comparison
(IS < IS0 of Step 3.1, or a minmod branch of Step 3.2) lies within rounding of
a tie.  The rule the tests apply:

  * stencil logs: wherever the GPU's logged choice differs from the oracle's,
    the oracle's margin of the deciding comparison (relative to its rounding
    scale) must satisfy |mu| < TIE_TOL = 1e-12; such faces are ties and are
    reported (count, largest |mu|);
  * the operator L(U): evaluated by the oracle on the same input, taking the
    GPU's choice at the ties, it agrees with the GPU's per variable within
    STAGE_TOL * max(max|L_oracle|, S) at every cell, where S is the size of
    the terms L is the difference of (the split fluxes over h, summed over
    the directions): a variable whose L is near zero next to its fluxes (rho
    of a state at rest, the momentum of a symmetric shear) is cancellation,
    and relative to its own maximum it is rounding noise (the error without
    taking the GPU's choice is printed too);
  * runs: the oracle's own SSP-RK3 run, taking the GPU's choice at the ties of
    every stage (the GPU's stage logs), agrees with the GPU's final state per
    variable within FINAL_TOL * max(1, max|U_oracle|), and every step's dt
    within DT_TOL relative.  Runs that do not take the GPU's choices drift
    apart beyond that: a rounding-level tie can switch a later decision whose
    margin is not small, and the switch moves the solution by the truncation
    error.

Helpers only: no test is collected from this module.
"""
import numpy as np

import oracle

TIE_TOL = oracle.TIE_TOL
STAGE_TOL = 1e-12
FINAL_TOL = 1e-10
DT_TOL = 1e-13


def host(t):
    return t.detach().cpu().numpy()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def rel_err_per_var(got, ref, floor=0.0):
    """max |got - ref| / max(floor, max |ref|) for each leading index."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    out = []
    for v in range(ref.shape[0]):
        scale = max(floor, float(np.abs(ref[v]).max()))
        err = float(np.abs(got[v] - ref[v]).max())
        out.append(err / scale if scale > 0 else err)
    return out


def assert_ties(rep, what):
    bad = np.abs(rep.mu) >= TIE_TOL
    assert not bad.any(), "%s: %d stencil choices differ from the oracle's with |mu| >= %g (largest %.3g at log " \
                          "position %d)" % (what, int(bad.sum()), TIE_TOL, float(np.abs(rep.mu).max()),
                                            int(rep.pos[np.argmax(np.abs(rep.mu))]))


def _euler_fluxes(U, gamma):
    """Face-normal fluxes of every direction of U ([3][n] or [4][ny][nx]) and
    each direction's largest |u_n| + c."""
    rho = U[0]
    if U.shape[0] == 3:
        u = U[1] / rho
        p = (gamma - 1.0) * (U[2] - 0.5 * U[1] * u)
        c = np.sqrt(gamma * p / rho)
        return [(np.stack([U[1], U[1] * u + p, (U[2] + p) * u]), float((np.abs(u) + c).max()))]
    u, v = U[1] / rho, U[2] / rho
    p = (gamma - 1.0) * (U[3] - 0.5 * (U[1] * u + U[2] * v))
    c = np.sqrt(gamma * p / rho)
    Fx = np.stack([U[1], U[1] * u + p, U[2] * u, (U[3] + p) * u])
    Fy = np.stack([U[2], U[1] * v, U[2] * v + p, (U[3] + p) * v])
    return [(Fx, float((np.abs(u) + c).max())), (Fy, float((np.abs(v) + c).max()))]


def flux_scale(U, hs, gamma=1.4, gravity=0.0):
    """Per variable: sum over the directions of max |G+-| / h, the size of
    the split fluxes whose differences L is made of (plus the source)."""
    U = np.asarray(U)
    out = np.zeros(U.shape[0])
    for (F, a), h in zip(_euler_fluxes(U, gamma), hs):
        for v in range(U.shape[0]):
            out[v] += float((0.5 * (np.abs(F[v]) + a * np.abs(U[v]))).max()) / h
    if gravity:
        out[2] += abs(gravity) * float(np.abs(U[0]).max())
        out[3] += abs(gravity) * float(np.abs(U[2]).max())
    return out


def assert_stage_close(got, ref, what, scale=None):
    """Per variable: |got - ref| <= STAGE_TOL max(max|ref|, scale).  Returns
    the errors relative to max|ref| (printed) and to the bound's scale."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    rel, rel_s = [], []
    for v in range(ref.shape[0]):
        m = float(np.abs(ref[v]).max())
        sc = max(m, float(scale[v]) if scale is not None else 0.0)
        err = float(np.abs(got[v] - ref[v]).max())
        rel.append(err / m if m > 0 else err)
        rel_s.append(err / sc if sc > 0 else err)
    assert max(rel_s) <= STAGE_TOL, (what, rel_s, rel)
    return rel_s


def check_euler2d_operator(order, U, hx, hy, L_gpu, log_gpu, what="euler2d", **kw):
    """The GPU's L(U) and stencil log of a 2D Euler problem against the
    oracle (ties followed).  kw: bcx, bcy, gamma and the operator switches.
    Returns the tie report."""
    L_gpu = np.asarray(L_gpu)
    log_gpu = np.asarray(log_gpu).reshape(-1)
    Lf, ix, iy, _, _, rep = oracle.euler2d_rhs_follow(order, U, hx, hy, log_gpu, **kw)
    own = np.concatenate([ix.reshape(-1), iy.reshape(-1)])
    assert own.size == log_gpu.size
    assert int((own != log_gpu).sum()) == rep.count
    assert_ties(rep, what)
    errs = assert_stage_close(L_gpu, Lf, what, flux_scale(U, (hx, hy), kw.get("gamma", 1.4), kw.get("gravity", 0.0)))
    Ln = oracle._euler2d(order, U, hx, hy, kw.get("gamma", 1.4), kw.get("bcx", oracle.PERIODIC),
                         kw.get("bcy", oracle.OUTFLOW), kw.get("componentwise", False), kw.get("per_field", False),
                         kw.get("gravity", 0.0), None, False)[0]
    print("%s order %d %s: ties %d of %d choices (max |mu| %.3g); L rel err %.3g (ties followed), %.3g (not)"
          % (what, order, "x".join(map(str, U.shape[1:][::-1])), rep.count, own.size, rep.max_abs_mu, max(errs),
             max(rel_err_per_var(L_gpu, Ln))), flush=True)
    return rep


def check_euler1d_operator(order, U, h, L_gpu, log_gpu, what="euler1d", **kw):
    L_gpu = np.asarray(L_gpu)
    log_gpu = np.asarray(log_gpu).reshape(-1)
    Lf, idx, _, rep = oracle.euler1d_rhs_follow(order, U, h, log_gpu, **kw)
    assert int((idx.reshape(-1) != log_gpu).sum()) == rep.count
    assert_ties(rep, what)
    errs = assert_stage_close(L_gpu, Lf, what, flux_scale(U, (h,), kw.get("gamma", 1.4)))
    print("%s order %d n %d: ties %d (max |mu| %.3g); L rel err %.3g"
          % (what, order, U.shape[1], rep.count, rep.max_abs_mu, max(errs)), flush=True)
    return rep


def check_scalar_operator(order, u, h, L_gpu, log_gpu, what="scalar", **kw):
    """Scalar laws: the GPU evaluates every flux as the oracle does, so with
    the ties followed the operator is bitwise equal."""
    L_gpu = np.asarray(L_gpu).reshape(-1)
    Lf, idx, _, rep = oracle.scalar_rhs(order, u, h, follow=np.asarray(log_gpu).reshape(-1), **kw)
    assert_ties(rep, what)
    assert np.array_equal(L_gpu, Lf), (what, float(np.abs(L_gpu - Lf).max()))
    return rep


def check_recon(order, sign, f, fhat_gpu, idx_gpu, what="recon"):
    got = np.asarray(fhat_gpu)
    fh, idx, rep = oracle.recon_faces(order, sign, f, follow=np.asarray(idx_gpu))
    assert_ties(rep, what)
    assert np.array_equal(got, fh), (what, float(np.abs(got - fh).max()))
    return rep


def follow_run_2d(ctx, prob, U0, nsteps, cfl=0.5, what="euler2d run", **kw):
    """nsteps SSP-RK3 steps on the GPU (dt from the CFL rule, stencil logs of
    every stage) and the oracle's own run taking the GPU's choices at the
    ties of every stage.  Checks each step's dt and the final state; returns
    (gpu final, oracle final, total ties, largest |mu|)."""
    import torch
    order, hx, hy = prob.order, prob.hx, prob.hy
    U = dev(U0)
    ib = prob.idx_bytes()
    log = torch.empty(3 * ib, dtype=torch.uint8, device="cuda")
    Uo = np.array(U0, dtype=np.float64, copy=True)
    gamma = kw.get("gamma", 1.4)
    ties, worst = 0, 0.0
    for step in range(nsteps):
        dtd = ctx.dt(prob, U, cfl)
        ctx.ssprk3_step(prob, U, dtd, log)
        ctx.check()
        logs = host(log)
        dt_g = float(host(dtd)[0])
        dt_o = oracle.dt_2d(Uo, hx, hy, cfl, gamma)
        assert abs(dt_g - dt_o) <= DT_TOL * dt_o, (what, step, dt_g, dt_o)
        un = Uo.copy()
        us = Uo.copy()
        for s in range(3):
            L, _, _, _, _, rep = oracle.euler2d_rhs_follow(order, us, hx, hy, logs[s * ib:(s + 1) * ib], **kw)
            assert_ties(rep, "%s step %d stage %d" % (what, step, s + 1))
            ties += rep.count
            worst = max(worst, rep.max_abs_mu)
            us = oracle.ssprk3_combine(s + 1, un, us, L, dt_o)
        Uo = us
        if prob.nx * prob.ny >= 1 << 20:
            # a progress line per step of the large runs (minutes of oracle time)
            print("%s step %d/%d: ties so far %d (max |mu| %.3g)" % (what, step + 1, nsteps, ties, worst), flush=True)
    got = host(U)
    errs = rel_err_per_var(got, Uo, floor=1.0)
    print("%s order %d %dx%d, %d steps: ties %d (max |mu| %.3g); final rel err %.3g"
          % (what, order, prob.nx, prob.ny, nsteps, ties, worst, max(errs)), flush=True)
    assert max(errs) <= FINAL_TOL, (what, errs)
    return got, Uo, ties, worst


def follow_run_1d(ctx, prob, U0, nsteps, cfl=0.5, what="euler1d run"):
    """follow_run_2d for a 1D Euler problem (recorded steps)."""
    import torch
    order, h, bc = prob.order, prob.hx, prob.bc_x
    n = prob.nx
    U = dev(U0)
    ib = prob.idx_bytes()
    stages = torch.empty((3, 3 * n), dtype=torch.float64, device="cuda")
    idx = torch.empty(3 * ib, dtype=torch.uint8, device="cuda")
    alpha = torch.empty(3, dtype=torch.float64, device="cuda")
    dtd = torch.empty(1, dtype=torch.float64, device="cuda")
    Uo = np.array(U0, dtype=np.float64, copy=True)
    ties, worst = 0, 0.0
    for step in range(nsteps):
        ctx.step_record(prob, U, cfl, stages, idx, alpha, dtd)
        ctx.check()
        logs = host(idx)
        dt_g = float(host(dtd)[0])
        dt_o = oracle.dt_1d(Uo, h, cfl)
        assert abs(dt_g - dt_o) <= DT_TOL * dt_o, (what, step, dt_g, dt_o)
        un = Uo.copy()
        us = Uo.copy()
        for s in range(3):
            L, _, _, rep = oracle.euler1d_rhs_follow(order, us, h, logs[s * ib:(s + 1) * ib], bc=bc)
            assert_ties(rep, "%s step %d stage %d" % (what, step, s + 1))
            ties += rep.count
            worst = max(worst, rep.max_abs_mu)
            us = oracle.ssprk3_combine(s + 1, un, us, L, dt_o)
        Uo = us
    got = host(U)
    errs = rel_err_per_var(got, Uo, floor=1.0)
    print("%s order %d n %d, %d steps: ties %d (max |mu| %.3g); final rel err %.3g"
          % (what, order, n, nsteps, ties, worst, max(errs)), flush=True)
    assert max(errs) <= FINAL_TOL, (what, errs)
    return got, Uo, ties, worst
