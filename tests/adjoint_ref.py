"""Oracle-side reference for the frozen-stencil adjoint of SSP-RK3 runs (test
helper; uses only the CPU oracle)."""
import numpy as np

import oracle

C13, C23 = 1.0 / 3.0, 2.0 / 3.0


def record_run(order, U0, h, nsteps, cfl=0.5, bc=oracle.OUTFLOW, dts=None):
    """Oracle SSP-RK3 run recording each stage's input, stencil log and alpha."""
    U = np.array(U0, dtype=np.float64, copy=True)
    rec = []
    for step in range(nsteps):
        dt = oracle.dt_1d(U, h, cfl) if dts is None else dts[step]
        un = U.copy()
        us = U.copy()
        stages = []
        for s in (1, 2, 3):
            L, idx, a = oracle.euler1d_rhs(order, us, h, bc=bc, with_idx=True)
            stages.append((us.copy(), idx.copy(), a))
            us = oracle.ssprk3_combine(s, un, us, L, dt)
        rec.append((dt, stages))
        U = us
    return U, rec


def frozen_run(order, U0, h, rec, bc=oracle.OUTFLOW):
    """The run with every stencil, alpha and dt held at the recorded values."""
    U = np.array(U0, dtype=np.float64, copy=True)
    for dt, stages in rec:
        un = U.copy()
        us = U.copy()
        for s, (_, idx, a) in zip((1, 2, 3), stages):
            L = oracle.euler1d_rhs_frozen(order, us, h, idx, a, bc=bc)
            us = oracle.ssprk3_combine(s, un, us, L, dt)
        U = us
    return U


def adjoint(order, h, rec, lam, bc=oracle.OUTFLOW):
    """lambda_0 = (dU_T/dU_0)^T lambda_T of the frozen run, from dense
    Jacobians of the frozen operator (tangents, transposed)."""
    lam = np.array(lam, dtype=np.float64).reshape(-1)
    for dt, stages in reversed(rec):
        (u0, i0, a0), (u1, i1, a1), (u2, i2, a2) = stages
        J2 = oracle.euler1d_rhs_frozen_jacobian(order, u2, h, i2, a2, bc=bc)
        J1 = oracle.euler1d_rhs_frozen_jacobian(order, u1, h, i1, a1, bc=bc)
        J0 = oracle.euler1d_rhs_frozen_jacobian(order, u0, h, i0, a0, bc=bc)
        l2 = C23 * lam + J2.T @ (C23 * dt * lam)
        ln = C13 * lam
        l1 = 0.25 * l2 + J1.T @ (0.25 * dt * l2)
        ln = ln + 0.75 * l2
        ln = ln + l1 + J0.T @ (dt * l1)
        lam = ln
    return lam
