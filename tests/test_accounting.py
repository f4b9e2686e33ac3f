"""The benchmark's algorithmic operation count (bench.line_ops and
bench.stage_tail_ops, applied to stencil logs) equals the oracle's
instrumented count of the same operator evaluation (orc_ops_begin /
orc_ops_end, counted as the method's steps run in the paper's order, the early
exit included, fma = 1).  No GPU: both sides use the oracle's own logs."""
import numpy as np
import pytest

import bench
import oracle
import workloads


def _field_hist(idx):
    """[4][256] counts of the logged candidates per field of idx [..][4][2]."""
    return np.stack([np.bincount(idx[..., q, :].reshape(-1).astype(np.int64), minlength=256)[:256]
                     for q in range(4)])


@pytest.mark.parametrize("order", [9, 17])
@pytest.mark.parametrize("bcx,bcy", [(oracle.PERIODIC, oracle.OUTFLOW), (oracle.OUTFLOW, oracle.OUTFLOW),
                                     (oracle.PERIODIC, oracle.PERIODIC)])
def test_log_based_count_equals_instrumented_oracle(order, bcx, bcy):
    nx, ny = 41, 30
    (x, y, hx, hy), U = workloads.euler2d_quadrants_vortices(order, nx, ny)
    _, ix, iy, ops = oracle.euler2d_rhs_ops(order, U, hx, hy, bcx=bcx, bcy=bcy)
    # ix: [ny][nx+1][4][2]; iy: [ny+1][nx][4][2]; a periodic line's last face repeats its first
    ixl = ix[:, :nx] if bcx == oracle.PERIODIC else ix
    iyl = iy[:ny] if bcy == oracle.PERIODIC else iy
    hx_ = _field_hist(ixl)
    hy_ = _field_hist(iyl)
    fx = ny * (nx if bcx == oracle.PERIODIC else nx + 1)
    fy = nx * (ny if bcy == oracle.PERIODIC else ny + 1)
    ox, _ = bench.line_ops(order, fx, nx * ny, hx_)
    oy, _ = bench.line_ops(order, fy, nx * ny, hy_)
    assert hx_[:, 1:].sum() > 0 and hy_[:, 1:].sum() > 0      # the data exercises the fallback
    assert hx_[2, 1:].sum() > 0                               # the shear field's fallback too
    assert ox == ops[0], (ox, ops[0])
    assert oy == ops[1], (oy, ops[1])
    assert ops[2] == nx * ny * bench.SUM_OPS and ops[3] == 0


def test_stage_combination_count():
    (x, y, hx, hy), U = workloads.euler2d_quadrants_vortices(3, 20, 17)
    L = oracle.euler2d_rhs(9, U, hx, hy)
    for stage in (1, 2, 3):
        cats = np.zeros(4)
        oracle.lib().orc_ops_begin()
        oracle.ssprk3_combine(stage, U, U, L, 1e-3)
        oracle.lib().orc_ops_end(oracle._p(cats))
        assert cats[3] == bench.stage_tail_ops(20 * 17, stage) - 20 * 17 * bench.SUM_OPS
        assert cats[:3].sum() == 0


def test_smooth_face_count_closed_form():
    # On smooth data every reconstruction takes the full stencil (C = 0).
    order, n = 17, 128
    r = (order + 1) // 2
    x = np.linspace(-1.0, 1.0, n, endpoint=False)
    X, Y = np.meshgrid(x, x)
    rho = 1.0 + 0.2 * np.sin(np.pi * X) * np.cos(np.pi * Y)
    u = 0.3 * np.sin(np.pi * (X + Y))
    v = 0.2 * np.cos(np.pi * X) + 0.1 * np.sin(np.pi * Y)
    p = 1.0 + 0.1 * np.sin(np.pi * Y) * np.cos(np.pi * X)
    U = np.stack([rho, rho * u, rho * v, p / 0.4 + 0.5 * rho * (u * u + v * v)])
    _, ix, iy, ops = oracle.euler2d_rhs_ops(order, U, 2.0 / n, 2.0 / n, bcx=oracle.PERIODIC,
                                           bcy=oracle.PERIODIC)
    assert not ix.any() and not iy.any()
    ny, nx = rho.shape
    w = 2 * r - 1
    # per face: Roe, projection of both windows onto every field, back-projection,
    # and 8 reconstructions of IS0 + b_l chain + compare + a_l chain
    per_face = 42 + 2 * w * 16 + (4 + 16) + 8 * (11 + (w + 1) + w)
    per_cell = (18 + 5 * 4) + 2 * 4       # staging and the difference, per line
    assert ops[0] == ny * nx * per_face + nx * ny * per_cell
    assert ops[1] == nx * ny * per_face + nx * ny * per_cell
    assert ops[2] == nx * ny * 4
    # about 2060 operations per cell and RK stage at order 17 (with the average stage combination)
    total = (ops[:3].sum() + nx * ny * (8 + 20 + 20) / 3) / (nx * ny)
    assert 2000 < total < 2100, total
