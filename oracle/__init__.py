"""CPU oracle for ENO-MR (H. Shen, arXiv 2311.15504) -- TEST INFRASTRUCTURE.

A plain, slow FP64 implementation of what the GPU library computes, used only
by the test suite, the smoke check and the CPU-baseline leg of the benchmark.
It shares no code with the GPU library (paper_2311_15504_amd) and never imports
it.  The heavy loops are plain C (enomr_oracle.c, built with gcc
-ffp-contract=off); the stencil coefficients are derived here in exact
rational arithmetic (coeffs.py) and handed to the C code as doubles.

Entry points (all numpy float64, C-contiguous):
  recon_faces(order, sign, f_with_halo)             Sec. 3.2 at n faces
  scalar_rhs(order, u, h, ...)                      Eq. (1DWENOFD) for a scalar law
  euler1d_rhs / euler2d_rhs / euler2d_rhs_cells     Euler right-hand sides
  euler1d_run / euler2d_run / scalar_*_run          SSP-RK3 / linear SSP-RK runs
  lssp_coefficients(m)                              Eq. (lSSPRK_Coe), exact
"""
import ctypes
import os
import subprocess
from fractions import Fraction

import numpy as np

from . import coeffs

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "enomr_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

PERIODIC, OUTFLOW = 0, 1
ADVECTION, BURGERS = 0, 1
SPLIT_NONE, SPLIT_LF = 0, 1
MAXW = 17

_dp = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_lp = ctypes.POINTER(ctypes.c_long)


class OracleError(RuntimeError):
    pass


def build(force=True):
    """Compile enomr_oracle.c into liboracle.so with gcc (plain FP64, no contraction)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    cmd = ["gcc", "-O2", "-std=c99", "-D_DEFAULT_SOURCE", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-o", LIB + ".tmp", SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        L.orc_table_new.restype = ctypes.c_void_p
        L.orc_table_new.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int), _dp, _dp]
        L.orc_table_free.argtypes = [ctypes.c_void_p]
        L.orc_recon_faces.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_long, _dp, _dp, _u8p]
        L.orc_scalar_rhs.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_long, ctypes.c_double, _dp, _dp, _u8p, _dp]
        L.orc_roe_eigen.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp, _dp, _dp]
        L.orc_euler1d_rhs.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_long,
                                      ctypes.c_double, _dp, _dp, _u8p, _dp]
        L.orc_ops_begin.restype = None
        L.orc_ops_begin.argtypes = []
        L.orc_ops_end.restype = ctypes.c_double
        L.orc_ops_end.argtypes = []
        L.orc_euler2d_rhs.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_long, ctypes.c_long, ctypes.c_double, ctypes.c_double,
                                      _dp, _dp, _u8p, _u8p, _dp, _dp]
        L.orc_euler1d_rhs_var.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_long,
                                          ctypes.c_double, _dp, _dp, _u8p, _dp, ctypes.c_int, ctypes.c_int]
        L.orc_euler1d_rhs_var.restype = ctypes.c_int
        L.orc_euler2d_rhs_var.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_long, ctypes.c_long, ctypes.c_double, ctypes.c_double,
                                          _dp, _dp, _u8p, _u8p, _dp, _dp, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_double]
        L.orc_euler2d_rhs_var.restype = ctypes.c_int
        L.orc_euler2d_rhs_cells.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_long, ctypes.c_long, ctypes.c_double, ctypes.c_double,
                                            _dp, ctypes.c_long, _lp, _dp]
        L.orc_euler1d_rhs_frozen.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_long,
                                             ctypes.c_double, _dp, _dp, _u8p, ctypes.c_double, _dp, _dp]
        L.orc_euler_maxspeed.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_long, _dp, _dp]
        L.orc_euler2d_maxspeeds.argtypes = [ctypes.c_double, ctypes.c_long, ctypes.c_long, _dp, _dp, _dp]
        L.orc_ssprk3_combine.restype = None
        L.orc_ssprk3_combine.argtypes = [ctypes.c_int, ctypes.c_long, _dp, _dp, _dp, ctypes.c_double, _dp]
        L.orc_scalar_lssp_run.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                          ctypes.c_int, ctypes.c_long, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_long, ctypes.c_int, _dp, _dp]
        L.orc_scalar_ssprk3_run.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                            ctypes.c_int, ctypes.c_long, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_double, ctypes.c_long, _dp]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _u8(a):
    return None if a is None else a.ctypes.data_as(_u8p)


def _check(st, what):
    if st != 0:
        raise OracleError("%s failed with status %d" % (what, st))


_tables = {}


def table(order):
    """C-side candidate table for `order` (a_l, b_l as correctly rounded doubles)."""
    if order not in _tables:
        rows = coeffs.double_table(order)
        nc = len(rows)
        mn = (ctypes.c_int * (2 * nc))(*[v for (m, n, _, _) in rows for v in (m, n)])
        a = np.zeros((nc, MAXW))
        b = np.zeros((nc, MAXW))
        for c, (m, n, al, bl) in enumerate(rows):
            a[c, :len(al)] = al
            b[c, :len(bl)] = bl
        ptr = lib().orc_table_new(order, nc, mn, _p(a), _p(b))
        if not ptr:
            raise OracleError("bad table for order %d" % order)
        _tables[order] = ptr
    return _tables[order]


def ncand(order):
    return len(coeffs.candidates(order))


# --------------------------------------------------------------------------
# Scalar reconstruction and scalar laws
# --------------------------------------------------------------------------

def recon_faces(order, sign, f_with_halo):
    """f-hat at n = len - (2r-1) faces; face i between array cells i+r-1, i+r."""
    f = np.ascontiguousarray(f_with_halo, dtype=np.float64)
    r = (order + 1) // 2
    n = f.size - (2 * r - 1)
    fhat = np.empty(max(n, 0))
    idx = np.empty(max(n, 0), dtype=np.uint8)
    _check(lib().orc_recon_faces(table(order), sign, n, _p(f), _p(fhat), _u8(idx)), "recon_faces")
    return fhat, idx


def scalar_rhs(order, u, h, flux=ADVECTION, a=1.0, split=SPLIT_LF, bc=PERIODIC, with_idx=False):
    """L(u) for a scalar law on one line; idx [n+1][2] if requested."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    n = u.size
    out = np.empty(n)
    idx = np.empty((n + 1) * 2, dtype=np.uint8) if with_idx else None
    alpha = ctypes.c_double()
    _check(lib().orc_scalar_rhs(table(order), flux, a, split, bc, n, 1.0 / h, _p(u), _p(out),
                                _u8(idx), ctypes.byref(alpha)), "scalar_rhs")
    if with_idx:
        return out, idx.reshape(n + 1, 2), alpha.value
    return out


def lssp_coefficients(m):
    """alpha_{m,0..m-1} of Eq. (lSSPRK_Coe) as exact Fractions.

    alpha_{2,0} = 0, alpha_{2,1} = 1; alpha_{m,k} = (2/k) alpha_{m-1,k-1} for
    k = 1..m-2; alpha_{m,m-1} = (2/m) alpha_{m-1,m-2} (the printed line drops
    the '='); alpha_{m,0} = 1 - sum_{k>=1} alpha_{m,k}.
    """
    a = {2: [Fraction(0), Fraction(1)]}
    for mm in range(3, m + 1):
        prev = a[mm - 1]
        cur = [Fraction(0)] * mm
        for k in range(1, mm - 1):
            cur[k] = Fraction(2, k) * prev[k - 1]
        cur[mm - 1] = Fraction(2, mm) * prev[mm - 2]
        cur[0] = 1 - sum(cur[1:])
        a[mm] = cur
    return a[m]


def scalar_lssp_run(order, u0, h, dt, nsteps, m, flux=ADVECTION, a=1.0, split=SPLIT_LF, bc=PERIODIC):
    u = np.array(u0, dtype=np.float64, copy=True)
    coef = np.array([float(c) for c in lssp_coefficients(m)])
    _check(lib().orc_scalar_lssp_run(table(order), flux, a, split, bc, u.size, 1.0 / h, dt, nsteps, m,
                                     _p(coef), _p(u)), "scalar_lssp_run")
    return u


def scalar_ssprk3_run(order, u0, h, dt, t_end=0.0, nsteps=0, flux=ADVECTION, a=1.0, split=SPLIT_LF,
                      bc=PERIODIC):
    u = np.array(u0, dtype=np.float64, copy=True)
    _check(lib().orc_scalar_ssprk3_run(table(order), flux, a, split, bc, u.size, 1.0 / h, dt, t_end,
                                       nsteps, _p(u)), "scalar_ssprk3_run")
    return u


def ssprk3_combine(stage, un, us, L, dt):
    out = np.empty_like(us)
    lib().orc_ssprk3_combine(stage, us.size, _p(un), _p(us), _p(L), dt, _p(out))
    return out


# --------------------------------------------------------------------------
# Euler
# --------------------------------------------------------------------------

def roe_eigen(UL, UR, gamma=1.4):
    nv = len(UL)
    UL = np.ascontiguousarray(UL, dtype=np.float64)
    UR = np.ascontiguousarray(UR, dtype=np.float64)
    Lm = np.empty(nv * nv)
    Rm = np.empty(nv * nv)
    _check(lib().orc_roe_eigen(nv, gamma, _p(UL), _p(UR), _p(Lm), _p(Rm)), "roe_eigen")
    return Lm.reshape(nv, nv), Rm.reshape(nv, nv)


def euler1d_rhs(order, U, h, gamma=1.4, bc=OUTFLOW, with_idx=False):
    U = np.ascontiguousarray(U, dtype=np.float64)
    n = U.shape[1]
    out = np.empty_like(U)
    idx = np.empty((n + 1) * 6, dtype=np.uint8) if with_idx else None
    alpha = ctypes.c_double()
    _check(lib().orc_euler1d_rhs(table(order), gamma, bc, n, 1.0 / h, _p(U), _p(out), _u8(idx),
                                 ctypes.byref(alpha)), "euler1d_rhs")
    if with_idx:
        return out, idx.reshape(n + 1, 3, 2), alpha.value
    return out


def euler1d_rhs_var(order, U, h, gamma=1.4, bc=OUTFLOW, componentwise=False, per_field=False):
    """1D Euler L(U) with the operator variants (component-wise reconstruction
    or per-field alphas, see enomr_oracle.c).  Returns (L, idx [n+1][3][2],
    alphas: one value, or three per-field values)."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    n = U.shape[1]
    out = np.empty_like(U)
    idx = np.empty((n + 1) * 6, dtype=np.uint8)
    alpha = np.zeros(3)
    _check(lib().orc_euler1d_rhs_var(table(order), gamma, bc, n, 1.0 / h, _p(U), _p(out), _u8(idx), _p(alpha),
                                     int(componentwise), int(per_field)), "euler1d_rhs_var")
    return out, idx.reshape(n + 1, 3, 2), (alpha if per_field else alpha[:1])


def euler1d_rhs_frozen(order, U, h, idx, alpha, dU=None, gamma=1.4, bc=OUTFLOW):
    """Frozen-stencil operator L(U; idx, alpha) and, if dU is given, its
    tangent dL/dU . dU (dual numbers).  Returns L or (L, dL)."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    n = U.shape[1]
    idx = np.ascontiguousarray(idx, dtype=np.uint8).reshape(-1)
    out = np.empty_like(U)
    dout = np.empty_like(U) if dU is not None else None
    dUc = None if dU is None else np.ascontiguousarray(dU, dtype=np.float64)
    _check(lib().orc_euler1d_rhs_frozen(table(order), gamma, bc, n, 1.0 / h, _p(U), _p(dUc), _u8(idx), alpha,
                                        _p(out), _p(dout)), "euler1d_rhs_frozen")
    return out if dU is None else (out, dout)


def euler1d_rhs_frozen_jacobian(order, U, h, idx, alpha, gamma=1.4, bc=OUTFLOW):
    """Dense Jacobian of the frozen operator, [3n][3n], column by column from tangents."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    n = U.shape[1]
    J = np.empty((3 * n, 3 * n))
    e = np.zeros_like(U)
    for col in range(3 * n):
        e.reshape(-1)[col] = 1.0
        _, dL = euler1d_rhs_frozen(order, U, h, idx, alpha, e, gamma, bc)
        J[:, col] = dL.reshape(-1)
        e.reshape(-1)[col] = 0.0
    return J


def euler2d_rhs(order, U, hx, hy, gamma=1.4, bcx=PERIODIC, bcy=OUTFLOW, with_idx=False):
    U = np.ascontiguousarray(U, dtype=np.float64)
    _, ny, nx = U.shape
    out = np.empty_like(U)
    ix = np.empty(ny * (nx + 1) * 8, dtype=np.uint8) if with_idx else None
    iy = np.empty((ny + 1) * nx * 8, dtype=np.uint8) if with_idx else None
    ax = np.empty(ny)
    ay = np.empty(nx)
    _check(lib().orc_euler2d_rhs(table(order), gamma, bcx, bcy, nx, ny, 1.0 / hx, 1.0 / hy, _p(U), _p(out),
                                 _u8(ix), _u8(iy), _p(ax), _p(ay)), "euler2d_rhs")
    if with_idx:
        return out, ix.reshape(ny, nx + 1, 4, 2), iy.reshape(ny + 1, nx, 4, 2), ax, ay
    return out


def euler2d_rhs_var(order, U, hx, hy, gamma=1.4, bcx=PERIODIC, bcy=OUTFLOW, componentwise=False,
                    per_field=False, gravity=0.0):
    """2D Euler L(U) with the operator variants (component-wise reconstruction,
    per-field alphas, gravity source g [0, 0, rho, rho v]).  Returns
    (L, ix, iy, ax, ay); with per_field ax is [3][ny] and ay [3][nx]."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    _, ny, nx = U.shape
    out = np.empty_like(U)
    ix = np.empty(ny * (nx + 1) * 8, dtype=np.uint8)
    iy = np.empty((ny + 1) * nx * 8, dtype=np.uint8)
    na = 3 if per_field else 1
    ax = np.empty((na, ny))
    ay = np.empty((na, nx))
    _check(lib().orc_euler2d_rhs_var(table(order), gamma, bcx, bcy, nx, ny, 1.0 / hx, 1.0 / hy, _p(U), _p(out),
                                     _u8(ix), _u8(iy), _p(ax), _p(ay), int(componentwise), int(per_field),
                                     float(gravity)), "euler2d_rhs_var")
    return out, ix.reshape(ny, nx + 1, 4, 2), iy.reshape(ny + 1, nx, 4, 2), ax, ay


def euler2d_rhs_ops(order, U, hx, hy, gamma=1.4, bcx=PERIODIC, bcy=OUTFLOW):
    """(L(U), ix, iy, ops): the operator with its stencil logs and the
    algorithmic operation count of evaluating it (see the counter in
    enomr_oracle.c)."""
    lib().orc_ops_begin()
    try:
        out, ix, iy, _, _ = euler2d_rhs(order, U, hx, hy, gamma, bcx, bcy, with_idx=True)
    finally:
        ops = lib().orc_ops_end()
    return out, ix, iy, ops


def euler2d_rhs_cells(order, U, hx, hy, cells, gamma=1.4, bcx=PERIODIC, bcy=OUTFLOW):
    """L(U) at the listed (x, y) cells only; returns [ncell][4]."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    _, ny, nx = U.shape
    cells = np.ascontiguousarray(np.asarray(cells, dtype=np.int64).reshape(-1, 2))
    out = np.empty((cells.shape[0], 4))
    _check(lib().orc_euler2d_rhs_cells(table(order), gamma, bcx, bcy, nx, ny, 1.0 / hx, 1.0 / hy, _p(U),
                                       cells.shape[0], cells.ctypes.data_as(_lp), _p(out)),
           "euler2d_rhs_cells")
    return out


def euler_maxspeed_1d(U, gamma=1.4):
    U = np.ascontiguousarray(U, dtype=np.float64)
    s = ctypes.c_double()
    _check(lib().orc_euler_maxspeed(U.shape[0], gamma, U.shape[1], _p(U), ctypes.byref(s)), "maxspeed")
    return s.value


def euler_maxspeeds_2d(U, gamma=1.4):
    U = np.ascontiguousarray(U, dtype=np.float64)
    sx, sy = ctypes.c_double(), ctypes.c_double()
    _check(lib().orc_euler2d_maxspeeds(gamma, U.shape[2], U.shape[1], _p(U), ctypes.byref(sx),
                                       ctypes.byref(sy)), "maxspeeds")
    return sx.value, sy.value


def dt_1d(U, h, cfl, gamma=1.4):
    """dt = CFL / (max(|u|+c) / h), evaluated as cfl / (smax * (1/h))."""
    return cfl / (euler_maxspeed_1d(U, gamma) * (1.0 / h))


def dt_2d(U, hx, hy, cfl, gamma=1.4):
    """dt = CFL / (max(|u|+c)/hx + max(|v|+c)/hy), with 1/h precomputed."""
    sx, sy = euler_maxspeeds_2d(U, gamma)
    return cfl / (sx * (1.0 / hx) + sy * (1.0 / hy))


def euler1d_run(order, U0, h, nsteps, cfl=0.5, gamma=1.4, bc=OUTFLOW, dts=None):
    """SSP-RK3 run; dt from the CFL rule at the start of each step.  Returns (U, dts)."""
    U = np.array(U0, dtype=np.float64, copy=True)
    used = []
    for step in range(nsteps):
        dt = dts[step] if dts is not None else dt_1d(U, h, cfl, gamma)
        used.append(dt)
        un = U.copy()
        us = U.copy()
        for s in (1, 2, 3):
            L = euler1d_rhs(order, us, h, gamma, bc)
            us = ssprk3_combine(s, un, us, L, dt)
        U = us
    return U, used


def euler2d_run(order, U0, hx, hy, nsteps, cfl=0.5, gamma=1.4, bcx=PERIODIC, bcy=OUTFLOW, componentwise=False,
                per_field=False, gravity=0.0):
    U = np.array(U0, dtype=np.float64, copy=True)
    used = []
    plain = not (componentwise or per_field or gravity)
    for step in range(nsteps):
        dt = dt_2d(U, hx, hy, cfl, gamma)
        used.append(dt)
        un = U.copy()
        us = U.copy()
        for s in (1, 2, 3):
            if plain:
                L = euler2d_rhs(order, us, hx, hy, gamma, bcx, bcy)
            else:
                L = euler2d_rhs_var(order, us, hx, hy, gamma, bcx, bcy, componentwise, per_field, gravity)[0]
            us = ssprk3_combine(s, un, us, L, dt)
        U = us
    return U, used
