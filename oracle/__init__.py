"""CPU oracle for ENO-MR (H. Shen, arXiv 2311.15504) -- TEST INFRASTRUCTURE.

A plain, slow implementation of what the GPU library computes, used only by
the test suite, the smoke check and the CPU-baseline leg of the benchmark.  It
shares no code with the GPU library (paper_2311_15504_amd) and never imports
it.  The loops are plain C (enomr_oracle.c, built with gcc -ffp-contract=off
and OpenMP over independent lines); the stencil coefficients are derived here
in exact rational arithmetic (coeffs.py) and handed to the C code as exact
fractions.  The same C file built with -DORC_QUAD runs the scalar path in
IEEE binary128 (liboracle_q.so).

Entry points (all numpy float64, C-contiguous):
  recon_faces(order, sign, f_with_halo)             Sec. 3.2 at n faces
  scalar_rhs(order, u, h, ...)                      Eq. (1DWENOFD) for a scalar law
  euler1d_rhs / euler2d_rhs (and _var variants)     Euler right-hand sides
  *_follow                                          the same, with a near-tie record
                                                    against another implementation's log
  euler1d_run / euler2d_run / scalar_*_run          SSP-RK3 / linear SSP-RK runs
  lssp_coefficients(m)                              Eq. (lSSPRK_Coe), exact
  quad_advection_errors(...)                        Sec. 4.1 convergence test in binary128
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
LIBQ = os.path.join(HERE, "liboracle_q.so")

PERIODIC, OUTFLOW = 0, 1
ADVECTION, BURGERS = 0, 1
SPLIT_NONE, SPLIT_LF = 0, 1
MAXW = 17

# Near-tie rule: two implementations may choose different stencils only where
# the deciding comparison's margin is below this, relative to its rounding scale.
TIE_TOL = 1e-12

_dp = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_i64p = ctypes.POINTER(ctypes.c_int64)
_ip = ctypes.POINTER(ctypes.c_int)
_vp = ctypes.c_void_p

CFLAGS = ["-O2", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


class OracleError(RuntimeError):
    pass


class _Ties(ctypes.Structure):
    _fields_ = [("follow", _vp), ("tol", ctypes.c_double), ("pos", _i64p), ("mu", _dp),
                ("max", ctypes.c_int64), ("count", ctypes.c_int64)]


class TieReport:
    """Where the oracle's choice differs from the followed log: positions in
    the log (ascending) and the margin mu of each deciding comparison."""

    def __init__(self, pos, mu):
        order = np.argsort(pos, kind="stable")
        self.pos = np.asarray(pos)[order]
        self.mu = np.asarray(mu)[order]

    @property
    def count(self):
        return int(self.pos.size)

    @property
    def max_abs_mu(self):
        return float(np.abs(self.mu).max()) if self.mu.size else 0.0

    def __repr__(self):
        return "TieReport(count=%d, max|mu|=%.3g)" % (self.count, self.max_abs_mu)


def build(force=True):
    """Compile enomr_oracle.c into liboracle.so (FP64) and liboracle_q.so
    (binary128 scalar path) with gcc: no contraction, OpenMP."""
    for out, extra, libs in ((LIB, [], ["-lm"]), (LIBQ, ["-DORC_QUAD"], ["-lquadmath", "-lm"])):
        if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(SRC):
            continue
        subprocess.check_call(["gcc"] + CFLAGS + extra + ["-o", out + ".tmp", SRC] + libs)
        os.replace(out + ".tmp", out)
    return LIB


_lib = None
_libq = None


def _stale(path):
    return not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(SRC)


def lib():
    global _lib
    if _lib is None:
        if _stale(LIB):
            build(force=False)
        L = ctypes.CDLL(LIB)
        L.orc_table_new.restype = _vp
        L.orc_table_new.argtypes = [ctypes.c_int, ctypes.c_int, _ip, _i64p, _i64p, _i64p]
        L.orc_table_free.argtypes = [_vp]
        L.orc_recon_faces.argtypes = [_vp, ctypes.c_int, ctypes.c_long, _dp, _dp, _u8p, _vp]
        L.orc_scalar_rhs.argtypes = [_vp, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_long,
                                     ctypes.c_double, _dp, _dp, _u8p, _dp, _vp]
        L.orc_roe_eigen.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp, _dp, _dp]
        L.orc_ops_begin.restype = None
        L.orc_ops_begin.argtypes = []
        L.orc_ops_end.restype = ctypes.c_double
        L.orc_ops_end.argtypes = [_dp]
        L.orc_set_threads.restype = None
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_max_threads.restype = ctypes.c_int
        L.orc_max_threads.argtypes = []
        L.orc_euler1d_rhs.argtypes = [_vp, ctypes.c_double, ctypes.c_int, ctypes.c_long, ctypes.c_double, _dp, _dp,
                                      _u8p, _dp, _vp]
        L.orc_euler1d_rhs_var.argtypes = [_vp, ctypes.c_double, ctypes.c_int, ctypes.c_long, ctypes.c_double, _dp,
                                          _dp, _u8p, _dp, ctypes.c_int, ctypes.c_int, _vp]
        L.orc_euler2d_rhs.argtypes = [_vp, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_long, ctypes.c_long,
                                      ctypes.c_double, ctypes.c_double, _dp, _dp, _u8p, _u8p, _dp, _dp, _vp]
        L.orc_euler2d_rhs_var.argtypes = [_vp, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_long,
                                          ctypes.c_long, ctypes.c_double, ctypes.c_double, _dp, _dp, _u8p, _u8p, _dp,
                                          _dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, _vp]
        L.orc_euler1d_rhs_frozen.argtypes = [_vp, ctypes.c_double, ctypes.c_int, ctypes.c_long, ctypes.c_double, _dp,
                                             _dp, _u8p, ctypes.c_double, _dp, _dp]
        L.orc_euler_maxspeed.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_long, _dp, _dp]
        L.orc_euler2d_maxspeeds.argtypes = [ctypes.c_double, ctypes.c_long, ctypes.c_long, _dp, _dp, _dp]
        L.orc_ssprk3_combine.restype = None
        L.orc_ssprk3_combine.argtypes = [ctypes.c_int, ctypes.c_long, _dp, _dp, _dp, ctypes.c_double, _dp]
        L.orc_scalar_lssp_run.argtypes = [_vp, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_long, ctypes.c_double, ctypes.c_double, ctypes.c_long,
                                          ctypes.c_int, _i64p, _i64p, _dp]
        L.orc_scalar_ssprk3_run.argtypes = [_vp, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_long, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_long, _dp]
        _lib = L
    return _lib


def libq():
    global _libq
    if _libq is None:
        if _stale(LIBQ):
            build(force=False)
        L = ctypes.CDLL(LIBQ)
        L.orc_table_new_q.restype = _vp
        L.orc_table_new_q.argtypes = [ctypes.c_int, ctypes.c_int, _ip, _i64p, _i64p, _i64p]
        L.orc_q_advection_errors.argtypes = [_vp, ctypes.c_int, ctypes.c_double, ctypes.c_long, ctypes.c_int,
                                             _i64p, _i64p, _dp, _dp]
        _libq = L
    return _libq


def set_threads(n):
    """OpenMP threads of the oracle's parallel loops (results do not depend on it)."""
    lib().orc_set_threads(int(n))


def max_threads():
    return int(lib().orc_max_threads())


def _p(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _u8(a):
    return None if a is None else a.ctypes.data_as(_u8p)


def _i64(a):
    return a.ctypes.data_as(_i64p)


def _check(st, what):
    if st != 0:
        raise OracleError("%s failed with status %d" % (what, st))


_tables = {}
_tables_q = {}


def _table_arrays(order):
    rows = coeffs.exact_table(order)
    nc = len(rows)
    mn = (ctypes.c_int * (2 * nc))(*[v for (m, n, _, _) in rows for v in (m, n)])
    anum = np.zeros((nc, MAXW), dtype=np.int64)
    aden = np.zeros((nc, MAXW), dtype=np.int64)
    bint = np.zeros((nc, MAXW), dtype=np.int64)
    for c, (m, n, al, bl) in enumerate(rows):
        for l, (a, b) in enumerate(zip(al, bl)):
            assert b.denominator == 1 and abs(a.numerator) < 2 ** 53 and a.denominator < 2 ** 53
            anum[c, l], aden[c, l], bint[c, l] = a.numerator, a.denominator, b.numerator
    return nc, mn, anum, aden, bint


def table(order):
    """C-side candidate table for `order` (a_l, b_l from exact fractions)."""
    if order not in _tables:
        nc, mn, anum, aden, bint = _table_arrays(order)
        ptr = lib().orc_table_new(order, nc, mn, _i64(anum), _i64(aden), _i64(bint))
        if not ptr:
            raise OracleError("bad table for order %d" % order)
        _tables[order] = ptr
    return _tables[order]


def table_q(order):
    if order not in _tables_q:
        nc, mn, anum, aden, bint = _table_arrays(order)
        ptr = libq().orc_table_new_q(order, nc, mn, _i64(anum), _i64(aden), _i64(bint))
        if not ptr:
            raise OracleError("bad table for order %d" % order)
        _tables_q[order] = ptr
    return _tables_q[order]


def ncand(order):
    return len(coeffs.candidates(order))


class _Follow:
    """A near-tie record for one call: follow `log` (uint8 array in the call's
    own log layout), taking its choice where |mu| < tol."""

    def __init__(self, log, tol, cap):
        self.log = np.ascontiguousarray(np.asarray(log, dtype=np.uint8).reshape(-1))
        self.cap = int(cap)
        self.pos = np.zeros(max(self.cap, 1), dtype=np.int64)
        self.mu = np.zeros(max(self.cap, 1))
        self.s = _Ties(self.log.ctypes.data, float(tol), _i64(self.pos), _p(self.mu), self.cap, 0)

    def ptr(self):
        return ctypes.byref(self.s)

    def report(self):
        n = int(self.s.count)
        if n > self.cap:
            return None
        return TieReport(self.pos[:n].copy(), self.mu[:n].copy())


def _with_follow(call, log, tol, cap=1 << 16):
    """Run call(ties_ptr) with a near-tie record against `log`; rerun with a
    larger record if the first one overflowed.  Returns (call's result, report)."""
    while True:
        f = _Follow(log, tol, cap)
        res = call(f.ptr())
        rep = f.report()
        if rep is not None:
            return res, rep
        cap = int(f.s.count) + 1


# --------------------------------------------------------------------------
# Scalar reconstruction and scalar laws
# --------------------------------------------------------------------------

def recon_faces(order, sign, f_with_halo, follow=None, tol=TIE_TOL):
    """f-hat at n = len - (2r-1) faces; face i between array cells i+r-1, i+r.
    With follow (another implementation's log of the n faces) also returns
    the near-tie report, and the values take its choices at ties."""
    f = np.ascontiguousarray(f_with_halo, dtype=np.float64)
    r = (order + 1) // 2
    n = f.size - (2 * r - 1)
    fhat = np.empty(max(n, 0))
    idx = np.empty(max(n, 0), dtype=np.uint8)

    def call(ties):
        _check(lib().orc_recon_faces(table(order), sign, n, _p(f), _p(fhat), _u8(idx), ties), "recon_faces")

    if follow is None:
        call(None)
        return fhat, idx
    _, rep = _with_follow(call, follow, tol)
    return fhat, idx, rep


def scalar_rhs(order, u, h, flux=ADVECTION, a=1.0, split=SPLIT_LF, bc=PERIODIC, with_idx=False, follow=None,
               tol=TIE_TOL):
    """L(u) for a scalar law on one line; idx [n+1][2] if requested.  With
    follow (a log [n+1][2]) returns (L, idx, alpha, report)."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    n = u.size
    out = np.empty(n)
    idx = np.empty((n + 1) * 2, dtype=np.uint8) if (with_idx or follow is not None) else None
    alpha = ctypes.c_double()

    def call(ties):
        _check(lib().orc_scalar_rhs(table(order), flux, a, split, bc, n, 1.0 / h, _p(u), _p(out), _u8(idx),
                                    ctypes.byref(alpha), ties), "scalar_rhs")

    if follow is not None:
        _, rep = _with_follow(call, follow, tol)
        return out, idx.reshape(n + 1, 2), alpha.value, rep
    call(None)
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


def _lssp_fracs(m):
    c = lssp_coefficients(m)
    num = np.array([x.numerator for x in c], dtype=np.int64)
    den = np.array([x.denominator for x in c], dtype=np.int64)
    assert all(abs(x.numerator) < 2 ** 53 and x.denominator < 2 ** 53 for x in c)
    return num, den


def scalar_lssp_run(order, u0, h, dt, nsteps, m, flux=ADVECTION, a=1.0, split=SPLIT_LF, bc=PERIODIC):
    u = np.array(u0, dtype=np.float64, copy=True)
    num, den = _lssp_fracs(m)
    _check(lib().orc_scalar_lssp_run(table(order), flux, a, split, bc, u.size, 1.0 / h, dt, nsteps, m, _i64(num),
                                     _i64(den), _p(u)), "scalar_lssp_run")
    return u


def quad_advection_errors(order, alpha, lam, n):
    """The Sec. 4.1 test in binary128: lam sin^alpha(pi x) on [-1, 1] with n
    nodes, linear SSP-RK(order+1, order), dt = h, t = 2.  Returns (L1, Linf)
    rounded to double (L1 over the n+1 points, the end point counted twice)."""
    num, den = _lssp_fracs(order + 1)
    l1, linf = ctypes.c_double(), ctypes.c_double()
    _check(libq().orc_q_advection_errors(table_q(order), int(alpha), float(lam), int(n), order + 1, _i64(num),
                                         _i64(den), ctypes.byref(l1), ctypes.byref(linf)), "quad_advection_errors")
    return l1.value, linf.value


def scalar_ssprk3_run(order, u0, h, dt, t_end=0.0, nsteps=0, flux=ADVECTION, a=1.0, split=SPLIT_LF,
                      bc=PERIODIC):
    u = np.array(u0, dtype=np.float64, copy=True)
    _check(lib().orc_scalar_ssprk3_run(table(order), flux, a, split, bc, u.size, 1.0 / h, dt, t_end,
                                       nsteps, _p(u)), "scalar_ssprk3_run")
    return u


def ssprk3_combine(stage, un, us, L, dt):
    un = np.ascontiguousarray(un, dtype=np.float64)
    us = np.ascontiguousarray(us, dtype=np.float64)
    L = np.ascontiguousarray(L, dtype=np.float64)
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


def _euler1d(order, U, h, gamma, bc, componentwise, per_field, ties):
    U = np.ascontiguousarray(U, dtype=np.float64)
    n = U.shape[1]
    out = np.empty_like(U)
    idx = np.empty((n + 1) * 6, dtype=np.uint8)
    alpha = np.zeros(3)
    _check(lib().orc_euler1d_rhs_var(table(order), gamma, bc, n, 1.0 / h, _p(U), _p(out), _u8(idx), _p(alpha),
                                     int(componentwise), int(per_field), ties), "euler1d_rhs")
    return out, idx.reshape(n + 1, 3, 2), (alpha if per_field else alpha[:1])


def euler1d_rhs(order, U, h, gamma=1.4, bc=OUTFLOW, with_idx=False):
    out, idx, alpha = _euler1d(order, U, h, gamma, bc, False, False, None)
    if with_idx:
        return out, idx, float(alpha[0])
    return out


def euler1d_rhs_var(order, U, h, gamma=1.4, bc=OUTFLOW, componentwise=False, per_field=False):
    """1D Euler L(U) with the operator variants (component-wise reconstruction
    or per-field alphas, see enomr_oracle.c).  Returns (L, idx [n+1][3][2],
    alphas: one value, or three per-field values)."""
    return _euler1d(order, U, h, gamma, bc, componentwise, per_field, None)


def euler1d_rhs_follow(order, U, h, follow, gamma=1.4, bc=OUTFLOW, componentwise=False, per_field=False,
                       tol=TIE_TOL):
    """(L, idx, alphas, report): the operator with a near-tie record against
    another implementation's log `follow` ([n+1][3][2]); L takes the other
    choice where |mu| < tol."""
    res, rep = _with_follow(lambda t: _euler1d(order, U, h, gamma, bc, componentwise, per_field, t), follow, tol)
    return res + (rep,)


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


def _euler2d(order, U, hx, hy, gamma, bcx, bcy, componentwise, per_field, gravity, ties, with_idx=True):
    U = np.ascontiguousarray(U, dtype=np.float64)
    _, ny, nx = U.shape
    out = np.empty_like(U)
    ix = np.empty(ny * (nx + 1) * 8, dtype=np.uint8) if with_idx else None
    iy = np.empty((ny + 1) * nx * 8, dtype=np.uint8) if with_idx else None
    na = 3 if per_field else 1
    ax = np.empty((na, ny))
    ay = np.empty((na, nx))
    _check(lib().orc_euler2d_rhs_var(table(order), gamma, bcx, bcy, nx, ny, 1.0 / hx, 1.0 / hy, _p(U), _p(out),
                                     _u8(ix), _u8(iy), _p(ax), _p(ay), int(componentwise), int(per_field),
                                     float(gravity), ties), "euler2d_rhs")
    if not with_idx:
        return out, None, None, ax, ay
    return out, ix.reshape(ny, nx + 1, 4, 2), iy.reshape(ny + 1, nx, 4, 2), ax, ay


def euler2d_rhs(order, U, hx, hy, gamma=1.4, bcx=PERIODIC, bcy=OUTFLOW, with_idx=False):
    out, ix, iy, ax, ay = _euler2d(order, U, hx, hy, gamma, bcx, bcy, False, False, 0.0, None, with_idx)
    if with_idx:
        return out, ix, iy, ax[0], ay[0]
    return out


def euler2d_rhs_var(order, U, hx, hy, gamma=1.4, bcx=PERIODIC, bcy=OUTFLOW, componentwise=False,
                    per_field=False, gravity=0.0):
    """2D Euler L(U) with the operator variants (component-wise reconstruction,
    per-field alphas, gravity source g [0, 0, rho, rho v]).  Returns
    (L, ix, iy, ax, ay); with per_field ax is [3][ny] and ay [3][nx]."""
    return _euler2d(order, U, hx, hy, gamma, bcx, bcy, componentwise, per_field, gravity, None)


def euler2d_rhs_follow(order, U, hx, hy, follow, gamma=1.4, bcx=PERIODIC, bcy=OUTFLOW, componentwise=False,
                       per_field=False, gravity=0.0, tol=TIE_TOL):
    """(L, ix, iy, ax, ay, report): the operator with a near-tie record against
    another implementation's log `follow` (x faces [ny][nx+1][4][2], then y
    faces [ny+1][nx][4][2], flat); L takes the other choice where |mu| < tol."""
    res, rep = _with_follow(lambda t: _euler2d(order, U, hx, hy, gamma, bcx, bcy, componentwise, per_field,
                                               gravity, t), follow, tol)
    return res + (rep,)


def euler2d_rhs_ops(order, U, hx, hy, gamma=1.4, bcx=PERIODIC, bcy=OUTFLOW):
    """(L(U), ix, iy, ops): the operator with its stencil logs and the
    algorithmic operation count of evaluating it, per category (x lines,
    y lines, the sum L_x + L_y, RK combination; see the counter in
    enomr_oracle.c)."""
    cats = np.zeros(4)
    lib().orc_ops_begin()
    try:
        out, ix, iy, _, _ = euler2d_rhs(order, U, hx, hy, gamma, bcx, bcy, with_idx=True)
    finally:
        lib().orc_ops_end(_p(cats))
    return out, ix, iy, cats


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
    """dt = CFL h / max(|u|+c) (the CFL rule, 1D)."""
    return cfl * h / euler_maxspeed_1d(U, gamma)


def dt_2d(U, hx, hy, cfl, gamma=1.4):
    """dt = CFL / (max(|u|+c)/hx + max(|v|+c)/hy)."""
    sx, sy = euler_maxspeeds_2d(U, gamma)
    return cfl / (sx / hx + sy / hy)


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
                per_field=False, gravity=0.0, dts=None):
    U = np.array(U0, dtype=np.float64, copy=True)
    used = []
    for step in range(nsteps):
        dt = dts[step] if dts is not None else dt_2d(U, hx, hy, cfl, gamma)
        used.append(dt)
        un = U.copy()
        us = U.copy()
        for s in (1, 2, 3):
            L = _euler2d(order, us, hx, hy, gamma, bcx, bcy, componentwise, per_field, gravity, None, False)[0]
            us = ssprk3_combine(s, un, us, L, dt)
        U = us
    return U, used
