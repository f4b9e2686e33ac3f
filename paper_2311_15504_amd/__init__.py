"""Python binding of libenomr (the MI355X ENO-MR library, include/enomr.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of libenomr.so.  PyTorch provides device memory and the stream; arrays are
torch float64 CUDA tensors laid out [variable][y][x].  If the library is
missing or cannot be loaded this module raises at first use: there is no CPU
fallback.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libenomr.so")

ADVECTION, BURGERS, EULER = 0, 1, 2
PERIODIC, OUTFLOW = 0, 1
SPLIT_NONE, SPLIT_LF = 0, 1
CHARACTERISTIC, COMPONENTWISE = 0, 1
ALPHA_LINE, ALPHA_FIELD = 0, 1

STATUS = {0: "ENOMR_OK", 1: "ENOMR_EINVAL", 2: "ENOMR_EORDER", 3: "ENOMR_ENOMEM", 4: "ENOMR_EHIP",
          5: "ENOMR_ENONPHYS", 6: "ENOMR_ENODEV"}


class EnomrError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (STATUS.get(status, status), message))
        self.status = status


class Problem(ctypes.Structure):
    """Mirror of enomr_problem."""
    _fields_ = [("ndim", ctypes.c_int32), ("system", ctypes.c_int32), ("nx", ctypes.c_int64),
                ("ny", ctypes.c_int64), ("hx", ctypes.c_double), ("hy", ctypes.c_double),
                ("order", ctypes.c_int32), ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32),
                ("split", ctypes.c_int32), ("gamma", ctypes.c_double), ("adv_speed", ctypes.c_double),
                ("recon", ctypes.c_int32), ("alpha_mode", ctypes.c_int32), ("gravity", ctypes.c_double)]

    @classmethod
    def scalar(cls, system, n, h, order, bc=PERIODIC, split=SPLIT_LF, adv_speed=1.0):
        return cls(1, system, n, 1, h, 0.0, order, bc, PERIODIC, split, 0.0, adv_speed)

    @classmethod
    def euler1d(cls, n, h, order, bc=OUTFLOW, gamma=1.4, componentwise=False, per_field=False):
        return cls(1, EULER, n, 1, h, 0.0, order, bc, PERIODIC, SPLIT_LF, gamma, 0.0,
                   COMPONENTWISE if componentwise else CHARACTERISTIC,
                   ALPHA_FIELD if per_field else ALPHA_LINE, 0.0)

    @classmethod
    def euler2d(cls, nx, ny, hx, hy, order, bc_x=PERIODIC, bc_y=OUTFLOW, gamma=1.4, componentwise=False,
                per_field=False, gravity=0.0):
        return cls(2, EULER, nx, ny, hx, hy, order, bc_x, bc_y, SPLIT_LF, gamma, 0.0,
                   COMPONENTWISE if componentwise else CHARACTERISTIC,
                   ALPHA_FIELD if per_field else ALPHA_LINE, float(gravity))

    @property
    def nvar(self):
        if self.system != EULER:
            return 1
        return 4 if self.ndim == 2 else 3

    @property
    def state_shape(self):
        if self.ndim == 2:
            return (self.nvar, self.ny, self.nx)
        return (self.nvar, self.nx)

    def idx_bytes(self):
        """Bytes of one stencil-index log (see enomr_rhs)."""
        if self.system != EULER:
            return (self.nx + 1) * 2
        if self.ndim == 1:
            return (self.nx + 1) * 6
        return self.ny * (self.nx + 1) * 8 + (self.ny + 1) * self.nx * 8


_lib = None
_vp = ctypes.c_void_p


def lib():
    """Load libenomr.so (built in-tree by build.py); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libenomr.so not built: run paper_2311_15504_amd/build.py "
                              "(or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        st = ctypes.c_int
        P = ctypes.POINTER(Problem)
        sig = {
            "enomr_create": ([ctypes.c_int, _vp, ctypes.POINTER(_vp)], st),
            "enomr_destroy": ([_vp], st),
            "enomr_set_stream": ([_vp, _vp], st),
            "enomr_last_error": ([], ctypes.c_char_p),
            "enomr_coefficients": ([ctypes.c_int, _vp, _vp, _vp, _vp], st),
            "enomr_recon_faces": ([_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int64, _vp, _vp, _vp], st),
            "enomr_workspace_size": ([P, ctypes.POINTER(ctypes.c_size_t)], st),
            "enomr_rhs": ([_vp, P, _vp, _vp, _vp, _vp], st),
            "enomr_rhs_noalloc": ([_vp, P, _vp, _vp, _vp], st),
            "enomr_dt": ([_vp, P, _vp, ctypes.c_double, _vp, _vp], st),
            "enomr_ssprk3_step": ([_vp, P, _vp, _vp, _vp, _vp], st),
            "enomr_advance": ([_vp, P, _vp, ctypes.c_double, ctypes.c_int64, ctypes.c_double, _vp, _vp], st),
            "enomr_check": ([_vp], st),
            "enomr_profile_start": ([_vp], st),
            "enomr_profile_stop": ([_vp, _vp, _vp], st),
            "enomr_lssp_workspace_size": ([P, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)], st),
            "enomr_lssp_advance": ([_vp, P, _vp, ctypes.c_double, ctypes.c_int64, ctypes.c_int, _vp], st),
            "enomr_rhs_adjoint": ([_vp, P, _vp, _vp, _vp, _vp, _vp, _vp], st),
            "enomr_record_steps": ([_vp, P, _vp, ctypes.c_double, ctypes.c_int64, _vp, _vp, _vp, _vp, _vp], st),
            "enomr_adjoint_steps": ([_vp, P, ctypes.c_int64, _vp, _vp, _vp, _vp, _vp, _vp], st),
            "enomr_batch_create": ([_vp, ctypes.c_int32, P, _vp, ctypes.c_int, ctypes.POINTER(_vp)], st),
            "enomr_batch_advance": ([_vp, ctypes.c_double, ctypes.c_int64], st),
            "enomr_batch_info": ([_vp, _vp, _vp, _vp], st),
            "enomr_batch_info2d": ([_vp, _vp, _vp, _vp], st),
            "enomr_batch_set_tile2d": ([_vp, ctypes.c_int32, ctypes.c_int32], st),
            "enomr_batch_destroy": ([_vp], st),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _call(name, *args):
    st = getattr(lib(), name)(*args)
    if st != 0:
        raise EnomrError(st, (lib().enomr_last_error() or b"").decode())
    return st


def coefficients(order):
    """(mn, a, b) as the library uses them; host only, no GPU needed."""
    import numpy as np
    nc = ctypes.c_int32()
    _call("enomr_coefficients", order, ctypes.cast(ctypes.byref(nc), _vp), None, None, None)
    mn = np.zeros(2 * nc.value, dtype=np.int32)
    a = np.zeros(nc.value * 17)
    b = np.zeros(nc.value * 17)
    _call("enomr_coefficients", order, ctypes.cast(ctypes.byref(nc), _vp), mn.ctypes.data, a.ctypes.data,
          b.ctypes.data)
    return mn.reshape(-1, 2), a.reshape(-1, 17), b.reshape(-1, 17)


def workspace_size(prob):
    n = ctypes.c_size_t()
    _call("enomr_workspace_size", ctypes.byref(prob), ctypes.byref(n))
    return n.value


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Context:
    """An enomr_ctx bound to a CUDA (HIP) device; calls follow torch's current stream."""

    def __init__(self, device=0):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        h = _vp()
        with torch.cuda.device(self.device):
            _call("enomr_create", device, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), ctypes.byref(h))
        self.handle = h
        self._ws = {}

    def close(self):
        if self.handle:
            lib().enomr_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_stream(self):
        s = self.torch.cuda.current_stream(self.device).cuda_stream
        _call("enomr_set_stream", self.handle, ctypes.c_void_p(s))

    def workspace(self, prob):
        key = bytes(prob)
        if key not in self._ws:
            self._ws[key] = self.torch.empty(workspace_size(prob), dtype=self.torch.uint8, device=self.device)
        return self._ws[key]

    def _check_state(self, prob, U):
        t = self.torch
        if U.dtype != t.float64 or not U.is_cuda or not U.is_contiguous() or tuple(U.shape) != prob.state_shape:
            raise ValueError("state must be a contiguous float64 CUDA tensor of shape %s" % (prob.state_shape,))

    # -- entry points -------------------------------------------------------

    def recon_faces(self, order, sign, f_with_halo, with_idx=True):
        t = self.torch
        r = (order + 1) // 2
        n = f_with_halo.numel() - (2 * r - 1)
        fhat = t.empty(max(n, 0), dtype=t.float64, device=self.device)
        idx = t.empty(max(n, 0), dtype=t.uint8, device=self.device) if with_idx else None
        self._sync_stream()
        _call("enomr_recon_faces", self.handle, order, sign, n, _ptr(f_with_halo), _ptr(fhat), _ptr(idx))
        return fhat, idx

    def rhs(self, prob, U, with_idx=False):
        t = self.torch
        self._check_state(prob, U)
        out = t.empty_like(U)
        idx = t.empty(prob.idx_bytes(), dtype=t.uint8, device=self.device) if with_idx else None
        self._sync_stream()
        _call("enomr_rhs", self.handle, ctypes.byref(prob), _ptr(U), _ptr(out), _ptr(idx), _ptr(self.workspace(prob)))
        return (out, idx) if with_idx else out

    def rhs_noalloc(self, prob, U, with_idx=False):
        """L(U) through enomr_rhs_noalloc (no workspace, no device allocation
        inside the library); the output tensor is allocated here."""
        t = self.torch
        self._check_state(prob, U)
        out = t.empty_like(U)
        idx = t.empty(prob.idx_bytes(), dtype=t.uint8, device=self.device) if with_idx else None
        self._sync_stream()
        _call("enomr_rhs_noalloc", self.handle, ctypes.byref(prob), _ptr(U), _ptr(out), _ptr(idx))
        return (out, idx) if with_idx else out

    def dt(self, prob, U, cfl):
        t = self.torch
        self._check_state(prob, U)
        d = t.empty(1, dtype=t.float64, device=self.device)
        self._sync_stream()
        _call("enomr_dt", self.handle, ctypes.byref(prob), _ptr(U), cfl, _ptr(d), _ptr(self.workspace(prob)))
        return d

    def ssprk3_step(self, prob, U, dt_dev, idx_log=None):
        self._check_state(prob, U)
        self._sync_stream()
        _call("enomr_ssprk3_step", self.handle, ctypes.byref(prob), _ptr(U), _ptr(dt_dev),
              _ptr(self.workspace(prob)), _ptr(idx_log))

    def advance(self, prob, U, cfl, nsteps, t_end=0.0, dt_log=None):
        self._check_state(prob, U)
        self._sync_stream()
        _call("enomr_advance", self.handle, ctypes.byref(prob), _ptr(U), cfl, nsteps, t_end,
              _ptr(self.workspace(prob)), _ptr(dt_log))

    def check(self):
        self._sync_stream()
        _call("enomr_check", self.handle)

    def lssp_advance(self, prob, U, dt, nsteps, m):
        """nsteps linear SSP-RK(m, m-1) steps of a scalar line with fixed dt, in place."""
        self._check_state(prob, U)
        n = ctypes.c_size_t()
        _call("enomr_lssp_workspace_size", ctypes.byref(prob), m, ctypes.byref(n))
        ws = self.torch.empty(n.value, dtype=self.torch.uint8, device=self.device)
        self._sync_stream()
        _call("enomr_lssp_advance", self.handle, ctypes.byref(prob), _ptr(U), dt, nsteps, m, _ptr(ws))
        self._sync_stream()
        self.torch.cuda.current_stream(self.device).synchronize()   # ws is freed on return

    # -- frozen-stencil adjoint (1D Euler) ------------------------------------

    def rhs_adjoint(self, prob, U, idx, alpha_dev, lam_dUdt):
        """(dL/dU)^T lam_dUdt of the operator with frozen stencils idx and alpha."""
        self._check_state(prob, U)
        out = self.torch.empty_like(U)
        self._sync_stream()
        _call("enomr_rhs_adjoint", self.handle, ctypes.byref(prob), _ptr(U), _ptr(idx), _ptr(alpha_dev),
              _ptr(lam_dUdt), _ptr(out), _ptr(self.workspace(prob)))
        return out

    def _check_log(self, prob, nsteps, stages, idx_log, alpha_log, dt_log):
        t = self.torch
        ns = 3 * prob.nx
        need = ((stages, t.float64, 3 * ns), (idx_log, t.uint8, 3 * prob.idx_bytes()),
                (alpha_log, t.float64, 3), (dt_log, t.float64, 1))
        for arr, dtype, per_step in need:
            if arr.dtype != dtype or not arr.is_cuda or not arr.is_contiguous() or arr.numel() < nsteps * per_step:
                raise ValueError("step log arrays must be contiguous CUDA tensors holding %d steps" % nsteps)

    def record_steps(self, prob, U, cfl, nsteps, stages, idx_log, alpha_log, dt_log):
        """nsteps SSP-RK3 steps of U in place, recording stages, stencil logs, alphas, dts."""
        self._check_state(prob, U)
        self._check_log(prob, nsteps, stages, idx_log, alpha_log, dt_log)
        self._sync_stream()
        _call("enomr_record_steps", self.handle, ctypes.byref(prob), _ptr(U), cfl, nsteps, _ptr(stages),
              _ptr(idx_log), _ptr(alpha_log), _ptr(dt_log), _ptr(self.workspace(prob)))

    def adjoint_steps(self, prob, nsteps, stages, idx_log, alpha_log, dt_log, lam):
        """lam <- adjoint through the recorded steps, last first (in place)."""
        self._check_state(prob, lam)
        self._check_log(prob, nsteps, stages, idx_log, alpha_log, dt_log)
        self._sync_stream()
        _call("enomr_adjoint_steps", self.handle, ctypes.byref(prob), nsteps, _ptr(stages), _ptr(idx_log),
              _ptr(alpha_log), _ptr(dt_log), _ptr(lam), _ptr(self.workspace(prob)))

    def step_record(self, prob, U, cfl, stages, idx_log, alpha_log, dt_dev):
        """One recorded step (record_steps with nsteps = 1)."""
        self.record_steps(prob, U, cfl, 1, stages, idx_log, alpha_log, dt_dev)

    def step_adjoint(self, prob, stages, idx_log, alpha_log, dt_dev, lam):
        """The adjoint of one recorded step (adjoint_steps with nsteps = 1)."""
        self.adjoint_steps(prob, 1, stages, idx_log, alpha_log, dt_dev, lam)

    # -- profiling ----------------------------------------------------------

    def profile_start(self):
        _call("enomr_profile_start", self.handle)

    def profile_stop(self):
        """{class: (milliseconds, launches)} for 'sweep_x', 'sweep_y', 'aux'."""
        ms = (ctypes.c_double * 3)()
        n = (ctypes.c_int64 * 3)()
        self._sync_stream()
        _call("enomr_profile_stop", self.handle, ctypes.cast(ms, _vp), ctypes.cast(n, _vp))
        return {k: (ms[i], n[i]) for i, k in enumerate(("sweep_x", "sweep_y", "aux"))}


class Batch:
    """Many independent 1D and 2D Euler problems advanced by graph-replayed
    launches (enomr_batch_*): one persistent launch for the 1D problems, a
    one-step graph per step for the 2D ones.  `states` are the
    problems' [3][n] or [4][ny][nx] float64 CUDA tensors; they stay bound to
    the batch and are advanced in place."""

    def __init__(self, ctx, problems, states, autotune=True, tile_faces=None):
        """autotune: time one step per 1D tile width (64/128/256) and per 2D
        tile shape (64x4, 32x8, 16x16 faces x lines) on scratch copies and
        keep the fastest of each; tile_faces: use that 1D width instead
        (autotune is then ignored; set_tile2d() picks a 2D shape)."""
        if len(problems) != len(states) or not problems:
            raise ValueError("one state per problem")
        for p, U in zip(problems, states):
            ctx._check_state(p, U)
        self.ctx = ctx
        self.states = list(states)
        n = len(problems)
        arr = (Problem * n)(*problems)
        ptrs = (ctypes.c_void_p * n)(*[U.data_ptr() for U in states])
        h = _vp()
        ctx._sync_stream()
        mode = int(tile_faces) if tile_faces is not None else (1 if autotune else 0)
        _call("enomr_batch_create", ctx.handle, n, arr, ctypes.cast(ptrs, _vp), mode, ctypes.byref(h))
        self.handle = h

    def advance(self, cfl, nsteps):
        self.ctx._sync_stream()
        _call("enomr_batch_advance", self.handle, cfl, nsteps)

    def info(self):
        tf = ctypes.c_int32()
        nb = ctypes.c_int32()
        ms = (ctypes.c_double * 3)()
        _call("enomr_batch_info", self.handle, ctypes.cast(ctypes.byref(tf), _vp), ctypes.cast(ctypes.byref(nb), _vp),
              ctypes.cast(ms, _vp))
        tf2 = ctypes.c_int32()
        tl2 = ctypes.c_int32()
        ms2 = (ctypes.c_double * 3)()
        _call("enomr_batch_info2d", self.handle, ctypes.cast(ctypes.byref(tf2), _vp),
              ctypes.cast(ctypes.byref(tl2), _vp), ctypes.cast(ms2, _vp))
        return {"tile_faces": tf.value, "workgroups": nb.value, "tune_ms": list(ms),
                "tile2d": (tf2.value, tl2.value), "tune2d_ms": list(ms2)}

    def set_tile2d(self, tile_faces, tile_lines):
        """Use the 2D sweeps' tile shape tile_faces x tile_lines (64x4, 32x8 or 16x16)."""
        self.ctx._sync_stream()
        _call("enomr_batch_set_tile2d", self.handle, int(tile_faces), int(tile_lines))

    def close(self):
        if self.handle:
            lib().enomr_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _solve_forward(ctx, prob, U0, cfl, nsteps, every):
    """Advance U0 by nsteps, keeping a copy of the state every `every` steps."""
    U = U0.detach().clone()
    ckpts = []
    done = 0
    while done < nsteps:
        ckpts.append(U.clone())
        k = min(every, nsteps - done)
        ctx.advance(prob, U, cfl, k)
        done += k
    return U, ckpts


def _solve_adjoint(ctx, prob, ckpts, cfl, nsteps, every, lam):
    """Reverse through the checkpointed run: each segment is recomputed from
    its checkpoint with recording, then its steps are transposed in reverse."""
    t = ctx.torch
    dev = ctx.device
    ns = lam.numel()
    ib = prob.idx_bytes()
    stages = t.empty((every, 3, ns), dtype=t.float64, device=dev)
    idx = t.empty((every, 3 * ib), dtype=t.uint8, device=dev)
    alpha = t.empty((every, 3), dtype=t.float64, device=dev)
    dts = t.empty((every, 1), dtype=t.float64, device=dev)
    lam = lam.detach().clone().contiguous()
    for seg in reversed(range(len(ckpts))):
        k = min(every, nsteps - seg * every)
        U = ckpts[seg].clone()
        ctx.record_steps(prob, U, cfl, k, stages, idx, alpha, dts)
        ctx.adjoint_steps(prob, k, stages, idx, alpha, dts, lam)
    return lam


def _autograd_function():
    import torch

    class EnoMRSolve(torch.autograd.Function):
        """U_T = SSP-RK3^nsteps(U_0) of a 1D Euler problem on the GPU.  The
        backward pass is the frozen-stencil discrete adjoint (stencil choices,
        per-stage alphas and step sizes of the forward run held fixed) with the
        run checkpointed every `checkpoint_every` steps."""

        @staticmethod
        def forward(fctx, U0, ctx, prob, cfl, nsteps, checkpoint_every):
            UT, ckpts = _solve_forward(ctx, prob, U0, cfl, nsteps, checkpoint_every)
            fctx.enomr = (ctx, prob, cfl, nsteps, checkpoint_every, ckpts)
            return UT

        @staticmethod
        def backward(fctx, grad):
            ctx, prob, cfl, nsteps, every, ckpts = fctx.enomr
            g = _solve_adjoint(ctx, prob, ckpts, cfl, nsteps, every, grad.contiguous())
            return g, None, None, None, None, None

    return EnoMRSolve


_EnoMRSolve = None


def solve(ctx, prob, U0, cfl, nsteps, checkpoint_every=20):
    """Differentiable SSP-RK3 run (see EnoMRSolve): returns U after nsteps."""
    global _EnoMRSolve
    if _EnoMRSolve is None:
        _EnoMRSolve = _autograd_function()
    if prob.system != EULER or prob.ndim != 1:
        raise ValueError("the differentiable solve is provided for 1D Euler problems")
    if prob.recon != CHARACTERISTIC or prob.alpha_mode != ALPHA_LINE or prob.gravity != 0.0:
        raise ValueError("the differentiable solve takes the default operator only")
    return _EnoMRSolve.apply(U0, ctx, prob, cfl, nsteps, checkpoint_every)

