"""Thin ctypes binding of the C ABI in include/lr.h (argument marshalling only).

Every step of the integration runs in the HIP library ``liblr.so`` built by
``paper_2508_18114_amd.build``; this module only converts Python values into
the ABI's structs and device pointers.  PyTorch provides device memory and
the stream.  Importing this module fails loudly if the library is missing.

Device arrays: a factor B (N x M, column-major as the ABI requires) is held
in a torch complex128 CUDA tensor of shape (M, N) (row j = column j of B);
use ``to_device`` / ``from_device`` to move numpy (N, M) arrays.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

# torch first: the library then binds to the HIP runtime torch already loaded
# (the one that owns the device memory and streams passed in), whatever
# module imports this one first
import torch  # noqa: F401

from . import inputs as _inp

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblr.so")

LR_OK = 0
LR_ERR_ARG = -1
LR_ERR_OOM = -2
LR_ERR_HIP = -3
LR_ERR_GRAM_NOT_PD = -4
LR_ERR_NONFINITE = -5
LR_ERR_PULSE = -6
LR_ERR_STATE = -7
LR_ERR_TIMEOUT = -8
LR_ERR_STEP = -9
LR_MAX_M = 32
LR_BATCH_PACKED = 1       # lr_batch_init_ex flag: one workgroup per trajectory
LR_BATCH_PACKED_MFMA64 = 2    # packed FP64 Gram terms on the matrix cores instead of the vector ALU
LR_PACKED_MAX_LM = 1536


def LR_BATCH_SPREAD_LAYERS(k: int) -> int:
    """lr_batch_init_ex flag: resonator layers per workgroup of the spread schedule."""
    return (int(k) & 0xFF) << 8


def LR_BATCH_PACKED_PARTS(p: int) -> int:
    """Packed-schedule flag: every FP64 packed trajectory split over p workgroups (layer ranges)."""
    return (int(p) & 0xFF) << 16

# every symbol include/lr.h declares
EXPORTS = ("lr_init", "lr_workspace_bytes", "lr_bind", "lr_rhs", "lr_integrate",
           "lr_observables", "lr_spectrum", "lr_status", "lr_profile_enable", "lr_profile_read",
           "lr_readout_loss", "lr_dense_workspace_bytes", "lr_dense_integrate", "lr_strerror", "lr_destroy",
           "lr_batch_init", "lr_batch_init_ex", "lr_batch_init_adaptive", "lr_batch_init_adaptive_ex",
           "lr_batch_adaptive_stats",
           "lr_batch_workspace_bytes", "lr_batch_graph", "lr_batch_bind", "lr_batch_run",
           "lr_batch_status", "lr_batch_profile_enable", "lr_batch_profile_read", "lr_batch_destroy",
           "lr_wait_limits", "lr_batch_wait_limits", "lr_apply_heff", "lr_integrate_noalloc")


class LrError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {lr_strerror(code)} ({code})")
        self.code = code


class lr_model_t(ctypes.Structure):
    _fields_ = [("d_q", ctypes.c_int32), ("d_r", ctypes.c_int32), ("d_f", ctypes.c_int32),
                ("kind", ctypes.c_int32),
                ("w_q", ctypes.c_double), ("alpha", ctypes.c_double),
                ("w_r", ctypes.c_double), ("w_f", ctypes.c_double),
                ("g", ctypes.c_double), ("G", ctypes.c_double),
                ("kappa_f", ctypes.c_double), ("gamma_1", ctypes.c_double),
                ("E_t", ctypes.c_double * _inp.MAX_DQ),
                ("n_t", ctypes.c_double * (_inp.MAX_DQ * _inp.MAX_DQ)),
                ("S", ctypes.c_double * 8)]


class lr_pulse_t(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("frame", ctypes.c_int32),
                ("w_d", ctypes.c_double), ("amp", ctypes.c_double),
                ("t_ramp", ctypes.c_double), ("T", ctypes.c_double),
                ("p", ctypes.c_double * 6),
                ("nh", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("sigma", ctypes.c_double), ("h", ctypes.c_double * (2 * _inp.PULSE_MAX_HEIGHTS))]


class lr_traj_t(ctypes.Structure):
    _fields_ = [("model", lr_model_t), ("M", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("pulse", lr_pulse_t), ("t0", ctypes.c_double), ("dt", ctypes.c_double),
                ("nsteps", ctypes.c_int64), ("d_B", ctypes.c_void_p), ("obs_stride", ctypes.c_int32),
                ("step0", ctypes.c_int32), ("d_obs", ctypes.c_void_p)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library {LIB_PATH} is missing: build it with "
                          "`python -m paper_2508_18114_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    sig = {
        "lr_init": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.POINTER(lr_model_t), i32, i32]),
        "lr_workspace_bytes": (sz, [vp]),
        "lr_bind": (ctypes.c_int, [vp, vp, sz, vp]),
        "lr_rhs": (ctypes.c_int, [vp, ctypes.POINTER(lr_pulse_t), dbl, vp, vp]),
        "lr_integrate": (ctypes.c_int, [vp, ctypes.POINTER(lr_pulse_t), dbl, dbl, i64, vp, i32, vp]),
        "lr_observables": (ctypes.c_int, [vp, vp, vp]),
        "lr_spectrum": (ctypes.c_int, [vp, vp, vp]),
        "lr_status": (ctypes.c_int, [vp, ctypes.POINTER(i64)]),
        "lr_profile_enable": (ctypes.c_int, [vp, i32]),
        "lr_profile_read": (ctypes.c_int, [vp, ctypes.POINTER(dbl), ctypes.POINTER(i64),
                                           ctypes.POINTER(dbl), ctypes.POINTER(i64)]),
        "lr_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "lr_readout_loss": (ctypes.c_int, [vp, vp, i64, i32, dbl, dbl, dbl, dbl, vp, vp]),
        "lr_dense_workspace_bytes": (sz, [ctypes.POINTER(lr_model_t)]),
        "lr_dense_integrate": (ctypes.c_int, [ctypes.POINTER(lr_model_t), ctypes.POINTER(lr_pulse_t), dbl, dbl, i64,
                                              vp, i32, vp, vp, sz, vp]),
        "lr_batch_init": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.POINTER(lr_traj_t), i32]),
        "lr_batch_init_ex": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.POINTER(lr_traj_t), i32, i32]),
        "lr_batch_init_adaptive": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.POINTER(lr_traj_t), i32, dbl, dbl]),
        "lr_batch_init_adaptive_ex": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.POINTER(lr_traj_t), i32, i32, dbl,
                                                     dbl]),
        "lr_batch_adaptive_stats": (ctypes.c_int, [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]),
        "lr_batch_graph": (ctypes.c_int, [vp, i32]),
        "lr_batch_workspace_bytes": (sz, [vp]),
        "lr_batch_bind": (ctypes.c_int, [vp, vp, sz, vp]),
        "lr_batch_run": (ctypes.c_int, [vp]),
        "lr_batch_status": (ctypes.c_int, [vp, ctypes.POINTER(i32), ctypes.POINTER(i64)]),
        "lr_batch_profile_enable": (ctypes.c_int, [vp, i32]),
        "lr_batch_profile_read": (ctypes.c_int, [vp, ctypes.POINTER(dbl), ctypes.POINTER(i64)]),
        "lr_batch_destroy": (None, [vp]),
        "lr_destroy": (None, [vp]),
        "lr_wait_limits": (ctypes.c_int, [vp, ctypes.c_uint32, i32]),
        "lr_batch_wait_limits": (ctypes.c_int, [vp, ctypes.c_uint32, i32]),
        "lr_apply_heff": (ctypes.c_int, [ctypes.POINTER(lr_model_t), ctypes.POINTER(lr_pulse_t), dbl, vp, i64, vp,
                                         vp]),
        "lr_integrate_noalloc": (ctypes.c_int, [ctypes.POINTER(lr_model_t), i32, i32, ctypes.POINTER(lr_pulse_t), dbl,
                                                dbl, i64, vp, i32, vp, vp, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def model_struct(m: _inp.ModelParams) -> lr_model_t:
    s = lr_model_t(m.d_q, m.d_r, m.d_f, int(getattr(m, "kind", 0)), m.w_q, m.alpha, m.w_r, m.w_f,
                   m.g, m.G, m.kappa_f, m.gamma_1)
    if s.kind in (_inp.MODEL_TRANSMON, _inp.MODEL_NORMAL):
        if m.d_q > _inp.MAX_DQ or len(m.E_t) != m.d_q or len(m.n_t) != m.d_q * m.d_q:
            raise ValueError("transmon model: E_t needs d_q values and n_t d_q * d_q (d_q <= MAX_DQ)")
        for k, x in enumerate(m.E_t):
            s.E_t[k] = float(x)
        for k, x in enumerate(m.n_t):
            s.n_t[k] = float(x)
    if s.kind == _inp.MODEL_NORMAL:
        if len(m.S) != 8:
            raise ValueError("normal-mode model: S needs the two rows of a and f (8 values)")
        for k, x in enumerate(m.S):
            s.S[k] = float(x)
    return s


def pulse_struct(p: _inp.PulseParams) -> lr_pulse_t:
    h = [0.0] * (2 * _inp.PULSE_MAX_HEIGHTS)
    hs = list(p.h)[:_inp.PULSE_MAX_HEIGHTS]
    for k, x in enumerate(hs):
        h[2 * k], h[2 * k + 1] = complex(x).real, complex(x).imag
    nh = len(p.h) if p.kind == _inp.PULSE_STEPWISE else 0  # too many heights: rejected by the library
    return lr_pulse_t(p.kind, p.frame, p.w_d, p.amp, p.t_ramp, p.T, (ctypes.c_double * 6)(*p.p), nh, 0,
                      p.sigma, (ctypes.c_double * (2 * _inp.PULSE_MAX_HEIGHTS))(*h))


# ---------------------------------------------------------------- raw ABI

def lr_strerror(code: int) -> str:
    return _lib.lr_strerror(code).decode()


def lr_init(model: _inp.ModelParams, M: int, precision: int = _inp.FP64) -> int:
    h = ctypes.c_void_p()
    ms = model_struct(model)
    rc = _lib.lr_init(ctypes.byref(h), ctypes.byref(ms), M, precision)
    if rc != LR_OK:
        raise LrError(rc, "lr_init")
    return h.value


def lr_workspace_bytes(ctx: int) -> int:
    return int(_lib.lr_workspace_bytes(ctx))


def lr_bind(ctx: int, d_ws: int, nbytes: int, stream: int) -> int:
    return _lib.lr_bind(ctx, d_ws, nbytes, stream)


def lr_rhs(ctx: int, pulse: _inp.PulseParams, t: float, d_B: int, d_dB: int) -> int:
    ps = pulse_struct(pulse)
    return _lib.lr_rhs(ctx, ctypes.byref(ps), t, d_B, d_dB)


def lr_integrate(ctx: int, pulse: _inp.PulseParams, t0: float, dt: float, nsteps: int,
                 d_B: int, obs_stride: int, d_obs: int) -> int:
    ps = pulse_struct(pulse)
    return _lib.lr_integrate(ctx, ctypes.byref(ps), t0, dt, nsteps, d_B, obs_stride, d_obs)


def lr_observables(ctx: int, d_B: int, d_out: int) -> int:
    return _lib.lr_observables(ctx, d_B, d_out)


def lr_spectrum(ctx: int, d_B: int, d_eval: int) -> int:
    return _lib.lr_spectrum(ctx, d_B, d_eval)


def lr_status(ctx: int):
    fs = ctypes.c_int64(-1)
    rc = _lib.lr_status(ctx, ctypes.byref(fs))
    return rc, fs.value


def lr_profile_enable(ctx: int, on: bool) -> int:
    return _lib.lr_profile_enable(ctx, 1 if on else 0)


def lr_profile_read(ctx: int):
    """-> (rc, stage_ms, stage_launches, solve_ms, solve_launches)"""
    sm, sl, vm, vl = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_int64()
    rc = _lib.lr_profile_read(ctx, ctypes.byref(sm), ctypes.byref(sl), ctypes.byref(vm), ctypes.byref(vl))
    return rc, sm.value, sl.value, vm.value, vl.value


def lr_destroy(ctx: int) -> None:
    _lib.lr_destroy(ctx)


def lr_batch_init(trajs, flags: int = 0, adaptive=None) -> int:
    """trajs: sequence of lr_traj_t; flags: 0 or LR_BATCH_PACKED (lr_batch_init_ex);
    adaptive: (rtol, atol) for lr_batch_init_adaptive (with flags: lr_batch_init_adaptive_ex)."""
    arr = (lr_traj_t * len(trajs))(*trajs)
    h = ctypes.c_void_p()
    if adaptive is not None and flags & ~LR_BATCH_PACKED:
        rc = _lib.lr_batch_init_adaptive_ex(ctypes.byref(h), arr, len(trajs), int(flags), float(adaptive[0]),
                                            float(adaptive[1]))
    elif adaptive is not None:
        rc = _lib.lr_batch_init_adaptive(ctypes.byref(h), arr, len(trajs), float(adaptive[0]), float(adaptive[1]))
    elif flags:
        rc = _lib.lr_batch_init_ex(ctypes.byref(h), arr, len(trajs), flags)
    else:
        rc = _lib.lr_batch_init(ctypes.byref(h), arr, len(trajs))
    if rc != LR_OK:
        raise LrError(rc, "lr_batch_init")
    return h.value


def lr_batch_workspace_bytes(batch: int) -> int:
    return int(_lib.lr_batch_workspace_bytes(batch))


def lr_batch_bind(batch: int, d_ws: int, nbytes: int, stream: int) -> int:
    return _lib.lr_batch_bind(batch, d_ws, nbytes, stream)


def lr_batch_run(batch: int) -> int:
    return _lib.lr_batch_run(batch)


def lr_batch_status(batch: int, n: int):
    codes = (ctypes.c_int32 * n)()
    steps = (ctypes.c_int64 * n)()
    rc = _lib.lr_batch_status(batch, codes, steps)
    return rc, list(codes), list(steps)


def lr_batch_profile_enable(batch: int, on: bool) -> int:
    return _lib.lr_batch_profile_enable(batch, 1 if on else 0)


def lr_batch_profile_read(batch: int):
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    rc = _lib.lr_batch_profile_read(batch, ctypes.byref(ms), ctypes.byref(n))
    return rc, ms.value, n.value


def lr_batch_destroy(batch: int) -> None:
    _lib.lr_batch_destroy(batch)


LOSS_KEYS = ("snr", "eps_sep", "eps_decay", "eps_a", "ionisation", "loss")


def readout_loss(obs_g, obs_e, d_q, h, kappa_f, gamma_1, eta=0.6, stream=None):
    """Figures of merit of a g/e pair on the device (lr_readout_loss).

    obs_g, obs_e: device float64 tensors (nsamples, LR_OBS_LEN(d_q)).
    Returns a dict of Python floats (synchronises the stream)."""
    import torch
    assert obs_g.shape == obs_e.shape and obs_g.dtype == torch.float64 and obs_g.is_cuda and obs_e.is_cuda
    assert obs_g.shape[1] == 6 + d_q and obs_g.is_contiguous() and obs_e.is_contiguous()
    out = torch.empty(6, dtype=torch.float64, device=obs_g.device)
    st = stream if stream is not None else torch.cuda.current_stream()
    rc = _lib.lr_readout_loss(obs_g.data_ptr(), obs_e.data_ptr(), obs_g.shape[0], d_q, h, kappa_f, gamma_1, eta,
                              out.data_ptr(), st.cuda_stream)
    if rc != LR_OK:
        raise LrError(rc, "lr_readout_loss")
    vals = out.cpu().tolist()
    return dict(zip(LOSS_KEYS, vals))


def lr_integrate_noalloc(model, M, precision, pulse, t0, dt, nsteps, d_B: int, obs_stride: int, d_obs: int,
                         d_status: int, stream: int) -> int:
    """Raw call of lr_integrate_noalloc (device pointers as integers)."""
    ms, ps = model_struct(model), pulse_struct(pulse)
    return _lib.lr_integrate_noalloc(ctypes.byref(ms), M, precision, ctypes.byref(ps), t0, dt, nsteps, d_B,
                                     obs_stride, d_obs or None, d_status or None, stream)


def apply_heff(model, pulse, t, B, Z=None, stream=None):
    """Z = H_eff(t) B on the device (lr_apply_heff).  B: device complex128 tensor (ncols, N) (column j of
    the factor is row j; several factors of one model may be stacked); Z: same shape, allocated if None."""
    import torch
    assert B.dtype == torch.complex128 and B.is_cuda and B.is_contiguous() and B.shape[-1] == model.N
    if Z is None:
        Z = torch.empty_like(B)
    assert Z.shape == B.shape and Z.dtype == B.dtype and Z.is_contiguous()
    ms, ps = model_struct(model), pulse_struct(pulse)
    st = stream if stream is not None else torch.cuda.current_stream()
    ncols = B.numel() // model.N
    rc = _lib.lr_apply_heff(ctypes.byref(ms), ctypes.byref(ps), float(t), B.data_ptr(), ncols, Z.data_ptr(),
                            st.cuda_stream)
    if rc != LR_OK:
        raise LrError(rc, "lr_apply_heff")
    return Z


def dense_integrate(model, pulse, t0, dt, nsteps, rho, obs_stride=0, obs=None, workspace=None, stream=None):
    """Dense full-Lindblad RK4 on the device (lr_dense_integrate).

    rho: device complex128 tensor (N, N), row-major, Hermitian; updated in
    place.  obs: device float64 tensor (nsteps // obs_stride + 1, 6 + d_q) when
    obs_stride > 0.  workspace: optional device uint8 tensor to reuse."""
    import torch
    N = model.N
    assert rho.shape == (N, N) and rho.dtype == torch.complex128 and rho.is_cuda and rho.is_contiguous()
    ms = model_struct(model)
    nbytes = _lib.lr_dense_workspace_bytes(ctypes.byref(ms))
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=rho.device)
    st = stream if stream is not None else torch.cuda.current_stream()
    ps = pulse_struct(pulse)
    rc = _lib.lr_dense_integrate(ctypes.byref(ms), ctypes.byref(ps), t0, dt, nsteps, rho.data_ptr(), obs_stride,
                                 obs.data_ptr() if obs is not None else None, workspace.data_ptr(), nbytes,
                                 st.cuda_stream)
    if rc != LR_OK:
        raise LrError(rc, "lr_dense_integrate")
    return workspace


# ---------------------------------------------------------------- helpers

def to_device(B: np.ndarray, device="cuda"):
    """numpy (N, M) complex -> torch (M, N) complex128 device tensor (column-major B)."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(B, dtype=np.complex128).T)).to(device)


def from_device(t) -> np.ndarray:
    """torch (M, N) device tensor -> numpy (N, M)."""
    return t.detach().cpu().numpy().T.copy()


def obs_len(model: _inp.ModelParams) -> int:
    return 6 + model.d_q


class Context:
    """One trajectory shape bound to torch-owned workspace on the current stream."""

    def __init__(self, model: _inp.ModelParams, M: int, precision: int = _inp.FP64, stream=None):
        import torch
        self.model, self.M, self.precision = model, M, precision
        self.handle = lr_init(model, M, precision)
        nbytes = lr_workspace_bytes(self.handle)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.workspace = _stream_buffer(nbytes + 256, self.stream)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        rc = lr_bind(self.handle, base + off, nbytes, self.stream.cuda_stream)
        if rc != LR_OK:
            raise LrError(rc, "lr_bind")

    def _check(self, rc, where):
        if rc != LR_OK:
            raise LrError(rc, where)

    def rhs(self, pulse, t, B_dev, dB_dev):
        self._check(lr_rhs(self.handle, pulse, t, B_dev.data_ptr(), dB_dev.data_ptr()), "lr_rhs")

    def integrate(self, pulse, t0, dt, nsteps, B_dev, obs_stride=0, obs_dev=None):
        d_obs = obs_dev.data_ptr() if obs_dev is not None else 0
        self._check(lr_integrate(self.handle, pulse, t0, dt, nsteps, B_dev.data_ptr(), obs_stride, d_obs),
                    "lr_integrate")

    def observables(self, B_dev, out_dev):
        self._check(lr_observables(self.handle, B_dev.data_ptr(), out_dev.data_ptr()), "lr_observables")

    def spectrum(self, B_dev, out_dev=None):
        """Eigenvalues p_1 >= ... >= p_M of B^ B (device tensor of M doubles):
        the weights of the low-rank density matrix; p_M / p_1 is the validity
        control quantity and sum p_j^2 the purity (supplement S1.B)."""
        import torch
        if out_dev is None:
            out_dev = torch.empty((self.M,), dtype=torch.float64, device=B_dev.device)
        self._check(lr_spectrum(self.handle, B_dev.data_ptr(), out_dev.data_ptr()), "lr_spectrum")
        return out_dev

    def status(self):
        return lr_status(self.handle)

    def wait_limits(self, spins=0, never=False):
        """Bounded waits of the group barriers (lr_wait_limits): `spins` polls (0: the default);
        never=True makes every wait expire (failure-handling tests)."""
        self._check(_lib.lr_wait_limits(self.handle, int(spins), 1 if never else 0), "lr_wait_limits")

    def new_obs(self, nsteps, obs_stride):
        import torch
        n = nsteps // obs_stride + 1 if obs_stride > 0 else 0
        return torch.zeros((n, obs_len(self.model)), dtype=torch.float64, device="cuda")

    def close(self):
        """Wait for the context's stream, then free the library handle and the workspace."""
        if self.handle:
            self.stream.synchronize()
            lr_destroy(self.handle)
            self.handle = None
        self.workspace = None

    def __del__(self):
        _finalize(self, lr_destroy)


def _stream_buffer(nbytes, stream):
    """Device workspace allocated on `stream` (the caching allocator then reuses it only after the work
    queued on that stream, whichever stream is current when it is freed)."""
    import torch
    with torch.cuda.stream(stream):
        return torch.empty(nbytes, dtype=torch.uint8, device="cuda")


def _finalize(obj, destroy):
    """Release of a handle by the garbage collector.  During interpreter shutdown the HIP runtime may
    already be gone, so nothing is called then (the process is ending; the handle's host memory goes
    with it)."""
    import sys
    h = getattr(obj, "handle", None)
    if not h or sys.is_finalizing():
        return
    try:
        obj.stream.synchronize()
        destroy(h)
        obj.handle = None
    except Exception:
        pass


def traj_struct(model, M, pulse, t0, dt, nsteps, B_dev, obs_stride=0, obs_dev=None,
                precision=_inp.FP64, step0=0) -> lr_traj_t:
    return lr_traj_t(model_struct(model), M, precision, pulse_struct(pulse), t0, dt, nsteps,
                     B_dev.data_ptr(), obs_stride, step0, obs_dev.data_ptr() if obs_dev is not None else 0)


class Batch:
    """A batch of trajectories bound to torch-owned workspace on one stream.

    items: sequence of dicts with keys model, M, pulse, dt, nsteps, B (device
    tensor (M, N) complex128), and optionally t0, obs_stride, obs (device
    tensor), precision (FP64 / FP32 / BF16X3), step0 (index of the first step
    when a trajectory is continued).  The tensors must stay alive while the
    batch is used.  packed=True: the packed schedule (LR_BATCH_PACKED), one
    workgroup per FP64 trajectory.  adaptive=(rtol, atol): adaptive
    Dormand-Prince steps (lr_batch_init_adaptive); dt is then the output grid.
    parts=p (p >= 2): every FP64 packed trajectory split over p workgroups
    (LR_BATCH_PACKED_PARTS), for latency when few trajectories are in flight.
    """

    def __init__(self, items, stream=None, packed=False, adaptive=None, flags=0, parts=0):
        import torch
        self.items = list(items)
        ts = [traj_struct(it["model"], it["M"], it["pulse"], it.get("t0", 0.0), it["dt"], it["nsteps"],
                          it["B"], it.get("obs_stride", 0), it.get("obs"), it.get("precision", _inp.FP64),
                          it.get("step0", 0))
              for it in self.items]
        flags = int(flags) | (LR_BATCH_PACKED_PARTS(parts) if parts else 0)
        self.handle = lr_batch_init(ts, (LR_BATCH_PACKED if packed else 0) | flags, adaptive)
        nbytes = lr_batch_workspace_bytes(self.handle)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.workspace = _stream_buffer(nbytes + 256, self.stream)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        rc = lr_batch_bind(self.handle, base + off, nbytes, self.stream.cuda_stream)
        if rc != LR_OK:
            raise LrError(rc, "lr_batch_bind")

    def run(self):
        rc = lr_batch_run(self.handle)
        if rc != LR_OK:
            raise LrError(rc, "lr_batch_run")

    def status(self):
        return lr_batch_status(self.handle, len(self.items))

    def wait_limits(self, spins=0, never=False):
        """lr_batch_wait_limits: bounded waits of the group barriers (spread schedule, layer-split trajectories)."""
        rc = _lib.lr_batch_wait_limits(self.handle, int(spins), 1 if never else 0)
        if rc != LR_OK:
            raise LrError(rc, "lr_batch_wait_limits")

    def graph(self, on=True):
        """Capture the launch sequence once and replay it on every run (packed batches)."""
        rc = _lib.lr_batch_graph(self.handle, 1 if on else 0)
        if rc != LR_OK:
            raise LrError(rc, "lr_batch_graph")

    def adaptive_stats(self):
        """(accepted, rejected) step counts per trajectory of an adaptive batch."""
        n = len(self.items)
        acc = (ctypes.c_int64 * n)()
        rej = (ctypes.c_int64 * n)()
        rc = _lib.lr_batch_adaptive_stats(self.handle, acc, rej)
        if rc != LR_OK:
            raise LrError(rc, "lr_batch_adaptive_stats")
        return list(acc), list(rej)

    def profile(self, on=True):
        rc = lr_batch_profile_enable(self.handle, on)
        if rc != LR_OK:
            raise LrError(rc, "lr_batch_profile_enable")

    def profile_read(self):
        """(summed kernel ms, launches) of the timed persistent-kernel chunks."""
        rc, ms, n = lr_batch_profile_read(self.handle)
        if rc != LR_OK:
            raise LrError(rc, "lr_batch_profile_read")
        return ms, n

    def close(self):
        """Wait for the batch's stream, then free the library handle and the workspace."""
        if self.handle:
            self.stream.synchronize()
            lr_batch_destroy(self.handle)
            self.handle = None
        self.workspace = None

    def __del__(self):
        _finalize(self, lr_batch_destroy)
