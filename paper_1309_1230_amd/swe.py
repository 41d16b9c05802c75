"""Thin ctypes binding of libswe.so (include/swe.h).

Every step of the solver runs in the HIP kernels of libswe.so; this module
only marshals arguments: it passes PyTorch device tensors' pointers and the
current HIP stream to the C ABI.  There is no CPU fallback: if the library
is not built, or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libswe.so")

SWE_OK, SWE_EINVAL, SWE_ENOMEM, SWE_EDEVICE, SWE_EUNSTABLE, SWE_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
SWE_F32, SWE_F64 = 1, 2
SWE_BC_WALL, SWE_BC_OPEN, SWE_BC_INFLOW = 0, 1, 2
SWE_PATH_FUSED, SWE_PATH_UNFUSED = 0, 1
FLAG_NAN, FLAG_CLIPPED, FLAG_BADDT, FLAG_STALL = 1, 2, 4, 8
NTRACE = 47
TRACE_NAMES = (
    ["S1.eta", "S1.qx", "S1.qy", "S2.h", "S2.r", "S2.u", "S2.v", "S3.nux", "S3.nuy",
     "S4.Deta", "S4.Dqx", "S4.Dqy", "S5.Fm", "S5.Fx", "S5.Fy", "S5.Px",
     "S6.Gm", "S6.Gx", "S6.Gy", "S6.Py", "S7.eta", "S7.qx", "S7.qy",
     "S9.h", "S9.r", "S9.u", "S9.v", "S10.Fm", "S10.Fx", "S10.Fy", "S10.Px",
     "S11.Gm", "S11.Gx", "S11.Gy", "S11.Py", "S12.eta", "S12.qx", "S12.qy",
     "S13.eta", "S13.qx", "S13.qy", "S14.eta", "S14.qx", "S14.qy",
     "S15.eta", "S15.qx", "S15.qy"])
SCALAR_NAMES = ["qin_n", "qin_n1", "rx", "ry", "defect_depth", "lam_max", "dt_next",
                "volume", "flags", "sigma", "t_next"]


class SweError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libswe error {code}: {msg}")
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("path", ctypes.c_int32), ("bc", ctypes.c_int32 * 4),
                ("inflow_lo", ctypes.c_int32 * 4), ("inflow_hi", ctypes.c_int32 * 4),
                ("hydro_len", ctypes.c_int32), ("tile_rows", ctypes.c_int32),
                ("pitch", ctypes.c_int64)] + [
                (f, ctypes.c_double) for f in
                ("dx", "dy", "g", "cfl", "h_dry", "kappa", "eps_max", "dt_max", "dt_fixed", "t0")] + [
                ("hydro_t", ctypes.POINTER(ctypes.c_double)),
                ("hydro_q", ctypes.POINTER(ctypes.c_double)),
                ("z", ctypes.c_void_p), ("n", ctypes.c_void_p), ("eta", ctypes.c_void_p),
                ("qx", ctypes.c_void_p), ("qy", ctypes.c_void_p), ("stream", ctypes.c_void_p),
                ("dry_skip", ctypes.c_int32), ("h_film", ctypes.c_double)]


class _Stats(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("steps", ctypes.c_int64), ("bad_step", ctypes.c_int64),
                ("flags", ctypes.c_uint32), ("pad_", ctypes.c_uint32)] + [
                (f, ctypes.c_double) for f in
                ("t", "dt", "dt_min", "dt_max", "volume", "defect", "lambda_max")] + [
                ("cells_skipped", ctypes.c_int64)]


class Checkpoint(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("flags", ctypes.c_uint32), ("pad_", ctypes.c_uint32),
                ("t", ctypes.c_double), ("dt", ctypes.c_double), ("defect", ctypes.c_double)]


@dataclasses.dataclass
class Stats:
    step: int
    steps: int
    bad_step: int
    flags: int
    t: float
    dt: float
    dt_min: float
    dt_max: float
    volume: float
    defect: float
    lambda_max: float
    cells_skipped: int = 0


class Gauges(ctypes.Structure):
    _fields_ = [("ngauge", ctypes.c_int32), ("obs_every", ctypes.c_int32),
                ("cells", ctypes.POINTER(ctypes.c_int64)), ("hobs", ctypes.c_void_p)]


#: every function include/swe.h declares
EXPORTS = ("swe_abi_version", "swe_config_init", "swe_create", "swe_destroy", "swe_step",
           "swe_run", "swe_run_dt", "swe_run_noalloc", "swe_get_stats", "swe_trace_step", "swe_trace_bytes", "swe_save",
           "swe_load", "swe_last_error", "swe_probe_copy", "swe_probe_stream", "swe_probe_march", "swe_grad", "swe_loss", "swe_ensemble_create",
           "swe_ensemble_destroy", "swe_ensemble_run", "swe_ensemble_capture",
           "swe_ensemble_replay", "swe_ensemble_stats", "swe_ensemble_tile_rows",
           "swe_ensemble_last_error")

_lib = None


def lib():
    """Load libswe.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1309_1230_amd._build` (no CPU fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        H = ctypes.c_void_p
        L.swe_abi_version.restype = ctypes.c_int
        L.swe_config_init.argtypes = [ctypes.POINTER(Config)]
        L.swe_config_init.restype = None
        L.swe_create.argtypes = [ctypes.POINTER(Config), ctypes.POINTER(H)]
        L.swe_create.restype = ctypes.c_int
        L.swe_destroy.argtypes = [H]
        L.swe_destroy.restype = None
        L.swe_step.argtypes = [H, ctypes.POINTER(ctypes.c_double)]
        L.swe_step.restype = ctypes.c_int
        L.swe_run.argtypes = [H, ctypes.c_int64, ctypes.c_double, ctypes.POINTER(_Stats)]
        L.swe_run.restype = ctypes.c_int
        L.swe_run_dt.argtypes = [H, ctypes.c_int64, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(_Stats)]
        L.swe_run_dt.restype = ctypes.c_int
        L.swe_run_noalloc.argtypes = [ctypes.POINTER(Config), ctypes.c_int64, ctypes.c_double,
                                      ctypes.POINTER(_Stats)]
        L.swe_run_noalloc.restype = ctypes.c_int
        L.swe_get_stats.argtypes = [H, ctypes.POINTER(_Stats)]
        L.swe_get_stats.restype = ctypes.c_int
        L.swe_trace_step.argtypes = [H, ctypes.c_void_p, ctypes.c_size_t,
                                     ctypes.POINTER(ctypes.c_double)]
        L.swe_trace_step.restype = ctypes.c_int
        L.swe_trace_bytes.argtypes = [H]
        L.swe_trace_bytes.restype = ctypes.c_size_t
        L.swe_save.argtypes = [H, ctypes.POINTER(Checkpoint)]
        L.swe_save.restype = ctypes.c_int
        L.swe_load.argtypes = [H, ctypes.POINTER(Checkpoint)]
        L.swe_load.restype = ctypes.c_int
        L.swe_last_error.argtypes = [H]
        L.swe_last_error.restype = ctypes.c_char_p
        L.swe_probe_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                     ctypes.c_void_p]
        L.swe_probe_copy.restype = ctypes.c_int
        L.swe_probe_stream.argtypes = [ctypes.POINTER(ctypes.c_void_p),
                                       ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t,
                                       ctypes.c_int, ctypes.c_void_p]
        L.swe_probe_stream.restype = ctypes.c_int
        L.swe_probe_march.argtypes = [ctypes.POINTER(ctypes.c_void_p),
                                      ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32,
                                      ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                                      ctypes.c_int32, ctypes.c_void_p]
        L.swe_probe_march.restype = ctypes.c_int
        L.swe_grad.argtypes = [H, ctypes.c_int64, ctypes.POINTER(Gauges), ctypes.c_int32,
                               ctypes.POINTER(ctypes.c_double), ctypes.c_void_p, ctypes.c_void_p]
        L.swe_grad.restype = ctypes.c_int
        E = ctypes.c_void_p
        L.swe_ensemble_create.argtypes = [ctypes.POINTER(Config), ctypes.c_int32, ctypes.c_int32,
                                          ctypes.POINTER(E)]
        L.swe_ensemble_create.restype = ctypes.c_int
        L.swe_ensemble_destroy.argtypes = [E]
        L.swe_ensemble_destroy.restype = None
        L.swe_ensemble_run.argtypes = [E, ctypes.c_int64, ctypes.c_double]
        L.swe_ensemble_run.restype = ctypes.c_int
        L.swe_ensemble_capture.argtypes = [E, ctypes.c_int64]
        L.swe_ensemble_capture.restype = ctypes.c_int
        L.swe_ensemble_replay.argtypes = [E]
        L.swe_ensemble_replay.restype = ctypes.c_int
        L.swe_ensemble_stats.argtypes = [E, ctypes.POINTER(_Stats)]
        L.swe_ensemble_stats.restype = ctypes.c_int
        L.swe_ensemble_tile_rows.argtypes = [E]
        L.swe_ensemble_tile_rows.restype = ctypes.c_int32
        L.swe_ensemble_last_error.argtypes = [E]
        L.swe_ensemble_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def last_error(handle=None) -> str:
    return lib().swe_last_error(handle).decode()


def default_config() -> Config:
    c = Config()
    lib().swe_config_init(ctypes.byref(c))
    return c


def _torch():
    import torch
    return torch


def _stream_ptr(stream) -> Optional[int]:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _make_config(z, n, eta, qx, qy, *, dx: float, dy: float, g: float = 9.81,
                 cfl: float = 0.5, h_dry: float = 1e-3, kappa: float = 0.5, eps_max: float = 0.25,
                 dt_max: float = 1.0, dt_fixed: float = 0.0, t0: float = 0.0,
                 bc=(SWE_BC_WALL,) * 4, inflow_lo=(0, 0, 0, 0), inflow_hi=None,
                 hydro_t=(), hydro_q=(), path: str = "fused", tile_rows: int = 0,
                 dry_skip: bool = False, h_film: float = 0.0):
    """Validate five field tensors and build a swe_config for them; returns
    (config, objects the config points into)."""
    torch = _torch()
    fields = (z, n, eta, qx, qy)
    dt0 = eta.dtype
    if dt0 not in (torch.float32, torch.float64):
        raise TypeError("fields must be float32 or float64")
    for f in fields:
        if f.dtype != dt0 or f.device != eta.device or f.dim() != 2 or not f.is_cuda:
            raise TypeError("z, n, eta, qx, qy must be 2-D CUDA tensors of one dtype and device")
        if f.shape != eta.shape or f.stride(1) != 1 or f.stride(0) != eta.stride(0):
            raise TypeError("fields must share shape and row pitch, unit stride along x")
    ny, nx = eta.shape
    c = default_config()
    c.nx, c.ny = nx, ny
    c.dtype = SWE_F32 if dt0 == torch.float32 else SWE_F64
    c.path = {"fused": SWE_PATH_FUSED, "unfused": SWE_PATH_UNFUSED}[path]
    c.pitch = eta.stride(0)
    c.tile_rows = int(tile_rows)
    c.dry_skip = 1 if dry_skip else 0
    if inflow_hi is None:
        inflow_hi = (ny, ny, nx, nx)
    for k in range(4):
        c.bc[k] = int(bc[k])
        c.inflow_lo[k] = int(inflow_lo[k])
        c.inflow_hi[k] = int(inflow_hi[k])
    c.h_film = float(h_film)
    c.dx, c.dy, c.g, c.cfl, c.h_dry = float(dx), float(dy), float(g), float(cfl), float(h_dry)
    c.kappa, c.eps_max, c.dt_max = float(kappa), float(eps_max), float(dt_max)
    c.dt_fixed, c.t0 = float(dt_fixed), float(t0)
    if len(hydro_t) != len(hydro_q):
        raise ValueError("hydro_t and hydro_q differ in length")
    ht = (ctypes.c_double * max(1, len(hydro_t)))(*[float(v) for v in hydro_t])
    hq = (ctypes.c_double * max(1, len(hydro_q)))(*[float(v) for v in hydro_q])
    c.hydro_len = len(hydro_t)
    c.hydro_t = ctypes.cast(ht, ctypes.POINTER(ctypes.c_double))
    c.hydro_q = ctypes.cast(hq, ctypes.POINTER(ctypes.c_double))
    c.z, c.n = z.data_ptr(), n.data_ptr()
    c.eta, c.qx, c.qy = eta.data_ptr(), qx.data_ptr(), qy.data_ptr()
    return c, [ht, hq] + list(fields)


def _problem_kwargs(p):
    return dict(dx=p.dx, dy=p.dy, g=p.g, cfl=p.cfl, h_dry=p.h_dry, kappa=p.kappa,
                eps_max=p.eps_max, dt_max=p.dt_max, dt_fixed=p.dt_fixed, bc=p.bc,
                inflow_lo=p.inflow_lo, inflow_hi=p.inflow_hi, hydro_t=p.hydro_t,
                hydro_q=p.hydro_q, h_film=getattr(p, "h_film", 0.0))


def run_noalloc(z, n, eta, qx, qy, nsteps: int, t_end: float = math.inf, *, tile_rows: int = 0,
                stream=None, check: bool = True, **kw) -> "Stats":
    """swe_run_noalloc: nsteps steps of the fused path over caller-owned
    tensors (eta, qx, qy advanced in place) without any device allocation;
    returns the statistics."""
    torch = _torch()
    c, keep = _make_config(z, n, eta, qx, qy, path="fused", tile_rows=tile_rows, **kw)
    st = _Stats()
    with torch.cuda.device(eta.device):
        c.stream = _stream_ptr(stream)
        rc = lib().swe_run_noalloc(ctypes.byref(c), int(nsteps), float(t_end), ctypes.byref(st))
    del keep
    if check and rc != SWE_OK:
        raise SweError(rc, last_error(None))
    return Solver._stats(st)


class Solver:
    """A libswe handle over caller-owned device tensors (eta, qx, qy are
    advanced in place; z and n are read)."""

    def __init__(self, z, n, eta, qx, qy, *, path: str = "fused", tile_rows: int = 0,
                 stream=None, **kw):
        torch = _torch()
        c, keep = _make_config(z, n, eta, qx, qy, path=path, tile_rows=tile_rows, **kw)
        self._keep = keep
        self.ny, self.nx = eta.shape
        self.dtype = eta.dtype
        with torch.cuda.device(eta.device):
            c.stream = _stream_ptr(stream)
            h = ctypes.c_void_p()
            rc = lib().swe_create(ctypes.byref(c), ctypes.byref(h))
        if rc != SWE_OK:
            raise SweError(rc, last_error(None))
        self._h = h
        self.eta, self.qx, self.qy, self.z, self.n = eta, qx, qy, z, n

    @classmethod
    def from_problem(cls, p, dtype=None, device="cuda", path: str = "fused", tile_rows: int = 0,
                     stream=None, dry_skip: bool = False):
        """Upload a workloads.Problem (float64 numpy arrays) and create a solver."""
        torch = _torch()
        dtype = dtype or torch.float64
        t = lambda a: torch.as_tensor(a, dtype=torch.float64).to(device=device, dtype=dtype).contiguous()
        return cls(t(p.z), t(p.n), t(p.eta), t(p.qx), t(p.qy), path=path, tile_rows=tile_rows,
                   stream=stream, dry_skip=dry_skip, **_problem_kwargs(p))

    def _check(self, rc):
        if rc != SWE_OK:
            raise SweError(rc, last_error(self._h))

    def run(self, nsteps: int, t_end: float = math.inf, check: bool = True) -> Stats:
        st = _Stats()
        rc = lib().swe_run(self._h, int(nsteps), float(t_end), ctypes.byref(st))
        if check:
            self._check(rc)
        return self._stats(st)

    def run_dt(self, dts, check: bool = True) -> Stats:
        """Steps on a prescribed time grid: step k takes dts[k] (swe_run_dt)."""
        import numpy as np
        d = np.ascontiguousarray(np.asarray(dts, dtype=np.float64).ravel())
        st = _Stats()
        rc = lib().swe_run_dt(self._h, int(d.size),
                              d.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                              ctypes.byref(st))
        if check:
            self._check(rc)
        return self._stats(st)

    def step(self, sync: bool = True) -> Optional[float]:
        if sync:
            d = ctypes.c_double()
            self._check(lib().swe_step(self._h, ctypes.byref(d)))
            return d.value
        self._check(lib().swe_step(self._h, None))
        return None

    def stats(self) -> Stats:
        st = _Stats()
        self._check(lib().swe_get_stats(self._h, ctypes.byref(st)))
        return self._stats(st)

    @staticmethod
    def _stats(st) -> Stats:
        return Stats(st.step, st.steps, st.bad_step, st.flags, st.t, st.dt, st.dt_min, st.dt_max,
                     st.volume, st.defect, st.lambda_max, st.cells_skipped)

    def trace_step(self):
        """One unfused step exposing every intermediate: (dict name -> (ny+2,
        nx+2) device tensor, dict name -> scalar)."""
        torch = _torch()
        nbytes = lib().swe_trace_bytes(self._h)
        buf = torch.empty(NTRACE, self.ny + 2, self.nx + 2, dtype=self.dtype, device=self.eta.device)
        assert buf.numel() * buf.element_size() == nbytes
        sc = (ctypes.c_double * 16)()
        self._check(lib().swe_trace_step(self._h, buf.data_ptr(), nbytes, sc))
        return ({nm: buf[k] for k, nm in enumerate(TRACE_NAMES)},
                {nm: sc[k] for k, nm in enumerate(SCALAR_NAMES)})

    def grad(self, nsteps: int, cells, obs_every: int, hobs, ckpt_every: int = 0):
        """Discrete adjoint: run nsteps steps (the state advances, as with
        run) and return (J, dJ/dn, dJ/dz) of the gauge-misfit loss, the time
        steps of the run held fixed.  cells: distinct flattened cells j*nx+i;
        hobs: (nsteps // obs_every, len(cells)) float64 device tensor of
        observed depths.  ckpt_every: checkpoint spacing of the forward run;
        0 keeps the whole FP64 trajectory when it fits in device memory (no
        recompute), else checkpoints every round(sqrt(nsteps)) steps; the
        gradient does not depend on it.  FP32 solvers run the forward in FP32
        and the reverse sweep in FP64, linearised at the promoted FP32 states;
        the gradients are float64 either way."""
        torch = _torch()
        import numpy as np
        cells = np.ascontiguousarray(np.asarray(cells, dtype=np.int64).ravel())
        ng = len(cells)
        nobs = int(nsteps) // int(obs_every)
        if hobs is None:
            hobs = torch.zeros(max(nobs, 1), max(ng, 1), dtype=torch.float64, device=self.eta.device)
        if hobs.dtype != torch.float64 or not hobs.is_cuda:
            raise TypeError("hobs must be a float64 CUDA tensor")
        hobs = hobs.contiguous()
        if nobs > 0 and ng > 0 and tuple(hobs.shape) != (nobs, ng):
            raise ValueError(f"hobs must have shape ({nobs}, {ng})")
        g = Gauges()
        g.ngauge = ng
        g.obs_every = int(obs_every)
        g.cells = cells.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) if ng else None
        g.hobs = hobs.data_ptr()
        gn = torch.zeros_like(self.eta, dtype=torch.float64)
        gz = torch.zeros_like(self.eta, dtype=torch.float64)
        J = ctypes.c_double()
        self._check(lib().swe_grad(self._h, int(nsteps), ctypes.byref(g), int(ckpt_every),
                                   ctypes.byref(J), gn.data_ptr(), gz.data_ptr()))
        return J.value, gn, gz

    def loss(self, nsteps: int, cells, obs_every: int, hobs) -> float:
        """The gauge-misfit loss of the next nsteps steps (swe_loss): the state
        advances as with run; the same J as grad, without the adjoint."""
        import numpy as np
        cells = np.ascontiguousarray(np.asarray(cells, dtype=np.int64).ravel())
        g = Gauges()
        g.ngauge = len(cells)
        g.obs_every = int(obs_every)
        g.cells = cells.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) if len(cells) else None
        g.hobs = hobs.contiguous().data_ptr()
        J = ctypes.c_double()
        self._check(lib().swe_loss(self._h, int(nsteps), ctypes.byref(g), ctypes.byref(J)))
        return J.value

    def save(self) -> Checkpoint:
        ck = Checkpoint()
        self._check(lib().swe_save(self._h, ctypes.byref(ck)))
        return ck

    def load(self, ck: Checkpoint):
        self._check(lib().swe_load(self._h, ctypes.byref(ck)))

    def close(self):
        if getattr(self, "_h", None):
            lib().swe_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def probe_stream(ins, outs, nontemporal=False, stream=None):
    """One pass of the library's 5-read / 3-write stream kernel over
    equally sized device tensors (bandwidth probe)."""
    nbytes = outs[0].numel() * outs[0].element_size()
    arr_in = (ctypes.c_void_p * 5)(*[t.data_ptr() for t in ins])
    arr_out = (ctypes.c_void_p * 3)(*[t.data_ptr() for t in outs])
    rc = lib().swe_probe_stream(arr_in, arr_out, nbytes, 1 if nontemporal else 0,
                                _stream_ptr(stream))
    if rc != SWE_OK:
        raise SweError(rc, last_error(None))


def probe_march(ins, outs, nx, ny, pitch, rows=0, stream=None):
    """One launch of the library's march-pattern probe (the step kernel's
    tiles, loads and stores without its arithmetic) over device tensors of
    ny * pitch elements; returns the tile height used."""
    arr_in = (ctypes.c_void_p * 5)(*[t.data_ptr() for t in ins])
    arr_out = (ctypes.c_void_p * 3)(*[t.data_ptr() for t in outs])
    rc = lib().swe_probe_march(arr_in, arr_out, nx, ny, pitch, outs[0].element_size(), rows,
                               _stream_ptr(stream))
    if rc <= 0:
        raise SweError(rc, last_error(None))
    return rc


def probe_copy(dst, src, stream=None):
    """Device copy through the library's plain copy kernel (bandwidth probe)."""
    nbytes = src.numel() * src.element_size()
    rc = lib().swe_probe_copy(dst.data_ptr(), src.data_ptr(), nbytes, _stream_ptr(stream))
    if rc != SWE_OK:
        raise SweError(rc, last_error(None))


def _make_loss_function():
    torch = _torch()

    class SweLoss(torch.autograd.Function):
        """Gauge-misfit loss of a run as a differentiable function of the
        Manning field n and the bed z (CUDA tensors).  forward runs the
        forward model and its loss only (swe_loss); backward, if it is
        called, runs the library's discrete adjoint (swe_grad) from the saved
        inputs.  The time steps of the run are held fixed.

            J = SweLoss.apply(n, z, eta0, qx0, qy0, solver_kwargs, nsteps,
                              cells, obs_every, hobs, ckpt_every)
        """

        @staticmethod
        def forward(ctx, n, z, eta0, qx0, qy0, solver_kwargs, nsteps, cells, obs_every, hobs,
                    ckpt_every=0):
            s = Solver(z.detach().contiguous(), n.detach().contiguous(), eta0.detach().clone(),
                       qx0.detach().clone(), qy0.detach().clone(), **solver_kwargs)
            try:
                J = s.loss(nsteps, cells, obs_every, hobs)
            finally:
                s.close()
            ctx.save_for_backward(n.detach(), z.detach(), eta0.detach(), qx0.detach(),
                                  qy0.detach(), hobs.detach())
            ctx.args = (solver_kwargs, nsteps, cells, obs_every, ckpt_every)
            return torch.tensor(J, dtype=torch.float64, device=n.device)

        @staticmethod
        def backward(ctx, gout):
            n, z, eta0, qx0, qy0, hobs = ctx.saved_tensors
            solver_kwargs, nsteps, cells, obs_every, ckpt_every = ctx.args
            s = Solver(z.contiguous(), n.contiguous(), eta0.clone(), qx0.clone(), qy0.clone(),
                       **solver_kwargs)
            try:
                _, gn, gz = s.grad(nsteps, cells, obs_every, hobs, ckpt_every)
            finally:
                s.close()
            return (gout * gn.to(n.dtype), gout * gz.to(z.dtype)) + (None,) * 9

    return SweLoss


_SweLoss = None


def SweLoss():
    """The torch.autograd.Function of the gauge-misfit loss (created on first
    use so that importing this module does not import torch)."""
    global _SweLoss
    if _SweLoss is None:
        _SweLoss = _make_loss_function()
    return _SweLoss


class Ensemble:
    """Many independent scenarios advanced together: one fused-kernel launch
    per time step for all of them (each keeps its own grid, fields,
    boundaries and CFL-adaptive dt).  Fields are caller-owned CUDA tensors,
    advanced in place; the ensemble runs on its own stream."""

    def __init__(self, scenarios, tile_rows: int = 0):
        """scenarios: list of (z, n, eta, qx, qy, kwargs) with the kwargs of
        Solver (dx, dy, bc, hydrograph, ...)."""
        cfgs = (Config * len(scenarios))()
        self._keep = []
        self.fields = []
        for k, (z, n, eta, qx, qy, kw) in enumerate(scenarios):
            c, keep = _make_config(z, n, eta, qx, qy, **kw)
            cfgs[k] = c
            self._keep += keep
            self.fields.append((eta, qx, qy))
        self.count = len(scenarios)
        h = ctypes.c_void_p()
        rc = lib().swe_ensemble_create(cfgs, self.count, int(tile_rows), ctypes.byref(h))
        if rc != SWE_OK:
            raise SweError(rc, (lib().swe_ensemble_last_error(None) or b"").decode())
        self._e = h

    @classmethod
    def from_problems(cls, problems, dtype=None, device="cuda", tile_rows: int = 0,
                      dry_skip: bool = False):
        torch = _torch()
        dtype = dtype or torch.float32
        t = lambda a: torch.as_tensor(a, dtype=torch.float64).to(device=device, dtype=dtype).contiguous()
        return cls([(t(p.z), t(p.n), t(p.eta), t(p.qx), t(p.qy),
                     dict(_problem_kwargs(p), dry_skip=dry_skip)) for p in problems],
                   tile_rows=tile_rows)

    def _check(self, rc):
        if rc != SWE_OK:
            raise SweError(rc, (lib().swe_ensemble_last_error(self._e) or b"").decode())

    @property
    def tile_rows(self) -> int:
        return int(lib().swe_ensemble_tile_rows(self._e))

    def run(self, nsteps: int, t_end: float = math.inf):
        """Enqueue nsteps steps of every scenario (asynchronous)."""
        self._check(lib().swe_ensemble_run(self._e, int(nsteps), float(t_end)))

    def capture(self, nsteps: int):
        """Capture an nsteps run (nsteps even) into a HIP graph."""
        self._check(lib().swe_ensemble_capture(self._e, int(nsteps)))

    def replay(self):
        """Launch the captured graph once (asynchronous)."""
        self._check(lib().swe_ensemble_replay(self._e))

    def stats(self, check: bool = True):
        """Synchronise; per-scenario Stats."""
        st = (_Stats * self.count)()
        rc = lib().swe_ensemble_stats(self._e, st)
        if check:
            self._check(rc)
        return [Solver._stats(x) for x in st]

    def close(self):
        if getattr(self, "_e", None):
            lib().swe_ensemble_destroy(self._e)
            self._e = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
