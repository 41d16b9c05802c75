"""Python front-end of the serial FP64 CPU oracle (swe_oracle.cpp).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline call this module; the GPU library never does.  It takes problems
from the shared seeded input generators (plain numpy arrays) and shares no
arithmetic with the GPU path.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "swe_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

FLAG_NAN, FLAG_CLIPPED, FLAG_BADDT = 1, 2, 4
NTRACE, NSCALAR = 47, 16
#: names of the traced arrays, in order, with the sub-step that writes them
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


LIB_OMP = os.path.join(HERE, "liboracle_omp.so")


def build(force: bool = False) -> str:
    """Compile swe_oracle.cpp with g++ (no FMA contraction, no fast-math);
    also the -fopenmp build whose cell sweeps use all host threads (for the
    benchmark's all-core CPU figure only)."""
    for lib_path, extra in ((LIB, []), (LIB_OMP, ["-fopenmp"])):
        if force or not os.path.exists(lib_path) or os.path.getmtime(lib_path) < os.path.getmtime(SRC):
            tmp = lib_path + ".tmp"
            subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off",
                                   "-fno-fast-math", "-fPIC", "-shared"] + extra + ["-o", tmp, SRC])
            os.replace(tmp, lib_path)
    return LIB


class _Cfg(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("bc", ctypes.c_int32 * 4), ("in_lo", ctypes.c_int32 * 4),
                ("in_hi", ctypes.c_int32 * 4), ("hydro_len", ctypes.c_int32),
                ("pad_", ctypes.c_int32)] + [
                (f, ctypes.c_double) for f in
                ("dx", "dy", "g", "cfl", "h_dry", "kappa", "eps_max", "dt_max", "dt_fixed")] + [
                ("hydro_t", ctypes.POINTER(ctypes.c_double)),
                ("hydro_q", ctypes.POINTER(ctypes.c_double)),
                ("h_film", ctypes.c_double)]


class _Stats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("bad_step", ctypes.c_int64),
                ("flags", ctypes.c_uint32), ("pad_", ctypes.c_uint32)] + [
                (f, ctypes.c_double) for f in
                ("t", "dt", "dt_min", "dt_max", "volume", "defect", "lambda_max",
                 "loop_seconds")]


_lib = None
_lib_omp = None


def lib_threads():
    """The -fopenmp build of the oracle (same source; its cell sweeps run on
    all host threads, the state bit for bit that of the serial build)."""
    global _lib_omp
    if _lib_omp is None:
        build()
        L = ctypes.CDLL(LIB_OMP)
        _declare(L)
        _lib_omp = L
    return _lib_omp


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        _declare(L)
        _lib = L
    return _lib


def _declare(L):
    """Argument and result types of the exported functions."""
    dp = ctypes.POINTER(ctypes.c_double)
    L.orc_run.argtypes = [ctypes.POINTER(_Cfg), dp, dp, dp, dp, dp, dp,
                          ctypes.POINTER(ctypes.c_int64), dp, ctypes.c_int64, ctypes.c_double,
                          ctypes.POINTER(_Stats)]
    L.orc_run.restype = ctypes.c_int
    L.orc_trace.argtypes = [ctypes.POINTER(_Cfg), dp, dp, dp, dp, dp, ctypes.c_double,
                            ctypes.c_int64, ctypes.c_double, dp, dp]
    L.orc_trace.restype = ctypes.c_int
    L.orc_initial_dt.argtypes = [ctypes.POINTER(_Cfg), dp, dp, dp, dp, dp, dp]
    L.orc_initial_dt.restype = ctypes.c_double
    L.orc_cbrt3.argtypes = [ctypes.c_double]
    L.orc_cbrt3.restype = ctypes.c_double
    L.orc_run_f32.argtypes = L.orc_run.argtypes
    L.orc_run_f32.restype = ctypes.c_int
    L.orc_run_record.argtypes = L.orc_run.argtypes + [dp]
    L.orc_run_record.restype = ctypes.c_int
    i64p = ctypes.POINTER(ctypes.c_int64)
    loss_args = [ctypes.POINTER(_Cfg), dp, dp, dp, dp, dp, ctypes.c_double, ctypes.c_int64,
                 ctypes.c_int64, dp, ctypes.c_int32, i64p, ctypes.c_int32, dp]
    L.orc_loss_tangent.argtypes = loss_args + [dp, dp, dp, dp]
    L.orc_loss_tangent.restype = ctypes.c_int
    L.orc_loss_gradient.argtypes = loss_args + [dp, dp, dp]
    L.orc_loss_gradient.restype = ctypes.c_int
    L.orc_threads.restype = ctypes.c_int


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _cfg(p, keep):
    c = _Cfg()
    c.nx, c.ny = p.nx, p.ny
    for k in range(4):
        c.bc[k] = int(p.bc[k])
        c.in_lo[k] = int(p.inflow_lo[k])
        c.in_hi[k] = int(p.inflow_hi[k])
    ht = np.ascontiguousarray(p.hydro_t, dtype=np.float64)
    hq = np.ascontiguousarray(p.hydro_q, dtype=np.float64)
    keep += [ht, hq]
    c.hydro_len = len(ht)
    c.hydro_t = _ptr(ht) if len(ht) else None
    c.hydro_q = _ptr(hq) if len(hq) else None
    for f in ("dx", "dy", "g", "cfl", "h_dry", "kappa", "eps_max", "dt_max", "dt_fixed"):
        setattr(c, f, float(getattr(p, f)))
    c.h_film = float(getattr(p, "h_film", 0.0))
    return c


@dataclasses.dataclass
class Stats:
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
    loop_seconds: float = 0.0
    step: int = 0


class State:
    """Oracle state of one problem: (eta, qx, qy), t^n, n and dt^n.
    binary32=True runs the same steps with every operation rounded to float
    (orc_run_f32: a rounding reference for FP32 state, not the oracle)."""

    def __init__(self, problem, t0: float = 0.0, step0: int = 0, binary32: bool = False,
                 threads: bool = False):
        self.p = problem
        self.binary32 = bool(binary32)
        self.threads = bool(threads)
        self.eta, self.qx, self.qy = problem.state()
        if self.binary32:
            for a in (self.eta, self.qx, self.qy):
                a[...] = a.astype(np.float32)
        self.t = float(t0)
        self.step = int(step0)
        # dt^0 (binary32: computed by the first orc_run_f32 call)
        self.dt = 0.0 if self.binary32 else initial_dt(problem, self.eta, self.qx, self.qy)

    def run(self, nsteps: int, t_end: float = math.inf) -> Stats:
        keep = []
        c = _cfg(self.p, keep)
        t = ctypes.c_double(self.t)
        n = ctypes.c_int64(self.step)
        dt = ctypes.c_double(self.dt)
        st = _Stats()
        L = lib_threads() if self.threads else lib()
        fn = L.orc_run_f32 if self.binary32 else L.orc_run
        rc = fn(ctypes.byref(c), _ptr(self.eta), _ptr(self.qx), _ptr(self.qy),
                           _ptr(self.p.z), _ptr(self.p.n), ctypes.byref(t), ctypes.byref(n),
                           ctypes.byref(dt), int(nsteps), float(t_end), ctypes.byref(st))
        if rc < 0:
            raise ValueError("oracle rejected its arguments")
        self.t, self.step, self.dt = t.value, n.value, dt.value
        return Stats(st.steps, st.bad_step, st.flags, st.t, st.dt, st.dt_min, st.dt_max,
                     st.volume, st.defect, st.lambda_max, st.loop_seconds, self.step)

    def trace(self):
        """One step with every intermediate: (dict name -> (ny+2, nx+2) array,
        dict name -> scalar).  Advances the state."""
        keep = []
        c = _cfg(self.p, keep)
        P, Q = self.p.nx + 2, self.p.ny + 2
        arrays = np.zeros((NTRACE, Q, P))
        scal = np.zeros(NSCALAR)
        rc = lib().orc_trace(ctypes.byref(c), _ptr(self.eta), _ptr(self.qx), _ptr(self.qy),
                             _ptr(self.p.z), _ptr(self.p.n), self.t, self.step, self.dt,
                             _ptr(arrays), _ptr(scal))
        if rc < 0:
            raise ValueError("oracle rejected its arguments")
        self.t = scal[10]
        self.dt = scal[6]
        self.step += 1
        return ({nm: arrays[k] for k, nm in enumerate(TRACE_NAMES)},
                {nm: scal[k] for k, nm in enumerate(SCALAR_NAMES)})


def initial_dt(problem, eta=None, qx=None, qy=None):
    keep = []
    c = _cfg(problem, keep)
    eta = problem.eta if eta is None else eta
    qx = problem.qx if qx is None else qx
    qy = problem.qy if qy is None else qy
    return lib().orc_initial_dt(ctypes.byref(c), _ptr(eta), _ptr(qx), _ptr(qy), _ptr(problem.z),
                                None, None)


def volume_and_lambda(problem, eta, qx, qy):
    keep = []
    c = _cfg(problem, keep)
    lam = ctypes.c_double()
    vol = ctypes.c_double()
    lib().orc_initial_dt(ctypes.byref(c), _ptr(eta), _ptr(qx), _ptr(qy), _ptr(problem.z),
                         ctypes.byref(lam), ctypes.byref(vol))
    return vol.value, lam.value


def run(problem, nsteps: int, t_end: float = math.inf):
    """Convenience: fresh state, nsteps steps; returns (State, Stats)."""
    s = State(problem)
    st = s.run(nsteps, t_end)
    return s, st


def cbrt3(x: float) -> float:
    """The friction step's cube root (exponent-thirding guess, two Halley steps)."""
    return lib().orc_cbrt3(float(x))


# ------------------------------------------------------------ derivatives

def run_record(problem, nsteps: int):
    """Adaptive forward run from the problem's state: (State, dts), dts[n] the
    time step dt^n each step used (the sequence the loss holds fixed)."""
    s = State(problem)
    keep = []
    c = _cfg(problem, keep)
    t = ctypes.c_double(s.t)
    n = ctypes.c_int64(s.step)
    dt = ctypes.c_double(s.dt)
    st = _Stats()
    dts = np.zeros(max(int(nsteps), 1))
    rc = lib().orc_run_record(ctypes.byref(c), _ptr(s.eta), _ptr(s.qx), _ptr(s.qy),
                              _ptr(problem.z), _ptr(problem.n), ctypes.byref(t), ctypes.byref(n),
                              ctypes.byref(dt), int(nsteps), math.inf, ctypes.byref(st),
                              _ptr(dts))
    if rc != 0 or st.steps != nsteps:
        raise ValueError("oracle forward run failed")
    s.t, s.step, s.dt = t.value, n.value, dt.value
    return s, dts[:nsteps]


@dataclasses.dataclass
class Gauges:
    """Gauge-misfit loss: cells (flattened j*nx + i), observed depths
    hobs[k, g] after steps (k+1)*every, and the fixed time steps dts."""
    cells: np.ndarray
    every: int
    hobs: np.ndarray
    dts: np.ndarray


def _loss_args(problem, G: Gauges, keep, eta0=None, qx0=None, qy0=None, z=None, nman=None):
    c = _cfg(problem, keep)
    eta0 = problem.eta if eta0 is None else eta0
    qx0 = problem.qx if qx0 is None else qx0
    qy0 = problem.qy if qy0 is None else qy0
    z = problem.z if z is None else z
    nman = problem.n if nman is None else nman
    cells = np.ascontiguousarray(G.cells, dtype=np.int64)
    hobs = np.ascontiguousarray(G.hobs, dtype=np.float64)
    dts = np.ascontiguousarray(G.dts, dtype=np.float64)
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (eta0, qx0, qy0, z, nman)]
    keep += [cells, hobs, dts] + arrs
    return [ctypes.byref(c)] + [_ptr(a) for a in arrs] + [
        0.0, 0, len(dts), _ptr(dts), len(cells),
        cells.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), int(G.every), _ptr(hobs)]


def loss(problem, G: Gauges, **fields) -> float:
    """The gauge-misfit loss (fields: optional eta0, qx0, qy0, z, nman)."""
    keep = []
    J = ctypes.c_double()
    rc = lib().orc_loss_tangent(*_loss_args(problem, G, keep, **fields), None, None,
                                ctypes.byref(J), None)
    if rc:
        raise ValueError("oracle rejected the loss arguments")
    return J.value


def loss_tangent(problem, G: Gauges, dn=None, dz=None, **fields):
    """(J, dJ): the loss and its derivative along (dn, dz), forward mode."""
    keep = []
    J, dJ = ctypes.c_double(), ctypes.c_double()
    dn = None if dn is None else np.ascontiguousarray(dn, dtype=np.float64)
    dz = None if dz is None else np.ascontiguousarray(dz, dtype=np.float64)
    keep += [dn, dz]
    rc = lib().orc_loss_tangent(*_loss_args(problem, G, keep, **fields),
                                None if dn is None else _ptr(dn), None if dz is None else _ptr(dz),
                                ctypes.byref(J), ctypes.byref(dJ))
    if rc:
        raise ValueError("oracle rejected the loss arguments")
    return J.value, dJ.value


def loss_gradient(problem, G: Gauges, **fields):
    """(J, dJ/dn, dJ/dz): the loss and its gradient, reverse mode."""
    keep = []
    J = ctypes.c_double()
    gn = np.zeros((problem.ny, problem.nx))
    gz = np.zeros((problem.ny, problem.nx))
    rc = lib().orc_loss_gradient(*_loss_args(problem, G, keep, **fields), ctypes.byref(J),
                                 _ptr(gn), _ptr(gz))
    if rc:
        raise ValueError("oracle rejected the loss arguments")
    return J.value, gn, gz
