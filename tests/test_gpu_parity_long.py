"""GPU against the oracle over the reservoir workload's full length: 1000
steps of the reservoir release at 512 x 512, dx = 40 m (the 20.48 km domain
of the 4096 x 4096 benchmark at one eighth of its resolution: same terrain
recipe and seed, same reservoir, open east edge, wet/dry fronts moving over
the hills for the whole run).

Every input is rounded to float32 first, so that the FP64 and FP32 solvers
and both CPU references start from the same numbers.

FP64: the GPU state after steps 100, 200 and 1000 matches the oracle to
max relative error 1e-11 (floor 1 m, 1 m^2/s), as on the shorter cases.

FP32: the FP32 state is held against the FP64 oracle on depth.  A float
implementation cannot follow the double trajectory on this workload for its
whole length: one rounding can flip a wet/dry threshold at a front, and the
flip then spreads.  The test therefore also runs the oracle's binary32
instantiation (the same sub-steps with every operation correctly rounded to
float) as the rounding reference, and requires the GPU's FP32 depth error
against the FP64 oracle to stay within 1.5 times that reference's own error
at every checkpoint (measured on MI355X: 0.98, 1.00 and 1.03 times at steps
100, 200 and 1000; the GPU's FP32 path uses the hardware reciprocal and
square root, the reference correctly rounded ones).  It asserts the 1e-4
relative L1 bar where the float reference itself meets it: at 100 and 200
steps (5.4e-5 and 8.9e-5) but not at 1000 (5.5e-4), where no float
implementation meets it on this workload.  The pointwise error (floor
10 h_dry) is printed, not asserted: at a front a cell that is dry in one run
and wet in the other gives values of order 1e2 for the reference as for the
GPU.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1309_1230_amd import swe
from paper_1309_1230_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CHECKS = (100, 200, 1000)


def note(msg):
    print(f"[parity-long] {msg}", flush=True)


def as_f32(p):
    q = p.copy()
    for k in ("z", "n", "eta", "qx", "qy"):
        setattr(q, k, getattr(p, k).astype(np.float32).astype(np.float64))
    return q


def l1_rel(a, b):
    return float(np.abs(a - b).sum() / np.abs(b).sum())


def max_rel(a, b, floor):
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), floor)))


def snapshots(run, state):
    out, done = {}, 0
    for k in CHECKS:
        run(k - done)
        done = k
        out[k] = [a.copy() for a in state()]
    return out


@pytest.fixture(scope="module")
def reservoir512():
    p = as_f32(W.reservoir_release(nx=512, ny=512, dx=40.0, hills=200, seed=1001))
    note("oracle FP64: reservoir 512x512, dx=40 m, 1000 steps")
    o = O.State(p)
    snap = snapshots(lambda k: o.run(k), lambda: (o.eta, o.qx, o.qy))
    return p, snap


def gpu_snapshots(p, dtype):
    s = swe.Solver.from_problem(p, dtype=dtype)
    flags = []

    def run(k):
        flags.append(s.run(k).flags)

    snap = snapshots(run, lambda: [t.double().cpu().numpy() for t in (s.eta, s.qx, s.qy)])
    s.close()
    return snap, flags


def test_reservoir512_fp64_1000_steps_matches_oracle(reservoir512):
    p, ref = reservoir512
    note("GPU FP64: reservoir 512x512, 1000 steps")
    got, flags = gpu_snapshots(p, torch.float64)
    assert all(f & swe.FLAG_NAN == 0 for f in flags)
    for k in CHECKS:
        errs = [max_rel(a, b, 1.0) for a, b in zip(got[k], ref[k])]
        note(f"step {k}: max rel error eta/qx/qy {errs[0]:.2e} {errs[1]:.2e} {errs[2]:.2e}")
        assert max(errs) <= 1e-11, k


def test_reservoir512_fp32_1000_steps_within_float_envelope(reservoir512):
    p, ref = reservoir512
    note("GPU FP32 and the oracle's binary32 run: reservoir 512x512, 1000 steps")
    got, _ = gpu_snapshots(p, torch.float32)
    f = O.State(p, binary32=True)
    flt = snapshots(lambda k: f.run(k), lambda: (f.eta, f.qx, f.qy))
    floor = 10 * p.h_dry
    for k in CHECKS:
        h64 = ref[k][0] - p.z
        h_gpu = got[k][0] - p.z
        h_flt = flt[k][0] - p.z
        e_gpu, e_flt = l1_rel(h_gpu, h64), l1_rel(h_flt, h64)
        m_gpu, m_flt = max_rel(h_gpu, h64, floor), max_rel(h_flt, h64, floor)
        note(f"step {k}: depth vs FP64 oracle, L1 rel: GPU FP32 {e_gpu:.3e}, binary32 "
             f"reference {e_flt:.3e}; pointwise (floor 10 h_dry): GPU {m_gpu:.3e}, "
             f"reference {m_flt:.3e}; GPU FP32 vs reference L1 {l1_rel(h_gpu, h_flt):.3e}")
        assert e_gpu <= 1.5 * e_flt + 1e-7, k
        if e_flt <= 1e-4:
            assert e_gpu <= 1e-4, k
