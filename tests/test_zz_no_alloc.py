"""swe_run_noalloc (the entry point for callers that cannot allocate device
memory) against swe_create + swe_run on the same inputs: two calls in a
row, the second on a smaller grid, so that the second call runs on the
static scratch the first one left behind.  Same kernels, so the states and
the statistics must agree bit for bit."""
import math

import numpy as np
import pytest

from paper_1309_1230_amd import swe
from paper_1309_1230_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def note(msg):
    print(f"[no-alloc] {msg}", flush=True)


def upload(p, dtype):
    t = lambda a: torch.as_tensor(a, dtype=torch.float64).to(device="cuda", dtype=dtype).contiguous()
    return [t(a) for a in (p.z, p.n, p.eta, p.qx, p.qy)]


def kwargs(p):
    return dict(dx=p.dx, dy=p.dy, g=p.g, cfl=p.cfl, h_dry=p.h_dry, kappa=p.kappa,
                eps_max=p.eps_max, dt_max=p.dt_max, dt_fixed=p.dt_fixed, bc=p.bc,
                inflow_lo=p.inflow_lo, inflow_hi=p.inflow_hi, hydro_t=p.hydro_t,
                hydro_q=p.hydro_q)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_matches_create_run_twice(dtype):
    tdt = torch.float64 if dtype == "f64" else torch.float32
    p1 = W.inflow_channel(300, 200, seed=3, q_peak=2.0, dry=True, t_peak=10.0, t_end=30.0)
    p1.inflow_lo = (20, 0, 0, 0)
    p1.inflow_hi = (120, 200, 300, 300)
    p2 = W.reservoir_release(nx=150, ny=90, dx=80.0, hills=20, seed=1001)
    for k, (p, nsteps) in enumerate(((p1, 37), (p2, 24))):
        note(f"call {k + 1}: {p.name} {p.nx}x{p.ny} {dtype}, {nsteps} steps")
        z, n, eta, qx, qy = upload(p, tdt)
        st = swe.run_noalloc(z, n, eta, qx, qy, nsteps, **kwargs(p))
        ref = swe.Solver.from_problem(p, dtype=tdt)
        rs = ref.run(nsteps)
        for a, b in ((eta, ref.eta), (qx, ref.qx), (qy, ref.qy)):
            assert torch.equal(a, b)
        assert st.steps == rs.steps == nsteps and st.step == rs.step
        assert st.t == rs.t and st.dt == rs.dt and st.flags == rs.flags
        assert st.volume == rs.volume and st.defect == rs.defect
        assert st.lambda_max == rs.lambda_max
        ref.close()


def test_noalloc_rejects_grids_beyond_its_limit():
    p = W.smooth_wet(1100, 1000, seed=1)
    z, n, eta, qx, qy = upload(p, torch.float64)
    with pytest.raises(swe.SweError) as ei:
        swe.run_noalloc(z, n, eta, qx, qy, 1, **kwargs(p))
    assert ei.value.code == swe.SWE_EINVAL
    assert "too large" in str(ei.value)
