"""Ensemble launches against single-grid runs and the oracle.

An ensemble step is one launch of the fused step kernel over the tiles of
every scenario, each scenario with its own arguments, control block and
time step.  Since the fused step's result does not depend on tiling, every
scenario of an ensemble must reproduce, bit for bit, the same scenario run
alone through the single-grid library, which is itself checked against the
oracle (FP64 to 1e-11, FP32 by tolerance).
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import oracle as O
from paper_1309_1230_amd import swe
from paper_1309_1230_amd import workloads as W


def note(msg):
    print(f"[gpu-ensemble] {msg}", flush=True)


def scenarios(sizes, dry=True):
    out = []
    for k, (nx, ny) in enumerate(sizes):
        p = W.flood_scenario(k, nx, ny)
        if not dry:
            p.eta = p.z + 0.3
        out.append(p)
    return out


SIZES = [(64, 64), (65, 70), (127, 64), (300, 97), (61, 250), (200, 129), (1024, 80), (96, 512)]


def alone(p, dtype, nsteps, t_end=math.inf):
    s = swe.Solver.from_problem(p, dtype=dtype)
    st = s.run(nsteps, t_end)
    return s, st


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_ensemble_equals_single_grid_runs(dtype):
    tdt = torch.float32 if dtype == "f32" else torch.float64
    probs = scenarios(SIZES, dry=False)
    note(f"{len(probs)} scenarios {dtype}, 60 steps, tile rows 32")
    e = swe.Ensemble.from_problems(probs, dtype=tdt, tile_rows=32)
    e.run(60)
    est = e.stats()
    for k, p in enumerate(probs):
        s, st = alone(p, tdt, 60)
        for a, b in zip(e.fields[k], (s.eta, s.qx, s.qy)):
            assert torch.equal(a, b), (k, p.name)
        assert est[k].t == st.t and est[k].dt == st.dt and est[k].step == st.step == 60
    e.close()


def test_ensemble_fp64_scenario_matches_oracle():
    p = scenarios([(90, 50)], dry=False)[0]
    note("FP64 ensemble scenario vs oracle, 80 steps")
    e = swe.Ensemble.from_problems([p, scenarios([(70, 66)])[0]], dtype=torch.float64,
                                   tile_rows=16)
    e.run(80)
    e.stats()
    o, _ = O.run(p, 80)
    for a, b in zip(e.fields[0], (o.eta, o.qx, o.qy)):
        a = a.cpu().numpy()
        err = np.abs(a - b).max() / max(np.abs(b).max(), 1.0)
        assert err <= 1e-11


def test_scenarios_keep_their_own_time_steps_and_stop_independently():
    probs = scenarios(SIZES[:5], dry=False)
    note("independent stops at t_end = 3 s")
    e = swe.Ensemble.from_problems(probs, dtype=torch.float64, tile_rows=16)
    e.run(400, t_end=3.0)
    est = e.stats()
    steps = set()
    for k, p in enumerate(probs):
        s, st = alone(p, torch.float64, 400, t_end=3.0)
        assert est[k].step == st.step and est[k].t == st.t and est[k].t >= 3.0
        steps.add(st.step)
        for a, b in zip(e.fields[k], (s.eta, s.qx, s.qy)):
            assert torch.equal(a, b)
    assert len(steps) > 1   # the scenarios really took different numbers of steps


def test_graph_replay_equals_eager_run():
    probs = scenarios(SIZES[:6])
    note("graph of 20 steps replayed 3 times vs eager 60 steps")
    g = swe.Ensemble.from_problems(probs, dtype=torch.float32, tile_rows=32)
    g.capture(20)
    for _ in range(3):
        g.replay()
        g.stats()          # eager host work and a synchronisation between replays
    gst = g.stats()
    e = swe.Ensemble.from_problems(probs, dtype=torch.float32, tile_rows=32)
    e.run(60)
    est = e.stats()
    for k in range(len(probs)):
        for a, b in zip(g.fields[k], e.fields[k]):
            assert torch.equal(a, b)
        assert gst[k].t == est[k].t and gst[k].step == est[k].step == 60


def test_autotuner_picks_a_candidate_and_keeps_the_state():
    probs = scenarios(SIZES[:4])
    note("autotuned tile rows")
    e = swe.Ensemble.from_problems(probs, dtype=torch.float32, tile_rows=0)
    assert e.tile_rows in (16, 32, 64, 128)
    st = e.stats()
    assert all(x.step == 0 and x.t == 0.0 for x in st)
    for k, p in enumerate(probs):
        assert torch.equal(e.fields[k][0].cpu().double(), torch.as_tensor(p.eta).float().double())
    e.run(10)
    e.stats()


def test_ensemble_rejects_mixed_dtypes():
    a = scenarios([(64, 64)])[0]
    t32 = lambda x: torch.as_tensor(x, dtype=torch.float32, device="cuda").contiguous()
    t64 = lambda x: torch.as_tensor(x, dtype=torch.float64, device="cuda").contiguous()
    kw = swe._problem_kwargs(a)
    note("mixed dtypes rejected")
    with pytest.raises(swe.SweError) as ei:
        swe.Ensemble([(t32(a.z), t32(a.n), t32(a.eta), t32(a.qx), t32(a.qy), kw),
                      (t64(a.z), t64(a.n), t64(a.eta), t64(a.qx), t64(a.qy), kw)], tile_rows=16)
    assert ei.value.code == swe.SWE_EINVAL
