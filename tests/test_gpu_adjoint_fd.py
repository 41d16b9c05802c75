"""Central finite differences of the GPU gradient on the Manning calibration
workload at its full size: 1024 x 1024, dx = 2 m, FP64, 2000 steps, 64
gauges observed every 10 steps, gradient with respect to the Manning field
at the first guess n = 0.05, checkpoint every 45 steps.

swe_grad differentiates the discrete step with the run's time steps held
fixed (dt comes from a CFL maximum, which is not differentiated), so each
perturbed forward run replays the unperturbed run's time steps through
swe_run_dt; otherwise the difference quotient would also contain the
sensitivity of dt.  The loss of a perturbed run is formed from the gauge
depths the GPU run produces, in FP64.

The loss is only piecewise smooth: the switch's |d2 eta|, the max and min of
the dissipation coefficient and the wet tests put kinks into it, and over
2000 steps of a million cells some fall within any difference step.  A step
sweep on MI355X (1e-3 n down to 1e-7 n, eight cells) gave: truncation and
kink crossings dominate above 1e-5 n (errors 1e-4 and more at 1e-4 n),
rounding noise below it (errors 1e-5 to 5e-4 at 1e-7 n), and at 1e-5 n the
central difference agrees with the adjoint to 1e-7 .. 1.1e-5 wherever the
loss is smooth at that scale; at one cell the forward and backward quotients
differed by a factor three (a kink at the evaluation point), and only
shrinking the step to 1e-7 n brought the difference to 4e-4 of the adjoint.
So the step is 1e-5 n, and a cell counts as smooth when its forward and
backward quotients agree to 1e-3 of the adjoint (a smooth loss gives
spreads of 1e-5 .. 1e-4 at this step).  Bar: on 20 random cells whose
derivative is at least 1e-3 of the largest, at most two are kinked, every
smooth cell agrees within 2e-5 and their median within 1e-5.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1309_1230_amd import swe
from paper_1309_1230_amd import workloads as W


def note(msg):
    print(f"[gpu-adjoint-fd] {msg}", flush=True)


def gauge_depths(s, cells_t, zc):
    return s.eta.reshape(-1)[cells_t] - zc


def observe(p, n, cells, every, nsteps):
    """Gauge depths of an adaptive run of p with Manning field n."""
    q = p.copy()
    q.n = n
    s = swe.Solver.from_problem(q, dtype=torch.float64)
    cells_t = torch.as_tensor(cells, device="cuda")
    zc = s.z.reshape(-1)[cells_t]
    obs = []
    for _ in range(nsteps // every):
        s.run(every)
        obs.append(gauge_depths(s, cells_t, zc))
    s.close()
    return torch.stack(obs).contiguous()


def loss_on_grid(p, n, cells, every, hobs, dts):
    """J of a run of p with Manning field n on the prescribed time grid dts."""
    q = p.copy()
    q.n = n
    s = swe.Solver.from_problem(q, dtype=torch.float64)
    cells_t = torch.as_tensor(cells, device="cuda")
    zc = s.z.reshape(-1)[cells_t]
    J = torch.zeros((), dtype=torch.float64, device="cuda")
    for k in range(len(dts) // every):
        s.run_dt(dts[k * every:(k + 1) * every])
        d = gauge_depths(s, cells_t, zc) - hobs[k]
        J = J + (d * d).sum()
    s.close()
    return float(J)


def test_calibration_gradient_matches_central_differences():
    c = W.calibration()
    p = c.problem
    nsteps, every = c.nsteps, c.obs_every
    note(f"{p.nx}x{p.ny}, {nsteps} steps: observations from the true field")
    hobs = observe(p, c.n_true, c.cells, every, nsteps)
    note("time steps of the first-guess run")
    s = swe.Solver.from_problem(p, dtype=torch.float64)
    dts = np.array([s.step() for _ in range(nsteps)])
    s.close()
    note(f"swe_grad, checkpoint every 45 (dt in [{dts.min():.4f}, {dts.max():.4f}] s)")
    g = swe.Solver.from_problem(p, dtype=torch.float64)
    J, gn, _ = g.grad(nsteps, c.cells, every, hobs, 45)
    g.close()
    gn = gn.cpu().numpy()
    J0 = loss_on_grid(p, p.n, c.cells, every, hobs, dts)
    note(f"J = {J:.10e}, replayed J = {J0:.10e}")
    # same depths, summed in another order
    assert J0 == pytest.approx(J, rel=1e-12), "the replayed time grid must reproduce the run"
    big = np.flatnonzero(np.abs(gn).ravel() >= 1e-3 * np.abs(gn).max())
    rng = np.random.default_rng(2024)
    cells = rng.choice(big, 20, replace=False)
    errs, kinks = [], 0
    for cell in cells:
        j, i = divmod(int(cell), p.nx)
        delta = 1e-5 * p.n[j, i]
        npl = p.n.copy()
        nmi = p.n.copy()
        npl[j, i] += delta
        nmi[j, i] -= delta
        Jp = loss_on_grid(p, npl, c.cells, every, hobs, dts)
        Jm = loss_on_grid(p, nmi, c.cells, every, hobs, dts)
        fd = (Jp - Jm) / (npl[j, i] - nmi[j, i])
        fwd = (Jp - J0) / (npl[j, i] - p.n[j, i])
        bwd = (J0 - Jm) / (p.n[j, i] - nmi[j, i])
        rel = abs(fd - gn[j, i]) / abs(gn[j, i])
        spread = abs(fwd - bwd) / abs(gn[j, i])
        kinked = spread > 1e-3
        kinks += kinked
        if not kinked:
            errs.append(rel)
        note(f"cell ({i},{j}): adjoint {gn[j, i]:+.10e}  central difference {fd:+.10e}  "
             f"rel {rel:.2e}  one-sided spread {spread:.2e}{'  (kink)' if kinked else ''}")
    errs = np.array(errs)
    note(f"smooth cells {len(errs)}: max rel error {errs.max():.2e}, median {np.median(errs):.2e}; "
         f"kinked cells {kinks}")
    assert kinks <= 2
    assert errs.max() <= 2e-5 and np.median(errs) <= 1e-5
