"""GPU discrete adjoint (swe_grad) against the oracle's reverse-mode gradient.

The loss is the gauge-misfit sum over observation steps with the time steps
of the run held fixed.  The FP64 forward run is bit-identical to the
oracle's, so both differentiate the same discrete trajectory; they differ
only in the rounding of the derivative arithmetic, accumulated over the
steps.  Tolerance: 1e-9 of the gradient's largest entry (the CPU pins show
the two oracle modes agree to 1e-12 and finite differences to 1e-9).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import oracle as O
from paper_1309_1230_amd import swe
from paper_1309_1230_amd import workloads as W


def note(msg):
    print(f"[gpu-adjoint] {msg}", flush=True)


def gauges_for(p, nsteps, every, ncell, seed, noise=0.01, cells=None):
    rng = np.random.default_rng(seed)
    _, dts = O.run_record(p, nsteps)
    if cells is None:
        cells = rng.choice(p.nx * p.ny, ncell, replace=False)
    hobs = np.zeros((nsteps // every, len(cells)))
    st = O.State(p)
    for k in range(nsteps // every):
        st.run(every)
        hobs[k] = (st.eta - p.z).ravel()[cells] + rng.normal(0.0, noise, len(cells))
    return O.Gauges(cells=np.asarray(cells), every=every, hobs=hobs, dts=dts)


def gpu_grad(p, G, nsteps, ckpt):
    s = swe.Solver.from_problem(p, dtype=torch.float64)
    hobs = torch.as_tensor(G.hobs, dtype=torch.float64, device="cuda")
    J, gn, gz = s.grad(nsteps, G.cells, G.every, hobs, ckpt)
    out = (J, gn.cpu().numpy(), gz.cpu().numpy(), s)
    return out


def prep(name):
    if name == "smooth":
        return W.smooth_wet(48, 36, seed=9)
    if name == "random":
        return W.random_valid_state(45, 33, seed=21)
    p = W.inflow_channel(40, 18, seed=3, q_peak=2.0, dry=True, t_peak=2.0, t_end=6.0)
    p.inflow_lo = (3, 0, 0, 0)
    p.inflow_hi = (14, 18, 40, 40)
    return p


@pytest.mark.parametrize("name", ["smooth", "random", "inflow"])
def test_gradient_matches_oracle(name):
    p = prep(name)
    nsteps, every = 24, 4
    G = gauges_for(p, nsteps, every, 15, seed=5)
    note(f"{name} {p.nx}x{p.ny}: {nsteps} steps, adjoint vs oracle")
    J, gn, gz, s = gpu_grad(p, G, nsteps, 7)
    Jo, gno, gzo = O.loss_gradient(p, G)
    assert J == pytest.approx(Jo, rel=1e-13)
    scale_n = np.abs(gno).max()
    scale_z = np.abs(gzo).max()
    assert scale_n > 0 and scale_z > 0
    en = np.abs(gn - gno).max() / scale_n
    ez = np.abs(gz - gzo).max() / scale_z
    note(f"max err / max |grad|: n {en:.2e}, z {ez:.2e}")
    assert en <= 1e-9 and ez <= 1e-9


def test_checkpoint_spacing_does_not_change_the_gradient():
    p = prep("random")
    G = gauges_for(p, 20, 5, 10, seed=6)
    note("checkpoint spacing 1, 6, 20")
    outs = [gpu_grad(p, G, 20, c) for c in (1, 6, 20)]
    for o in outs[1:]:
        assert o[0] == outs[0][0]
        assert np.array_equal(o[1], outs[0][1]) and np.array_equal(o[2], outs[0][2])


def test_kept_traces_and_replay_give_the_same_gradient(monkeypatch):
    p = prep("inflow")
    G = gauges_for(p, 20, 4, 10, seed=9)
    note("segment traces kept vs replayed per step")
    a = gpu_grad(p, G, 20, 6)
    monkeypatch.setenv("SWE_GRAD_KEEP", "0")
    b = gpu_grad(p, G, 20, 6)
    assert a[0] == b[0]
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


def test_state_after_grad_equals_run():
    p = prep("smooth")
    G = gauges_for(p, 12, 3, 6, seed=7)
    note("state after swe_grad vs swe_run")
    _, _, _, s = gpu_grad(p, G, 12, 5)
    r = swe.Solver.from_problem(p, dtype=torch.float64)
    r.run(12)
    for a, b in ((s.eta, r.eta), (s.qx, r.qx), (s.qy, r.qy)):
        assert torch.equal(a, b)
    assert s.stats().step == r.stats().step == 12


def test_lake_at_rest_closed_form_on_gpu():
    p = W.lake_at_rest(40, 30, seed=8, dry_banks=True)
    h0 = (p.eta - p.z).ravel()
    wet = np.flatnonzero(h0 > 10 * p.h_dry)
    cells = np.random.default_rng(5).choice(wet, 12, replace=False)
    G = gauges_for(p, 24, 6, 12, seed=6, noise=0.05, cells=cells)
    note("lake at rest closed-form gradient")
    J, gn, gz, _ = gpu_grad(p, G, 24, 8)
    assert np.all(gn == 0.0)
    expect = np.zeros(p.nx * p.ny)
    for k in range(G.hobs.shape[0]):
        np.add.at(expect, cells, -2.0 * (h0[cells] - G.hobs[k]))
    np.testing.assert_allclose(gz.ravel(), expect, rtol=1e-13, atol=1e-15)


def test_autograd_function_matches_solver_grad():
    p = prep("smooth")
    G = gauges_for(p, 12, 4, 8, seed=8)
    note("SweLoss autograd")
    t = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda").contiguous()
    n = t(p.n).requires_grad_(True)
    z = t(p.z).requires_grad_(True)
    kw = dict(dx=p.dx, dy=p.dy, g=p.g, cfl=p.cfl, h_dry=p.h_dry, kappa=p.kappa,
              eps_max=p.eps_max, dt_max=p.dt_max, dt_fixed=p.dt_fixed, bc=p.bc,
              inflow_lo=p.inflow_lo, inflow_hi=p.inflow_hi, hydro_t=p.hydro_t, hydro_q=p.hydro_q)
    hobs = t(G.hobs)
    J = swe.SweLoss().apply(n, z, t(p.eta), t(p.qx), t(p.qy), kw, 12, G.cells, G.every, hobs, 5)
    (3.0 * J).backward()
    Jr, gn, gz, _ = gpu_grad(p, G, 12, 5)
    assert float(J.detach()) == Jr
    assert torch.equal(n.grad, 3.0 * torch.as_tensor(gn, device="cuda"))
    assert torch.equal(z.grad, 3.0 * torch.as_tensor(gz, device="cuda"))


def test_grad_rejects_bad_gauges():
    p = prep("smooth")
    note("swe_grad argument errors")
    s64 = swe.Solver.from_problem(p, dtype=torch.float64)
    hobs = torch.zeros(2, 2, dtype=torch.float64, device="cuda")
    for cells in ([3, 3], [1, p.nx * p.ny]):
        with pytest.raises(swe.SweError) as ei:
            s64.grad(4, cells, 2, hobs)
        assert ei.value.code == swe.SWE_EINVAL


# ---- FP32 forward, FP64 reverse sweep (linearised at the promoted FP32 states)

def gpu_grad32(p, G, nsteps, ckpt):
    s = swe.Solver.from_problem(p, dtype=torch.float32)
    hobs = torch.as_tensor(G.hobs, dtype=torch.float64, device="cuda")
    J, gn, gz = s.grad(nsteps, G.cells, G.every, hobs, ckpt)
    assert gn.dtype == torch.float64 and gz.dtype == torch.float64
    return J, gn.cpu().numpy(), gz.cpu().numpy(), s


def test_mixed_lake_at_rest_closed_form():
    p = W.lake_at_rest(40, 30, seed=8, dry_banks=True)
    e32 = p.eta.astype(np.float32).astype(np.float64)
    z32 = p.z.astype(np.float32).astype(np.float64)
    h0 = (e32 - z32).ravel()
    wet = np.flatnonzero(h0 > 10 * p.h_dry)
    cells = np.random.default_rng(5).choice(wet, 12, replace=False)
    G = gauges_for(p, 24, 6, 12, seed=6, noise=0.05, cells=cells)
    note("FP32 forward / FP64 adjoint: lake at rest closed form")
    J, gn, gz, s = gpu_grad32(p, G, 24, 8)
    assert np.all(gn == 0.0)
    expect = np.zeros(p.nx * p.ny)
    for k in range(G.hobs.shape[0]):
        np.add.at(expect, cells, -2.0 * (h0[cells] - G.hobs[k]))
    np.testing.assert_allclose(gz.ravel(), expect, rtol=1e-13, atol=1e-15)
    assert J == pytest.approx(float(((h0[cells][None, :] - G.hobs) ** 2).sum()), rel=1e-13)


@pytest.mark.parametrize("name", ["smooth", "inflow"])
def test_mixed_gradient_close_to_fp64(name):
    """The FP32 trajectory differs from the FP64 one by FP32 rounding, so the
    two gradients agree to that order (1e-3 of the largest entry), not bitwise;
    the FP64 one is itself pinned to the oracle."""
    p = prep(name)
    G = gauges_for(p, 24, 4, 15, seed=5)
    note(f"{name}: FP32-forward gradient vs FP64 gradient")
    J32, gn32, gz32, _ = gpu_grad32(p, G, 24, 7)
    J64, gn64, gz64, _ = gpu_grad(p, G, 24, 7)
    assert J32 == pytest.approx(J64, rel=1e-3)
    en = np.abs(gn32 - gn64).max() / np.abs(gn64).max()
    ez = np.abs(gz32 - gz64).max() / np.abs(gz64).max()
    note(f"max diff / max |grad|: n {en:.2e}, z {ez:.2e}")
    assert en <= 1e-3 and ez <= 1e-3


def test_mixed_state_and_checkpoint_spacing():
    p = prep("random")
    G = gauges_for(p, 20, 5, 10, seed=6)
    note("FP32 forward: state after grad equals run; checkpoint spacing 1, 6, 20")
    outs = [gpu_grad32(p, G, 20, c) for c in (1, 6, 20)]
    for o in outs[1:]:
        assert o[0] == outs[0][0]
        assert np.array_equal(o[1], outs[0][1]) and np.array_equal(o[2], outs[0][2])
    r = swe.Solver.from_problem(p, dtype=torch.float32)
    r.run(20)
    s = outs[0][3]
    for a, b in ((s.eta, r.eta), (s.qx, r.qx), (s.qy, r.qy)):
        assert torch.equal(a, b)


@pytest.mark.parametrize("name,nx,ny,nsteps", [("smooth", 64, 64, 60), ("random", 64, 64, 60),
                                               ("smooth", 128, 128, 100),
                                               ("random", 128, 128, 100)])
def test_gradient_matches_oracle_elementwise(name, nx, ny, nsteps):
    """64 x 64 and 128 x 128, up to 100 steps: every entry of both gradients
    against the oracle's reverse-mode gradient, relative to the entry itself
    with a floor of 1e-6 of the largest entry (below that, an entry is a sum
    of cancelling terms whose rounding is not its own size), at most 1e-10."""
    if name == "smooth":
        p = W.smooth_wet(nx, ny, seed=9)
    else:
        p = W.random_valid_state(nx, ny, seed=21)
    every = 4
    G = gauges_for(p, nsteps, every, 24, seed=5)
    note(f"{name} {nx}x{ny}: {nsteps} steps, elementwise adjoint vs oracle")
    J, gn, gz, _ = gpu_grad(p, G, nsteps, 10)
    Jo, gno, gzo = O.loss_gradient(p, G)
    assert J == pytest.approx(Jo, rel=1e-13)
    for nm, a, b in (("dJ/dn", gn, gno), ("dJ/dz", gz, gzo)):
        floor = 1e-6 * np.abs(b).max()
        err = np.abs(a - b) / np.maximum(np.abs(b), floor)
        note(f"{nm}: max elementwise rel error {err.max():.2e} (floor {floor:.2e}), "
             f"max err / max |grad| {np.abs(a - b).max() / np.abs(b).max():.2e}")
        assert err.max() <= 1e-10, nm


def test_loss_alone_equals_grad_loss_and_advances_like_run():
    """swe_loss: the same J as swe_grad (same misfits, same order) from one
    forward run, and the handle's state advances exactly as swe_run's."""
    p = prep("inflow")
    G = gauges_for(p, 20, 4, 10, seed=9)
    note("swe_loss vs swe_grad's loss")
    hobs = torch.as_tensor(G.hobs, dtype=torch.float64, device="cuda")
    for dtype in (torch.float64, torch.float32):
        a = swe.Solver.from_problem(p, dtype=dtype)
        J = a.loss(20, G.cells, G.every, hobs)
        b = swe.Solver.from_problem(p, dtype=dtype)
        Jg, _, _ = b.grad(20, G.cells, G.every, hobs, 6)
        r = swe.Solver.from_problem(p, dtype=dtype)
        r.run(20)
        assert J == Jg
        for x, y in ((a.eta, r.eta), (a.qx, r.qx), (a.qy, r.qy)):
            assert torch.equal(x, y)
        for s in (a, b, r):
            s.close()
