"""The dry-tile skip of the fused step against the dense step.

With the skip on, a tile of the fused kernel whose cells and whose eight
neighbour tiles' cells were all dry after the previous step, and that lies at
least two cells from every edge, is not computed: the step maps such a tile
to itself.  The dense step is checked against the oracle elsewhere, so the
property tested here is bit equality of the two (fields and every reported
scalar: t, dt, volume, defect, lambda_max), over one call, over several calls
with the state edited in between, with an inflow boundary, in FP32 and FP64,
for single grids and ensembles (eager and graph replay); plus the exact count
of skipped cell updates on a domain that is dry everywhere.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import oracle as O
from paper_1309_1230_amd import swe
from paper_1309_1230_amd import workloads as W

KOUTW = 60   # output columns per tile of the fused kernel


def note(msg):
    print(f"[gpu-dry] {msg}", flush=True)


def dry_land_case(nx=720, ny=320, seed=5):
    """Reservoir released onto hills, with dry cells of every kind the skip
    must reproduce: h = 0 land, thin films 0 < h <= h_dry on a sloping bed
    (their pressure terms are not zero), a flat patch with z = eta = -0, and
    a still wet pond out on the dry land."""
    p = W.reservoir_release(nx=nx, ny=ny, dx=5.0, seed=seed)
    rng = np.random.default_rng(seed)
    film = (slice(ny // 5, ny // 2), slice(nx // 2, 3 * nx // 4))
    p.eta[film] = p.z[film] + rng.uniform(0.0, 0.9 * p.h_dry, p.z[film].shape)
    nz = (slice(3 * ny // 5, 3 * ny // 5 + 40), slice(nx // 2, nx // 2 + 70))
    p.z[nz] = -0.0
    p.eta[nz] = -0.0
    pond = (slice(ny - 60, ny - 40), slice(nx - 90, nx - 70))
    p.eta[pond] = p.z[pond].max() + 0.5
    return p


def fields(s):
    return [t.clone() for t in (s.eta, s.qx, s.qy)]


def same(a, b, what):
    for k, (x, y) in enumerate(zip(a, b)):
        assert torch.equal(x, y), (what, ("eta", "qx", "qy")[k],
                                   float((x - y).abs().max()))


def same_stats(a, b, what):
    for f in ("step", "steps", "t", "dt", "volume", "defect", "lambda_max", "dt_min", "dt_max"):
        assert getattr(a, f) == getattr(b, f), (what, f, getattr(a, f), getattr(b, f))


@pytest.mark.parametrize("dtype,tile_rows", [("f64", 16), ("f64", 0), ("f32", 16), ("f32", 32)])
def test_skip_is_bitwise_equal_to_dense(dtype, tile_rows):
    tdt = torch.float64 if dtype == "f64" else torch.float32
    p = dry_land_case()
    note(f"reservoir 720x320 {dtype} tile_rows={tile_rows}: 150 steps, skip vs dense")
    dense = swe.Solver.from_problem(p, dtype=tdt, tile_rows=tile_rows)
    skip = swe.Solver.from_problem(p, dtype=tdt, tile_rows=tile_rows, dry_skip=True)
    sd = dense.run(150)
    ss = skip.run(150)
    same(fields(skip), fields(dense), "one call")
    same_stats(ss, sd, "one call")
    assert sd.cells_skipped == 0
    frac = ss.cells_skipped / (150 * p.nx * p.ny)
    note(f"skipped fraction {frac:.3f}")
    assert frac > 0.2   # much of the land stays dry


def test_skip_across_calls_with_state_edits():
    p = dry_land_case(seed=9)
    note("reservoir 720x320 f64: calls of 7, 1, 13 steps, state edit, 30 steps")
    dense = swe.Solver.from_problem(p, tile_rows=16)
    skip = swe.Solver.from_problem(p, tile_rows=16, dry_skip=True)
    for k, n in enumerate((7, 1, 13)):
        if n == 1:
            dense.step()
            skip.step()
        else:
            sd = dense.run(n)
            ss = skip.run(n)
            same_stats(ss, sd, f"call {k}")
        same(fields(skip), fields(dense), f"call {k}")
    # pour water onto land that the skip has been leaving out: the next call
    # must see it (flags are rebuilt at the start of every call)
    for s in (dense, skip):
        s.eta[100:130, 430:460] += 3.0
        s.qx[100:130, 430:460] = 0.25
    sd = dense.run(30)
    ss = skip.run(30)
    same(fields(skip), fields(dense), "after edit")
    same_stats(ss, sd, "after edit")
    assert ss.cells_skipped > 0


def test_skip_with_inflow_boundary_matches_oracle():
    p = W.flood_scenario(3, 250, 190)
    note("flood scenario 250x190 f64 (inflow west): skip vs dense vs oracle, 200 steps")
    dense = swe.Solver.from_problem(p, tile_rows=16)
    skip = swe.Solver.from_problem(p, tile_rows=16, dry_skip=True)
    sd = dense.run(200)
    ss = skip.run(200)
    same(fields(skip), fields(dense), "flood")
    same_stats(ss, sd, "flood")
    assert ss.cells_skipped > 0
    o, _ = O.run(p, 200)
    for a, b in zip(fields(skip), (o.eta, o.qx, o.qy)):
        a = a.cpu().numpy()
        assert np.abs(a - b).max() / max(np.abs(b).max(), 1.0) <= 1e-11


def expected_skipped(nx, ny, H, nsteps):
    """Cell updates the skip leaves out on a domain dry everywhere: the first
    step of a call computes every tile; from the second on, every tile that
    is not an edge strip, not the first or last chunk, and at least two
    cells from the south and north edges is skipped."""
    gx, gy = (nx + KOUTW - 1) // KOUTW, (ny + H - 1) // H
    per_step = 0
    for s in range(gx):
        x0 = s * KOUTW
        if x0 - 2 <= 0 or x0 + 62 >= nx or s < 1 or s + 1 >= gx:
            continue
        for c in range(1, gy - 1):
            y0, y1 = c * H, min(c * H + H, ny)
            if H >= 2 and y0 >= 2 and y1 + 2 <= ny:
                per_step += (y1 - y0) * KOUTW
    return per_step * (nsteps - 1)


@pytest.mark.parametrize("nx,ny,H", [(481, 300, 16), (245, 130, 32), (600, 97, 16)])
def test_skipped_cell_count_on_a_dry_domain(nx, ny, H):
    rng = np.random.default_rng(nx + ny)
    z = W.gaussian_hills(nx, ny, 1.0, 1.0, rng, 12, (0.0, 3.0), (5.0, 40.0))
    p = W.Problem(nx=nx, ny=ny, dx=1.0, dy=1.0, z=z, n=np.full((ny, nx), 0.03), eta=z.copy(),
                  qx=np.zeros((ny, nx)), qy=np.zeros((ny, nx)), name="dry")
    note(f"dry {nx}x{ny} H={H}: skipped-cell count over 9 steps")
    s = swe.Solver.from_problem(p, tile_rows=H, dry_skip=True)
    st = s.run(9)
    assert st.cells_skipped == expected_skipped(nx, ny, H, 9)
    assert torch.equal(s.eta.cpu(), torch.as_tensor(p.eta))
    assert bool((s.qx == 0).all()) and bool((s.qy == 0).all())


def test_ensemble_skip_eager_and_graph():
    sizes = [(300, 200), (190, 256), (64, 64), (420, 130)]
    probs = [W.flood_scenario(k, nx, ny) for k, (nx, ny) in enumerate(sizes)]
    note("flood ensemble of 4 f32: skip vs dense, 40 eager steps, 2 x 40-step graph replays")
    dense = swe.Ensemble.from_problems(probs, dtype=torch.float32, tile_rows=16)
    skip = swe.Ensemble.from_problems(probs, dtype=torch.float32, tile_rows=16, dry_skip=True)
    dense.run(40)
    skip.run(40)
    a, b = dense.stats(), skip.stats()
    for k in range(len(probs)):
        same(skip.fields[k], dense.fields[k], f"eager {k}")
        same_stats(b[k], a[k], f"eager {k}")
    assert sum(x.cells_skipped for x in b) > 0
    dense.capture(40)
    skip.capture(40)
    for r in range(2):
        dense.replay()
        skip.replay()
        a, b = dense.stats(), skip.stats()
        for k in range(len(probs)):
            same(skip.fields[k], dense.fields[k], f"replay {r} scenario {k}")
            assert a[k].t == b[k].t and a[k].volume == b[k].volume
    dense.close()
    skip.close()
