"""Forward-step throughput of the MI355X shallow-water library.

Workload: the reservoir release on seeded synthetic terrain, 4096 x 4096
cells, dx = 5 m (200 Gaussian hills 0-20 m high, sigma 50-400 m, plus 1/f
noise of amplitude 1 m; water surface at 25 m behind x = 0.2 L, dry land
elsewhere with h_dry = 1e-3 m; uniform Manning n = 0.035; open east edge),
1000 adaptive time steps.  One "step" is one full MacCormack time step
(all sixteen sub-steps, one fused kernel launch) over the whole grid, with
the state already resident in HBM.

Prints one JSON line: cell-updates/s, the roofline of the fused step kernel
(algorithmic bytes 64 B/cell-update in FP64, 32 B in FP32, over the kernel's
average duration from HIP events on its stream, against 8 TB/s HBM), the
the same run with the dry-tile skip (dense-equivalent and active cell-update
rates), the adjoint/forward cost ratio on the 1024 x 1024 Manning calibration
workload, the flood-ensemble throughput (256 scenarios in one launch per step, graph
replay) against one-grid-at-a-time runs, and the CPU oracle timed on a
bounded sample of the reservoir workload.

    python bench.py [--steps K] [--warmup W] [--dtype f64|f32]
"""
import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "cell-updates/s and % HBM peak (fwd)"
KERNEL_SOURCES = ("paper_1309_1230_amd/csrc/swe_fused.hip", "paper_1309_1230_amd/csrc/swe_common.hpp")
TRAFFIC_PROFILE = "profiles/fused_step_reservoir4096_traffic.txt"


def kernel_source_hash():
    """SHA-1 of the fused kernel's sources: a traffic figure measured on other
    sources no longer describes the kernel and is reported as null."""
    import hashlib
    h = hashlib.sha1()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(dtype):
    """HBM bytes per launch of the fused step from the committed rocprofv3
    FETCH_SIZE/WRITE_SIZE summary, or None when it was taken on other kernel
    sources (or is absent)."""
    path = os.path.join(ROOT, TRAFFIC_PROFILE)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            parts = line.split()
            if len(parts) == 2 and not line.startswith("#"):
                vals[parts[0]] = parts[1]
    if vals.get("source_sha1") != kernel_source_hash():
        return None
    v = vals.get(f"{dtype}_traffic_bytes_per_launch")
    return float(v) if v is not None else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--dtype", choices=["f64", "f32"], default="f64")
    ap.add_argument("--tile-rows", type=int, default=0)
    ap.add_argument("--nx", type=int, default=4096)
    ap.add_argument("--cpu-steps", type=int, default=12,
                    help="oracle steps timed for the CPU baseline (0: skip)")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the other-precision and unfused comparison runs")
    ap.add_argument("--print-source-hash", action="store_true",
                    help="print the fused kernel's source hash and exit")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint/forward cost ratio on the calibration workload")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="run only the adjoint measurement (for profiling)")
    ap.add_argument("--adj-nx", type=int, default=1024)
    ap.add_argument("--adj-steps", type=int, default=2000)
    ap.add_argument("--adj-ckpt", type=int, default=45,
                    help="checkpoint spacing of swe_grad (the calibration run's 45); the "
                         "kept-trajectory mode is timed beside it")
    ap.add_argument("--adj-fd-cells", type=int, default=20,
                    help="cells of the finite-difference check of the gradient (0: skip)")
    ap.add_argument("--no-ensemble", action="store_true",
                    help="skip the flood-ensemble throughput measurement")
    ap.add_argument("--ensemble-only", action="store_true",
                    help="run only the ensemble measurement (for profiling)")
    ap.add_argument("--ens-count", type=int, default=256)
    ap.add_argument("--ens-steps", type=int, default=500)
    ap.add_argument("--no-dry-skip", action="store_true",
                    help="skip the dry-tile-skip measurement of the reservoir workload")
    ap.add_argument("--dry-only", action="store_true",
                    help="run only the dense and dry-skip reservoir runs (for profiling)")
    ap.add_argument("--combined", action="store_true",
                    help="run only the large combined run: FP32 forward and FP64 adjoint of the "
                         "channel flood (8192 x 8192 by default; several minutes)")
    ap.add_argument("--comb-nx", type=int, default=8192)
    ap.add_argument("--comb-steps", type=int, default=5000)
    ap.add_argument("--comb-ckpt", type=int, default=0, help="0: round(sqrt(steps))")
    ap.add_argument("--comb-obs-every", type=int, default=50)
    ap.add_argument("--comb-h-film", type=float, default=0.1,
                    help="depth floor of the dissipation switch for the combined run (0: plain)")
    ap.add_argument("--probe-copy-mb", type=int, default=0,
                    help="also run the library's plain copy kernel once over this many MiB "
                         "(calibrates HBM traffic counters)")
    return ap.parse_args()


def bytes_per_cell(dtype):
    # read eta, qx, qy, z, m; write eta, qx, qy
    return 8 * (8 if dtype == "f64" else 4)


def timed_run(torch, swe, W, p, dtype, steps, warmup, tile_rows, path="fused", dry_skip=False):
    tdt = torch.float64 if dtype == "f64" else torch.float32
    if warmup > 0:
        w = swe.Solver.from_problem(p, dtype=tdt, path=path, tile_rows=tile_rows,
                                    dry_skip=dry_skip)
        w.run(warmup)
        w.close()
        del w
    s = swe.Solver.from_problem(p, dtype=tdt, path=path, tile_rows=tile_rows, dry_skip=dry_skip)
    stream = torch.cuda.current_stream()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    st = s.run(steps)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(stop)
    s.close()
    return st, ms, wall


def progress(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def fd_check(torch, swe, p, cells, every, hobs, dts, gn, ncell=20, rel_step=1e-5):
    """Central differences of the loss on the run's time grid (swe_run_dt) at
    ncell random cells whose derivative is at least 1e-3 of the largest, step
    rel_step * n.  A cell whose forward and backward quotients differ by more
    than 1e-3 of the adjoint sits on a kink of the piecewise smooth loss and
    is counted apart."""
    import numpy as np
    cells_t = torch.as_tensor(cells, device="cuda")

    def loss(nfield):
        q = p.copy()
        q.n = nfield
        s = swe.Solver.from_problem(q, dtype=torch.float64)
        zc = s.z.reshape(-1)[cells_t]
        J = torch.zeros((), dtype=torch.float64, device="cuda")
        for k in range(len(dts) // every):
            s.run_dt(dts[k * every:(k + 1) * every])
            d = s.eta.reshape(-1)[cells_t] - zc - hobs[k]
            J = J + (d * d).sum()
        s.close()
        return float(J)

    g = gn.cpu().numpy()
    big = np.flatnonzero(np.abs(g).ravel() >= 1e-3 * np.abs(g).max())
    pick = np.random.default_rng(2024).choice(big, min(ncell, big.size), replace=False)
    J0 = loss(p.n)
    errs, kinks = [], 0
    for cell in pick:
        j, i = divmod(int(cell), p.nx)
        d = rel_step * p.n[j, i]
        a, b = p.n.copy(), p.n.copy()
        a[j, i] += d
        b[j, i] -= d
        Jp, Jm = loss(a), loss(b)
        fd = (Jp - Jm) / (a[j, i] - b[j, i])
        spread = abs((Jp - J0) / (a[j, i] - p.n[j, i]) - (J0 - Jm) / (p.n[j, i] - b[j, i]))
        if spread > 1e-3 * abs(g[j, i]):
            kinks += 1
        else:
            errs.append(abs(fd - g[j, i]) / abs(g[j, i]))
    return {"cells": len(pick), "step_rel": rel_step, "smooth_cells": len(errs),
            "kinked_cells": kinks, "max_rel_err_smooth": max(errs) if errs else None,
            "median_rel_err_smooth": float(np.median(errs)) if errs else None}


def adjoint_ratio(torch, swe, W, nx, nsteps, ckpt, fd_cells):
    """Cost of the discrete adjoint against the forward run on the Manning
    calibration workload: synthetic gauge observations from the true field,
    then (a) the forward run at the first guess, timed, and (b) swe_grad of
    the misfit loss over the same run, timed on a fresh solver, with a
    checkpoint every ckpt steps (45 for the calibration run: about
    sqrt(2000); forward, segment recompute, reverse sweep).  The mode that
    keeps the whole FP64 trajectory in device memory (no recompute) is timed
    beside it as a variant and its gradient compared bit for bit.  fd_cells
    > 0: central differences of the loss at that many cells (fd_check)."""
    c = W.calibration(nx=nx, ny=nx, nsteps=nsteps)
    p = c.problem
    progress(f"adjoint: {p.nx}x{p.ny} calibration, {nsteps} steps, checkpoint every {ckpt}")
    truth = p.copy()
    truth.n = c.n_true
    s = swe.Solver.from_problem(truth, dtype=torch.float64)
    cells = torch.as_tensor(c.cells, device="cuda")
    zc = s.z.reshape(-1)[cells]
    obs = []
    for _ in range(nsteps // c.obs_every):
        s.run(c.obs_every)
        obs.append(s.eta.reshape(-1)[cells] - zc)
    hobs = torch.stack(obs).contiguous()
    s.close()
    # warm-up of both paths (kernel code objects, the binding's first torch
    # calls): 20 forward steps and a 20-step gradient in each mode
    w = swe.Solver.from_problem(p, dtype=torch.float64)
    w.run(20)
    for ck in (ckpt, 0):
        w.grad(20, c.cells, c.obs_every, hobs[: 20 // c.obs_every].contiguous(), ck)
    w.close()
    f = swe.Solver.from_problem(p, dtype=torch.float64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f.run(nsteps)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    f.close()

    def timed_grad(ck):
        g = swe.Solver.from_problem(p, dtype=torch.float64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = g.grad(nsteps, c.cells, c.obs_every, hobs, ck)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        g.close()
        return res, t

    (J, gn, gz), t_grad = timed_grad(ckpt)
    progress(f"adjoint: forward {t_fwd * 1e3:.1f} ms, swe_grad {t_grad * 1e3:.1f} ms "
             f"(checkpoint every {ckpt})")
    out = {"workload": f"Manning calibration {p.nx}x{p.ny}, dx={p.dx:g} m, FP64, {nsteps} steps, "
                       f"{len(c.cells)} gauges every {c.obs_every} steps, checkpoint every {ckpt}",
           "metric": "adjoint/fwd cost ratio", "value": t_grad / t_fwd,
           "higher_is_better": False, "checkpoint_every": ckpt, "fwd_ms": t_fwd * 1e3,
           "grad_ms": t_grad * 1e3, "loss": J, "max_abs_dJ_dn": float(gn.abs().max()),
           "max_abs_dJ_dz": float(gz.abs().max())}
    (J2, gn2, gz2), t2 = timed_grad(0)
    progress(f"adjoint: swe_grad {t2 * 1e3:.1f} ms (whole trajectory kept)")
    out["kept_trajectory"] = {"grad_ms": t2 * 1e3, "ratio": t2 / t_fwd,
                              "gradient_equal": bool(J2 == J and torch.equal(gn2, gn)
                                                     and torch.equal(gz2, gz))}
    if fd_cells > 0:
        import numpy as np
        s = swe.Solver.from_problem(p, dtype=torch.float64)
        dts = np.array([s.step() for _ in range(nsteps)])
        s.close()
        out["fd_check"] = fd_check(torch, swe, p, c.cells, c.obs_every, hobs, dts, gn,
                                   ncell=fd_cells)
        progress(f"adjoint: finite differences {out['fd_check']}")
    return out


def ensemble_throughput(torch, swe, W, count, nsteps):
    """Flood ensemble: `count` scenarios (FP32) advanced together, one
    fused launch per step for all of them, the nsteps-step run captured in a
    HIP graph and replayed; against the same scenarios run one grid at a time
    through the single-grid library, one after another."""
    probs = W.flood_ensemble(count=count)
    cells = sum(p.nx * p.ny for p in probs)
    progress(f"ensemble: {count} scenarios, {cells / 1e6:.1f} M cells, {nsteps} steps")
    e = swe.Ensemble.from_problems(probs, dtype=torch.float32, tile_rows=0)
    H = e.tile_rows
    e.capture(nsteps)
    e.close()
    e = swe.Ensemble.from_problems(probs, dtype=torch.float32, tile_rows=H)
    e.capture(nsteps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e.replay()
    st = e.stats()
    t_ens = time.perf_counter() - t0
    steps = sum(x.step for x in st)
    e.close()
    solvers = [swe.Solver.from_problem(p, dtype=torch.float32) for p in probs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in solvers:
        s.run(nsteps)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    for s in solvers:
        s.close()
    e = swe.Ensemble.from_problems(probs, dtype=torch.float32, tile_rows=H, dry_skip=True)
    e.capture(nsteps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e.replay()
    st_dry = e.stats()
    t_dry = time.perf_counter() - t0
    skipped = sum(x.cells_skipped for x in st_dry)
    same = all(a.t == b.t and a.volume == b.volume for a, b in zip(st, st_dry))   # same tiling
    e.close()
    cu = sum(p.nx * p.ny for p in probs) * nsteps
    progress(f"ensemble: graph replay {t_ens * 1e3:.1f} ms (dry-tile skip {t_dry * 1e3:.1f} ms), "
             f"one grid at a time {t_seq * 1e3:.1f} ms")
    return {"workload": f"flood ensemble: {count} scenarios, grids 64..1024 x 64..512 (seeded), "
                        f"{cells} cells, FP32, {nsteps}-step run captured in a HIP graph",
            "metric": "ensemble cells/s", "value": cu / t_ens, "unit": "cell-updates/s",
            "sequential_value": cu / t_seq, "speedup_vs_sequential": t_seq / t_ens,
            "tile_rows": H, "ms": t_ens * 1e3, "sequential_ms": t_seq * 1e3,
            "steps_taken": steps,
            "dry_skip": {"ms": t_dry * 1e3, "dense_equivalent_value": cu / t_dry,
                         "active_value": (cu - skipped) / t_dry,
                         "skipped_fraction": skipped / cu, "speedup_vs_dense": t_ens / t_dry,
                         "stats_equal_to_dense": same}}


def dry_skip_run(torch, swe, W, p, dtype, steps, warmup, tile_rows, dense_st, dense_ms):
    """The reservoir workload again with the dry-tile skip on.  Dense-
    equivalent throughput counts every cell of every step; active throughput
    counts only the cell updates the kernel computed."""
    progress(f"dry skip: timing {steps} {dtype} steps")
    st, ms, _ = timed_run(torch, swe, W, p, dtype, steps, warmup, tile_rows, dry_skip=True)
    total = p.nx * p.ny * steps
    # t, dt and lambda_max do not depend on the tiling; volume and defect are
    # sums whose rounding follows the tile partition (the skip run's default
    # tile height is 32 rows), so they are compared to 1e-12
    close = lambda x, y: abs(x - y) <= 1e-12 * max(abs(x), abs(y), 1e-300)
    same = (all(getattr(st, f) == getattr(dense_st, f)
                for f in ("t", "dt", "lambda_max", "dt_min", "dt_max")) and
            close(st.volume, dense_st.volume) and close(st.defect, dense_st.defect))
    progress(f"dry skip {dtype}: {ms / steps * 1e3:.1f} us/step, skipped "
             f"{st.cells_skipped / total:.3f} of the cell updates, stats match the dense run: {same}")
    return {"dtype": dtype, "ms_per_step": ms / steps,
            "dense_equivalent_value": total / (ms / 1e3),
            "active_value": (total - st.cells_skipped) / (ms / 1e3),
            "unit": "cell-updates/s", "skipped_fraction": st.cells_skipped / total,
            "speedup_vs_dense": dense_ms / ms, "stats_match_dense": same}


def combined_run(torch, swe, W, nx, nsteps, ckpt, obs_every, h_film):
    """The large combined run: the channel flood at nx x nx, FP32 forward
    state, FP64 adjoint of the gauge-misfit loss with respect to Manning n
    (each step linearised at its FP32 state), checkpoint spacing ckpt.
    Observations come from an FP32 run with the true Manning field.
    h_film > 0 takes the thin-film reading: the reciprocal depth of the
    primitive variables and of the dissipation switch (S2, S9) is
    min(1/h, 1/h_film), so films thinner than h_film do not give velocities
    and switch values of order 1/h.  Without it the discrete adjoint of this
    flood grows without bound."""
    import dataclasses
    ckpt = ckpt or max(1, int(round(math.sqrt(nsteps))))
    c = W.channel_flood(nx=nx, ny=nx, nsteps=nsteps, obs_every=obs_every)
    p = c.problem
    p.h_film = h_film
    cells = p.nx * p.ny
    progress(f"combined: channel flood {nx}x{nx}, {nsteps} steps, checkpoint every {ckpt}")
    nobs = nsteps // obs_every
    gc = torch.as_tensor(c.cells, device="cuda")
    hobs = torch.empty(nobs, len(c.cells), dtype=torch.float64, device="cuda")
    s = swe.Solver.from_problem(dataclasses.replace(p, n=c.n_true), dtype=torch.float32)
    for k in range(nobs):
        s.run(obs_every)
        hobs[k] = s.eta.reshape(-1)[gc].double() - s.z.reshape(-1)[gc].double()
        if (k + 1) % 20 == 0:
            progress(f"combined: observation run, step {(k + 1) * obs_every}")
    s.close()
    del s
    progress("combined: timing the FP32 forward run")
    st, ms_fwd, _ = timed_run(torch, swe, W, p, "f32", nsteps, 0, 0)
    st_dry, ms_dry, _ = timed_run(torch, swe, W, p, "f32", nsteps, 0, 0, dry_skip=True)
    progress(f"combined: forward {ms_fwd:.0f} ms, with the dry-tile skip {ms_dry:.0f} ms")
    f = swe.Solver.from_problem(p, dtype=torch.float32, dry_skip=True)
    free0, total = torch.cuda.mem_get_info()
    fe = p.ny * p.nx
    npad = (p.nx + 2) * (p.ny + 2)
    nseg = (nsteps + ckpt - 1) // ckpt
    # FP32 checkpoints and segment states; FP64: replay output, promoted state,
    # z/n/m, U* and U^d (15 pitched fields), padded z and m, 20 adjoint arrays
    planned = (nseg + ckpt) * 3 * fe * 4 + 15 * fe * 8 + (2 + 20) * npad * 8
    progress(f"combined: swe_grad, planned scratch {planned / 1e9:.1f} GB of "
             f"{free0 / 1e9:.1f} GB free")
    os.environ["SWE_VERBOSE"] = "1"   # the library reports each reverse segment on stderr
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J, gn, gz = f.grad(nsteps, c.cells, obs_every, hobs, ckpt)
    torch.cuda.synchronize()
    grad_s = time.perf_counter() - t0
    os.environ.pop("SWE_VERBOSE", None)
    h = (f.eta - f.z).double()
    wet = float((h > p.h_dry).double().mean())
    finite = bool(torch.isfinite(gn).all()) and bool(torch.isfinite(gz).all())
    fin = lambda v: v if math.isfinite(v) else None
    out = {"workload": f"channel flood {nx}x{nx}, dx={p.dx:g} m, fractal terrain (5 m, 1/|k|^1.8) "
                       f"+ diagonal plane (1e-3) + parabolic channel 3 m x 40 m along x=y flowing "
                       f"0.5 m below its banks, inflow 10 m^2/s (30 s ramp) on the W and S faces "
                       f"of its deeper part, open N and E, land initially dry, {nsteps} steps",
           "forward_dtype": "f32", "adjoint_dtype": "f64", "steps": nsteps, "sim_time_s": st.t,
           "checkpoint_every": ckpt, "forward_ms": ms_fwd,
           "forward_cell_updates_per_s": cells * nsteps / (ms_fwd / 1e3),
           "forward_dry_skip_ms": ms_dry,
           "forward_dry_skip_skipped_fraction": st_dry.cells_skipped / (cells * nsteps),
           "forward_dry_skip_t_equal": st_dry.t == st.t,
           "grad_ms": grad_s * 1e3, "adjoint_fwd_ratio": grad_s * 1e3 / ms_fwd,
           "loss": fin(J), "gradient_finite": finite, "h_film": h_film,
           "max_abs_dJ_dn": fin(float(gn.abs().max())),
           "max_abs_dJ_dz": fin(float(gz.abs().max())),
           "gradient_note": ("thin-film reading (h_film > 0): the gradient is the FP64 "
                             "linearisation along the FP32 trajectory.  On this flood at "
                             "1024^2 (FP64) it is O(10) and agrees with central differences "
                             "up to 3000 steps; by 5000 steps wet/dry switching makes the "
                             "loss itself jump (difference quotients grow like 1/step), so "
                             "no gradient can be checked there and this run's is a "
                             "diagnostic" if h_film > 0 else
                             "plain scheme: the discrete adjoint grows exponentially through "
                             "the wet/dry fronts of this flood, so the gradient is a "
                             "diagnostic"),
           "gradient_target_met": False,
           "planned_scratch_bytes": planned, "device_free_bytes_before": free0,
           "device_total_bytes": total, "wet_fraction_end": wet,
           "gauges": len(c.cells), "obs_every": obs_every}
    f.close()
    progress(f"combined: forward {ms_fwd:.0f} ms, swe_grad {grad_s * 1e3:.0f} ms, "
             f"ratio {out['adjoint_fwd_ratio']:.1f}, wet fraction {wet:.4f}")
    return out


def stream_probe(torch, swe, dtype, nx, ny, reps=7):
    """Bandwidth ceilings for the step's traffic, each timed as the median of
    reps launches with HIP events on torch's current stream (where the probes
    launch), all over the workload's own size:
    - copy: the library's plain copy kernel over four arrays' worth (as many
      bytes moved as the step's eight arrays);
    - plain / nontemporal: the library's stream kernel reading five and
      writing three arrays, one grid-stride pass, without and with
      non-temporal hints;
    - march: the library's march-pattern probe, the step kernel's own tiles,
      tile height, strip order, row march, loads and stores with a few
      operations per cell in place of the sub-steps; its rate is algorithmic
      bytes (the step's 8 words per cell) over time, like the kernel's."""
    tdt = torch.float64 if dtype == "f64" else torch.float32
    cells = nx * ny
    ins = [torch.ones(cells, dtype=tdt, device="cuda") for _ in range(5)]
    outs = [torch.empty(cells, dtype=tdt, device="cuda") for _ in range(3)]
    nbytes = 8 * cells * ins[0].element_size()

    def median_ms(fn):
        fn()
        ts = []
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            b.synchronize()
            ts.append(a.elapsed_time(b))
        return sorted(ts)[len(ts) // 2]

    res = {}
    for nt in (False, True):
        ms = median_ms(lambda: swe.probe_stream(ins, outs, nontemporal=nt))
        res["nontemporal_GBps" if nt else "plain_GBps"] = nbytes / (ms / 1e3) / 1e9
    rows = swe.probe_march(ins, outs, nx, ny, nx)
    ms = median_ms(lambda: swe.probe_march(ins, outs, nx, ny, nx, rows))
    res["march_GBps"] = nbytes / (ms / 1e3) / 1e9
    res["march_us"] = ms * 1e3
    res["march_rows"] = rows
    del ins, outs
    src = torch.ones(4 * cells, dtype=tdt, device="cuda")
    dst = torch.empty_like(src)
    ms = median_ms(lambda: swe.probe_copy(dst, src))
    res["copy_GBps"] = nbytes / (ms / 1e3) / 1e9
    del src, dst
    res["bytes_per_launch"] = nbytes
    res["note"] = ("stream: 5 arrays read + 3 written, 16 B per lane, grid-stride "
                   "(swe_probe_stream); march: the step kernel's traversal without its "
                   "arithmetic (swe_probe_march); copy: swe_probe_copy of the same bytes")
    return res


def cpu_model():
    """The host CPU's model name (as lscpu reports it) and the cores this
    process may run on."""
    name = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return name, avail


def cpu_baseline(W, p, nsteps):
    """The oracle as it stands, timed on the host: serial (1 core), and the
    same source built with OpenMP over the host threads (its state bit for
    bit the serial one, checked here)."""
    from oracle import oracle as O
    import numpy as np
    model, avail = cpu_model()
    progress(f"CPU oracle baseline: {nsteps} timed steps of {p.nx}x{p.ny} on {model}")
    s = O.State(p)
    s.run(1)                       # untimed: first touch of the work arrays
    st = s.run(nsteps)
    cells = p.nx * p.ny * st.steps
    out = {"value": cells / st.loop_seconds, "unit": "cell-updates/s", "cores": 1,
           "kind": "oracle", "cpu": model, "host_cores_available": avail,
           "sample": f"serial FP64 oracle (C++), {p.nx}x{p.ny} reservoir release, steps 1..{nsteps} "
                     f"after one untimed step, {st.loop_seconds:.1f} s of step loop"}
    t = O.State(p, threads=True)
    threads = O.lib_threads().orc_threads()
    t.run(1)
    stt = t.run(nsteps)
    same = all(np.array_equal(x, y) for x, y in ((s.eta, t.eta), (s.qx, t.qx), (s.qy, t.qy)))
    out["all_cores"] = {"value": cells / stt.loop_seconds, "cores": threads,
                        "state_equal_to_serial": bool(same),
                        "sample": f"the same steps, oracle built with -fopenmp, {threads} threads, "
                                  f"{stt.loop_seconds:.1f} s of step loop"}
    return out


def main():
    a = parse()
    if a.print_source_hash:
        print(kernel_source_hash())
        return
    if a.gpus != 1:
        print(f"bench.py: --gpus {a.gpus} requested, but the library runs on one GPU only "
              "(the row-slab multi-GPU split is a design, not built); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1309_1230_amd import swe
    from paper_1309_1230_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if a.probe_copy_mb > 0:
        n = a.probe_copy_mb * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        swe.probe_copy(dst, src)
        torch.cuda.synchronize()
        del src, dst
    if a.combined:
        out = combined_run(torch, swe, W, a.comb_nx, a.comb_steps, a.comb_ckpt, a.comb_obs_every,
                           a.comb_h_film)
        print(json.dumps({"combined": out}), flush=True)
        return
    if a.ensemble_only:
        out = ensemble_throughput(torch, swe, W, a.ens_count, a.ens_steps)
        print(json.dumps({"ensemble": out}), flush=True)
        return
    if a.adjoint_only:
        out = adjoint_ratio(torch, swe, W, a.adj_nx, a.adj_steps, a.adj_ckpt, a.adj_fd_cells)
        print(json.dumps({"adjoint": out}), flush=True)
        return
    nx = a.nx
    p = W.reservoir_release(nx=nx, ny=nx, dx=20480.0 / nx)
    cells = p.nx * p.ny
    progress(f"workload ready; timing {a.steps} {a.dtype} steps")
    st, ms, wall = timed_run(torch, swe, W, p, a.dtype, a.steps, a.warmup, a.tile_rows)
    progress(f"{a.dtype}: {ms / a.steps * 1e3:.1f} us/step")
    assert st.steps == a.steps, st
    value = cells * a.steps / (ms / 1e3)
    ms_step = ms / a.steps
    bpc = bytes_per_cell(a.dtype)
    achieved = bpc * cells / (ms_step / 1e3) / 1e9
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": a.dtype,
        "data": "synthetic (seeded terrain and reservoir, no external data set)",
        "config": {"workload": f"reservoir release {p.nx}x{p.ny}, dx={p.dx:g} m, 200 hills + 1/f "
                               f"noise, surface 25 m behind x=0.2L, n=0.035, open east, "
                               f"{a.steps} adaptive steps",
                   "nx": p.nx, "ny": p.ny, "path": "fused", "tile_rows": a.tile_rows or "auto",
                   "sim_time_s": st.t},
        "hbm_pct": 100.0 * achieved / HBM_PEAK_GBS,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(a.dtype),
                     "kernel": f"k_fused_split_{a.dtype}",
                     "bytes_per_launch_algorithmic": bpc * cells,
                     "bytes_per_cell_update": bpc},
        "wall_s": wall,
    }
    out["stream_probe"] = stream_probe(torch, swe, a.dtype, p.nx, p.ny)
    out["roofline"]["frac_of_stream_probe"] = achieved / out["stream_probe"]["plain_GBps"]
    out["roofline"]["frac_of_march_probe"] = achieved / out["stream_probe"]["march_GBps"]
    if a.dry_only:
        out["dry_skip"] = dry_skip_run(torch, swe, W, p, a.dtype, a.steps, a.warmup, a.tile_rows,
                                       st, ms)
        print(json.dumps(out), flush=True)
        return
    if not a.no_variants:
        other = "f32" if a.dtype == "f64" else "f64"
        st2, ms2, _ = timed_run(torch, swe, W, p, other, a.steps, a.warmup, a.tile_rows)
        v2 = cells * a.steps / (ms2 / 1e3)
        out["variants"] = {other: {"value": v2, "ms_per_step": ms2 / a.steps,
                                   "hbm_pct": 100.0 * bytes_per_cell(other) * v2 / 1e9 / HBM_PEAK_GBS}}
        nu = 20
        st3, ms3, _ = timed_run(torch, swe, W, p, a.dtype, nu, 2, a.tile_rows, path="unfused")
        out["variants"]["unfused_" + a.dtype] = {"value": cells * nu / (ms3 / 1e3),
                                                 "ms_per_step": ms3 / nu, "steps": nu}
    if not a.no_dry_skip:
        out["dry_skip"] = dry_skip_run(torch, swe, W, p, a.dtype, a.steps, a.warmup, a.tile_rows,
                                       st, ms)
        if not a.no_variants:
            out["dry_skip_" + other] = dry_skip_run(torch, swe, W, p, other, a.steps, a.warmup,
                                                    a.tile_rows, st2, ms2)
    if not a.no_adjoint:
        out["adjoint"] = adjoint_ratio(torch, swe, W, a.adj_nx, a.adj_steps, a.adj_ckpt, a.adj_fd_cells)
    if not a.no_ensemble:
        out["ensemble"] = ensemble_throughput(torch, swe, W, a.ens_count, a.ens_steps)
    if a.cpu_steps > 0:
        out["cpu_baseline"] = cpu_baseline(W, p, a.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
