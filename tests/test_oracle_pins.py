"""Pins of the CPU oracle against what physics and mathematics fix.

The oracle is the reference the GPU library is checked against, so it is
itself checked here against facts that do not come from it: exact discrete
invariants of a conservative scheme (still water, mass and momentum budgets),
closed forms (Stoker's dam break, the linear wave speed sqrt(g h), the first
seiche period, the Manning friction decay ODE, the first time step of a still
dam break) and exact symmetries.  A plausible slip anywhere in the scheme (a
dropped or sign-flipped term, a wrong index or a transposed operand) breaks at
least one of them.  The switch and dissipation sub-steps (S3, S4) and the
time-step speed sum (S16) are also pinned value by value on small inputs
worked out by hand, so that the oracle is held to its written reading of the
scheme; that reading itself (the switch's form and the coefficient kappa)
has no source beyond the loose Stoker accuracy, since the paper defers the
equations to a thesis that is not available.
"""
import math
import os

import numpy as np
import pytest
from scipy.optimize import brentq

from oracle import oracle as O
from paper_1309_1230_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------- closed forms

def stoker_closed_form(hl=1.0, hr=0.5, g=9.81):
    cl = math.sqrt(g * hl)

    def f(hm):
        return 2.0 * (cl - math.sqrt(g * hm)) - (hm - hr) * math.sqrt(0.5 * g * (hm + hr) / (hm * hr))

    hm = brentq(f, hr, hl, xtol=1e-15)
    um = 2.0 * (cl - math.sqrt(g * hm))
    return hm, um, hm * um / (hm - hr), cl


def stoker_profile(x, t, x0=64.0, hl=1.0, hr=0.5, g=9.81):
    hm, um, S, cl = stoker_closed_form(hl, hr, g)
    cm = math.sqrt(g * hm)
    xi = (x - x0) / t
    fan = ((2.0 * cl - xi) / 3.0) ** 2 / g
    return np.where(xi < -cl, hl, np.where(xi < um - cm, fan, np.where(xi < S, hm, hr)))


def test_stoker_golden_fixture_matches_closed_form():
    vals = {}
    with open(os.path.join(GOLDEN, "stoker_h1_h05_g981.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                vals[k] = float(v)
    hm, um, S, cl = stoker_closed_form()
    assert abs(vals["h_m"] - hm) < 1e-6
    assert abs(vals["u_m"] - um) < 1e-6
    assert abs(vals["S"] - S) < 1e-6
    assert abs(vals["rarefaction_head"] + cl) < 1e-6
    assert abs(vals["rarefaction_tail"] - (um - math.sqrt(9.81 * hm))) < 1e-6


# ------------------------------------------------------------- still water

@pytest.mark.parametrize("dry_banks", [False, True])
def test_lake_at_rest_is_bitwise_still(dry_banks):
    p = W.lake_at_rest(48, 40, seed=7, dry_banks=dry_banks)
    if dry_banks:
        assert np.any(p.eta - p.z <= p.h_dry) and np.any(p.eta - p.z > p.h_dry)
    s = O.State(p)
    st = s.run(300)
    assert st.flags & O.FLAG_NAN == 0
    assert np.array_equal(s.eta, p.eta)
    assert not np.any(s.qx) and not np.any(s.qy)
    assert st.defect == 0.0


def test_lake_at_rest_flat_bed_long():
    p = W.lake_at_rest(24, 20, seed=3, dry_banks=False)
    p.z[:] = 0.0
    p.eta[:] = 2.0
    s = O.State(p)
    s.run(1000)
    assert np.array_equal(s.eta, p.eta) and not np.any(s.qx) and not np.any(s.qy)


def test_first_time_step_of_still_dam_break():
    # lam = (|u| + c)/dx + (|v| + c)/dy with u = v = 0 and the deepest cell h = 1
    p = W.stoker()
    assert O.initial_dt(p) == pytest.approx(0.5 / (2.0 * math.sqrt(9.81)), rel=1e-15)


# ------------------------------------------------------------ conservation

def test_closed_basin_mass_conserved_to_roundoff():
    p = W.smooth_wet(64, 64, seed=11)
    assert p.kappa > 0 and p.n.min() > 0
    v0, _ = O.volume_and_lambda(p, p.eta, p.qx, p.qy)
    s = O.State(p)
    st = s.run(200)
    assert st.defect == 0.0 and st.flags == 0
    assert abs(st.volume - v0) / v0 < 1e-12


def test_inflow_mass_budget_from_hydrograph():
    """Walls everywhere except an inflow band: the volume gained over a step is
    dt * width of the band * mean of q_in at the two stage times, plus the clip
    defect -- all of it fixed by the hydrograph alone."""
    p = W.inflow_channel(40, 24, seed=5, q_peak=1.5, dry=True, t_peak=3.0, t_end=9.0)
    p.bc = (W.INFLOW, W.WALL, W.WALL, W.WALL)
    p.inflow_lo = (6, 0, 0, 0)
    p.inflow_hi = (18, 24, 40, 40)
    s = O.State(p)
    v_prev, _ = O.volume_and_lambda(p, s.eta, s.qx, s.qy)
    total_in = 0.0
    for _ in range(60):
        t0, dt = s.t, s.dt
        st = s.run(1)
        qin = lambda t: float(np.interp(t, p.hydro_t, p.hydro_q))
        inflow = dt * (12 * p.dy) * 0.5 * (qin(t0) + qin(t0 + dt))
        total_in += inflow
        assert st.volume - v_prev == pytest.approx(inflow + st.defect, abs=1e-9 * max(1.0, st.volume))
        v_prev = st.volume
    assert total_in > 1.0


def test_open_boundary_mass_budget():
    """Open east edge: the outflow over a step is the mean of the predictor and
    corrector boundary-face fluxes, which the open-edge rule takes from the
    edge cells of U^n and U* (a copy ghost makes either donor the edge cell)."""
    p = W.smooth_wet(32, 24, seed=2, vel=0.6)
    p.bc = (W.WALL, W.OPEN, W.WALL, W.WALL)
    s = O.State(p)
    for _ in range(5):
        v0, _ = O.volume_and_lambda(p, s.eta, s.qx, s.qy)
        dt = s.dt
        tr, sc = s.trace()
        e_n = tr["S1.qx"][1:-1, -2]     # east edge cells of U^n
        e_s = tr["S7.qx"][1:-1, -2]     # east edge cells of U*
        assert np.all(tr["S1.eta"][1:-1, -2] - p.z[:, -1] > p.h_dry)
        out = dt * p.dy * 0.5 * (e_n.sum() + e_s.sum())
        v1 = sc["volume"]
        assert v1 - v0 == pytest.approx(-out + sc["defect_depth"] * p.dx * p.dy, abs=1e-10 * v0)


def test_flat_bed_momentum_budget_pins_pressure_form():
    """On a flat bed with walls, x-momentum changes only through the wall
    hydrostatic thrust g h^2/2 of the edge cells, in each stage; a pressure
    term with the wrong face depth, sign or side breaks this to O(1)."""
    p = W.smooth_wet(36, 20, seed=4)
    p.z[:] = 0.0
    p.n[:] = 0.0
    p.kappa = 0.0
    g = p.g
    s = O.State(p)
    for _ in range(4):
        dt = s.dt
        tr, _ = s.trace()
        hn = tr["S1.eta"][1:-1, 1:-1]
        hs = tr["S7.eta"][1:-1, 1:-1]
        thrust = lambda h: (0.5 * g * h[:, -1] ** 2 - 0.5 * g * h[:, 0] ** 2).sum()
        expect = -(dt / p.dx) * 0.5 * (thrust(hn) + thrust(hs))
        m0 = tr["S1.qx"][1:-1, 1:-1].sum()
        m1 = tr["S15.qx"][1:-1, 1:-1].sum()
        scale = np.abs(tr["S1.qx"]).sum() + abs(expect)
        assert m1 - m0 == pytest.approx(expect, abs=1e-12 * scale)


def test_dissipation_conserves_mass():
    p = W.random_valid_state(30, 22, seed=9)
    s = O.State(p)
    tr, _ = s.trace()
    d = tr["S4.Deta"][1:-1, 1:-1]
    assert np.abs(d).max() > 0
    assert abs(d.sum()) < 1e-13 * np.abs(d).sum()


# ------------------------------------------------------------- closed forms

def test_stoker_dam_break_accuracy():
    p = W.stoker()  # 128 x 128, the full first workload
    s = O.State(p)
    st = s.run(200)
    assert st.flags & O.FLAG_NAN == 0 and st.defect == 0.0
    t = s.t
    assert 14.0 < t < 17.0
    xc = (np.arange(p.nx) + 0.5) * p.dx
    h = s.eta - p.z
    assert np.all(h == h[0:1, :])            # stays uniform in y
    h = h[0]
    hx = stoker_profile(xc, t)
    hm, um, S, cl = stoker_closed_form()
    assert np.sum(np.abs(h - hx)) * p.dx <= 1e-2 * 1.0 * (p.nx * p.dx)
    tail = 64.0 + (um - math.sqrt(9.81 * hm)) * t
    bore = 64.0 + S * t
    plateau = h[(xc > tail + 4) & (xc < bore - 4)]
    assert abs(plateau.mean() - hm) < 0.01 * hm
    front = xc[np.where(h > 0.5 * (hm + 0.5))[0].max()]
    assert abs(front - bore) <= 2.0 * p.dx


def test_stoker_converges_under_refinement():
    errs = []
    for n in (128, 256, 512):
        p = W.stoker(nx=n, ny=4, dx=128.0 / n)
        s = O.State(p)
        s.run(10 ** 6, t_end=12.0)
        xc = (np.arange(n) + 0.5) * p.dx
        errs.append(np.sum(np.abs(s.eta[1] - stoker_profile(xc, s.t))) * p.dx)
    assert errs[1] < 0.75 * errs[0] and errs[2] < 0.75 * errs[1]


def test_linear_wave_speed():
    p = W.gaussian_hump(nx=2048, ny=4, amp=1e-4, width=20.0, dt_fixed=0.1)
    s = O.State(p)
    T = 100.0
    s.run(int(round(T / 0.1)))
    xc = (np.arange(p.nx) + 0.5) * p.dx
    x0 = 0.5 * p.nx * p.dx
    a = s.eta[1] - 1.0
    right = np.where(xc > x0 + 50)[0]
    k = right[np.argmax(a[right])]
    y0, y1, y2 = a[k - 1], a[k], a[k + 1]
    xpk = xc[k] + 0.5 * (y0 - y2) / (y0 - 2 * y1 + y2) * p.dx
    speed = (xpk - x0) / s.t
    assert speed == pytest.approx(math.sqrt(9.81 * 1.0), rel=5e-3)
    # the pulse splits in two halves of equal height, a/2 each
    assert a[k] == pytest.approx(0.5e-4, rel=0.05)


def test_seiche_period():
    p = W.seiche(nx=200, ny=4, h0=1.0, amp=1e-4, dt_fixed=0.05)
    s = O.State(p)
    T = 2 * 200.0 / math.sqrt(9.81)
    ts, ys = [0.0], [s.eta[1, 0] - 1.0]
    while s.t < 1.6 * T:
        s.run(1)
        ts.append(s.t)
        ys.append(s.eta[1, 0] - 1.0)
    ts, ys = np.array(ts), np.array(ys)
    cross = []
    for k in range(len(ys) - 1):
        if ys[k] > 0 >= ys[k + 1] or ys[k] < 0 <= ys[k + 1]:
            cross.append(ts[k] + (ts[k + 1] - ts[k]) * ys[k] / (ys[k] - ys[k + 1]))
    assert len(cross) >= 3
    period = 2.0 * (cross[2] - cross[1])
    assert period == pytest.approx(T, rel=5e-3)


def test_friction_matches_manning_decay_closed_form():
    """Uniform flow on a flat bed with open edges feels friction alone:
    dq/dt = -m q |q| h^(-7/3), so 1/q grows linearly: 1/q(t) = 1/q0 + m h^(-7/3) t.
    A point-implicit step q' = q / (1 + dt m |q| h^(-7/3)) advances 1/q by
    exactly dt m h^(-7/3), so the discrete decay equals the closed form to
    round-off for every dt; a wrong depth exponent or coefficient does not."""
    for h, q0, nm, T in ((0.8, 1.2, 0.05, 20.0), (1.5, -0.7, 0.08, 35.0)):
        m = 9.81 * nm * nm
        exact = q0 / (1.0 + abs(q0) * m * h ** (-7.0 / 3.0) * T)
        for dt in (0.2, 0.05):
            p = W.uniform_flow(12, 10, h=h, q=q0, manning=nm, dt_fixed=dt)
            s = O.State(p)
            s.run(int(round(T / dt)))
            assert s.t == pytest.approx(T, rel=1e-12)
            assert np.all(s.eta == h)             # mass untouched
            assert np.all(s.qx == s.qx[0, 0]) and not np.any(s.qy)
            assert abs(s.qx[0, 0] - exact) < 1e-13 * abs(q0)
            assert abs(exact - q0) > 0.2 * abs(q0)


# --------------------------------------------------------------- symmetries

def test_y_uniform_problem_stays_bitwise_uniform():
    p = W.stoker(nx=64, ny=9, dx=2.0)
    s = O.State(p)
    s.run(60)
    for a in (s.eta, s.qx, s.qy):
        assert np.all(a == a[0:1, :])
    assert not np.any(s.qy)


def test_transposed_dam_break_is_bitwise_transposed():
    px = W.stoker(nx=64, ny=10, dx=2.0, axis="x")
    py = W.stoker(nx=10, ny=64, dx=2.0, axis="y")
    sx, sy = O.State(px), O.State(py)
    assert sx.dt == sy.dt
    sx.run(80)
    sy.run(80)
    assert np.array_equal(sx.eta, sy.eta.T)
    assert np.array_equal(sx.qx, sy.qy.T)
    assert np.array_equal(sx.qy, sy.qx.T)


def test_radial_dam_break_is_transpose_symmetric():
    n = 48
    xc = (np.arange(n) + 0.5)
    X, Y = np.meshgrid(xc, xc)
    h = np.where((X - 24) ** 2 + (Y - 24) ** 2 < 100, 2.0, 1.0)
    p = W.Problem(nx=n, ny=n, dx=1.0, dy=1.0, z=np.zeros((n, n)), n=np.full((n, n), 0.02),
                  eta=h, qx=np.zeros((n, n)), qy=np.zeros((n, n)))
    s = O.State(p)
    s.run(40)
    scale = np.abs(s.qx).max()
    assert scale > 0.1
    assert np.abs(s.eta - s.eta.T).max() < 1e-12
    assert np.abs(s.qx - s.qy.T).max() < 1e-12 * scale


def test_friction_cube_root_accuracy():
    """The friction step's cube root (a fixed guess-plus-Halley sequence, so
    that every implementation reproduces it bit for bit) against numpy's cbrt
    over the range of reciprocal depths a wet cell can have."""
    rng = np.random.default_rng(12)
    xs = np.exp(rng.uniform(np.log(1e-6), np.log(1e6), 20000))
    xs = np.concatenate([xs, [1.0, 8.0, 27.0, 0.125, 1e3, 1e-3, 2.0 ** -20, 2.0 ** 30]])
    got = np.array([O.cbrt3(x) for x in xs])
    assert np.max(np.abs(got / np.cbrt(xs) - 1.0)) < 1e-14
    assert O.cbrt3(8.0) == pytest.approx(2.0, rel=1e-15)
    assert O.cbrt3(1e3) == pytest.approx(10.0, rel=1e-15)


# ------------------------------------------------ hand-computed sub-steps

def test_cfl_speed_sum_of_a_moving_state():
    """S16 on a uniform moving state: every wet cell has u = -1.5, v = 0.7
    and c = sqrt(2 g), so lam = (|u| + c)/dx + (|v| + c)/dy and
    dt^0 = cfl/lam.  dx != dy and u != v make a dropped |u| or |v|, a
    missing absolute value, or the two speeds paired with the wrong cell
    size change dt by 3% to 20%.  A dry cell with a huge discharge (h below
    h_dry) must not count."""
    nx, ny, dx, dy, h = 6, 5, 2.0, 5.0, 2.0
    eta = np.full((ny, nx), h)
    qx = np.full((ny, nx), -1.5 * h)
    qy = np.full((ny, nx), 0.7 * h)
    z = np.zeros((ny, nx))
    z[2, 3] = 10.0
    eta[2, 3] = 10.0 + 0.5e-3          # a thin film: dry at h_dry = 1e-3
    qx[2, 3] = 50.0
    p = W.Problem(nx=nx, ny=ny, dx=dx, dy=dy, z=z, n=np.zeros((ny, nx)), eta=eta, qx=qx, qy=qy,
                  cfl=0.5, h_dry=1e-3, dt_max=100.0)
    c = math.sqrt(9.81 * h)
    lam = (1.5 + c) / dx + (0.7 + c) / dy
    _, lam_o = O.volume_and_lambda(p, p.eta, p.qx, p.qy)
    assert lam_o == pytest.approx(lam, rel=1e-14)
    assert O.initial_dt(p) == pytest.approx(0.5 / lam, rel=1e-14)
    # the slips this pin excludes, each far outside the tolerance above
    for wrong in ((c / dx + (0.7 + c) / dy), ((1.5 + c) / dy + (0.7 + c) / dx),
                  ((-1.5 + c) / dx + (0.7 + c) / dy), ((1.5 + c) / dx + c / dy)):
        assert abs(wrong / lam - 1.0) > 0.03
    # the fastest wet cell sets lam: one cell twice as fast along y
    p2 = p.copy()
    p2.qy[4, 0] = -2.0 * 0.7 * h
    _, lam2 = O.volume_and_lambda(p2, p2.eta, p2.qx, p2.qy)
    assert lam2 == pytest.approx((1.5 + c) / dx + (1.4 + c) / dy, rel=1e-14)
    # dt_max caps the step; dt_fixed replaces it
    p3 = p.copy()
    p3.dt_max = 0.01
    assert O.initial_dt(p3) == 0.01
    p3.dt_fixed = 0.037
    assert O.initial_dt(p3) == 0.037


def _four_by_four():
    """A 4 x 4 walled basin, dx = dy = 1, flat bed except one dry cell (z =
    eta = 5 at i = 0, j = 3) and depths 1, 2 or 4, so that every reciprocal
    depth, switch, coefficient and dissipation term is a short binary
    fraction and the values below are exact.  Rows are j = 0 (south) up."""
    eta = np.array([[1.0, 2.0, 4.0, 2.0],
                    [2.0, 2.0, 2.0, 1.0],
                    [4.0, 1.0, 2.0, 2.0],
                    [5.0, 1.0, 1.0, 4.0]])
    z = np.zeros((4, 4))
    z[3, 0] = 5.0
    qx = np.zeros((4, 4))
    qx[1, 1] = 1.0
    qx[2, 2] = 2.0
    qy = np.zeros((4, 4))
    qy[1, 3] = -1.0
    return W.Problem(nx=4, ny=4, dx=1.0, dy=1.0, z=z, n=np.zeros((4, 4)), eta=eta, qx=qx, qy=qy,
                     kappa=0.5, eps_max=0.25, h_dry=1e-3)


def test_switch_and_dissipation_hand_computed():
    """S3 and S4 of the scheme's reading, worked out by hand on the 4 x 4
    basin above (the ghost ring copies eta, so a boundary second difference
    has one term).  S3: nu_x = 0.25 |(eta_E - eta_C) - (eta_C - eta_W)| r_C
    with r_C = 1/h_C of the centre cell (0 when dry), nu_y alike.  S4: the
    face coefficient eps = min(kappa max(nu_L, nu_R), eps_max) when both
    sides are wet, 0 on boundary faces and at the dry cell; then
    D = (eps_E dU_E - eps_W dU_W) + (eps_N dU_N - eps_S dU_S) for eta, qx, qy.
    Example, cell (1, 2): nu_x = 0.25 |(2 - 1) - (1 - 4)| * 1 = 1, so both its
    x faces have eps = min(0.5 * 1, 0.25) = 0.25 (the cap), and
    D_eta = (0.25 (2 - 1) - 0.25 (1 - 4)) + (0.125 (1 - 1) - 0.125 (1 - 2))
          = 1.125.
    Dropping the 0.25, taking r of a neighbour instead of the centre, the
    cap, the wet test or a sign breaks these values."""
    p = _four_by_four()
    tr, _ = O.State(p).trace()
    inner = lambda nm: tr[nm][1:-1, 1:-1]
    nux = np.array([[0.25, 0.125, 0.25, 0.25],
                    [0.0, 0.0, 0.125, 0.25],
                    [0.1875, 1.0, 0.125, 0.0],
                    [0.0, 1.0, 0.75, 0.1875]])
    nuy = np.array([[0.25, 0.0, 0.125, 0.125],
                    [0.125, 0.125, 0.25, 0.5],
                    [0.0625, 0.25, 0.125, 0.125],
                    [0.0, 0.0, 0.25, 0.125]])
    d_eta = np.array([[0.25, 0.125, -0.75, 0.0],
                      [0.0, -0.125, 0.125, 0.625],
                      [-0.875, 1.125, -0.375, -0.125],
                      [0.0, 0.0, 0.875, -0.875]])
    d_qx = np.array([[0.0, 0.0625, 0.0, 0.0],
                     [0.0, -0.25, 0.3125, 0.0],
                     [0.0, 0.625, -1.125, 0.125],
                     [0.0, 0.0, 0.25, 0.0]])
    d_qy = np.array([[0.0, 0.0, 0.0, -0.25],
                     [0.0, 0.0, -0.125, 0.625],
                     [0.0, 0.0, 0.0, -0.25],
                     [0.0, 0.0, 0.0, 0.0]])
    r = np.array([[1.0, 0.5, 0.25, 0.5],
                  [0.5, 0.5, 0.5, 1.0],
                  [0.25, 1.0, 0.5, 0.5],
                  [0.0, 1.0, 1.0, 0.25]])
    assert np.array_equal(inner("S2.r"), r)
    assert np.array_equal(inner("S3.nux"), nux)
    assert np.array_equal(inner("S3.nuy"), nuy)
    assert np.array_equal(inner("S4.Deta"), d_eta)
    assert np.array_equal(inner("S4.Dqx"), d_qx)
    assert np.array_equal(inner("S4.Dqy"), d_qy)


# ------------------------------------------- binary32 rounding reference

def test_binary32_run_keeps_still_water_still():
    """The oracle's binary32 instantiation (every operation rounded to float)
    keeps a lake at rest bitwise still, dry banks included: the same exact
    cancellation as in double."""
    p = W.lake_at_rest(120, 90, seed=8, dry_banks=True)
    s = O.State(p, binary32=True)
    e0 = s.eta.copy()
    st = s.run(200)
    assert np.array_equal(s.eta, e0)
    assert not np.any(s.qx) and not np.any(s.qy)
    assert st.defect == 0.0


def test_binary32_run_is_float_rounding_of_the_double_step():
    """On the dam break the binary32 run stays within float rounding of the
    double run (relative L1 depth difference of order 1e-7, far below the
    scheme's own error) and holds float values only; a double operation
    leaking into it, or a float one into the double step, would show as an
    exact match or as non-float values."""
    p = W.stoker()
    o, st = O.run(p, 200)
    f = O.State(p, binary32=True)
    sf = f.run(200)
    for a in (f.eta, f.qx, f.qy):
        assert np.array_equal(a, a.astype(np.float32).astype(np.float64))
    h64, h32 = o.eta - p.z, f.eta - p.z
    d = float(np.abs(h32 - h64).sum() / np.abs(h64).sum())
    assert 1e-9 < d < 1e-5
    assert sf.t == pytest.approx(st.t, rel=1e-6)


def test_threaded_build_gives_the_serial_state_bit_for_bit():
    """The -fopenmp build of the same source (the benchmark's all-core CPU
    figure) runs the cell sweeps on several threads; every cell of a sweep
    depends on the previous sweep alone, so the state is the serial one bit
    for bit."""
    p = W.random_valid_state(90, 70, seed=4)
    a = O.State(p)
    b = O.State(p, threads=True)
    sa, sb = a.run(25), b.run(25)
    for x, y in ((a.eta, b.eta), (a.qx, b.qx), (a.qy, b.qy)):
        assert np.array_equal(x, y)
    assert sa.t == sb.t and sa.dt == sb.dt
