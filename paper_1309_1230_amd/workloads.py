"""Seeded synthetic inputs for the shallow-water step.

This module only builds problem definitions: grids, bed elevation, Manning
field, initial state, boundary kinds and the inflow hydrograph.  It holds none
of the solver's arithmetic, so both the GPU library and the CPU oracle can be
fed from it.

The paper's five data sets (Table 1) are not published; every input here is a
synthetic stand-in with the shape and structure of the workloads the solver is
measured on: a wet-bed dam break on a flat bed, a reservoir released onto
seeded hilly terrain, and small still-water and wave cases that have closed
forms.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

WALL, OPEN, INFLOW = 0, 1, 2
EDGE_W, EDGE_E, EDGE_S, EDGE_N = 0, 1, 2, 3

#: default switched-dissipation coefficient and its per-direction cap
KAPPA = 0.5
EPS_MAX = 0.25


@dataclasses.dataclass
class Problem:
    """One shallow-water problem: parameters plus float64 host arrays (ny, nx)."""

    nx: int
    ny: int
    dx: float
    dy: float
    z: np.ndarray
    n: np.ndarray
    eta: np.ndarray
    qx: np.ndarray
    qy: np.ndarray
    g: float = 9.81
    cfl: float = 0.5
    h_dry: float = 1e-3
    kappa: float = KAPPA
    eps_max: float = EPS_MAX
    dt_max: float = 1.0
    dt_fixed: float = 0.0
    h_film: float = 0.0
    bc: tuple = (WALL, WALL, WALL, WALL)
    inflow_lo: tuple = (0, 0, 0, 0)
    inflow_hi: Optional[tuple] = None
    hydro_t: Sequence[float] = ()
    hydro_q: Sequence[float] = ()
    name: str = ""

    def __post_init__(self):
        if self.inflow_hi is None:
            self.inflow_hi = (self.ny, self.ny, self.nx, self.nx)
        for a in ("z", "n", "eta", "qx", "qy"):
            arr = np.ascontiguousarray(getattr(self, a), dtype=np.float64)
            if arr.shape != (self.ny, self.nx):
                raise ValueError(f"{a} has shape {arr.shape}, expected {(self.ny, self.nx)}")
            setattr(self, a, arr)

    @property
    def cells(self) -> int:
        return self.nx * self.ny

    def copy(self) -> "Problem":
        p = dataclasses.replace(self)
        for a in ("z", "n", "eta", "qx", "qy"):
            setattr(p, a, getattr(self, a).copy())
        return p

    def state(self):
        return self.eta.copy(), self.qx.copy(), self.qy.copy()


# --------------------------------------------------------------------------
# Stoker wet-bed dam break: 128 x 128, dx = dy = 1 m, flat bed, walls,
# h = 1.0 m for x < 64 m and 0.5 m beyond, n = 0, g = 9.81, CFL 0.5.

def stoker(nx: int = 128, ny: int = 128, dx: float = 1.0, x_dam: float = 64.0,
           h_left: float = 1.0, h_right: float = 0.5, axis: str = "x") -> Problem:
    """Dam break along x (or along y with axis='y').  Cell centres sit at
    (i + 1/2) dx, so the dam lies on the face at x_dam when x_dam/dx is whole."""
    n_along = nx if axis == "x" else ny
    xc = (np.arange(n_along) + 0.5) * dx
    prof = np.where(xc < x_dam, h_left, h_right)
    if axis == "x":
        h = np.broadcast_to(prof[None, :], (ny, nx)).copy()
    else:
        h = np.broadcast_to(prof[:, None], (ny, nx)).copy()
    z = np.zeros((ny, nx))
    return Problem(nx=nx, ny=ny, dx=dx, dy=dx, z=z, n=np.zeros((ny, nx)), eta=h,
                   qx=np.zeros((ny, nx)), qy=np.zeros((ny, nx)), name=f"stoker{nx}x{ny}")


# --------------------------------------------------------------------------
# Terrain: a sum of Gaussian hills plus a 1/f fractal layer.

def gaussian_hills(nx: int, ny: int, dx: float, dy: float, rng: np.random.Generator,
                   count: int, height: tuple, sigma: tuple) -> np.ndarray:
    """Sum of `count` Gaussian hills with centres uniform over the domain,
    heights U(height) and widths U(sigma) (metres).  Each hill is separable, so
    the sum is one (ny x K) @ (K x nx) product."""
    Lx, Ly = nx * dx, ny * dy
    cx = rng.uniform(0.0, Lx, count)
    cy = rng.uniform(0.0, Ly, count)
    a = rng.uniform(height[0], height[1], count)
    s = rng.uniform(sigma[0], sigma[1], count)
    xc = (np.arange(nx) + 0.5) * dx
    yc = (np.arange(ny) + 0.5) * dy
    gx = np.exp(-0.5 * ((xc[None, :] - cx[:, None]) / s[:, None]) ** 2)  # K x nx
    gy = np.exp(-0.5 * ((yc[:, None] - cy[None, :]) / s[None, :]) ** 2)  # ny x K
    return (gy * a[None, :]) @ gx


def fractal_noise(nx: int, ny: int, rng: np.random.Generator, amplitude: float,
                  exponent: float = 1.0) -> np.ndarray:
    """Fractal noise by spectral synthesis: amplitude proportional to
    1/|k|^exponent (1: 1/f noise), random phases, zero mean, scaled so that
    max |noise| = amplitude."""
    kx = np.fft.rfftfreq(nx)
    ky = np.fft.fftfreq(ny)
    kk = np.sqrt(kx[None, :] ** 2 + ky[:, None] ** 2)
    kk[0, 0] = np.inf
    spec = (1.0 / kk ** exponent) * np.exp(2j * np.pi * rng.uniform(0.0, 1.0, kk.shape))
    spec[0, 0] = 0.0
    f = np.fft.irfft2(spec, s=(ny, nx))
    f -= f.mean()
    m = np.abs(f).max()
    return f * (amplitude / m) if m > 0 else f


def reservoir_release(nx: int = 4096, ny: int = 4096, dx: float = 5.0, seed: int = 1001,
                      hills: int = 200, hill_height=(0.0, 20.0), hill_sigma=(50.0, 400.0),
                      noise_amp: float = 1.0, surface: float = 25.0, dam_frac: float = 0.2,
                      manning: float = 0.035, h_dry: float = 1e-3) -> Problem:
    """Reservoir released onto seeded hilly terrain.  The default is the
    4096 x 4096, dx = 5 m workload: 200 Gaussian hills (height 0-20 m, sigma
    50-400 m) plus 1/f noise of amplitude 1 m; water surface at 25 m for cell
    centres with x < 0.2 L, dry land beyond (h = 0 there); uniform Manning
    n = 0.035; open east edge, walls elsewhere.  Smaller grids keep the
    physical recipe (hill sizes in metres) at the given dx."""
    rng = np.random.default_rng(seed)
    z = gaussian_hills(nx, ny, dx, dx, rng, hills, hill_height, hill_sigma)
    z += fractal_noise(nx, ny, rng, noise_amp)
    L = nx * dx
    xc = (np.arange(nx) + 0.5) * dx
    behind = (xc < dam_frac * L)[None, :]
    eta = np.where(behind, np.maximum(surface, z), z)
    return Problem(nx=nx, ny=ny, dx=dx, dy=dx, z=z, n=np.full((ny, nx), manning), eta=eta,
                   qx=np.zeros((ny, nx)), qy=np.zeros((ny, nx)), h_dry=h_dry,
                   bc=(WALL, OPEN, WALL, WALL), name=f"reservoir{nx}x{ny}")


# --------------------------------------------------------------------------
# Cases with closed forms or exact invariants.

def lake_at_rest(nx: int, ny: int, seed: int, level: float = 1.0, dry_banks: bool = True,
                 dx: float = 1.0) -> Problem:
    """Still water at elevation `level` over a random bed; with dry_banks the
    bed rises above the surface in places (those cells are dry, h = 0)."""
    rng = np.random.default_rng(seed)
    z = gaussian_hills(nx, ny, dx, dx, rng, max(4, (nx * ny) // 200), (0.0, 1.6 if dry_banks else 0.8),
                       (2.0 * dx, 0.25 * min(nx, ny) * dx))
    z -= 0.2
    eta = np.maximum(level, z)
    n = rng.uniform(0.01, 0.05, (ny, nx))
    return Problem(nx=nx, ny=ny, dx=dx, dy=dx, z=z, n=n, eta=eta, qx=np.zeros((ny, nx)),
                   qy=np.zeros((ny, nx)), name=f"lake{nx}x{ny}")


def smooth_wet(nx: int, ny: int, seed: int, dx: float = 1.0, manning: float = 0.03,
               amp: float = 0.2, vel: float = 0.3) -> Problem:
    """A random smooth, everywhere-wet moving state over a hilly bed (depth
    stays above ~0.5 m), used for conservation and parity checks."""
    rng = np.random.default_rng(seed)
    z = gaussian_hills(nx, ny, dx, dx, rng, 12, (0.0, 0.5), (0.1 * nx * dx, 0.3 * nx * dx))
    surf = 1.5 + gaussian_hills(nx, ny, dx, dx, rng, 6, (-amp, amp), (0.1 * nx * dx, 0.25 * nx * dx))
    h = np.maximum(surf - z, 0.5)
    eta = z + h
    u = gaussian_hills(nx, ny, dx, dx, rng, 6, (-vel, vel), (0.15 * nx * dx, 0.3 * nx * dx))
    v = gaussian_hills(nx, ny, dx, dx, rng, 6, (-vel, vel), (0.15 * nx * dx, 0.3 * nx * dx))
    n = rng.uniform(0.5 * manning, 1.5 * manning, (ny, nx))
    return Problem(nx=nx, ny=ny, dx=dx, dy=dx, z=z, n=n, eta=eta, qx=u * h, qy=v * h,
                   name=f"smooth{nx}x{ny}")


def gaussian_hump(nx: int = 2048, ny: int = 8, dx: float = 1.0, h0: float = 1.0,
                  amp: float = 1e-4, width: float = 20.0, dt_fixed: float = 0.1) -> Problem:
    """Small Gaussian hump on still water of depth h0 in a walled channel."""
    xc = (np.arange(nx) + 0.5) * dx
    x0 = 0.5 * nx * dx
    prof = h0 + amp * np.exp(-0.5 * ((xc - x0) / width) ** 2)
    eta = np.broadcast_to(prof[None, :], (ny, nx)).copy()
    return Problem(nx=nx, ny=ny, dx=dx, dy=dx, z=np.zeros((ny, nx)), n=np.zeros((ny, nx)),
                   eta=eta, qx=np.zeros((ny, nx)), qy=np.zeros((ny, nx)), dt_fixed=dt_fixed,
                   kappa=0.0, name="hump")


def seiche(nx: int = 200, ny: int = 6, dx: float = 1.0, h0: float = 1.0, amp: float = 1e-4,
           dt_fixed: float = 0.05) -> Problem:
    """First closed-basin mode: eta = h0 + amp cos(pi x / L)."""
    L = nx * dx
    xc = (np.arange(nx) + 0.5) * dx
    prof = h0 + amp * np.cos(np.pi * xc / L)
    eta = np.broadcast_to(prof[None, :], (ny, nx)).copy()
    return Problem(nx=nx, ny=ny, dx=dx, dy=dx, z=np.zeros((ny, nx)), n=np.zeros((ny, nx)),
                   eta=eta, qx=np.zeros((ny, nx)), qy=np.zeros((ny, nx)), dt_fixed=dt_fixed,
                   kappa=0.0, name="seiche")


def uniform_flow(nx: int, ny: int, h: float, q: float, manning: float, dt_fixed: float,
                 dx: float = 1.0) -> Problem:
    """Uniform depth h and discharge (q, 0) on a flat bed with open edges."""
    eta = np.full((ny, nx), h)
    return Problem(nx=nx, ny=ny, dx=dx, dy=dx, z=np.zeros((ny, nx)),
                   n=np.full((ny, nx), manning), eta=eta, qx=np.full((ny, nx), q),
                   qy=np.zeros((ny, nx)), dt_fixed=dt_fixed, bc=(OPEN, OPEN, OPEN, OPEN),
                   name="uniform")


def inflow_channel(nx: int, ny: int, seed: int, q_peak: float = 2.0, dry: bool = True,
                   dx: float = 2.0, t_peak: float = 20.0, t_end: float = 60.0) -> Problem:
    """Sloping channel fed by a triangular inflow hydrograph on the west edge
    (0 at t = 0, q_peak at t_peak, 0 again at t_end), open east edge, walls
    north and south; initially dry unless dry=False."""
    rng = np.random.default_rng(seed)
    xc = (np.arange(nx) + 0.5) * dx
    z = np.broadcast_to((1e-3 * (nx * dx - xc))[None, :], (ny, nx)).copy()
    z += gaussian_hills(nx, ny, dx, dx, rng, 6, (0.0, 0.3), (0.05 * nx * dx, 0.2 * nx * dx))
    eta = z.copy() if dry else z + 0.5
    n = rng.uniform(0.02, 0.06) * np.ones((ny, nx))
    return Problem(nx=nx, ny=ny, dx=dx, dy=dx, z=z, n=n, eta=eta, qx=np.zeros((ny, nx)),
                   qy=np.zeros((ny, nx)), bc=(INFLOW, OPEN, WALL, WALL),
                   hydro_t=(0.0, t_peak, t_end), hydro_q=(0.0, q_peak, 0.0), name="inflow")


def gaussian_random_field(nx: int, ny: int, dx: float, corr: float,
                          rng: np.random.Generator) -> np.ndarray:
    """Smooth stationary random field: white noise filtered by a Gaussian
    kernel of standard deviation `corr` metres (spectral multiplication),
    rescaled to [0, 1]."""
    kx = np.fft.rfftfreq(nx, d=dx)
    ky = np.fft.fftfreq(ny, d=dx)
    k2 = kx[None, :] ** 2 + ky[:, None] ** 2
    filt = np.exp(-2.0 * (np.pi * corr) ** 2 * k2)
    f = np.fft.irfft2(np.fft.rfft2(rng.standard_normal((ny, nx))) * filt, s=(ny, nx))
    f -= f.min()
    m = f.max()
    return f / m if m > 0 else f


@dataclasses.dataclass
class Calibration:
    """A friction-calibration case: the problem at the first-guess Manning
    field, the true field the observations come from, the gauge cells and
    observation stride, and the run length."""
    problem: Problem
    n_true: np.ndarray
    cells: np.ndarray
    obs_every: int
    nsteps: int


def calibration(nx: int = 1024, ny: int = 1024, dx: float = 2.0, seed: int = 1003,
                nsteps: int = 2000, ngauge: int = 64, obs_every: int = 10, depth: float = 1.5,
                slope: float = 1e-3, n_guess: float = 0.05, n_range=(0.02, 0.08),
                corr: float = 100.0, hill_height=(0.0, 1.0), dt_fixed: float = 0.0) -> Calibration:
    """Manning-field calibration: 1024 x 1024, dx = 2 m by default.  Bed: a
    plane sloping down along x at `slope` plus Gaussian hills up to 1 m.  True
    Manning field: a Gaussian random field with 100 m correlation length
    mapped to [0.02, 0.08].  Initial state: depth 1.5 m everywhere with the
    uniform-flow discharge q = h^(5/3) sqrt(slope) / n_guess along x; the
    west edge feeds that discharge in, the east edge is open, north and south
    are walls; everything stays wet.  64 distinct gauge cells, observed every
    10 steps of a 2000-step run.  The problem carries the first guess
    n = 0.05 everywhere (where the gradient is evaluated)."""
    rng = np.random.default_rng(seed)
    L = nx * dx
    xc = (np.arange(nx) + 0.5) * dx
    z = np.broadcast_to((slope * (L - xc))[None, :], (ny, nx)).copy()
    z += gaussian_hills(nx, ny, dx, dx, rng, 40, hill_height, (0.02 * L, 0.1 * L))
    n_true = n_range[0] + (n_range[1] - n_range[0]) * gaussian_random_field(nx, ny, dx, corr, rng)
    q = depth ** (5.0 / 3.0) * math.sqrt(slope) / n_guess
    eta = z + depth
    cells = rng.choice(nx * ny, ngauge, replace=False)
    p = Problem(nx=nx, ny=ny, dx=dx, dy=dx, z=z, n=np.full((ny, nx), n_guess), eta=eta,
                qx=np.full((ny, nx), q), qy=np.zeros((ny, nx)), dt_fixed=dt_fixed,
                bc=(INFLOW, OPEN, WALL, WALL), hydro_t=(0.0,), hydro_q=(q,),
                name=f"calibration{nx}x{ny}")
    return Calibration(problem=p, n_true=n_true, cells=np.sort(cells), obs_every=obs_every,
                       nsteps=nsteps)


def channel_flood(nx: int = 8192, ny: int = 8192, dx: float = 1.0, seed: int = 1005,
                  nsteps: int = 5000, ngauge: int = 64, obs_every: int = 50,
                  noise_amp: float = 5.0, noise_exponent: float = 1.8, slope: float = 1e-3,
                  depth: float = 3.0, width: float = 40.0, freeboard: float = 0.5,
                  q_in: float = 10.0, ramp: float = 30.0, dt_max: float = 0.1,
                  n_guess: float = 0.035, n_range=(0.02, 0.08),
                  corr: float = 100.0) -> Calibration:
    """The large combined run: 8192 x 8192, dx = 1 m by default.  Bed:
    fractal noise of amplitude 5 m (amplitude spectrum 1/|k|^1.8, a terrain-
    like Hurst exponent of 0.8) plus a plane descending along the diagonal
    from the south-west corner at `slope`, with a channel 40 m wide carved
    along x = y: inside it the bed is the lower of the terrain and a parabolic
    cross-section 3 m below the plane on the axis.  The channel starts
    flowing 0.5 m below its banks at the uniform-flow discharge of the first
    guess n along the axis; all land outside it is dry.  Inflow 10 m^2/s
    through the west and south boundary faces of the channel's deeper part
    (starting depth >= 1 m), ramped up linearly over the first 30 s,
    overtops the channel and floods the land; north and east open;
    dt_max = 0.1 s.  True Manning field: a Gaussian
    random field with 100 m correlation length mapped to [0.02, 0.08]; the
    problem carries the first guess n = 0.035.  64 gauges on the channel
    axis, the first 400 m from the corner, observed every 50 steps of a
    5000-step run."""
    rng = np.random.default_rng(seed)
    xc = (np.arange(nx) + 0.5) * dx
    yc = (np.arange(ny) + 0.5) * dx
    plane = slope * ((nx * dx - xc)[None, :] + (ny * dx - yc)[:, None]) / math.sqrt(2.0)
    z = fractal_noise(nx, ny, rng, noise_amp, noise_exponent) + plane
    dist = np.abs(xc[None, :] - yc[:, None]) / math.sqrt(2.0)
    inside = dist < 0.5 * width
    # carved bed: parabolic cross-section `depth` below the plane on the axis
    bed = plane - depth * (1.0 - (2.0 * dist / width) ** 2)
    z = np.where(inside, np.minimum(z, bed), z)
    n_true = n_range[0] + (n_range[1] - n_range[0]) * gaussian_random_field(nx, ny, dx, corr, rng)
    # inflow faces: those of the channel band where the starting depth is at
    # least 1 m (the parabolic section's inner part; the shallow bank cells
    # would turn 10 m^2/s into a thin, very fast jet)
    inner = 0.5 * width * math.sqrt(max(0.0, 1.0 - (freeboard + 1.0) / depth))
    band_w = int(np.count_nonzero(np.abs(0.5 * dx - yc) / math.sqrt(2.0) < inner))
    band_s = int(np.count_nonzero(np.abs(xc - 0.5 * dx) / math.sqrt(2.0) < inner))
    diag = np.unique(np.linspace(8, min(nx, ny, int(400 / dx)) - 1, ngauge).astype(np.int64))
    cells = diag * nx + diag
    # the channel flows bank-full less the freeboard at uniform-flow discharge
    # along the axis; the land around it is dry
    eta = np.where(inside, np.maximum(z, plane - freeboard), z)
    h = eta - z
    q = np.where(h > 0.0, h ** (5.0 / 3.0) * math.sqrt(slope) / n_guess, 0.0) / math.sqrt(2.0)
    p = Problem(nx=nx, ny=ny, dx=dx, dy=dx, z=z, n=np.full((ny, nx), n_guess), eta=eta,
                qx=q.copy(), qy=q, dt_max=dt_max,
                bc=(INFLOW, OPEN, INFLOW, OPEN), inflow_lo=(0, 0, 0, 0),
                inflow_hi=(band_w, ny, band_s, nx), hydro_t=(0.0, ramp), hydro_q=(0.0, q_in),
                name=f"channel{nx}x{ny}")
    return Calibration(problem=p, n_true=n_true, cells=np.sort(cells), obs_every=obs_every,
                       nsteps=nsteps)


def flood_scenario(index: int, nx: int, ny: int, dx: float = 2.0, seed_base: int = 100000,
                   hills: int = 20, slope: float = 1e-3) -> Problem:
    """One scenario of the flood ensemble: initially dry ground (a plane
    sloping down along x plus `hills` Gaussian hills of height U(0, 5) m and
    width U(0.05, 0.2) of the shorter side), a uniform Manning field
    n ~ U(0.02, 0.06), a triangular inflow hydrograph on the whole west edge
    (0 at t = 0, peak Q ~ U(0.5, 5) m^2/s at 20 s, 0 again at 60 s), open
    east edge, walls north and south.  Seeded by seed_base + index."""
    rng = np.random.default_rng(seed_base + index)
    Lx, Ly = nx * dx, ny * dx
    xc = (np.arange(nx) + 0.5) * dx
    z = np.broadcast_to((slope * (Lx - xc))[None, :], (ny, nx)).copy()
    side = min(Lx, Ly)
    z += gaussian_hills(nx, ny, dx, dx, rng, hills, (0.0, 5.0), (0.05 * side, 0.2 * side))
    n = np.full((ny, nx), rng.uniform(0.02, 0.06))
    qp = rng.uniform(0.5, 5.0)
    return Problem(nx=nx, ny=ny, dx=dx, dy=dx, z=z, n=n, eta=z.copy(), qx=np.zeros((ny, nx)),
                   qy=np.zeros((ny, nx)), bc=(INFLOW, OPEN, WALL, WALL),
                   hydro_t=(0.0, 20.0, 60.0), hydro_q=(0.0, qp, 0.0),
                   name=f"flood{index}_{nx}x{ny}")


def flood_ensemble(count: int = 256, seed: int = 1002, nx_range=(64, 1024), ny_range=(64, 512),
                   dx: float = 2.0) -> list:
    """The flood ensemble: `count` scenarios whose grid sizes are drawn from
    `seed` uniformly in nx_range x ny_range (integers, non-square allowed),
    each built by flood_scenario."""
    rng = np.random.default_rng(seed)
    nxs = rng.integers(nx_range[0], nx_range[1] + 1, count)
    nys = rng.integers(ny_range[0], ny_range[1] + 1, count)
    return [flood_scenario(k, int(nxs[k]), int(nys[k]), dx=dx) for k in range(count)]


def random_valid_state(nx: int, ny: int, seed: int, dry_fraction: float = 0.2,
                       dx: float = 1.0) -> Problem:
    """Rough random state with wet, thin and dry cells, banks and every
    boundary kind, for sub-step-by-sub-step parity checks."""
    rng = np.random.default_rng(seed)
    z = rng.uniform(0.0, 0.6, (ny, nx))
    h = rng.uniform(0.05, 1.0, (ny, nx))
    dry = rng.uniform(0.0, 1.0, (ny, nx)) < dry_fraction
    thin = rng.uniform(0.0, 1.0, (ny, nx)) < 0.05
    h = np.where(dry, 0.0, h)
    h = np.where(thin, rng.uniform(0.0, 2e-3, (ny, nx)), h)
    eta = z + h
    qx = rng.normal(0.0, 0.3, (ny, nx)) * (h > 1e-3)
    qy = rng.normal(0.0, 0.3, (ny, nx)) * (h > 1e-3)
    n = rng.uniform(0.0, 0.06, (ny, nx))
    return Problem(nx=nx, ny=ny, dx=dx, dy=1.25 * dx, z=z, n=n, eta=eta, qx=qx, qy=qy,
                   bc=(INFLOW, OPEN, WALL, INFLOW), inflow_lo=(1, 0, 0, 2),
                   inflow_hi=(ny - 1, ny, nx, nx - 3), hydro_t=(0.0, 0.05, 10.0),
                   hydro_q=(0.1, 0.4, 0.0), name=f"random{nx}x{ny}")
