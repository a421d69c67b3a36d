"""Seeded synthetic inputs: parameters, wall masks and initial fields.

This module is shared by the oracle tests, the GPU tests and the benchmark.  It
builds inputs only (geometry, initial density/velocity, parameter values) and
contains none of the lattice Boltzmann arithmetic.

Workloads follow the paper's two experiments: a droplet on a smooth insulating
substrate (Figs. 1-3) and electrolyte driven through a channel whose two walls
carry rectangular steps of width ``a``, height ``b`` and pitch ``p`` (Fig. 4,
periodic left/right).  The paper's own parameter values use a Green-function
normalisation under which G = -0.52 gives a density ratio of several thousand;
the workloads here use the standard weighted form G_alpha = G * w_alpha
(G/9 on axes, G/36 on diagonals) with G around -5, and a wall strength with the
paper's ratio w/G = 0.14/0.52.

Random numbers come from SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014): ``mix64`` below is its output
function and ``GOLDEN`` its increment.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field

import numpy as np

MASK64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15

# Lattice weights w_alpha only to scale G and W by direction class (axis/diagonal).
W_AXIS = 1.0 / 9.0
W_DIAG = 1.0 / 36.0
# Paper's ratio of fluid-wall to fluid-fluid strength (w = -0.14 with G = -0.52).
WALL_TO_FLUID = 0.14 / 0.52

ELEC_BOTTOM = 1
ELEC_TOP = 2

# psi-Maxwell coexistence densities (rho_v, rho_l) of psi = 1 - exp(-rho) with
# p = rho/3 + G psi^2 / 6, used only to choose initial densities.
_COEX_G = np.array([-6.0, -5.5, -5.25, -5.0, -4.75, -4.5])
_COEX_V = np.array([0.073345, 0.104813, 0.127145, 0.156413, 0.196282, 0.254125])
_COEX_L = np.array([2.649024, 2.307522, 2.125327, 1.932442, 1.724739, 1.494301])


def coexistence(G: float) -> tuple[float, float]:
    """(rho_v, rho_l) for interaction strength G, linearly interpolated."""
    if not (-6.0 <= G <= -4.5):
        raise ValueError(f"G={G} outside the tabulated range [-6, -4.5]")
    return float(np.interp(G, _COEX_G, _COEX_V)), float(np.interp(G, _COEX_G, _COEX_L))


# --------------------------------------------------------------------------- RNG
def mix64(z):
    """SplitMix64 output function on a Python int or a numpy uint64 array."""
    if isinstance(z, np.ndarray):
        z = z.astype(np.uint64)
        with np.errstate(over="ignore"):
            z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
            z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


class SplitMix64:
    """Sequential SplitMix64 stream; ``randint(a, b)`` draws from {a..b}."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next(self) -> int:
        self.state = (self.state + GOLDEN) & MASK64
        return mix64(self.state)

    def randint(self, a: int, b: int) -> int:
        return a + self.next() % (b - a + 1)

    def uniform(self) -> float:
        return (self.next() >> 11) * 2.0 ** -53


def uniform_field(seed: int, n: int) -> np.ndarray:
    """Counter-based uniforms in [0,1): u_i from mix64(seed + (i+1)*GOLDEN)."""
    i = np.arange(1, n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & MASK64) + i * np.uint64(GOLDEN)
    return (mix64(z) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def noise(seed: int, shape, amplitude: float) -> np.ndarray:
    """Uniform noise in [-amplitude, amplitude), indexed row-major (i = y*nx + x)."""
    n = int(np.prod(shape))
    return (2.0 * amplitude) * (uniform_field(seed, n) - 0.5).reshape(shape)


# ----------------------------------------------------------------------- params
@dataclass
class Params:
    """Model parameters; field names match ``lbm_params`` in include/lbm.h."""

    nx: int
    ny: int
    tau: float = 1.0
    rho0: float = 1.0
    g_axis: float = -5.0 * W_AXIS
    g_diag: float = -5.0 * W_DIAG
    w_axis: float = WALL_TO_FLUID * -5.0 * W_AXIS
    w_diag: float = WALL_TO_FLUID * -5.0 * W_DIAG
    rho_c: float = 1.0
    f_elec: float = 0.0
    elec_layers: int = 1
    elec_walls: int = ELEC_BOTTOM | ELEC_TOP
    accel_x: float = 0.0
    accel_y: float = 0.0
    storage: int = 0  # 0 = fp32, 1 = fp16, 2 = bf16
    rho_ref: float = 0.0  # stored deviations are f - w rho_ref (0: raw f for fp32, rho0 for 16-bit)
    collision: int = 0  # 0: BGK with the velocity shift of eq. (10); 1: TRT, 2: MRT, both with Guo forcing
    trt_magic: float = 3.0 / 16.0  # Lambda of the TRT operator (and the s_q of MRT)
    elec_normal: int = 0  # 0: electric force towards the electrode wall; 1: along the local face normal
    rounding: int = 0  # 16-bit storage: 0 nearest even, 1 stochastic (unbiased; see lbm_params.rounding)
    mrt_s_e: float = 1.64  # MRT rate of the energy moment e (bulk viscosity); Lallemand & Luo's value
    mrt_s_eps: float = 1.54  # MRT rate of the moment eps; Lallemand & Luo's value

    def replace(self, **kw) -> "Params":
        return dataclasses.replace(self, **kw)


def params_for_G(nx: int, ny: int, G: float, **kw) -> Params:
    """Weighted Green function G*w_alpha and wall strength at the paper's ratio."""
    return Params(nx=nx, ny=ny, g_axis=G * W_AXIS, g_diag=G * W_DIAG,
                  w_axis=WALL_TO_FLUID * G * W_AXIS, w_diag=WALL_TO_FLUID * G * W_DIAG, **kw)


# --------------------------------------------------------------------- geometry
def flat_channel(nx: int, ny: int) -> np.ndarray:
    """Solid rows y=0 and y=ny-1, fluid elsewhere (uint8, 1 = solid)."""
    s = np.zeros((ny, nx), np.uint8)
    s[0, :] = 1
    s[ny - 1, :] = 1
    return s


def periodic_bumps(nx: int, ny: int, a: int, b: int, p: int, seed: int) -> np.ndarray:
    """Flat walls plus steps of width a, height b, pitch p on both walls.

    Phases of the bottom and top rows are drawn in that order from
    SplitMix64(seed) as U{0..p-1}; bumps wrap periodically in x.
    """
    s = flat_channel(nx, ny)
    if b == 0:
        return s
    rng = SplitMix64(seed)
    ph_bot = rng.randint(0, p - 1)
    ph_top = rng.randint(0, p - 1)
    for ph, top in ((ph_bot, False), (ph_top, True)):
        for x0 in range(ph - p, nx, p):
            cols = np.arange(x0, x0 + a) % nx
            if top:
                s[ny - 1 - b:ny - 1, cols] = 1
            else:
                s[1:1 + b, cols] = 1
    return s


def random_bumps(nx: int, ny: int, seed: int, bmin: int = 2, bmax: int = 8,
                 pmin: int = 16, pmax: int = 64) -> np.ndarray:
    """Flat walls plus a sequence of steps with random pitch and height.

    Each wall draws, from its own SplitMix64 stream (bottom: seed, top:
    seed + 1), pitch p_i ~ U{pmin..pmax} then height b_i ~ U{bmin..bmax}; the
    step covers columns [x_i, x_i + p_i // 4) and the next starts at x_i + p_i.
    The sequence starts at x = 0 and is truncated at nx.
    """
    s = flat_channel(nx, ny)
    for top, sd in ((False, seed), (True, seed + 1)):
        rng = SplitMix64(sd)
        x = 0
        while x < nx:
            p = rng.randint(pmin, pmax)
            b = rng.randint(bmin, bmax)
            a = p // 4
            x1 = min(x + a, nx)
            if top:
                s[ny - 1 - b:ny - 1, x:x1] = 1
            else:
                s[1:1 + b, x:x1] = 1
            x += p
    return s


def chebyshev_dilate(solid: np.ndarray, k: int) -> np.ndarray:
    """Periodic mask of sites within Chebyshev distance <= k of a solid site."""
    out = solid.astype(bool).copy()
    for dy in range(-k, k + 1):
        for dx in range(-k, k + 1):
            out |= np.roll(np.roll(solid.astype(bool), dy, axis=0), dx, axis=1)
    return out


# ------------------------------------------------------------------ init fields
def droplet_density(nx: int, ny: int, R: float, rho_l: float, rho_v: float,
                    width: float = 2.0, cx: float | None = None, cy: float = 0.5) -> np.ndarray:
    """tanh profile of a circular droplet centred at (cx, cy) (default: mid-x, on the wall plane)."""
    if cx is None:
        cx = (nx - 1) / 2.0
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    r = np.hypot(x - cx, y - cy)
    return 0.5 * (rho_l + rho_v) - 0.5 * (rho_l - rho_v) * np.tanh(2.0 * (r - R) / width)


@dataclass
class Case:
    """One simulation input: parameters, solid mask and initial fields."""

    params: Params
    solid: np.ndarray                 # uint8 [ny][nx]
    rho: np.ndarray                   # float64 [ny][nx]
    ux: np.ndarray = None             # float64 [ny][nx] (zeros if None)
    uy: np.ndarray = None
    name: str = ""
    meta: dict = field(default_factory=dict)

    def __post_init__(self):
        ny, nx = self.solid.shape
        assert (ny, nx) == (self.params.ny, self.params.nx)
        self.solid = np.ascontiguousarray(self.solid, np.uint8)
        self.rho = np.ascontiguousarray(np.where(self.solid != 0, 0.0, self.rho), np.float64)
        if self.ux is None:
            self.ux = np.zeros((ny, nx))
        if self.uy is None:
            self.uy = np.zeros((ny, nx))
        self.ux = np.ascontiguousarray(np.where(self.solid != 0, 0.0, self.ux), np.float64)
        self.uy = np.ascontiguousarray(np.where(self.solid != 0, 0.0, self.uy), np.float64)


# The paper's droplet run: a 100 x 50 box, calG = -0.52, w = -0.14, tau = 0.9,
# rho0 = 1, rho_c = 1, a homogeneous density of 0.85.  Reading of eq. (4)
# used for it (the printed 2 calG / calG diverges, see tests/test_golden_paper.py):
# the 2 : 1 ratio of axis to diagonal Green function with calG on the axes,
# G_a = calG (|e| = 1), calG / 2 (|e| = sqrt 2), and W_a = w, w / 2 likewise.
PAPER_G, PAPER_W, PAPER_TAU, PAPER_RHO = -0.52, -0.14, 0.9, 0.85


def paper_params(nx: int = 100, ny: int = 50, f_elec: float = 0.0, **kw) -> Params:
    """Parameters of the paper's droplet run under the reading above: the
    electric force acts on the single layer next to the bottom substrate."""
    base = dict(nx=nx, ny=ny, tau=PAPER_TAU, rho0=1.0, g_axis=PAPER_G, g_diag=PAPER_G / 2,
                w_axis=PAPER_W, w_diag=PAPER_W / 2, rho_c=1.0, f_elec=f_elec, elec_layers=1,
                elec_walls=ELEC_BOTTOM)
    base.update(kw)
    return Params(**base)


def paper_droplet_case(seed: int = 0, nx: int = 100, ny: int = 50, noise_amp: float = 1e-3) -> Case:
    """The paper's initial state: homogeneous density 0.85 (plus seeded noise of
    +-noise_amp) between a solid substrate (row 0) and a solid top row."""
    p = paper_params(nx, ny)
    solid = flat_channel(nx, ny)
    rho = np.full((ny, nx), PAPER_RHO)
    if noise_amp:
        rho = rho + noise(seed, rho.shape, noise_amp)
    return Case(p, solid, rho, name=f"paper_droplet{nx}x{ny}_s{seed}")


# Flat-interface coexistence densities of the lattice model under reading R29
# (vapour, liquid), from a settled slab in the oracle (tests/test_oracle_paper_droplet.py).
PAPER_COEX = (0.0426, 2.83)
PAPER_BODY_FORCE = 8.0e-6      # the rightward body force f_b of the paper's channel runs


def paper_channel_case(nx: int = 256, ny: int = 80, f_elec: float = 0.0, seed: int = 0, a: int = 8, b: int = 4,
                       p: int = 32, vapor_layer: int = 2, noise_amp: float = 1e-3, storage: int = 0) -> Case:
    """The paper's rough-wall channel run under reading R29: steps of width a,
    height b and pitch p on both walls (random phases), width ny, periodic in
    x; liquid with a vapour layer within ``vapor_layer`` nodes of the walls;
    both walls electrodes with the electric force on the single fluid layer
    next to them; the rightward body force f_b = 8e-6 applied as rho g with
    g = f_b (per unit density, the form of the other channel runs)."""
    solid = periodic_bumps(nx, ny, a, b, p, seed)
    rv, rl = PAPER_COEX
    near = chebyshev_dilate(solid, vapor_layer)
    rho = np.where(near, rv, rl).astype(np.float64)
    prm = paper_params(nx, ny, f_elec=f_elec, elec_walls=ELEC_BOTTOM | ELEC_TOP, accel_x=PAPER_BODY_FORCE,
                       storage=storage, rho_ref=rl)
    if noise_amp:
        rho = rho + noise(seed, rho.shape, noise_amp)
    return Case(prm, solid, rho, name=f"paper_channel{nx}x{ny}_f{f_elec:g}_s{seed}")


def attraction_field(nx: int, ny: int, g: float, solid: np.ndarray | None = None,
                     cx: float | None = None, cy: float = 0.5) -> np.ndarray:
    """Acceleration of magnitude g towards the point (cx, cy) (default: the
    middle of the substrate, on the wall plane), [2][ny][nx] float32, zero on
    solid nodes: the artificial attraction that gathers the fluid into one
    droplet in the middle of the substrate."""
    if cx is None:
        cx = (nx - 1) / 2.0
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    dx, dy = cx - x, cy - y
    r = np.hypot(dx, dy)
    r = np.where(r > 0, r, 1.0)
    a = np.stack([g * dx / r, g * dy / r])
    if solid is not None:
        a[:, solid != 0] = 0.0
    return a.astype(np.float32)


def droplet_case(f_elec: float = 0.0, seed: int = 0, nx: int = 128, ny: int = 64,
                 R: float = 20.0, noise_amp: float = 1e-3, G: float = -5.0,
                 rho_l: float = 2.0, rho_v: float = 0.15, layers: int = 2) -> Case:
    """Sessile droplet on a smooth bottom electrode (128x64, R = 20, G = -5).

    Rows 0 and ny-1 are solid; the droplet is centred at ((nx-1)/2, 0.5), i.e. on
    the bottom wall plane under halfway bounce-back.  The electric force acts on
    liquid within ``layers`` cells of the bottom wall.
    """
    p = params_for_G(nx, ny, G, f_elec=f_elec, elec_layers=layers, elec_walls=ELEC_BOTTOM)
    solid = flat_channel(nx, ny)
    rho = droplet_density(nx, ny, R, rho_l, rho_v)
    if noise_amp:
        rho = rho + noise(seed, rho.shape, noise_amp)
    return Case(p, solid, rho, name=f"droplet{nx}x{ny}_f{f_elec:g}_s{seed}")


def channel_case(nx: int, ny: int, solid: np.ndarray, G: float = -5.0, f_elec: float = 0.0,
                 accel: float = 1e-6, seed: int = 0, noise_amp: float = 1e-3,
                 vapor_layer: int = 2, layers: int = 2, tau: float = 1.0, storage: int = 0,
                 name: str = "channel", rho_ref: float | None = None) -> Case:
    """Liquid-filled channel with a vapour layer within ``vapor_layer`` cells of the walls.

    With ``rho_ref`` None, populations are stored as deviations from the rest
    state of the majority phase (the median initial fluid density), so that the
    stored numbers are small on most nodes; pass 0 for the format's default."""
    rv, rl = coexistence(G)
    near = chebyshev_dilate(solid, vapor_layer)
    rho = np.where(near, rv, rl).astype(np.float64)
    if rho_ref is None:
        rho_ref = float(np.median(rho[solid == 0])) if (solid == 0).any() else 0.0
    p = params_for_G(nx, ny, G, f_elec=f_elec, elec_layers=layers,
                     elec_walls=ELEC_BOTTOM | ELEC_TOP, accel_x=accel, tau=tau, storage=storage,
                     rho_ref=rho_ref)
    if noise_amp:
        rho = rho + noise(seed, rho.shape, noise_amp)
    return Case(p, solid, rho, name=name)


def rough_channel_case(nx: int = 1024, ny: int = 128, f_elec: float = 0.0, seed: int = 0,
                       a: int = 8, b: int = 4, p: int = 32, **kw) -> Case:
    """Rough-wall channel with periodic steps (1024x128, a=8, b=4, p=32 by default)."""
    solid = periodic_bumps(nx, ny, a, b, p, seed)
    return channel_case(nx, ny, solid, f_elec=f_elec, seed=seed,
                        name=f"rough{nx}x{ny}_f{f_elec:g}_s{seed}", **kw)


def random_channel_case(nx: int = 8192, ny: int = 2048, f_elec: float = 1e-3, seed: int = 0,
                        storage: int = 0, **kw) -> Case:
    """Large channel with random step roughness (height 2..8, pitch 16..64)."""
    solid = random_bumps(nx, ny, seed)
    return channel_case(nx, ny, solid, f_elec=f_elec, seed=seed, storage=storage,
                        name=f"random{nx}x{ny}_s{seed}", **kw)


def sweep_table(n: int = 256, seed: int = 0):
    """Channel descriptors of the batched sweep, drawn in order from SplitMix64(seed).

    Per channel: width W ~ U{32..256}, length L ~ U{512..4096}, step height
    b ~ U{0..8}, field strength f ~ U(0, 3e-3), G ~ U[-5.5, -4.5], and a seed.
    """
    rng = SplitMix64(seed)
    rows = []
    for i in range(n):
        W = rng.randint(32, 256)
        L = rng.randint(512, 4096)
        b = rng.randint(0, 8)
        f = 3e-3 * rng.uniform()
        G = -5.5 + rng.uniform()
        rows.append(dict(index=i, ny=W, nx=L, b=b, f_elec=f, G=G, seed=(seed << 16) + i))
    return rows


def sweep_case(row: dict, storage: int = 1, accel: float = 1e-6, noise_amp: float = 1e-3,
               rounding: int = 0) -> Case:
    """Build one channel of the sweep table (steps a = 8, pitch 32, random phases)."""
    nx, ny = row["nx"], row["ny"]
    solid = periodic_bumps(nx, ny, 8, row["b"], 32, row["seed"])
    c = channel_case(nx, ny, solid, G=row["G"], f_elec=row["f_elec"], accel=accel,
                     seed=row["seed"], noise_amp=noise_amp, storage=storage,
                     name=f"sweep{row['index']}")
    c.params = c.params.replace(rounding=rounding)
    return c


def warm_row(seed: int) -> dict:
    """Channel descriptor of the warm-start data set, drawn in order from
    SplitMix64(seed): step height b ~ U{0..8} (steps of width 8, pitch 32),
    field strength f ~ U(0, 3e-3), G ~ U[-5.5, -4.5], and the seed of the step
    phases."""
    rng = SplitMix64(seed)
    b = rng.randint(0, 8)
    f = 3e-3 * rng.uniform()
    G = -5.5 + rng.uniform()
    geo = rng.next() >> 32                  # stream of the step phases
    return dict(seed=seed, b=b, f_elec=f, G=G, geo_seed=geo)


def warm_case(seed: int, nx: int = 256, ny: int = 64, storage: int = 0, accel: float = 1e-6) -> Case:
    """One 256 x 64 channel of the warm-start data set (see ``warm_row``)."""
    row = warm_row(seed)
    solid = periodic_bumps(nx, ny, 8, row["b"], 32, row["geo_seed"])
    c = channel_case(nx, ny, solid, G=row["G"], f_elec=row["f_elec"], accel=accel, seed=seed,
                     storage=storage, name=f"warm{seed}")
    c.meta.update(row)
    return c
