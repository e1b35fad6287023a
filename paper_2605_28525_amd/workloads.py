"""Seeded synthetic inputs for the sparse-grid MPM step.

This module only *places* material: it draws particle positions, builds the
terrain heightmap and records the physical constants of each workload.  It holds
none of the method's arithmetic (no shape functions, no transfers, no stress),
so that both the FP64 reference used by the tests and the HIP path can start from
the same arrays.

Workloads (stand-ins for the paper's examples, whose geometry is not printed):

* ``collapse_2d``      granular column collapse in 2D (the paper's collapse
                       example, Results "Low sparsity examples"): 512x128 cells,
                       dx = 0.01 m, a 32x32-cell column at 4 particles/cell.
* ``collapse_3d``      the same in 3D: 512x128x128 cells, a 64^3-cell column at
                       8 particles/cell (2,097,152 particles); ``scale=2`` gives the
                       1/8-volume copy (256x64x64 cells, 32^3-cell column).
* ``landslide``        synthetic stand-in for the Blatten rock-ice avalanche
                       (Results "Blatten landslide simulation"): 2048x2048x256
                       cells at dx = 1 m over a fractal terrain, a 250x250x40 m
                       release at 8 particles/cell (20,000,000 particles).
* ``landslide_crop``   a small window of the same terrain and release for
                       reference checks on the CPU.
* ``elastic_bar_2d``   a free-free elastic bar for the wave-speed check.

Particle state is SoA float32, component-major: ``x[a, p]``; ``C`` and ``F`` are
row-major d x d per particle (``F[r*d + c, p]``); ``tau`` holds the symmetric
Kirchhoff stress as (xx, yy, xy) in 2D and (xx, yy, zz, xy, yz, xz) in 3D.
Boundary conditions are named by strings (``"none"``, ``"sticky"``, ``"slip"``,
``"separate"``) per axis and side, so that each consumer maps them to its own
enumeration.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np


@dataclass
class Workload:
    name: str
    dim: int
    dx: float
    cells: tuple            # cells per axis (len == dim)
    gravity: tuple          # m/s^2, len 3 (unused components zero)
    dt: float
    steps: int
    model: str              # "dp" | "elastic"
    E: float
    nu: float
    rho: float
    friction_deg: float
    ppc: int
    p_vol0: float
    p_mass: float
    bound: int = 3
    bc: tuple = (("separate", "separate"), ("sticky", "separate"), ("separate", "separate"))
    heightmap: np.ndarray | None = None     # float32 (cells[0]+1, cells[1]+1), node heights
    mu_terrain: float = 0.0
    x: np.ndarray = field(default=None, repr=False)
    v: np.ndarray = field(default=None, repr=False)
    C: np.ndarray = field(default=None, repr=False)
    F: np.ndarray = field(default=None, repr=False)
    tau: np.ndarray = field(default=None, repr=False)
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[1])

    @property
    def n_stress(self) -> int:
        return 3 if self.dim == 2 else 6

    def state(self) -> dict:
        """Copy of the particle state arrays (float32, SoA)."""
        return {k: getattr(self, k).copy() for k in ("x", "v", "C", "F", "tau")}


def rest_state(x: np.ndarray) -> dict:
    """Material at rest, undeformed and unstressed: v = 0, C = 0, F = I, tau = 0."""
    d, n = x.shape
    F = np.zeros((d * d, n), np.float32)
    for a in range(d):
        F[a * d + a] = 1.0
    return {
        "x": np.ascontiguousarray(x, dtype=np.float32),
        "v": np.zeros((d, n), np.float32),
        "C": np.zeros((d * d, n), np.float32),
        "F": F,
        "tau": np.zeros((3 if d == 2 else 6, n), np.float32),
    }


def stratified_cells(cells_lo, cells_hi, dx, per_axis, rng) -> np.ndarray:
    """Jittered particles in every cell of the box [lo, hi) (cell indices).

    Each cell is split into ``per_axis**d`` sub-cells and one particle is placed
    uniformly at random inside each sub-cell.  Returns float32 (d, N), cell-major.
    """
    d = len(cells_lo)
    axes = [np.arange(cells_lo[a], cells_hi[a], dtype=np.float64) for a in range(d)]
    cell = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, d)
    sub = np.stack(np.meshgrid(*([np.arange(per_axis, dtype=np.float64)] * d), indexing="ij"),
                   axis=-1).reshape(-1, d)
    jit = rng.random((cell.shape[0], sub.shape[0], d))
    pos = (cell[:, None, :] + (sub[None, :, :] + jit) / per_axis) * dx
    return np.ascontiguousarray(pos.reshape(-1, d).T.astype(np.float32))


def stratified_columns(i_range, j_range, k0, thickness, dx, per_axis, rng) -> np.ndarray:
    """Jittered particles in vertical cell columns (i, j) from cell k0[i, j] upwards."""
    ii, jj = np.meshgrid(np.arange(*i_range), np.arange(*j_range), indexing="ij")
    ii = ii.ravel()
    jj = jj.ravel()
    kk0 = k0.ravel()
    kz = np.arange(thickness)
    ci = np.repeat(ii, thickness).astype(np.float64)
    cj = np.repeat(jj, thickness).astype(np.float64)
    ck = (kk0[:, None] + kz[None, :]).ravel().astype(np.float64)
    cell = np.stack([ci, cj, ck], axis=1)
    sub = np.stack(np.meshgrid(*([np.arange(per_axis, dtype=np.float64)] * 3), indexing="ij"),
                   axis=-1).reshape(-1, 3)
    out = np.empty((3, cell.shape[0] * sub.shape[0]), np.float32)
    chunk = 1 << 20
    for s in range(0, cell.shape[0], chunk):
        c = cell[s:s + chunk]
        jit = rng.random((c.shape[0], sub.shape[0], 3))
        pos = (c[:, None, :] + (sub[None, :, :] + jit) / per_axis) * dx
        out[:, s * sub.shape[0]:(s + c.shape[0]) * sub.shape[0]] = pos.reshape(-1, 3).T
    return out


def _smoothstep(t):
    return t * t * (3.0 - 2.0 * t)


def value_noise_fbm(nx, ny, spacing, base_wavelength, octaves, lacunarity, gain, amplitude, rng):
    """Fractal (fBm) value noise on an nx x ny node lattice, peak amplitude ``amplitude``.

    Each octave draws uniform lattice values in [-1, 1] at its wavelength and
    interpolates them with a smoothstep blend; octave o has weight gain**o,
    normalised so that the weights sum to ``amplitude``.
    """
    X = np.arange(nx, dtype=np.float64) * spacing
    Y = np.arange(ny, dtype=np.float64) * spacing
    weights = np.array([gain ** o for o in range(octaves)])
    weights *= amplitude / weights.sum()
    total = np.zeros((nx, ny))
    wl = float(base_wavelength)
    for o in range(octaves):
        gx = int(math.ceil(X[-1] / wl)) + 2
        gy = int(math.ceil(Y[-1] / wl)) + 2
        lat = rng.uniform(-1.0, 1.0, size=(gx, gy))
        fx = X / wl
        fy = Y / wl
        ix = np.floor(fx).astype(np.int64)
        iy = np.floor(fy).astype(np.int64)
        tx = _smoothstep(fx - ix)[:, None]
        ty = _smoothstep(fy - iy)[None, :]
        v00 = lat[ix[:, None], iy[None, :]]
        v10 = lat[ix[:, None] + 1, iy[None, :]]
        v01 = lat[ix[:, None], iy[None, :] + 1]
        v11 = lat[ix[:, None] + 1, iy[None, :] + 1]
        total += weights[o] * ((v00 * (1 - tx) + v10 * tx) * (1 - ty) + (v01 * (1 - tx) + v11 * tx) * ty)
        wl /= lacunarity
    return total


# ---------------------------------------------------------------------------
# material shared by the collapse workloads
_SAND = dict(model="dp", E=1.0e6, nu=0.3, rho=2000.0, friction_deg=30.0)


def collapse_2d(seed: int = 0) -> Workload:
    """2D granular column collapse: 512x128 cells, 32x32-cell column, 4 ppc (4096 particles)."""
    dx = 0.01
    rng = np.random.default_rng(seed)
    x = stratified_cells((3, 3), (35, 35), dx, 2, rng)
    vol = dx * dx / 4
    w = Workload(name="collapse_2d", dim=2, dx=dx, cells=(512, 128), gravity=(0.0, -9.81, 0.0),
                 dt=1e-4, steps=200, ppc=4, p_vol0=vol, p_mass=_SAND["rho"] * vol,
                 bc=(("separate", "separate"), ("sticky", "separate"), ("none", "none")), **_SAND)
    for k, a in rest_state(x).items():
        setattr(w, k, a)
    return w


def collapse_3d(seed: int = 1, scale: int = 1) -> Workload:
    """3D granular column collapse: 512x128x128 cells, 64^3-cell column, 8 ppc.

    ``scale=2`` halves every length (256x64x64 cells, 32^3-cell column,
    262,144 particles) for the reference copy.
    """
    dx = 0.01
    rng = np.random.default_rng(seed)
    s = scale
    cells = (512 // s, 128 // s, 128 // s)
    lo = (3, 3, 32 // s)
    hi = (3 + 64 // s, 3 + 64 // s, 32 // s + 64 // s)
    x = stratified_cells(lo, hi, dx, 2, rng)
    vol = dx ** 3 / 8
    w = Workload(name="collapse_3d" + ("" if s == 1 else f"_1of{s ** 3}"), dim=3, dx=dx, cells=cells,
                 gravity=(0.0, -9.81, 0.0), dt=1e-4, steps=2000, ppc=8, p_vol0=vol,
                 p_mass=_SAND["rho"] * vol,
                 bc=(("separate", "separate"), ("sticky", "separate"), ("separate", "separate")), **_SAND)
    for k, a in rest_state(x).items():
        setattr(w, k, a)
    return w


def landslide_terrain(cells=(2048, 2048), dx=1.0, seed=2):
    """Node heightmap: a planar slope from z = 205 m down to a runout plain at z = 5 m,
    plus 5 octaves of value-noise fBm (base wavelength 256 m, lacunarity 2, gain 0.5,
    peak amplitude 4 m).  The slope angle is drawn from U[25, 40] degrees."""
    rng = np.random.default_rng(seed)
    theta = np.deg2rad(rng.uniform(25.0, 40.0))
    nx, ny = cells[0] + 1, cells[1] + 1
    X = np.arange(nx, dtype=np.float64) * dx
    profile = np.maximum(205.0 - X * np.tan(theta), 5.0)
    noise = value_noise_fbm(nx, ny, dx, 256.0, 5, 2.0, 0.5, 4.0, rng)
    return (profile[:, None] + noise).astype(np.float32), float(np.rad2deg(theta))


def landslide(seed_terrain: int = 2, seed_particles: int = 102, window=None,
              footprint=((20, 270), (899, 1149)), thickness: int = 40, h: int = 1) -> Workload:
    """Synthetic landslide: 2048x2048x256 cells at dx = 1 m, a 250x250 m footprint,
    40 m thick, 8 ppc (20,000,000 particles) released on the slope at rest.

    ``h`` (1, 2 or 4) coarsens the same slide to dx = h metres: the terrain
    sampled at every h-th node, 256 / h cells high, the default footprint and
    thickness divided by h (rounded to whole cells), 8 ppc, dt = h ms.

    ``window=((i0, i1), (j0, j1))`` restricts the potential domain to that range
    of node columns of the (coarsened) terrain (cell counts i1-i0, j1-j0; height
    kept), with ``footprint`` and ``thickness`` given in the window's own cells.
    """
    if h not in (1, 2, 4):
        raise ValueError("h must be 1, 2 or 4")
    hm_full, theta = landslide_terrain((2048, 2048), 1.0, seed_terrain)
    hm_h = hm_full if h == 1 else np.ascontiguousarray(hm_full[::h, ::h])
    dx = float(h)
    if window is None:
        hm = hm_h
        cells = (2048 // h, 2048 // h, 256 // h)
        if h != 1:
            (a0, a1), (b0, b1) = footprint
            footprint = ((round(a0 / h), round(a1 / h)), (round(b0 / h), round(b1 / h)))
            thickness = round(thickness / h)
    else:
        (i0, i1), (j0, j1) = window
        hm = np.ascontiguousarray(hm_h[i0:i1 + 1, j0:j1 + 1])
        cells = (i1 - i0, j1 - j0, 256 // h)
    rng = np.random.default_rng(seed_particles)
    (fi0, fi1), (fj0, fj1) = footprint
    # lowest cell of each column lies on or above the terrain at all four corner nodes
    corner = np.maximum(np.maximum(hm[fi0:fi1, fj0:fj1], hm[fi0 + 1:fi1 + 1, fj0:fj1]),
                        np.maximum(hm[fi0:fi1, fj0 + 1:fj1 + 1], hm[fi0 + 1:fi1 + 1, fj0 + 1:fj1 + 1]))
    k0 = np.ceil(corner.astype(np.float64) / dx).astype(np.int64)
    x = stratified_columns((fi0, fi1), (fj0, fj1), k0, thickness, dx, 2, rng)
    vol = dx ** 3 / 8
    name = "landslide" if h == 1 else f"landslide_h{h}"
    if window is not None:
        name += "_crop"
    w = Workload(name=name, dim=3, dx=dx, cells=cells,
                 gravity=(0.0, 0.0, -9.81), dt=1e-3 * h, steps=5000, ppc=8, p_vol0=vol,
                 p_mass=2000.0 * vol, model="dp", E=5.0e7, nu=0.3, rho=2000.0, friction_deg=32.0,
                 bc=(("separate", "separate"), ("separate", "separate"), ("sticky", "separate")),
                 heightmap=hm, mu_terrain=0.4)
    w.meta["slope_deg"] = theta
    for k, a in rest_state(x).items():
        setattr(w, k, a)
    return w


def landslide_crop(seed_particles: int = 102) -> Workload:
    """A 64x64x256-cell window of the landslide terrain (nodes i in [0, 64],
    j in [992, 1056]) with a 16x16x8-cell release at 8 ppc (16,384 particles)."""
    return landslide(window=((0, 64), (992, 1056)), footprint=((20, 36), (24, 40)), thickness=8,
                     seed_particles=seed_particles)


SLIDE_MU = float(np.tan(np.deg2rad(15.0)))   # Coulomb coefficient of the sliding-block plane


def sliding_block(theta_deg: float, seed: int = 21, dx: float = 0.02, block_cells=(10, 5, 5),
                  E: float = 5.0e5, rho: float = 1000.0) -> Workload:
    """Elastic block released at rest on a plane inclined at ``theta_deg`` about the
    y axis: terrain z = 0.6 m - x tan(theta) over a 40x16x40-cell grid at dx = 0.02 m,
    Coulomb friction mu = tan 15 deg.  The block, 0.2 x 0.1 x 0.1 m (10x5x5 cells
    of dx along slope, across and normal), holds 8 particles per dx^3, stratified-
    jittered in the slope's own frame, the lowest ones within dx/2 above the plane;
    its upslope face starts 0.18 m down the plane from its x = 0 edge.  E = 5e5 Pa
    (nu = 0.3, rho = 1000 kg/m^3): stiff enough that the block's elastic settling
    after its release moves it by millimetres, so that it behaves as the rigid
    block of the closed form.
    ``meta``: the downslope unit vector and the slope angle."""
    th = np.deg2rad(theta_deg)
    rng = np.random.default_rng(seed)
    cells = (40, 16, 40)
    z0 = 0.6
    t_hat = np.array([np.cos(th), 0.0, -np.sin(th)])
    n_hat = np.array([np.sin(th), 0.0, np.cos(th)])
    local = stratified_cells((0, 0, 0), block_cells, dx, 2, rng).astype(np.float64)   # (s, w, n)
    s0, w0 = 0.1 + 4 * dx, 0.1
    anchor = np.array([s0 * np.cos(th), w0, z0 - s0 * np.sin(th)])
    x = anchor[:, None] + t_hat[:, None] * local[0] + np.array([0.0, 1.0, 0.0])[:, None] * local[1] \
        + n_hat[:, None] * local[2]
    X = np.arange(cells[0] + 1, dtype=np.float64) * dx
    hm = np.repeat((z0 - X * np.tan(th))[:, None], cells[1] + 1, axis=1).astype(np.float32)
    vol = dx ** 3 / 8
    w = Workload(name=f"sliding_block_{theta_deg:g}", dim=3, dx=dx, cells=cells, gravity=(0.0, 0.0, -9.81),
                 dt=0.3 * dx / float(np.sqrt(E * 0.7 / (1.3 * 0.4 * rho))), steps=0, ppc=8, p_vol0=vol,
                 p_mass=rho * vol, model="elastic", E=E, nu=0.3, rho=rho, friction_deg=0.0,
                 bc=(("separate", "separate"), ("separate", "separate"), ("separate", "separate")),
                 heightmap=hm, mu_terrain=SLIDE_MU)
    w.meta["downslope"] = t_hat
    w.meta["slope_deg"] = float(theta_deg)
    for k, a in rest_state(x.astype(np.float32)).items():
        setattr(w, k, a)
    return w


def elastic_bar_2d(length_cells: int = 128, thick_cells: int = 4, amplitude: float = 2.3e-3,
                   seed: int = 7) -> Workload:
    """Free-free elastic bar in 2D (plane strain) carrying its fundamental
    longitudinal mode v_x = A cos(pi (x - x0) / L); no wall within reach."""
    dx = 0.01
    rng = np.random.default_rng(seed)
    x0c, y0c = 8, 8
    x = stratified_cells((x0c, y0c), (x0c + length_cells, y0c + thick_cells), dx, 2, rng)
    cells = (length_cells + 16, thick_cells + 16)
    vol = dx * dx / 4
    w = Workload(name="elastic_bar_2d", dim=2, dx=dx, cells=cells, gravity=(0.0, 0.0, 0.0), dt=1e-4,
                 steps=0, ppc=4, p_vol0=vol, p_mass=1000.0 * vol, model="elastic", E=1.0e6, nu=0.3,
                 rho=1000.0, friction_deg=0.0,
                 bc=(("none", "none"), ("none", "none"), ("none", "none")))
    st = rest_state(x)
    L = length_cells * dx
    xs = x[0].astype(np.float64) - x0c * dx
    st["v"][0] = (amplitude * np.cos(np.pi * xs / L)).astype(np.float32)
    for k, a in st.items():
        setattr(w, k, a)
    w.meta.update(L=L, amplitude=amplitude, x0=x0c * dx)
    return w


def tiny_3d(n: int = 48, seed: int = 11, ties: bool = True) -> Workload:
    """A few dozen particles over a 16^3-cell box at dx = 0.25 m (a power of two,
    so that positions on half-cell ties are exact), including particles placed
    exactly on ties, on block corners and in cells with local index 3."""
    dx = 0.25
    rng = np.random.default_rng(seed)
    pts = rng.uniform(3.2, 12.8, size=(n, 3)) * dx
    if ties:
        # half-cell ties on every axis, and on single axes
        pts[0] = np.array([5.5, 7.5, 9.5]) * dx
        pts[1] = np.array([4.5, 6.3, 8.1]) * dx
        pts[2] = np.array([7.9, 7.5, 4.2]) * dx
        # block corners: base local index 3 on all axes (cells 7, 11)
        pts[3] = np.array([7.6, 11.7, 7.9]) * dx
        pts[4] = np.array([8.0, 8.0, 8.0]) * dx
        pts[5] = np.array([11.51, 3.52, 7.53]) * dx
    x = np.ascontiguousarray(pts.T.astype(np.float32))
    vol = dx ** 3 / 8
    w = Workload(name="tiny_3d", dim=3, dx=dx, cells=(16, 16, 16), gravity=(0.0, -9.81, 0.0), dt=1e-3,
                 steps=10, ppc=8, p_vol0=vol, p_mass=2000.0 * vol,
                 bc=(("separate", "separate"), ("sticky", "separate"), ("separate", "separate")), **_SAND)
    st = rest_state(x)
    st["v"] = rng.normal(0, 0.2, size=st["v"].shape).astype(np.float32)
    st["C"] = rng.normal(0, 0.5, size=st["C"].shape).astype(np.float32)
    F = st["F"] + rng.normal(0, 0.02, size=st["F"].shape).astype(np.float32)
    st["F"] = F.astype(np.float32)
    st["tau"] = rng.normal(0, 100.0, size=st["tau"].shape).astype(np.float32)
    for k, a in st.items():
        setattr(w, k, a)
    return w


def perturbed(w: Workload, seed: int, v_scale=0.05, C_scale=1.0, F_scale=1e-3, tau_scale=200.0) -> Workload:
    """Same geometry with a random but physically small state (velocity, affine
    matrix, deformation and stress), so that every term of the step is exercised."""
    rng = np.random.default_rng(seed)
    d, n = w.x.shape
    w.v = rng.normal(0, v_scale, size=(d, n)).astype(np.float32)
    w.C = rng.normal(0, C_scale, size=(d * d, n)).astype(np.float32)
    w.F = (w.F + rng.normal(0, F_scale, size=(d * d, n))).astype(np.float32)
    w.tau = rng.normal(0, tau_scale, size=w.tau.shape).astype(np.float32)
    return w


def differentiable_3d(seed: int = 3) -> Workload:
    """Calibration workload: the 3D column collapse at 1/8 volume (256x64x64
    cells, 32^3-cell column, 8 ppc, 262,144 particles), 400 steps."""
    w = collapse_3d(seed=seed, scale=2)
    w.name = "differentiable_3d"
    w.steps = 400
    return w


def differentiable_fd_copy(seed: int = 3) -> Workload:
    """Small copy for finite-difference checks: an 8^3-cell column at 8 ppc
    (4096 particles) in a 64x32x32-cell grid."""
    dx = 0.01
    rng = np.random.default_rng(seed)
    x = stratified_cells((3, 3, 12), (11, 11, 20), dx, 2, rng)
    vol = dx ** 3 / 8
    w = Workload(name="differentiable_fd_copy", dim=3, dx=dx, cells=(64, 32, 32), gravity=(0.0, -9.81, 0.0),
                 dt=1e-4, steps=400, ppc=8, p_vol0=vol, p_mass=_SAND["rho"] * vol,
                 bc=(("separate", "separate"), ("sticky", "separate"), ("separate", "separate")), **_SAND)
    for k, a in rest_state(x).items():
        setattr(w, k, a)
    return w


def calibration_target_velocity(n: int, dim: int = 3, seed: int = 1003) -> np.ndarray:
    """Initial velocity of the target run: (0.5, 0, 0) m/s plus N(0, 0.05^2) per
    particle and component."""
    rng = np.random.default_rng(seed)
    v = rng.normal(0.0, 0.05, size=(dim, n))
    v[0] += 0.5
    return v.astype(np.float32)


# ---------------------------------------------------------------------------
# ensembles of independent simulations
@dataclass
class Ensemble:
    """Independent 3D column collapses on identical potential grids.

    ``members[i]`` is instance i as a stand-alone workload (its own particles,
    material and dt); ``x .. tau`` hold every member's particles together and
    ``inst[p]`` names the instance of particle p.  The members' particles keep
    their relative order inside the combined arrays.
    """
    name: str
    members: list
    steps: int
    x: np.ndarray = field(default=None, repr=False)
    v: np.ndarray = field(default=None, repr=False)
    C: np.ndarray = field(default=None, repr=False)
    F: np.ndarray = field(default=None, repr=False)
    tau: np.ndarray = field(default=None, repr=False)
    inst: np.ndarray = field(default=None, repr=False)

    @property
    def n(self) -> int:
        return int(self.x.shape[1])

    @property
    def n_instances(self) -> int:
        return len(self.members)

    def state(self) -> dict:
        return {k: getattr(self, k).copy() for k in ("x", "v", "C", "F", "tau")}

    def member_positions(self, i: int) -> np.ndarray:
        """Positions in the combined arrays of instance i's particles, in member order."""
        return np.nonzero(self.inst == i)[0]


def ensemble(seed: int = 4, n_instances: int = 64, n_range=(5.0e4, 1.0e6), cells=(1020, 252, 252),
             steps: int = 1000, interleave: bool = False) -> Ensemble:
    """Batched column collapses: per instance N_i = round(exp U[ln a, ln b]) target
    particles, aspect a_i ~ U[0.5, 4], footprint L_i = round((N_i / (8 a_i))^(1/3))
    cells, height round(a_i L_i) cells (8 ppc, so the realised count is 8 L_i^2 H_i),
    friction angle U[20, 40] degrees, E_i = exp U[ln 1e6, ln 1e8] Pa, nu = 0.3,
    rho = 2000 kg/m^3, dt_i = 0.3 dx / c_P,i with c_P = sqrt((lambda + 2 mu) / rho),
    dx = 0.01 m.  Every instance has the same potential grid (``cells``) and
    walls; its column stands on the sticky floor y = 3 dx against the x = 3 dx
    wall, centred in z.  ``interleave`` mixes the instances' particles in the
    combined arrays (random merge that keeps each member's order)."""
    dx = 0.01
    rho, nu = 2000.0, 0.3
    rng = np.random.default_rng(seed)
    vol = dx ** 3 / 8
    members = []
    for i in range(n_instances):
        n_t = float(np.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1]))))
        a = float(rng.uniform(0.5, 4.0))
        L = max(1, int(round((n_t / (8 * a)) ** (1 / 3))))
        H = max(1, int(round(a * L)))
        phi = float(rng.uniform(20.0, 40.0))
        E = float(np.exp(rng.uniform(math.log(1e6), math.log(1e8))))
        mu = E / (2 * (1 + nu))
        lam = E * nu / ((1 + nu) * (1 - 2 * nu))
        dt = 0.3 * dx / math.sqrt((lam + 2 * mu) / rho)
        z0 = cells[2] // 2 - L // 2
        if 3 + L > cells[0] - 3 or 3 + H > cells[1] - 3 or z0 < 3 or z0 + L > cells[2] - 3:
            raise ValueError(f"instance {i}: a {L}x{H}x{L}-cell column does not fit {cells}")
        x = stratified_cells((3, 3, z0), (3 + L, 3 + H, z0 + L), dx, 2, rng)
        w = Workload(name=f"ensemble_member_{i}", dim=3, dx=dx, cells=tuple(cells), gravity=(0.0, -9.81, 0.0),
                     dt=dt, steps=steps, ppc=8, p_vol0=vol, p_mass=rho * vol,
                     bc=(("separate", "separate"), ("sticky", "separate"), ("separate", "separate")),
                     model="dp", E=E, nu=nu, rho=rho, friction_deg=phi,
                     meta={"aspect": a, "footprint_cells": L, "height_cells": H})
        for k, arr in rest_state(x).items():
            setattr(w, k, arr)
        members.append(w)
    counts = [m.n for m in members]
    inst = np.repeat(np.arange(n_instances, dtype=np.uint32), counts)
    ens = Ensemble(name=f"ensemble_{n_instances}", members=members, steps=steps)
    if interleave:
        inst = inst[rng.permutation(inst.size)]
    ens.inst = np.ascontiguousarray(inst)
    if interleave:
        pos = [np.nonzero(ens.inst == i)[0] for i in range(n_instances)]
    for k in ("x", "v", "C", "F", "tau"):
        if not interleave:
            setattr(ens, k, np.ascontiguousarray(np.concatenate([getattr(m, k) for m in members], axis=1)))
            continue
        rows = getattr(members[0], k).shape[0]
        out = np.empty((rows, inst.size), np.float32)
        for i, m in enumerate(members):
            out[:, pos[i]] = getattr(m, k)
        setattr(ens, k, out)
    return ens


def ensemble_small(seed: int = 5, n_instances: int = 6, interleave: bool = True) -> Ensemble:
    """A few small members (200 .. 3000 target particles) on a 64x32x32-cell
    grid, for reference checks."""
    return ensemble(seed=seed, n_instances=n_instances, n_range=(200.0, 3000.0), cells=(64, 32, 32), steps=20,
                    interleave=interleave)
