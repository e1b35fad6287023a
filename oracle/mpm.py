"""Dense-grid explicit MPM step in float64 (test infrastructure only).

The sparse method changes only where nodal quantities are stored, not what is
computed (Methods 3.1, closing paragraph; Methods 3.2, "the sparse
representation does not change the original MPM formulation"; Results 2.2.1,
sparse and dense results identical).  This module is therefore the plain
definition: a dense background grid over the whole potential domain and the
update of Methods 3.1 (Eqs. 6-17 in display order), with

* quadratic B-spline shape functions (Methods 3.1; textbook piecewise form),
* APIC transfers (Eqs. 6-8, 13-16),
* internal and external nodal forces (Eqs. 9-10) and explicit Euler (Eqs. 11-12),
* the deformation-gradient update with the exact shape-function gradient (Eq. 17),
* Hencky elasticity or a Drucker-Prager return map on Hencky strain (the paper
  names the models, Methods 3.1, but prints no formulas; the forms used are
  stated in the functions below).

Where the paper is silent the readings are:

* base node and index arithmetic: b = floor(x * (1/dx) - 0.5) evaluated in
  float64 with each operation rounded separately, from float32 positions;
* the particle support used for the active set is the full 3^d stencil from b
  (it includes the node of zero weight at exact half-cell ties);
* the stress term of Eq. 9 uses sigma_p V_p = tau_p V0_p (Kirchhoff stress of
  the elastic deformation gradient times the initial volume);
* Eq. 17 multiplies the elastic deformation gradient left by the previous
  return map; the time integration is symplectic Euler (grid first, Eq. 12,
  then positions with the new velocity, Eq. 14);
* boundary conditions (not in the paper): walls are the nodes within ``bound``
  of each face, each face sticky / slip / separating or free, plus an optional
  heightmap level set with Coulomb friction.

Layout: positions (N, d), velocities (N, d), C, F and tau as (N, d, d).
"""
from __future__ import annotations

from dataclasses import dataclass
import itertools

import numpy as np

MODEL_ELASTIC = "elastic"
MODEL_DP = "dp"
BC_NONE, BC_STICKY, BC_SLIP, BC_SEPARATE = "none", "sticky", "slip", "separate"


class DomainError(RuntimeError):
    """A particle's support leaves the potential domain."""


class InvertedError(RuntimeError):
    """A trial deformation gradient has det <= 0."""


@dataclass
class Params:
    dim: int
    dx: float
    cells: tuple
    gravity: tuple
    dt: float
    p_mass: float
    p_vol0: float
    model: str = MODEL_DP
    E: float = 1.0e6
    nu: float = 0.3
    friction_deg: float = 30.0
    bound: int = 3
    bc: tuple = ((BC_NONE, BC_NONE),) * 3
    heightmap: np.ndarray | None = None
    mu_terrain: float = 0.0

    @property
    def nodes(self) -> tuple:
        return tuple(c + 1 for c in self.cells[: self.dim])

    @classmethod
    def from_workload(cls, w) -> "Params":
        return cls(dim=w.dim, dx=w.dx, cells=tuple(w.cells), gravity=tuple(w.gravity), dt=w.dt,
                   p_mass=w.p_mass, p_vol0=w.p_vol0, model=w.model, E=w.E, nu=w.nu,
                   friction_deg=w.friction_deg, bound=w.bound, bc=tuple(tuple(s) for s in w.bc),
                   heightmap=None if w.heightmap is None else np.asarray(w.heightmap, np.float64),
                   mu_terrain=w.mu_terrain)


def lame(E: float, nu: float):
    """Lame parameters (mu, lambda) of an isotropic material."""
    return E / (2.0 * (1.0 + nu)), E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))


# ---------------------------------------------------------------------------
# state conversion between the SoA float32 layout and (N, d, d) float64
def tau_from_soa(t: np.ndarray, d: int) -> np.ndarray:
    t = np.asarray(t, np.float64)
    n = t.shape[1]
    out = np.zeros((n, d, d))
    if d == 2:
        out[:, 0, 0], out[:, 1, 1] = t[0], t[1]
        out[:, 0, 1] = out[:, 1, 0] = t[2]
    else:
        out[:, 0, 0], out[:, 1, 1], out[:, 2, 2] = t[0], t[1], t[2]
        out[:, 0, 1] = out[:, 1, 0] = t[3]
        out[:, 1, 2] = out[:, 2, 1] = t[4]
        out[:, 0, 2] = out[:, 2, 0] = t[5]
    return out


def tau_to_soa(t: np.ndarray) -> np.ndarray:
    d = t.shape[1]
    if d == 2:
        return np.stack([t[:, 0, 0], t[:, 1, 1], t[:, 0, 1]])
    return np.stack([t[:, 0, 0], t[:, 1, 1], t[:, 2, 2], t[:, 0, 1], t[:, 1, 2], t[:, 0, 2]])


def state_from_soa(st: dict, d: int) -> dict:
    """float32 SoA arrays -> float64 (N, ...) arrays (exact widening)."""
    n = st["x"].shape[1]
    return {
        "x": np.asarray(st["x"], np.float64).T.copy(),
        "v": np.asarray(st["v"], np.float64).T.copy(),
        "C": np.asarray(st["C"], np.float64).T.reshape(n, d, d).copy(),
        "F": np.asarray(st["F"], np.float64).T.reshape(n, d, d).copy(),
        "tau": tau_from_soa(st["tau"], d),
    }


def state_to_soa(st: dict) -> dict:
    n, d = st["x"].shape
    return {
        "x": st["x"].T.copy(),
        "v": st["v"].T.copy(),
        "C": st["C"].reshape(n, d * d).T.copy(),
        "F": st["F"].reshape(n, d * d).T.copy(),
        "tau": tau_to_soa(st["tau"]),
    }


# ---------------------------------------------------------------------------
# quadratic B-spline (Methods 3.1: "quadratic B-splines")
def bspline(u):
    """1D quadratic B-spline N(u), support |u| < 3/2 (textbook piecewise form)."""
    a = np.abs(u)
    return np.where(a < 0.5, 0.75 - a * a, np.where(a < 1.5, 0.5 * (1.5 - a) ** 2, 0.0))


def bspline_deriv(u):
    """dN/du of the quadratic B-spline."""
    a = np.abs(u)
    s = np.sign(u)
    return np.where(a < 0.5, -2.0 * u, np.where(a < 1.5, -s * (1.5 - a), 0.0))


def base_node(x: np.ndarray, dx: float) -> np.ndarray:
    """Lowest node of the 3-node stencil per axis: floor(x * (1/dx) - 0.5).

    ``x`` holds float32 positions widened exactly to float64; the reciprocal,
    the product and the difference are each rounded to float64 (no fused
    multiply-add), which is the index arithmetic both implementations share.
    """
    r = 1.0 / dx
    s = np.asarray(x, np.float64) * r
    s = s - 0.5
    return np.floor(s).astype(np.int64)


def stencil_offsets(d: int):
    return list(itertools.product(range(3), repeat=d))


def check_domain(b: np.ndarray, p: Params):
    hi = np.array(p.cells[: p.dim])
    bad = (b < 0) | (b + 2 > hi)
    if bad.any():
        raise DomainError(f"{int(bad.any(axis=1).sum())} particle(s) with support outside the grid")


def shape_at(x: np.ndarray, n: np.ndarray, dx: float):
    """N_n(x_p) and grad N_n(x_p) for node indices n (N, d) at positions x (N, d).

    Tensor-product form N = prod_a N(x_a/dx - n_a), dN/dx_a = N'(.)/dx prod_{e!=a} N(.).
    """
    r = 1.0 / dx
    u = x * r - n
    w = bspline(u)
    dw = bspline_deriv(u) * r
    N = np.prod(w, axis=1)
    d = x.shape[1]
    g = np.empty_like(x)
    for a in range(d):
        g[:, a] = dw[:, a] * np.prod(np.delete(w, a, axis=1), axis=1)
    return N, g


# ---------------------------------------------------------------------------
# P2G (Eqs. 6, 7, 9, 10)
def p2g(state: dict, p: Params) -> dict:
    """Scatter mass, APIC momentum and forces onto the dense node grid.

    Returns m (nodes), mv (nodes + (d,)), f_int and f_ext (nodes + (d,)).
    """
    x, v, C, tau = state["x"], state["v"], state["C"], state["tau"]
    n_p, d = x.shape
    shape = p.nodes
    n_nodes = int(np.prod(shape))
    b = base_node(x, p.dx)
    check_domain(b, p)
    g = np.array(p.gravity[:d], np.float64)
    m = np.zeros(n_nodes)
    mv = np.zeros((n_nodes, d))
    fint = np.zeros((n_nodes, d))
    fext = np.zeros((n_nodes, d))
    for off in stencil_offsets(d):
        node = b + np.array(off)
        N, gradN = shape_at(x, node, p.dx)
        flat = np.ravel_multi_index(tuple(node.T), shape)
        xn = node * p.dx
        # Eq. 6
        m += np.bincount(flat, weights=N * p.p_mass, minlength=n_nodes)
        # Eq. 7: N m_p [v_p + C_p (x_n - x_p)]
        mom = v + np.einsum("pij,pj->pi", C, xn - x)
        # Eq. 9: -grad N sigma_p V_p with sigma_p V_p = tau_p V0_p
        f = -p.p_vol0 * np.einsum("pij,pj->pi", tau, gradN)
        for a in range(d):
            mv[:, a] += np.bincount(flat, weights=N * p.p_mass * mom[:, a], minlength=n_nodes)
            fint[:, a] += np.bincount(flat, weights=f[:, a], minlength=n_nodes)
            # Eq. 10
            fext[:, a] += np.bincount(flat, weights=N * p.p_mass * g[a], minlength=n_nodes)
    return {"m": m.reshape(shape), "mv": mv.reshape(shape + (d,)),
            "f_int": fint.reshape(shape + (d,)), "f_ext": fext.reshape(shape + (d,))}


# ---------------------------------------------------------------------------
# boundary conditions (not in the paper; see module docstring)
def node_coords(p: Params):
    return np.stack(np.meshgrid(*[np.arange(n) for n in p.nodes], indexing="ij"), axis=-1)


def terrain_normal(hm: np.ndarray, i: np.ndarray, j: np.ndarray, dx: float):
    """Unit upward normal of z = H(x, y) at node columns (i, j), by central
    differences (one-sided at the heightmap edges)."""
    ni, nj = hm.shape
    il, ih = np.maximum(i - 1, 0), np.minimum(i + 1, ni - 1)
    jl, jh = np.maximum(j - 1, 0), np.minimum(j + 1, nj - 1)
    hx = (hm[ih, j] - hm[il, j]) / ((ih - il) * dx)
    hy = (hm[i, jh] - hm[i, jl]) / ((jh - jl) * dx)
    n = np.stack([-hx, -hy, np.ones_like(hx)], axis=-1)
    return n / np.linalg.norm(n, axis=-1, keepdims=True)


def coulomb(v: np.ndarray, n: np.ndarray, mu: float) -> np.ndarray:
    """Frictional contact of velocities v with a surface of unit normal n:
    separating motion is free; otherwise the normal approach is removed and the
    tangential velocity is reduced by mu times the removed normal speed, or
    stopped when that exceeds it (Coulomb stick)."""
    vn = np.sum(v * n, axis=-1)
    vt = v - vn[..., None] * n
    tn = np.linalg.norm(vt, axis=-1)
    out = v.copy()
    approach = vn < 0
    stick = approach & (tn <= -mu * vn)
    slide = approach & ~stick
    out[stick] = 0.0
    scale = 1.0 + mu * vn[slide] / tn[slide]
    out[slide] = vt[slide] * scale[:, None]
    return out


def apply_bc(vel: np.ndarray, p: Params) -> np.ndarray:
    """Boundary conditions on nodal velocities (nodes + (d,)); terrain first, then walls."""
    d = p.dim
    v = vel.copy()
    idx = node_coords(p)
    if p.heightmap is not None and d == 3:
        hm = p.heightmap
        z = idx[..., 2] * p.dx
        inside = z <= hm[idx[..., 0], idx[..., 1]]
        if inside.any():
            ii, jj = idx[..., 0][inside], idx[..., 1][inside]
            n = terrain_normal(hm, ii, jj, p.dx)
            v[inside] = coulomb(v[inside], n, p.mu_terrain)
    for a in range(d):
        for side in (0, 1):
            kind = p.bc[a][side]
            if kind == BC_NONE:
                continue
            sel = idx[..., a] < p.bound if side == 0 else idx[..., a] > p.cells[a] - p.bound
            if kind == BC_STICKY:
                v[sel] = 0.0
            elif kind == BC_SLIP:
                v[sel, a] = 0.0
            elif kind == BC_SEPARATE:
                v[sel, a] = np.maximum(v[sel, a], 0.0) if side == 0 else np.minimum(v[sel, a], 0.0)
            else:
                raise ValueError(kind)
    return v


# ---------------------------------------------------------------------------
# grid update (Eqs. 8, 11, 12)
def grid_update(grid: dict, p: Params) -> np.ndarray:
    """v_n = (m v)_n / m_n; v_n^{n+1} = v_n + dt/m_n (f_int + f_ext); zero where m_n = 0;
    then boundary conditions.  Returns the new nodal velocity (nodes + (d,))."""
    m = grid["m"][..., None]
    has = m > 0
    safe = np.where(has, m, 1.0)
    v = np.where(has, grid["mv"] / safe, 0.0)
    vnew = np.where(has, v + p.dt / safe * (grid["f_int"] + grid["f_ext"]), 0.0)
    return apply_bc(vnew, p)


# ---------------------------------------------------------------------------
# constitutive models (Methods 3.1 names them; forms are the standard ones cited)
def svd_proper(F: np.ndarray):
    """SVD F = U diag(s) V^T with s > 0; raises if det F <= 0."""
    det = np.linalg.det(F)
    if (det <= 0).any():
        raise InvertedError(f"{int((det <= 0).sum())} deformation gradient(s) with det <= 0")
    U, s, Vt = np.linalg.svd(F)
    return U, s, Vt


def dp_alpha(friction_deg: float) -> float:
    """Drucker-Prager cone coefficient matched to a Mohr-Coulomb friction angle,
    alpha = sqrt(2/3) * 2 sin(phi) / (3 - sin(phi)) (Klar et al. 2016, SIGGRAPH,
    "Drucker-Prager elastoplasticity for sand animation")."""
    s = np.sin(np.deg2rad(friction_deg))
    return np.sqrt(2.0 / 3.0) * 2.0 * s / (3.0 - s)


def project_strain(eps: np.ndarray, p: Params) -> np.ndarray:
    """Return map of principal Hencky strains eps (N, d) onto the cohesionless
    Drucker-Prager cone (no hardening), Klar et al. 2016:

    tr eps > 0 (tension)             -> eps' = 0 (cone tip);
    else dgamma = |dev eps| + (d lambda + 2 mu)/(2 mu) tr(eps) alpha;
         dgamma <= 0                 -> eps' = eps (elastic);
         else                        -> eps' = eps - dgamma dev(eps)/|dev eps|.
    """
    if p.model == MODEL_ELASTIC:
        return eps.copy()
    mu, lam = lame(p.E, p.nu)
    d = eps.shape[1]
    alpha = dp_alpha(p.friction_deg)
    tr = eps.sum(axis=1)
    dev = eps - tr[:, None] / d
    nd = np.linalg.norm(dev, axis=1)
    dgamma = nd + (d * lam + 2 * mu) / (2 * mu) * tr * alpha
    out = eps.copy()
    tip = tr > 0
    plastic = (~tip) & (dgamma > 0)
    out[tip] = 0.0
    out[plastic] = eps[plastic] - (dgamma[plastic] / nd[plastic])[:, None] * dev[plastic]
    return out


def constitutive(F_trial: np.ndarray, p: Params):
    """Elastic deformation gradient after the return map, and Kirchhoff stress:
    F^E = U diag(exp eps') V^T, tau = U diag(2 mu eps' + lambda tr eps') U^T
    (Hencky strain eps = log s of the singular values)."""
    mu, lam = lame(p.E, p.nu)
    U, s, Vt = svd_proper(F_trial)
    eps = np.log(s)
    eps_new = project_strain(eps, p)
    Fe = np.einsum("pij,pj,pjk->pik", U, np.exp(eps_new), Vt)
    diag = 2 * mu * eps_new + lam * eps_new.sum(axis=1, keepdims=True)
    tau = np.einsum("pij,pj,pkj->pik", U, diag, U)
    return Fe, tau


# ---------------------------------------------------------------------------
# G2P (Eqs. 13-17)
def g2p(state: dict, vgrid: np.ndarray, p: Params) -> dict:
    """Gather the updated nodal velocity back to the particles and advance them."""
    x, F = state["x"], state["F"]
    n_p, d = x.shape
    b = base_node(x, p.dx)
    check_domain(b, p)
    vp = np.zeros((n_p, d))
    Bp = np.zeros((n_p, d, d))
    Dp = np.zeros((n_p, d, d))
    gradv = np.zeros((n_p, d, d))
    for off in stencil_offsets(d):
        node = b + np.array(off)
        N, gradN = shape_at(x, node, p.dx)
        vn = vgrid[tuple(node.T)]
        dxn = node * p.dx - x
        vp += N[:, None] * vn                                   # Eq. 13
        Bp += N[:, None, None] * vn[:, :, None] * dxn[:, None, :]  # Eq. 15 numerator
        Dp += N[:, None, None] * dxn[:, :, None] * dxn[:, None, :]  # Eq. 16
        gradv += vn[:, :, None] * gradN[:, None, :]             # Eq. 17 sum
    Cp = Bp @ np.linalg.inv(Dp)                                 # Eq. 15
    x_new = x + p.dt * vp                                        # Eq. 14
    F_trial = (np.eye(d)[None] + p.dt * gradv) @ F               # Eq. 17
    Fe, tau = constitutive(F_trial, p)
    return {"x": x_new, "v": vp, "C": Cp, "F": Fe, "tau": tau, "F_trial": F_trial, "gradv": gradv}


def step(state: dict, p: Params, return_grid: bool = False):
    """One explicit step: P2G -> grid update -> G2P."""
    grid = p2g(state, p)
    vgrid = grid_update(grid, p)
    out = g2p(state, vgrid, p)
    if return_grid:
        return out, grid, vgrid
    return out
