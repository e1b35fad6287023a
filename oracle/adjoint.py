"""Reverse mode of the FP64 dense-grid step (test infrastructure only).

The paper has no adjoint; this is the exact derivative of the oracle's
discrete step (``oracle.mpm.step``), written out by hand in the forward's own
order reversed, so that gradients of a loss on the final positions with
respect to the initial velocities, Young's modulus and the friction angle can
be checked.  Pinned in ``tests/test_oracle_adjoint.py`` by central finite
differences of the forward step (dot-product tests).

Conventions: the state is (x, v, C, F, tau) with tau a full d x d matrix; the
adjoint of tau is with respect to that full matrix.  The step's inputs are the
state at step n; its outputs are the state at step n + 1 (tau' = tau(F^E')).
Walls are differentiated (sticky / slip / separating); terrain boundaries are
not supported here.

Derivatives used
----------------
* Shape functions: N, grad N and the Hessian of the tensor-product B-spline
  (second derivative of the 1D quadratic B-spline: -2 on |u| < 1/2, +1 on
  1/2 <= |u| < 3/2).
* Grid update: u = p/m + dt g (m > 0), v = BC(u) with a diagonal 0/1 Jacobian
  for the walls; p_bar = u_bar / m, m_bar = -u_bar . (u - dt g) / m.
* Constitutive map: with b = F F^T = Q diag(lam) Q^T, eps = log(lam)/2,
  eps' = P(eps) (the return map), the stress tau = Q diag(t) Q^T with
  t = 2 mu eps' + lambda tr(eps') 1 and the elastic gradient F^E = Q diag(h) Q^T F
  with h = exp(eps' - eps) are isotropic functions of b.  Their adjoint is
  Q S Q^T with S_jj = sum_i J_ij Y_ii and S_ij = K_ij Y_ij (i != j), where
  Y = Q^T Ybar Q, J = d(t or h)/d lam and K_ij = (f_i - f_j)/(lam_i - lam_j),
  replaced by its limit J_ii - J_ij when the eigenvalues coincide
  (Daleckii-Krein formula for isotropic symmetric tensor functions).
"""
from __future__ import annotations

import numpy as np

from .mpm import (Params, base_node, check_domain, lame, dp_alpha, stencil_offsets, bspline, bspline_deriv,
                  node_coords, BC_NONE, BC_STICKY, BC_SLIP, BC_SEPARATE, MODEL_DP, project_strain)


def bspline_deriv2(u):
    a = np.abs(u)
    return np.where(a < 0.5, -2.0, np.where(a < 1.5, 1.0, 0.0))


def shape_with_hessian(x, n, dx):
    """N, grad N and the Hessian of N_n at x (N, d)."""
    r = 1.0 / dx
    u = x * r - n
    w = bspline(u)
    dw = bspline_deriv(u) * r
    ddw = bspline_deriv2(u) * r * r
    d = x.shape[1]
    N = np.prod(w, axis=1)
    g = np.empty_like(x)
    H = np.empty((len(x), d, d))
    for a in range(d):
        g[:, a] = dw[:, a] * np.prod(np.delete(w, a, axis=1), axis=1)
        for b in range(d):
            if a == b:
                H[:, a, a] = ddw[:, a] * np.prod(np.delete(w, a, axis=1), axis=1)
            else:
                rest = [e for e in range(d) if e not in (a, b)]
                H[:, a, b] = dw[:, a] * dw[:, b] * (np.prod(w[:, rest], axis=1) if rest else 1.0)
    return N, g, H


# ---------------------------------------------------------------------------
# constitutive map and its adjoint
def _strain_jacobian(eps, p):
    """eps' = P(eps), d eps'/d eps (N, d, d) and d eps'/d alpha (N, d) per branch."""
    n, d = eps.shape
    eps2 = project_strain(eps, p)
    J = np.tile(np.eye(d), (n, 1, 1))
    da = np.zeros((n, d))
    if p.model != MODEL_DP:
        return eps2, J, da
    mu, lam = lame(p.E, p.nu)
    alpha = dp_alpha(p.friction_deg)
    c = (d * lam + 2 * mu) / (2 * mu)
    tr = eps.sum(1)
    dev = eps - tr[:, None] / d
    nd = np.linalg.norm(dev, axis=1)
    dgamma = nd + c * tr * alpha
    tip = tr > 0
    plastic = (~tip) & (dgamma > 0)
    J[tip] = 0.0
    if plastic.any():
        nh = dev[plastic] / nd[plastic, None]
        trp = tr[plastic]
        Pdev = np.eye(d) - np.ones((d, d)) / d
        dn = (Pdev[None] - nh[:, :, None] * nh[:, None, :]) / nd[plastic, None, None]
        # eps'_i = tr/d - c alpha tr nh_i
        J[plastic] = (np.ones((d, d)) / d)[None] - c * alpha * (nh[:, :, None] * np.ones(d)[None, None, :]
                                                                  + trp[:, None, None] * dn)
        da[plastic] = -c * trp[:, None] * nh
    return eps2, J, da


def _iso_adjoint(Q, lam, f, Jf, Ybar, tol=1e-9):
    """Adjoint of S -> Q diag(f(lam)) Q^T at S = Q diag(lam) Q^T."""
    Y = np.einsum("pji,pjk,pkl->pil", Q, 0.5 * (Ybar + np.transpose(Ybar, (0, 2, 1))), Q)
    n, d = lam.shape
    S = np.zeros_like(Y)
    diagY = np.einsum("pii->pi", Y)
    S[:, range(d), range(d)] = np.einsum("pij,pi->pj", Jf, diagY)
    for i in range(d):
        for j in range(d):
            if i == j:
                continue
            dl = lam[:, i] - lam[:, j]
            close = np.abs(dl) < tol * np.maximum(1.0, np.abs(lam[:, i]))
            K = np.where(close, Jf[:, i, i] - Jf[:, i, j], (f[:, i] - f[:, j]) / np.where(close, 1.0, dl))
            S[:, i, j] = K * Y[:, i, j]
    return np.einsum("pij,pjk,plk->pil", Q, S, Q)


def constitutive_forward(F, p):
    """F^E and tau from the eigen-decomposition of b = F F^T (same map as
    oracle.mpm.constitutive), plus the pieces the adjoint needs."""
    mu, lam_ = lame(p.E, p.nu)
    n, d = F.shape[0], F.shape[1]
    b = F @ np.transpose(F, (0, 2, 1))
    lam, Q = np.linalg.eigh(b)
    eps = 0.5 * np.log(lam)
    eps2, Jeps, da = _strain_jacobian(eps, p)
    t = 2 * mu * eps2 + lam_ * eps2.sum(1, keepdims=True)
    h = np.exp(eps2 - eps)
    tau = np.einsum("pij,pj,pkj->pik", Q, t, Q)
    Hm = np.einsum("pij,pj,pkj->pik", Q, h, Q)
    Fe = Hm @ F
    return Fe, tau, dict(Q=Q, lam=lam, eps=eps, eps2=eps2, Jeps=Jeps, da=da, t=t, h=h, Hm=Hm)


def constitutive_adjoint(F, Fe_bar, tau_bar, p):
    """Returns F_bar, E_bar, phi_bar (phi in degrees) of (F^E, tau)(F; E, phi)."""
    mu, lam_ = lame(p.E, p.nu)
    n, d = F.shape[0], F.shape[1]
    Fe, tau, k = constitutive_forward(F, p)
    Q, lam, Jeps, da, t, h, Hm = k["Q"], k["lam"], k["Jeps"], k["da"], k["t"], k["h"], k["Hm"]
    Cmat = 2 * mu * np.eye(d) + lam_ * np.ones((d, d))
    dlam = 1.0 / (2.0 * lam)                                        # d eps_j / d lam_j
    Jt = np.einsum("ik,pkj->pij", Cmat, Jeps) * dlam[:, None, :]   # d t_i / d lam_j
    Jh = h[:, :, None] * (Jeps - np.eye(d)[None]) * dlam[:, None, :]
    tau_bar_s = 0.5 * (tau_bar + np.transpose(tau_bar, (0, 2, 1)))
    H_bar = Fe_bar @ np.transpose(F, (0, 2, 1))
    F_bar = Hm @ Fe_bar
    b_bar = _iso_adjoint(Q, lam, t, Jt, tau_bar_s) + _iso_adjoint(Q, lam, h, Jh, H_bar)
    b_bar = 0.5 * (b_bar + np.transpose(b_bar, (0, 2, 1)))
    F_bar = F_bar + 2 * b_bar @ F
    # parameters: tau is proportional to E (eps' does not depend on E)
    E_bar = np.sum(tau_bar_s * tau) / p.E
    Yt = np.einsum("pji,pjk,pki->pi", Q, tau_bar_s, Q)
    Yh = np.einsum("pji,pjk,pki->pi", Q, 0.5 * (H_bar + np.transpose(H_bar, (0, 2, 1))), Q)
    dt_da = np.einsum("ik,pk->pi", Cmat, da)
    dh_da = h * da
    a_bar = np.sum(Yt * dt_da) + np.sum(Yh * dh_da)
    phi = np.deg2rad(p.friction_deg)
    dalpha_dphi = np.sqrt(2.0 / 3.0) * 6.0 * np.cos(phi) / (3.0 - np.sin(phi)) ** 2 * (np.pi / 180.0)
    return F_bar, E_bar, a_bar * dalpha_dphi


# ---------------------------------------------------------------------------
def bc_mask(u, p):
    """Diagonal Jacobian (0/1 per node and component) of the wall projection at u."""
    d = p.dim
    mask = np.ones_like(u)
    idx = node_coords(p)
    for a in range(d):
        for side in (0, 1):
            kind = p.bc[a][side]
            if kind == BC_NONE:
                continue
            sel = idx[..., a] < p.bound if side == 0 else idx[..., a] > p.cells[a] - p.bound
            if kind == BC_STICKY:
                mask[sel] = 0.0
            elif kind == BC_SLIP:
                mask[sel, a] = 0.0
            elif kind == BC_SEPARATE:
                clamp = (u[..., a] < 0) if side == 0 else (u[..., a] > 0)
                mask[sel & clamp, a] = 0.0
    return mask


def step_adjoint(state, out_bar, p: Params):
    """Adjoint of one oracle step.  state: dict x, v, C, F, tau (float64, N-major,
    tau full); out_bar: adjoints of the step's outputs (same keys).  Returns
    (in_bar dict, E_bar, phi_bar)."""
    if p.heightmap is not None:
        raise NotImplementedError("terrain boundaries are not differentiated")
    x, v, C, F, tau = state["x"], state["v"], state["C"], state["F"], state["tau"]
    n_p, d = x.shape
    shape = p.nodes
    n_nodes = int(np.prod(shape))
    b = base_node(x, p.dx)
    check_domain(b, p)
    g = np.array(p.gravity[:d], np.float64)
    offs = stencil_offsets(d)
    # ---- forward recompute: P2G
    m = np.zeros(n_nodes)
    pp = np.zeros((n_nodes, d))
    cache = []
    for off in offs:
        node = b + np.array(off)
        N, G, Hs = shape_with_hessian(x, node, p.dx)
        flat = np.ravel_multi_index(tuple(node.T), shape)
        dxn = node * p.dx - x
        cache.append((flat, N, G, Hs, dxn))
        m += np.bincount(flat, weights=N * p.p_mass, minlength=n_nodes)
        mom = N[:, None] * p.p_mass * (v + np.einsum("pij,pj->pi", C, dxn)) \
            - p.dt * p.p_vol0 * np.einsum("pij,pj->pi", tau, G)
        for a in range(d):
            pp[:, a] += np.bincount(flat, weights=mom[:, a], minlength=n_nodes)
    has = m > 0
    msafe = np.where(has, m, 1.0)
    u = np.where(has[:, None], pp / msafe[:, None] + p.dt * g, 0.0)
    from .mpm import apply_bc
    vg = apply_bc(u.reshape(shape + (d,)), p).reshape(-1, d)
    mask = bc_mask(u.reshape(shape + (d,)), p).reshape(-1, d) * has[:, None]
    # ---- forward recompute: G2P pieces
    vp = np.zeros((n_p, d))
    Bm = np.zeros((n_p, d, d))
    W = np.zeros((n_p, d, d))
    for flat, N, G, Hs, dxn in cache:
        vn = vg[flat]
        vp += N[:, None] * vn
        Bm += N[:, None, None] * vn[:, :, None] * dxn[:, None, :]
        W += vn[:, :, None] * G[:, None, :]
    Ftr = (np.eye(d)[None] + p.dt * W) @ F
    # ---- reverse: constitutive
    Ftr_bar, E_bar, phi_bar = constitutive_adjoint(Ftr, out_bar["F"], out_bar["tau"], p)
    F_bar = np.transpose(np.eye(d)[None] + p.dt * W, (0, 2, 1)) @ Ftr_bar
    W_bar = p.dt * Ftr_bar @ np.transpose(F, (0, 2, 1))
    vp_bar = out_bar["v"] + p.dt * out_bar["x"]
    B_bar = (4.0 / (p.dx * p.dx)) * out_bar["C"]       # C = B D^-1 with D = (dx^2/4) I
    x_bar = out_bar["x"].copy()
    vg_bar = np.zeros((n_nodes, d))
    for flat, N, G, Hs, dxn in cache:
        vn = vg[flat]
        contrib = N[:, None] * vp_bar + N[:, None] * np.einsum("pab,pb->pa", B_bar, dxn) \
            + np.einsum("pab,pb->pa", W_bar, G)
        for a in range(d):
            vg_bar[:, a] += np.bincount(flat, weights=contrib[:, a], minlength=n_nodes)
        x_bar += G * np.sum(vn * vp_bar, 1)[:, None]
        x_bar += G * np.einsum("pa,pab,pb->p", vn, B_bar, dxn)[:, None]
        x_bar -= N[:, None] * np.einsum("pab,pa->pb", B_bar, vn)
        x_bar += np.einsum("pbc,pab,pa->pc", Hs, W_bar, vn)
    # ---- reverse: grid update
    u_bar = mask * vg_bar
    p_bar = u_bar / msafe[:, None]
    m_bar = -np.sum(u_bar * (u - p.dt * g), 1) / msafe
    m_bar = np.where(has, m_bar, 0.0)
    # ---- reverse: P2G
    v_bar = np.zeros((n_p, d))
    C_bar = np.zeros((n_p, d, d))
    tau_bar = np.zeros((n_p, d, d))
    for flat, N, G, Hs, dxn in cache:
        pb = p_bar[flat]
        mb = m_bar[flat]
        v_bar += p.p_mass * N[:, None] * pb
        C_bar += p.p_mass * N[:, None, None] * pb[:, :, None] * dxn[:, None, :]
        tau_bar -= p.dt * p.p_vol0 * pb[:, :, None] * G[:, None, :]
        x_bar += (mb * p.p_mass)[:, None] * G
        x_bar += p.p_mass * G * np.sum(pb * (v + np.einsum("pij,pj->pi", C, dxn)), 1)[:, None]
        x_bar -= p.p_mass * N[:, None] * np.einsum("pab,pa->pb", C, pb)
        x_bar -= p.dt * p.p_vol0 * np.einsum("pbc,pab,pa->pc", Hs, tau, pb)
    in_bar = {"x": x_bar, "v": v_bar, "C": C_bar, "F": F_bar, "tau": tau_bar}
    return in_bar, E_bar, phi_bar


def run_with_gradient(state0, p: Params, steps: int, target_x: np.ndarray):
    """Loss L = (1/N) sum_p |x_p(T) - x*_p|^2 / 2 after `steps` oracle steps from
    state0, and dL/dv0 (N, d), dL/dE, dL/dphi (per degree)."""
    from .mpm import step
    states = [state0]
    st = state0
    for _ in range(steps):
        st = step(st, p)
        st = {k: st[k] for k in ("x", "v", "C", "F", "tau")}
        states.append(st)
    n = len(st["x"])
    diff = st["x"] - target_x
    L = 0.5 * np.sum(diff * diff) / n
    bar = {k: np.zeros_like(st[k]) for k in st}
    bar["x"] = diff / n
    E_bar = 0.0
    phi_bar = 0.0
    for k in range(steps - 1, -1, -1):
        bar, eb, pb = step_adjoint(states[k], bar, p)
        E_bar += eb
        phi_bar += pb
    return L, bar["v"], E_bar, phi_bar
