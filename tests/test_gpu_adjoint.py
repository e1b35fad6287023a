"""GPU reverse mode against the FP64 oracle's reverse mode (which is itself
pinned to finite differences in test_oracle_adjoint.py).

Bar: per adjoint field, normwise max|a - b| <= 2e-3 max|b| for one step from the
same float32 state; for a multi-step rollout, dL/dE and dL/dphi within 1e-3
relative and dL/dv0 with cosine >= 0.999.
"""
import numpy as np
import pytest

from oracle import adjoint as oa
from oracle import mpm as om
from paper_2605_28525_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _announce(*a):
    print("CASE", *a, flush=True)


def _tau_full_to_comp(t):
    d = t.shape[1]
    if d == 2:
        return np.stack([t[:, 0, 0], t[:, 1, 1], t[:, 0, 1] + t[:, 1, 0]])
    return np.stack([t[:, 0, 0], t[:, 1, 1], t[:, 2, 2], t[:, 0, 1] + t[:, 1, 0], t[:, 1, 2] + t[:, 2, 1],
                     t[:, 0, 2] + t[:, 2, 0]])


def _tau_comp_to_full(c, d):
    n = c.shape[1]
    t = np.zeros((n, d, d))
    if d == 2:
        t[:, 0, 0], t[:, 1, 1] = c[0], c[1]
        t[:, 0, 1] = t[:, 1, 0] = 0.5 * c[2]
    else:
        t[:, 0, 0], t[:, 1, 1], t[:, 2, 2] = c[0], c[1], c[2]
        t[:, 0, 1] = t[:, 1, 0] = 0.5 * c[3]
        t[:, 1, 2] = t[:, 2, 1] = 0.5 * c[4]
        t[:, 0, 2] = t[:, 2, 0] = 0.5 * c[5]
    return t


def _consistent_state(w, seed, v_scale=0.05, C_scale=0.5, strain=3e-3):
    """Random but consistent state: F a rotation times a small stretch, tau = tau(F)."""
    rng = np.random.default_rng(seed)
    d, n = w.dim, w.n
    st = w.state()
    st["v"] = rng.normal(0, v_scale, (d, n)).astype(np.float32)
    st["C"] = rng.normal(0, C_scale, (d * d, n)).astype(np.float32)
    F = np.empty((n, d, d))
    for p in range(n):
        q, r = np.linalg.qr(rng.normal(size=(d, d)))
        q = q * np.sign(np.diag(r))
        if np.linalg.det(q) < 0:
            q[:, 0] = -q[:, 0]
        F[p] = q @ np.diag(np.exp(rng.normal(0, strain, d) - strain))
    F = F.astype(np.float32).astype(np.float64)
    p_ = om.Params.from_workload(w)
    _, tau = om.constitutive(F, p_)
    st["F"] = F.reshape(n, d * d).T.astype(np.float32)
    st["tau"] = om.tau_to_soa(tau).astype(np.float32)
    return st


def _check_step_adjoint(w, st, seed):
    import torch
    from paper_2605_28525_amd import mpm as M
    d, n = w.dim, w.n
    rng = np.random.default_rng(seed)
    # adjoints of the step outputs, per particle (oracle order = input order)
    ob = {"x": rng.normal(size=(d, n)), "v": rng.normal(size=(d, n)), "C": rng.normal(size=(d * d, n)) * 1e-2,
          "F": rng.normal(size=(d * d, n)), "tau": rng.normal(size=(3 if d == 2 else 6, n)) * 1e-5}
    p = om.Params.from_workload(w)
    ost = om.state_from_soa(st, d)
    ob_full = {"x": ob["x"].T, "v": ob["v"].T, "C": ob["C"].T.reshape(n, d, d), "F": ob["F"].T.reshape(n, d, d),
               "tau": _tau_comp_to_full(ob["tau"], d)}
    ref, E_ref, phi_ref = oa.step_adjoint(ost, ob_full, p)
    params = M.params_from_workload(w, flags=M.MPM_FLAG_ADJOINT)
    ctx = M.mpm_create(params)
    try:
        pin = M.ParticleSet.from_arrays(st)
        M.mpm_sparse_build(ctx, pin.view())
        M.mpm_p2g(ctx, pin.view())  # records the G2P output permutation of this build
        order = torch.zeros(n, dtype=torch.int32, device="cuda")
        M.mpm_get_order(ctx, order, n)
        o = order.cpu().numpy().astype(np.int64)
        obar = M.ParticleSet(d, n)
        for k in ob:
            getattr(obar, k).copy_(torch.from_numpy(ob[k][:, o].astype(np.float32)))
        ibar = M.ParticleSet(d, n)
        pb = torch.zeros(2, dtype=torch.float32, device="cuda")
        M.mpm_step_adj(ctx, pin.view(), obar.view(), ibar.view(), pb)
        rc, flags = M.mpm_get_status(ctx)
        assert rc == 0, flags
        got = ibar.to_arrays()
        pbh = pb.cpu().numpy().astype(np.float64)
    finally:
        M.mpm_destroy(ctx)
    errs = {}
    refs = {"x": ref["x"].T, "v": ref["v"].T, "C": ref["C"].reshape(n, d * d).T, "F": ref["F"].reshape(n, d * d).T,
            "tau": _tau_full_to_comp(ref["tau"])}
    for k, r in refs.items():
        e = np.max(np.abs(got[k] - r)) / max(np.max(np.abs(r)), 1e-30)
        errs[k] = e
        assert e <= 2e-3, (k, e)
    for name, g, r in (("E", pbh[0], E_ref), ("phi", pbh[1], phi_ref)):
        e = abs(g - r) / max(abs(r), 1e-30)
        errs[name] = e
        assert e <= 2e-3, (name, g, r)
    return errs


def test_step_adjoint_tiny_3d():
    # no particles on half-cell ties: the B-spline's second derivative jumps at
    # its knots, so the position adjoint (which uses it) is undefined there
    w = wl.tiny_3d(n=48, ties=False)
    w.E = 5e4
    st = _consistent_state(w, 1)
    _announce("step adjoint tiny_3d", w.n)
    print(_check_step_adjoint(w, st, 2))


def test_step_adjoint_2d_window():
    w = wl.collapse_2d()
    sel = (w.x[0] < 0.15) & (w.x[1] < 0.15)
    for k in ("x", "v", "C", "F", "tau"):
        setattr(w, k, getattr(w, k)[:, sel].copy())
    w.E = 5e4
    st = _consistent_state(w, 3)
    _announce("step adjoint collapse_2d window", w.n)
    print(_check_step_adjoint(w, st, 4))


def test_step_adjoint_fd_copy_3d():
    w = wl.differentiable_fd_copy()
    st = _consistent_state(w, 5, v_scale=0.02, C_scale=0.2)
    _announce("step adjoint differentiable_fd_copy", w.n)
    print(_check_step_adjoint(w, st, 6))


def test_rollout_gradient_matches_oracle():
    """30-step checkpointed rollout (segments of 10) of the 4096-particle copy
    (E = 2e5 Pa, dt = 2e-4 s, target-run initial velocity): gradients of
    L = (1/N) sum |x(T) - x*|^2 / 2 (x* = x0 + N(0, 0.01^2) per particle) with
    respect to E, phi and v0, against the oracle's FP64 reverse pass chained
    along the GPU's own trajectory (so that float32 forward drift does not
    enter the comparison)."""
    import torch
    from paper_2605_28525_amd import autograd as AG
    from paper_2605_28525_amd import mpm as M
    w = wl.differentiable_fd_copy()
    w.E, w.dt = 2.0e5, 2.0e-4
    steps, K = 30, 10
    n, d = w.n, w.dim
    v0 = wl.calibration_target_velocity(n, seed=1003)
    rng = np.random.default_rng(1004)
    target = w.x.astype(np.float64) + rng.normal(0, 0.01, size=w.x.shape)      # (d, n), caller order
    _announce("rollout gradient", n, steps)
    roll = AG.Rollout(w, steps=steps, checkpoint=K)
    try:
        E = torch.tensor(float(w.E), dtype=torch.float64, requires_grad=True)
        phi = torch.tensor(float(w.friction_deg), dtype=torch.float64, requires_grad=True)
        vt = torch.from_numpy(v0).cuda().requires_grad_(True)
        xT = AG.rollout(E, phi, vt, roll)
        tgt = torch.from_numpy(target.astype(np.float32)).cuda()
        loss = 0.5 * torch.sum((xT.double() - tgt.double()) ** 2) / n
        loss.backward()
        gE, gphi, gv0 = float(E.grad), float(phi.grad), vt.grad.detach().cpu().numpy().astype(np.float64)
    finally:
        roll.close()
    # the GPU trajectory, every step
    sim = M.Simulation(w)
    sim.a.v.copy_(torch.from_numpy(v0))
    states, ids = [], []
    for k in range(steps + 1):
        states.append(sim.a.to_arrays())
        ids.append(sim.a.ids().astype(np.int64))
        if k < steps:
            sim.step(1)
    sim.close()
    p = om.Params.from_workload(w)
    xT_np = states[-1]["x"].astype(np.float64)
    bar = {"x": ((xT_np - target[:, ids[-1]]) / n).T}
    for key, shp in (("v", (n, d)), ("C", (n, d, d)), ("F", (n, d, d)), ("tau", (n, d, d))):
        bar[key] = np.zeros(shp)
    E_bar = phi_bar = 0.0
    for k in range(steps - 1, -1, -1):
        pos_next = np.empty(n, np.int64)
        pos_next[ids[k + 1]] = np.arange(n)
        perm = pos_next[ids[k]]                 # state_{k+1} position of each particle of state_k
        ob = {key: val[perm] for key, val in bar.items()}
        ist, eb, pb = oa.step_adjoint(om.state_from_soa(states[k], d), ob, p)
        E_bar += eb
        phi_bar += pb
        bar = ist
    v0_ref = bar["v"].T                           # state_0 order = caller order
    print("dE", gE, E_bar, "dphi", gphi, phi_bar)
    assert abs(gE - E_bar) <= 1e-3 * abs(E_bar)
    assert abs(gphi - phi_bar) <= 1e-3 * abs(phi_bar)
    cos = np.sum(gv0 * v0_ref) / (np.linalg.norm(gv0) * np.linalg.norm(v0_ref))
    rel = np.linalg.norm(gv0 - v0_ref) / np.linalg.norm(v0_ref)
    print("dL/dv0 cosine", cos, "relative", rel)
    assert cos >= 0.999
