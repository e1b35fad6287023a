"""Pins of the oracle's reverse mode against central finite differences of the
oracle's forward step (FP64).  The forward's return map goes through an SVD of
F, the adjoint through the eigen-decomposition of F F^T, so these tests also
cross two independent formulations of the constitutive map."""
import numpy as np
import pytest

from oracle import adjoint as oa
from oracle import mpm as om
from paper_2605_28525_amd import workloads as wl


def _rot(rng, d):
    q, r = np.linalg.qr(rng.normal(size=(d, d)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def _P(d, model="dp", **kw):
    base = dict(dim=d, dx=0.25, cells=(24,) * d, gravity=(0.0, -9.81, 0.0)[:3], dt=2e-3, p_mass=0.7,
                p_vol0=0.25 ** d / 8, model=model, E=2.0e4, nu=0.3, friction_deg=30.0)
    base.update(kw)
    return om.Params(**base)


def _branch_cases(rng, d, n=40):
    """Deformation gradients in the elastic, plastic and cone-tip branches, plus
    F = I and F = R exactly (repeated singular values)."""
    Fs = []
    for _ in range(n):
        R, Q = _rot(rng, d), _rot(rng, d)
        kind = rng.integers(3)
        if kind == 0:      # near-hydrostatic compression: elastic
            s = np.exp(-0.01 + rng.normal(0, 1e-4, d))
        elif kind == 1:    # shear dominated: plastic
            s = np.exp(rng.normal(0, 0.02, d) - 0.002)
        else:              # tension: cone tip
            s = np.exp(0.01 + rng.normal(0, 1e-3, d))
        Fs.append(R @ np.diag(s) @ Q)
    Fs.append(np.eye(d))
    Fs.append(_rot(rng, d))
    Fs.append(_rot(rng, d) @ np.diag(np.exp(np.full(d, -0.003))))
    return np.array(Fs)


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("model", ["elastic", "dp"])
def test_constitutive_adjoint_matches_fd(d, model):
    rng = np.random.default_rng(7 + d)
    p = _P(d, model)
    F = _branch_cases(rng, d)
    if model == "dp":
        # F = I and F = R sit on the cone apex (eps = 0), where the elastic,
        # plastic and tip branches meet and the return map has a kink
        F = np.concatenate([F[:-3], F[-1:]])
    Fe_bar = rng.normal(size=F.shape)
    tau_bar = rng.normal(size=F.shape) * 1e-4
    F_bar, E_bar, phi_bar = oa.constitutive_adjoint(F, Fe_bar, tau_bar, p)

    def loss(Fx, pp):
        Fe, tau = om.constitutive(Fx, pp)
        return np.sum(Fe_bar * Fe) + np.sum(tau_bar * tau)

    dF = rng.normal(size=F.shape)
    h = 1e-7
    fd = (loss(F + h * dF, p) - loss(F - h * dF, p)) / (2 * h)
    assert abs(fd - np.sum(F_bar * dF)) <= 1e-6 * (1 + abs(fd))
    # per-matrix check (no cancellation across particles)
    for i in range(len(F)):
        one = np.zeros_like(dF)
        one[i] = dF[i]
        fdi = (loss(F + h * one, p) - loss(F - h * one, p)) / (2 * h)
        assert abs(fdi - np.sum(F_bar[i] * dF[i])) <= 1e-6 * (1 + abs(fdi)), i
    # parameters
    pE = [om.Params(**{**p.__dict__, "E": p.E * (1 + s * 1e-6)}) for s in (1, -1)]
    fdE = (loss(F, pE[0]) - loss(F, pE[1])) / (2e-6 * p.E)
    assert abs(fdE - E_bar) <= 1e-6 * (1 + abs(fdE))
    pP = [om.Params(**{**p.__dict__, "friction_deg": p.friction_deg + s * 1e-5}) for s in (1, -1)]
    fdP = (loss(F, pP[0]) - loss(F, pP[1])) / 2e-5
    assert abs(fdP - phi_bar) <= 1e-5 * (1 + abs(fdP))
    if model == "dp":
        assert abs(phi_bar) > 0


def _state(rng, d, n, p):
    x = rng.uniform(2.2, 3.8, size=(n, d))
    F = np.stack([_rot(rng, d) @ np.diag(np.exp(rng.normal(0, 0.004, d) - 0.002)) for _ in range(n)])
    _, tau = om.constitutive(F, p)
    return {"x": x, "v": rng.normal(0, 0.3, (n, d)), "C": rng.normal(0, 0.5, (n, d, d)), "F": F, "tau": tau}


@pytest.mark.parametrize("d", [2, 3])
def test_step_adjoint_dot_product(d):
    rng = np.random.default_rng(30 + d)
    p = _P(d, bc=(("sticky", "separate"), ("sticky", "separate"), ("separate", "separate")))
    n = 30
    st = _state(rng, d, n, p)
    out_bar = {k: rng.normal(size=st[k].shape) for k in st}
    out_bar["tau"] *= 1e-3
    in_bar, E_bar, phi_bar = oa.step_adjoint(st, out_bar, p)

    def L(s, pp):
        o = om.step(s, pp)
        return sum(np.sum(out_bar[k] * o[k]) for k in out_bar)

    h = 1e-7
    for key in ("x", "v", "C", "F", "tau"):
        du = rng.normal(size=st[key].shape)
        if key == "tau":
            du = du + np.transpose(du, (0, 2, 1))
        if key == "x":
            du *= p.dx
        sp = {k: v.copy() for k, v in st.items()}
        sm = {k: v.copy() for k, v in st.items()}
        sp[key] = st[key] + h * du
        sm[key] = st[key] - h * du
        fd = (L(sp, p) - L(sm, p)) / (2 * h)
        an = np.sum(in_bar[key] * du)
        assert abs(fd - an) <= 2e-6 * (1 + abs(fd)), (key, fd, an)
    pE = [om.Params(**{**p.__dict__, "E": p.E * (1 + s * 1e-6)}) for s in (1, -1)]
    fdE = (L(st, pE[0]) - L(st, pE[1])) / (2e-6 * p.E)
    assert abs(fdE - E_bar) <= 1e-5 * (1 + abs(fdE))
    pP = [om.Params(**{**p.__dict__, "friction_deg": p.friction_deg + s * 1e-5}) for s in (1, -1)]
    fdP = (L(st, pP[0]) - L(st, pP[1])) / 2e-5
    assert abs(fdP - phi_bar) <= 1e-5 * (1 + abs(fdP))


def test_multistep_gradient_matches_fd():
    """dL/dv0, dL/dE, dL/dphi of a 6-step 2D collapse window against central
    differences of the loss (h = 1e-6 relative for E and phi, 1e-6 m/s for v0)."""
    rng = np.random.default_rng(44)
    w = wl.collapse_2d()
    sel = (w.x[0] < 0.12) & (w.x[1] < 0.12)
    p = om.Params.from_workload(w)
    p.E = 5e4
    p.dt = 5e-4
    st0 = om.state_from_soa({k: v[:, sel] for k, v in w.state().items()}, 2)
    st0["v"] = rng.normal(0, 0.05, st0["v"].shape)
    steps = 6
    target = st0["x"] + rng.normal(0, 1e-3, st0["x"].shape)
    L, v0_bar, E_bar, phi_bar = oa.run_with_gradient(st0, p, steps, target)

    def loss(s0, pp):
        s = s0
        for _ in range(steps):
            s = om.step(s, pp)
        diff = s["x"] - target
        return 0.5 * np.sum(diff * diff) / len(diff)

    for _ in range(4):
        dv = rng.normal(size=st0["v"].shape)
        h = 1e-6
        sp = dict(st0, v=st0["v"] + h * dv)
        sm = dict(st0, v=st0["v"] - h * dv)
        fd = (loss(sp, p) - loss(sm, p)) / (2 * h)
        assert abs(fd - np.sum(v0_bar * dv)) <= 1e-5 * abs(fd) + 1e-14
    pE = [om.Params(**{**p.__dict__, "E": p.E * (1 + s * 1e-6)}) for s in (1, -1)]
    fdE = (loss(st0, pE[0]) - loss(st0, pE[1])) / (2e-6 * p.E)
    assert abs(fdE - E_bar) <= 1e-5 * abs(fdE) + 1e-16
    pP = [om.Params(**{**p.__dict__, "friction_deg": p.friction_deg * (1 + s * 1e-6)}) for s in (1, -1)]
    fdP = (loss(st0, pP[0]) - loss(st0, pP[1])) / (2e-6 * p.friction_deg)
    assert abs(fdP - phi_bar) <= 1e-5 * abs(fdP) + 1e-14


def test_fd_copy_gradient_matches_central_differences():
    """The 4096-particle calibration copy: dL/dv0 (two random directions), dL/dE
    and dL/dphi of a 10-step rollout from the oracle's reverse mode against FP64
    central differences (h = 1e-5 relative for E and phi, 1e-6 m/s for v0).
    Over several steps some particles sit near a kink of the return map or of a
    separating wall, so central differences drift with h (1e-4 .. 1e-3 relative
    at h = 1e-4 .. 1e-5, converging as h shrinks); 1e-4 at h = 1e-6 still rejects
    any missing or wrong term, which shows up at the 1e-2 .. 1e0 level."""
    w = wl.differentiable_fd_copy()
    w.E, w.dt = 2.0e5, 2.0e-4
    p = om.Params.from_workload(w)
    n, d = w.n, w.dim
    rng = np.random.default_rng(1004)
    v0 = wl.calibration_target_velocity(n, seed=1003).astype(np.float64).T
    st0 = om.state_from_soa(w.state(), d)
    st0["v"] = v0
    target = st0["x"] + rng.normal(0, 0.01, size=st0["x"].shape)
    steps = 10
    L, v0_bar, E_bar, phi_bar = oa.run_with_gradient(st0, p, steps, target)

    def loss(s0, pp):
        s = s0
        for _ in range(steps):
            s = om.step(s, pp)
        diff = s["x"] - target
        return 0.5 * np.sum(diff * diff) / len(diff)

    for _ in range(2):
        dv = rng.normal(size=v0.shape)
        sp = dict(st0, v=v0 + 1e-6 * dv)
        sm = dict(st0, v=v0 - 1e-6 * dv)
        fd = (loss(sp, p) - loss(sm, p)) / 2e-6
        assert abs(fd - np.sum(v0_bar * dv)) <= 1e-4 * abs(fd)
    # parameters: h = 1e-5 relative (at 1e-6 the loss difference for phi sits at
    # the float64 round-off floor of the loss)
    pE = [om.Params(**{**p.__dict__, "E": p.E * (1 + s * 1e-5)}) for s in (1, -1)]
    fdE = (loss(st0, pE[0]) - loss(st0, pE[1])) / (2e-5 * p.E)
    assert abs(fdE - E_bar) <= 1e-4 * abs(fdE)
    pP = [om.Params(**{**p.__dict__, "friction_deg": p.friction_deg * (1 + s * 1e-5)}) for s in (1, -1)]
    fdP = (loss(st0, pP[0]) - loss(st0, pP[1])) / (2e-5 * p.friction_deg)
    assert abs(fdP - phi_bar) <= 1e-4 * abs(fdP)
