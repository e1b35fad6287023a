"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Each case prints its name, seed and size before touching the GPU.
"""
import numpy as np
import pytest

from oracle import mpm as om
from oracle import sparse as osp
from paper_2605_28525_amd import workloads as wl
from parity_util import compare_step, gpu_step_parts

pytestmark = pytest.mark.gpu


def _sim(w, **kw):
    import torch
    from paper_2605_28525_amd import mpm as M
    assert torch.cuda.is_available()
    return M.Simulation(w, **kw)


def _announce(*a):
    print("CASE", *a, flush=True)


@pytest.mark.parametrize("ties", [True, False])
def test_tiny_3d_one_step(ties):
    w = wl.tiny_3d(n=48, ties=ties)
    _announce("tiny_3d", w.n, ties)
    sim = _sim(w)
    parts = gpu_step_parts(sim)
    assert parts["status"][0] == 0, parts["status"]
    errs = compare_step(w, parts)
    print(errs)
    sim.close()


def test_dense_cells_one_step():
    """64 particles per cell over 8^3 cells (32,768 particles): 4096 per owner
    block, so P2G reads the permutation from HBM instead of its LDS copy, and
    cells past the 32 interleaved ranks of the output layout; two steps (the
    second after an incremental re-sort)."""
    w = wl.tiny_3d(n=48, ties=False)
    rng = np.random.default_rng(41)
    x = wl.stratified_cells((4, 4, 4), (12, 12, 12), w.dx, 4, rng)
    for k, a in wl.rest_state(x).items():
        setattr(w, k, a)
    w.ppc, w.p_vol0 = 64, w.dx ** 3 / 64
    w.p_mass = 2000.0 * w.p_vol0
    w = wl.perturbed(w, seed=43, v_scale=0.05, C_scale=0.2, F_scale=1e-3, tau_scale=50.0)
    _announce("dense cells", w.n)
    sim = _sim(w)
    for k in range(2):
        parts = gpu_step_parts(sim)
        assert parts["status"][0] == 0, (k, parts["status"])
        print(k, compare_step(w, parts))
        sim.a, sim.b = sim.b, sim.a
    sim.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_large_and_small_elastic_strain_one_step(dim):
    """Deformation gradients R diag(exp(s)) with principal log-stretches s of
    0.1 to 0.3 (|F F^T - I| beyond the series path's 1/8: eigen path) mixed in
    the same waves with near-identity ones (series path), elastic and
    Drucker-Prager, against the oracle."""
    rng = np.random.default_rng(17 + dim)
    for model in ("elastic", "dp"):
        w = wl.tiny_3d(n=64, ties=False)
        if dim == 2:
            w = _tiny_2d_from(w)
        w.model = model
        n, d = w.n, w.dim
        F = np.empty((n, d, d))
        for p in range(n):
            q, r = np.linalg.qr(rng.normal(size=(d, d)))
            q = q * np.sign(np.diag(r))
            if np.linalg.det(q) < 0:
                q[:, 0] = -q[:, 0]
            s = rng.normal(0, 0.2 if p % 2 else 0.01, d)
            F[p] = q @ np.diag(np.exp(s))
        w.F = F.reshape(n, d * d).T.astype(np.float32)
        _announce("large/small strain", dim, model, n)
        sim = _sim(w)
        parts = gpu_step_parts(sim)
        assert parts["status"][0] == 0, parts["status"]
        print(compare_step(w, parts))
        sim.close()


def _tiny_2d_from(w3):
    st = w3.state()
    x = st["x"][:2] + 0.4
    w = wl.Workload(name="tiny_2d", dim=2, dx=w3.dx, cells=(16, 16), gravity=(0.0, -9.81, 0.0), dt=1e-3,
                    steps=1, model="dp", E=1e6, nu=0.3, rho=2000.0, friction_deg=30.0, ppc=4,
                    p_vol0=w3.dx ** 2 / 4, p_mass=2000 * w3.dx ** 2 / 4,
                    bc=(("separate", "separate"), ("sticky", "separate"), ("none", "none")))
    rng = np.random.default_rng(4)
    n = x.shape[1]
    w.x = x.astype(np.float32)
    w.v = rng.normal(0, 0.2, (2, n)).astype(np.float32)
    w.C = rng.normal(0, 0.5, (4, n)).astype(np.float32)
    w.F = np.tile(np.array([[1.0], [0.0], [0.0], [1.0]], np.float32), (1, n))
    w.tau = rng.normal(0, 100.0, (3, n)).astype(np.float32)
    return w


def test_tiny_2d_one_step():
    w3 = wl.tiny_3d(n=40)
    w = wl.collapse_2d()
    # 2D copy of the tiny case: drop z, keep the 2D grid
    st = w3.state()
    d = 2
    x = st["x"][:2] + 0.4  # into the 2D domain
    w = wl.Workload(name="tiny_2d", dim=2, dx=w3.dx, cells=(16, 16), gravity=(0.0, -9.81, 0.0), dt=1e-3,
                    steps=1, model="dp", E=1e6, nu=0.3, rho=2000.0, friction_deg=30.0, ppc=4,
                    p_vol0=w3.dx ** 2 / 4, p_mass=2000 * w3.dx ** 2 / 4,
                    bc=(("separate", "separate"), ("sticky", "separate"), ("none", "none")))
    rng = np.random.default_rng(3)
    n = x.shape[1]
    w.x = x.astype(np.float32)
    w.v = rng.normal(0, 0.2, (2, n)).astype(np.float32)
    w.C = rng.normal(0, 0.5, (4, n)).astype(np.float32)
    w.F = (np.array([1, 0, 0, 1], np.float32)[:, None] + rng.normal(0, 0.02, (4, n))).astype(np.float32)
    w.tau = rng.normal(0, 100.0, (3, n)).astype(np.float32)
    _announce("tiny_2d", n)
    sim = _sim(w)
    parts = gpu_step_parts(sim)
    assert parts["status"][0] == 0, parts["status"]
    print(compare_step(w, parts))
    sim.close()


def test_collapse_2d_steps():
    """Every step of the 2D column collapse (200 steps, 4096 particles)
    compared with the oracle started from the GPU's state of that step."""
    w = wl.collapse_2d()
    _announce("collapse_2d", w.n, w.steps)
    sim = _sim(w)
    worst = {}
    for k in range(w.steps):
        parts = gpu_step_parts(sim)
        assert parts["status"][0] == 0, (k, parts["status"])
        errs = compare_step(w, parts)
        for f, e in errs.items():
            worst[f] = max(worst.get(f, 0.0), e)
        sim.a, sim.b = sim.b, sim.a
    print("worst normwise errors over 200 steps:", worst)
    sim.close()


def test_collapse_3d_eighth_scale_steps():
    """The 1/8-volume 3D collapse (262,144 particles): steps 0-2 compared, then
    the GPU runs ahead to step 50 and steps 50-51 are compared."""
    w = wl.perturbed(wl.collapse_3d(scale=2), seed=21, v_scale=0.05, C_scale=1.0, F_scale=2e-3, tau_scale=500.0)
    _announce("collapse_3d_1of8 perturbed", w.n)
    sim = _sim(w)
    for k in range(2):
        parts = gpu_step_parts(sim)
        assert parts["status"][0] == 0, (k, parts["status"])
        print(k, compare_step(w, parts))
        sim.a, sim.b = sim.b, sim.a
    sim.step(48)
    parts = gpu_step_parts(sim)
    assert parts["status"][0] == 0, parts["status"]
    print(50, compare_step(w, parts))
    sim.close()


def test_collapse_3d_eighth_scale_long_run():
    """The 1/8-volume 3D collapse from rest (262,144 particles) over its whole
    run: steps 0, 1, 100, 500, 1000 and 1999 compared with the oracle started
    from the GPU's state of that step (the GPU runs ahead in between), so the
    late, spread-out states with plastic flow are covered, not only the
    release."""
    w = wl.collapse_3d(scale=2)
    _announce("collapse_3d_1of8 long run", w.n)
    sim = _sim(w)
    at = 0
    for k in (0, 1, 100, 500, 1000, 1999):
        if k > at:
            sim.step(k - at)
            at = k
        parts = gpu_step_parts(sim)
        assert parts["status"][0] == 0, (k, parts["status"])
        print(k, parts["nb"], compare_step(w, parts), flush=True)
        sim.a, sim.b = sim.b, sim.a
        at += 1
    sim.close()


def test_dense_matches_sparse_and_oracle():
    """Dense-grid mode (every block of the potential domain) gives the oracle's
    step too; sparse and dense GPU particle results agree."""
    from paper_2605_28525_amd import mpm as M
    w = wl.perturbed(wl.collapse_2d(), seed=5)
    _announce("collapse_2d dense", w.n)
    sim_d = _sim(w, grid_mode=M.MPM_GRID_DENSE)
    parts_d = gpu_step_parts(sim_d, sparse=False)
    assert parts_d["status"][0] == 0
    print(compare_step(w, parts_d, sparse=False))
    sim_s = _sim(w)
    parts_s = gpu_step_parts(sim_s)
    od, os_ = parts_d["order"], parts_s["order"]
    for k in ("x", "v", "C", "F", "tau"):
        a = parts_d["state_out"][k][:, np.argsort(od)]
        b = parts_s["state_out"][k][:, np.argsort(os_)]
        assert np.max(np.abs(a - b)) <= 1e-5 * max(1e-30, np.max(np.abs(b))) + (5.0 if k == "tau" else 0.0)
    sim_d.close()
    sim_s.close()


def test_landslide_crop_terrain_steps():
    """Terrain level set with Coulomb friction: a 64x64x256-cell window of the
    landslide workload, 3 compared steps after 20 GPU steps of motion."""
    w = wl.landslide_crop()
    _announce("landslide_crop", w.n)
    sim = _sim(w)
    sim.step(20)
    for k in range(3):
        parts = gpu_step_parts(sim)
        assert parts["status"][0] == 0, parts["status"]
        print(k, compare_step(w, parts))
        sim.a, sim.b = sim.b, sim.a
    sim.close()
