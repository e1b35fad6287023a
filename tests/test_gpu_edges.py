"""GPU edge cases of the step: an empty particle set, a single particle,
block-capacity overflow (latched in the status word; with
MPM_FLAG_SYNC_REBUILD the build grows the table and the capacity and the step
still matches the oracle), and the domain and not-a-number flags.
"""
import numpy as np
import pytest

from paper_2605_28525_amd import workloads as wl
from parity_util import compare_step, gpu_step_parts

pytestmark = pytest.mark.gpu


def _announce(*a):
    print("CASE", *a, flush=True)


def _subset(w, sel):
    for k in ("x", "v", "C", "F", "tau"):
        setattr(w, k, np.ascontiguousarray(getattr(w, k)[:, sel]))
    return w


def test_empty_set():
    from paper_2605_28525_amd import mpm as M
    w = _subset(wl.tiny_3d(n=48, ties=False), np.zeros(48, bool))
    _announce("empty set", w.n)
    params = M.params_from_workload(w, max_particles=64)
    ctx = M.mpm_create(params)
    try:
        a, b = M.ParticleSet(3, 0), M.ParticleSet(3, 0)
        M.mpm_sparse_build(ctx, a.view())
        assert M.mpm_active_count(ctx)[0] == 0
        M.mpm_p2g(ctx, a.view())
        M.mpm_grid_update(ctx)
        M.mpm_g2p(ctx, a.view(), b.view())
        M.mpm_step(ctx, a.view(), b.view(), 3)
        rc, flags = M.mpm_get_status(ctx)
        assert rc == 0, flags
    finally:
        M.mpm_destroy(ctx)


@pytest.mark.parametrize("dim", [2, 3])
def test_single_particle(dim):
    from paper_2605_28525_amd import mpm as M
    w = wl.tiny_3d(n=48, ties=False) if dim == 3 else wl.perturbed(wl.collapse_2d(), seed=5, v_scale=0.3)
    sel = np.zeros(w.n, bool)
    sel[w.n // 2] = True
    w = _subset(w, sel)
    _announce("single particle", dim)
    sim = M.Simulation(w)
    try:
        for k in range(2):
            parts = gpu_step_parts(sim)
            assert parts["status"][0] == 0, (k, parts["status"])
            assert parts["nb"] >= 1
            print(k, compare_step(w, parts))
            sim.a, sim.b = sim.b, sim.a
    finally:
        sim.close()


def test_overflow_flag_and_sync_rebuild():
    """tiny_3d touches more than 4 blocks: with a 4-block capacity the build
    raises MPM_FLAG_OVERFLOW; with MPM_FLAG_SYNC_REBUILD it doubles the table
    and the capacity until the blocks fit, and the step matches the oracle."""
    from paper_2605_28525_amd import mpm as M
    w = wl.tiny_3d(n=48, ties=False)
    _announce("overflow", w.n)
    ctx = M.mpm_create(M.params_from_workload(w, block_capacity=4, hash_capacity_log2=3))
    try:
        a = M.ParticleSet.from_arrays(w.state())
        M.mpm_sparse_build(ctx, a.view())
        rc, flags = M.mpm_get_status(ctx)
        assert rc == M.MPM_ERR_OVERFLOW and flags & M.MPM_FLAG_OVERFLOW, (rc, flags)
        M.mpm_clear_status(ctx)
        rc, flags = M.mpm_get_status(ctx)
        assert rc == 0, flags
    finally:
        M.mpm_destroy(ctx)
    sim = M.Simulation(w, block_capacity=4, hash_capacity_log2=3, flags=M.MPM_FLAG_SYNC_REBUILD)
    try:
        for k in range(2):
            parts = gpu_step_parts(sim)
            assert parts["status"][0] == 0, (k, parts["status"])
            assert parts["nb"] > 4
            print(k, compare_step(w, parts))
            sim.a, sim.b = sim.b, sim.a
    finally:
        sim.close()


@pytest.mark.parametrize("case", ["domain", "nan"])
def test_domain_and_nan_flags(case):
    from paper_2605_28525_amd import mpm as M
    w = wl.tiny_3d(n=48, ties=False)
    st = w.state()
    if case == "domain":
        st["x"][:, 7] = np.float32(-3.0 * w.dx)      # below the grid's origin
        want_rc, want_flag = M.MPM_ERR_DOMAIN, M.MPM_FLAG_DOMAIN
    else:
        st["x"][1, 7] = np.float32(np.nan)
        want_rc, want_flag = M.MPM_ERR_NAN, M.MPM_FLAG_NAN
    _announce("status flag", case)
    ctx = M.mpm_create(M.params_from_workload(w))
    try:
        a, b = M.ParticleSet.from_arrays(st), M.ParticleSet(3, w.n)
        M.mpm_step(ctx, a.view(), b.view(), 1)
        rc, flags = M.mpm_get_status(ctx)
        assert flags & want_flag, (case, rc, flags)
        assert rc == want_rc or (flags & (want_flag - 1)), (case, rc, flags)
    finally:
        M.mpm_destroy(ctx)
