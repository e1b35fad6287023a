"""GPU: the reverse-mode tape (mpm_tape_forward / mpm_tape_adjoint) against
the per-step path (mpm_step, then mpm_step_adj step by step in reverse) on one
checkpoint segment.

The tape's forward steps are the same kernels on the same inputs as
mpm_step, and the sparse P2G has no atomics, so the recorded states must equal
the per-step ones bit for bit.  The reverse sweep reads the recorded builds
instead of rebuilding; its reverse scatter sums float32 contributions with
atomics, so the adjoints agree to 1e-5 normwise (max|a - b| <= 1e-5 max|b|), as
do the parameter adjoints.
"""
import numpy as np
import pytest

from paper_2605_28525_amd import workloads as wl
from test_gpu_adjoint import _consistent_state

pytestmark = pytest.mark.gpu

FIELDS = ("x", "v", "C", "F", "tau")


def _announce(*a):
    print("CASE", *a, flush=True)


def _workload(name):
    if name == "tiny_3d":
        w = wl.tiny_3d(n=48, ties=False)
        w.E = 5e4
        return w, _consistent_state(w, 1)
    if name == "fd_copy_3d":
        w = wl.differentiable_fd_copy()
        return w, _consistent_state(w, 5, v_scale=0.02, C_scale=0.2)
    w = wl.collapse_2d()
    sel = (w.x[0] < 0.15) & (w.x[1] < 0.15)
    for k in FIELDS:
        setattr(w, k, getattr(w, k)[:, sel].copy())
    w.E = 5e4
    return w, _consistent_state(w, 3)


def _normwise(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-30))


@pytest.mark.parametrize("name,k", [("tiny_3d", 4), ("fd_copy_3d", 5), ("collapse_2d_window", 3)])
def test_tape_matches_per_step_adjoint(name, k):
    import torch
    from paper_2605_28525_amd import mpm as M
    w, st = _workload(name)
    d, n = w.dim, w.n
    _announce("tape vs per-step adjoint", name, n, k)
    params = M.params_from_workload(w, flags=M.MPM_FLAG_ADJOINT)
    tape_ctx = M.mpm_create(params)
    step_ctx = M.mpm_create(params)
    try:
        M.mpm_tape_reserve(tape_ctx, k + 1)
        ta = [M.ParticleSet(d, n) for _ in range(k + 1)]
        sa = [M.ParticleSet(d, n) for _ in range(k + 1)]
        ta[0].copy_(M.ParticleSet.from_arrays(st))
        sa[0].copy_(ta[0])
        M.mpm_tape_forward(tape_ctx, [s.view() for s in ta])
        for j in range(k):
            M.mpm_step(step_ctx, sa[j].view(), sa[j + 1].view(), 1)
        for j in range(k + 1):
            A, B = ta[j].to_arrays(), sa[j].to_arrays()
            for f in FIELDS:
                assert np.array_equal(A[f], B[f]), (j, f)
            assert np.array_equal(ta[j].ids(), sa[j].ids()), j
        rng = np.random.default_rng(11)
        ob = M.ParticleSet(d, n)
        for f, sc in (("x", 1.0), ("v", 1.0), ("C", 1e-2), ("F", 1.0), ("tau", 1e-5)):
            t = getattr(ob, f)
            t.copy_(torch.from_numpy((rng.normal(size=tuple(t.shape)) * sc).astype(np.float32)))
        tbar, tspare = M.ParticleSet(d, n), M.ParticleSet(d, n)
        tbar.copy_(ob)
        pb_t = torch.zeros(2, dtype=torch.float32, device="cuda")
        M.mpm_tape_adjoint(tape_ctx, [s.view() for s in ta], tbar.view(), tspare.view(), pb_t)
        sbar, sspare = M.ParticleSet(d, n), M.ParticleSet(d, n)
        sbar.copy_(ob)
        pb_s = torch.zeros(2, dtype=torch.float32, device="cuda")
        for j in range(k - 1, -1, -1):
            M.mpm_step_adj(step_ctx, sa[j].view(), sbar.view(), sspare.view(), pb_s)
            sbar, sspare = sspare, sbar
        for c in (tape_ctx, step_ctx):
            rc, flags = M.mpm_get_status(c)
            assert rc == 0, flags
        A, B = tbar.to_arrays(), sbar.to_arrays()
        errs = {f: _normwise(A[f], B[f]) for f in FIELDS}
        pt, ps = pb_t.cpu().numpy().astype(np.float64), pb_s.cpu().numpy().astype(np.float64)
        errs["E"] = abs(pt[0] - ps[0]) / max(abs(ps[0]), 1e-30)
        errs["phi"] = abs(pt[1] - ps[1]) / max(abs(ps[1]), 1e-30)
        print(errs)
        for key, e in errs.items():
            assert e <= 1e-5, (key, e)
    finally:
        M.mpm_destroy(tape_ctx)
        M.mpm_destroy(step_ctx)


def test_tape_argument_checks():
    from paper_2605_28525_amd import mpm as M
    w, st = _workload("tiny_3d")
    d, n = w.dim, w.n
    _announce("tape argument checks", n)
    ctx = M.mpm_create(M.params_from_workload(w, flags=M.MPM_FLAG_ADJOINT))
    plain = M.mpm_create(M.params_from_workload(w))
    try:
        sets = [M.ParticleSet(d, n) for _ in range(4)]
        sets[0].copy_(M.ParticleSet.from_arrays(st))
        M.mpm_tape_reserve(ctx, 2)
        with pytest.raises(M.MPMError):
            M.mpm_tape_forward(ctx, [s.view() for s in sets])            # 3 steps, 2 slots
        with pytest.raises(M.MPMError):
            M.mpm_tape_forward(ctx, [sets[0].view(), sets[0].view()])    # the same set twice
        with pytest.raises(M.MPMError):
            M.mpm_tape_reserve(plain, 2)                                  # not an adjoint context
        M.mpm_tape_forward(ctx, [s.view() for s in sets[:3]])
        with pytest.raises(M.MPMError):
            M.mpm_p2g(ctx, sets[0].view())                                # no build is current
        rc, flags = M.mpm_get_status(ctx)
        assert rc == 0, flags
    finally:
        M.mpm_destroy(ctx)
        M.mpm_destroy(plain)
