"""GPU: the allocation-free scan query (mpm_scan_active_static, static device
scratch) against mpm_scan_active (the context's scratch), two calls in a row
with the second on a smaller input, and its size limit."""
import numpy as np
import pytest

from paper_2605_28525_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _announce(*a):
    print("CASE", *a, flush=True)


def _query(fn, ctx, pset):
    import torch
    n = fn(ctx, pset.view(), None, None, 0)            # count only
    k = torch.full((max(n, 1),), -1, dtype=torch.int64, device="cuda")
    m = torch.full_like(k, -1)
    assert fn(ctx, pset.view(), k, m, n) == n
    return k[:n].cpu().numpy().view(np.uint64).copy(), m[:n].cpu().numpy().view(np.uint64).copy()


def _subset(w, stride):
    """Every `stride`-th particle of w, as a new particle set."""
    from paper_2605_28525_amd import mpm as M
    st = {k: np.ascontiguousarray(v[:, ::stride]) for k, v in w.state().items()}
    return M.ParticleSet.from_arrays(st)


def _static_no_alloc(M, ctx, pset, cap):
    """One static query into preallocated outputs; the free device memory is
    the same before and after it (the static array was mapped by an earlier
    call)."""
    import torch
    k = torch.full((max(cap, 1),), -1, dtype=torch.int64, device="cuda")
    m = torch.full_like(k, -1)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    n = M.mpm_scan_active_static(ctx, pset.view(), k, m, cap)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0, "device memory changed across the static query"
    return n, k[:min(n, cap)].cpu().numpy().view(np.uint64).copy(), m[:min(n, cap)].cpu().numpy().view(np.uint64).copy()


@pytest.mark.parametrize("name", ["collapse_2d", "fd_copy", "landslide_crop"])
def test_static_scan_equals_scan_active(name):
    from paper_2605_28525_amd import mpm as M
    w = {"collapse_2d": lambda: wl.perturbed(wl.collapse_2d(), seed=5),
         "fd_copy": wl.differentiable_fd_copy,
         "landslide_crop": wl.landslide_crop}[name]()
    _announce("static scan query", name, w.n)
    ref = M.Simulation(w, flags=M.MPM_FLAG_SCAN_BUILD)   # mpm_scan_active needs the context scratch
    plain = M.Simulation(w)                               # no scan scratch of its own
    try:
        M.mpm_scan_active_static(plain.ctx, ref.a.view(), None, None, 0)   # maps the static array if first
        for pset, label in ((ref.a, "full"), (_subset(w, 7), "every 7th")):
            ks, ms = _query(M.mpm_scan_active, ref.ctx, pset)
            n, kz, mz = _static_no_alloc(M, plain.ctx, pset, len(ks))
            print(label, pset.n, "blocks", len(ks), n, flush=True)
            assert len(ks) > 0 and n == len(ks)
            assert np.array_equal(kz, ks) and np.array_equal(mz, ms)
            # a capacity below the count: the first entries only, count unchanged
            n2, kc, mc = _static_no_alloc(M, plain.ctx, pset, len(ks) // 2)
            assert n2 == len(ks)
            assert np.array_equal(kc, ks[:len(ks) // 2]) and np.array_equal(mc, ms[:len(ks) // 2])
        rc, flags = plain.status()
        assert rc == 0, flags
    finally:
        ref.close()
        plain.close()


def test_static_scan_rejects_a_box_beyond_its_scratch():
    """Two particles at opposite corners of the landslide's 2048 x 2048 x 256
    grid: the mask domain (about 12 M blocks) exceeds the static scratch, so
    the call returns MPM_ERR_OVERFLOW and writes nothing; a following call on a
    small set succeeds."""
    import torch
    from paper_2605_28525_amd import mpm as M
    w = wl.landslide_crop()
    w.cells = (2048, 2048, 256)
    w.heightmap = None
    x = np.array([[10.2, 2000.7], [11.3, 2001.1], [12.6, 200.4]], dtype=np.float32)
    st = wl.rest_state(x)
    for k, a in st.items():
        setattr(w, k, a)
    _announce("static scan too large", w.n)
    sim = M.Simulation(w)
    try:
        k = torch.full((8,), -1, dtype=torch.int64, device="cuda")
        m = torch.full_like(k, -1)
        import ctypes
        nb = ctypes.c_int(-7)
        rc = M.lib.mpm_scan_active_static(sim.ctx, ctypes.byref(sim.a.view()), ctypes.c_void_p(k.data_ptr()),
                                          ctypes.c_void_p(m.data_ptr()), 8, ctypes.byref(nb), None)
        assert rc == M.MPM_ERR_OVERFLOW and nb.value == 0
        assert np.all(k.cpu().numpy() == -1) and np.all(m.cpu().numpy() == -1)
        one = _subset(w, 2)      # the first particle alone: a 2 x 2 x 2-block domain
        kz, mz = _query(M.mpm_scan_active_static, sim.ctx, one)
        assert len(kz) >= 1
    finally:
        sim.close()
