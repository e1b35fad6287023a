"""GPU: the scan-based active set (Algorithms 1-4: block mask over the
bounding box of the owner blocks, exclusive scan, compaction) against the hash
table's (Algorithms 5-6): the same blocks and node masks, bit for bit, on the
workloads of the parity tests and on the full-size landslide."""
import numpy as np
import pytest

from paper_2605_28525_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _sets(sim):
    import torch
    from paper_2605_28525_amd import mpm as M
    M.mpm_sparse_build(sim.ctx, sim.a.view())
    nb, _ = M.mpm_active_count(sim.ctx)
    kh = torch.empty(max(nb, 1), dtype=torch.int64, device="cuda")
    mh = torch.empty_like(kh)
    M.mpm_get_active(sim.ctx, kh, mh, nb)
    n_scan = M.mpm_scan_active(sim.ctx, sim.a.view(), kh, mh, 0)   # count only
    ks = torch.empty(max(n_scan, 1), dtype=torch.int64, device="cuda")
    ms = torch.empty_like(ks)
    assert M.mpm_scan_active(sim.ctx, sim.a.view(), ks, ms, n_scan) == n_scan
    torch.cuda.synchronize()
    rc, flags = sim.status()
    assert rc == 0, flags
    h = dict(zip(kh[:nb].cpu().numpy().view(np.uint64).tolist(), mh[:nb].cpu().numpy().view(np.uint64).tolist()))
    s = dict(zip(ks[:n_scan].cpu().numpy().view(np.uint64).tolist(), ms[:n_scan].cpu().numpy().view(np.uint64).tolist()))
    return nb, n_scan, h, s


@pytest.mark.parametrize("name", ["tiny_3d", "collapse_2d", "fd_copy", "landslide_crop", "landslide_h4"])
def test_scan_equals_hash(name):
    from paper_2605_28525_amd import mpm as M
    w = {"tiny_3d": lambda: wl.tiny_3d(n=48, ties=True),
         "collapse_2d": lambda: wl.perturbed(wl.collapse_2d(), seed=5),
         "fd_copy": wl.differentiable_fd_copy,
         "landslide_crop": wl.landslide_crop,
         "landslide_h4": lambda: wl.landslide(h=4)}[name]()
    print("CASE scan vs hash", name, w.n, flush=True)
    sim = M.Simulation(w)
    try:
        for k in range(2):      # the initial state, then after 5 steps of motion
            nb, n_scan, h, s = _sets(sim)
            print(name, k, "blocks", nb, n_scan, flush=True)
            assert nb == n_scan and len(s) == n_scan, (nb, n_scan, len(s))
            assert h == s
            sim.step(5)
    finally:
        sim.close()


def test_scan_equals_hash_landslide_full():
    from paper_2605_28525_amd import mpm as M
    w = wl.landslide()
    print("CASE scan vs hash landslide", w.n, flush=True)
    sim = M.Simulation(w, block_capacity=1 << 18)
    try:
        sim.step(3)
        nb, n_scan, h, s = _sets(sim)
        print("blocks", nb, n_scan, flush=True)
        assert nb == n_scan and h == s
    finally:
        sim.close()
