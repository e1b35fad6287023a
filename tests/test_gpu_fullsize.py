"""GPU at the landslide's full size, in the launch configuration bench.py times
(20,000,000 particles, 2048 x 2048 x 256 cells, block capacity 2^18, shape
chosen by mpm_autotune), after 10 steps and after 2500 steps (half of the
configuration's 5000, the slide spread out and accelerated to about 20 m/s).

Properties of the whole step that hold at any size: the status word is clear,
the output is a permutation of the input carrying the ids, every output is
finite, total grid mass equals N m_p and total grid momentum equals
sum m_p v_p (the APIC and internal-force terms sum to zero over the nodes).

Sampled outputs against the FP64 oracle: a 40 x 40-column window of the slide
(every particle whose base node lies in it, about 0.4 M, shifted to the
window's origin) is stepped by the oracle on the same terrain crop; nodes
whose contributing particles all lie in the window (and away from the
window's faces) are compared with the GPU's grid, node by node (mass,
momentum, updated velocity, and the active node masks of the blocks there),
and particles whose 27 nodes are all such nodes with the GPU's output, at the
parity tolerance.  The landslide coarsened to dx = 4 m and 2 m gets the same
window comparison after 10 steps.
"""
import numpy as np
import pytest

from oracle import mpm as om
from paper_2605_28525_amd import workloads as wl
from parity_util import (RTOL, assert_field, block_coords_of, compare_step, gpu_step_parts, grid_nodes,
                         oracle_reference, tau_floor)

pytestmark = pytest.mark.gpu

I0, J0, W = 120, 1000, 40   # window origin (multiples of the block size) and width in cells


def _base(x, dx):
    s = x.astype(np.float64) * (1.0 / dx) - 0.5
    return np.floor(s).astype(np.int64)


def check_window(w, parts, i0, j0, width, h=1):
    """One step of a window of the slide on the FP64 oracle against the GPU's
    step: every particle whose base node lies in the window (shifted to its
    origin, an exact shift by whole cells), stepped on the same terrain crop;
    nodes whose contributing particles all lie in the window compared node by
    node (mass, momentum, updated velocity, active node masks of the blocks
    there), and particles whose 27 nodes are all such nodes.  Returns the
    errors and counts."""
    I0, J0, W = i0, j0, width
    n, d, dx = w.n, w.dim, w.dx
    sin, sout = parts["state_in"], parts["state_out"]
    order = parts["order"].astype(np.int64)
    g1 = parts["grid_p2g"].reshape(-1, 4).astype(np.float64)
    g2 = parts["grid_upd"].reshape(-1, 4)
    b_in = _base(sin["x"], dx)
    sel = np.nonzero((b_in[0] >= I0 + 3) & (b_in[0] < I0 + W - 3) &
                     (b_in[1] >= J0 + 3) & (b_in[1] < J0 + W - 3))[0]
    ww = wl.landslide(h=h, window=((I0, I0 + W), (J0, J0 + W)), footprint=((0, 1), (0, 1)), thickness=1)
    sub = {k: np.ascontiguousarray(sin[k][:, sel]) for k in ("x", "v", "C", "F", "tau")}
    sub["x"] = sub["x"].copy()
    sub["x"][0] = (sin["x"][0, sel].astype(np.float64) - I0 * dx).astype(np.float32)
    sub["x"][1] = (sin["x"][1, sel].astype(np.float64) - J0 * dx).astype(np.float32)
    # the shift is exact (whole cells), so base nodes shift by (I0, J0)
    assert np.array_equal(_base(sub["x"], dx)[0], b_in[0, sel] - I0)
    for k, a in sub.items():
        setattr(ww, k, a)
    print("window particles", len(sel), flush=True)
    p, out, grid, vgrid, okeys, omasks = oracle_reference(ww, sub)

    # complete nodes: every particle with base in [node - 2, node] is in the window
    lo, hi = 5, W - 4
    blocks = block_coords_of(parts["keys"], d)                  # global block coordinates
    nodes = grid_nodes(blocks, d).reshape(-1, d)
    wx, wy = nodes[:, 0] - I0, nodes[:, 1] - J0
    inner = (wx >= lo) & (wx <= hi) & (wy >= lo) & (wy <= hi) & (nodes[:, 2] <= w.cells[2])
    idx = (wx[inner], wy[inner], nodes[inner, 2])
    pref = grid["mv"] + p.dt * grid["f_int"]
    errs = {"nodes": int(inner.sum())}
    errs["m"] = assert_field("grid m", g1[inner, 3], grid["m"][idx])
    errs["p"] = assert_field("grid p", g1[inner, :d], pref[idx])
    errs["v_grid"] = assert_field("grid v", g2[inner, :d], vgrid[idx])
    # every oracle node with mass in the complete region lies in a GPU block
    region = grid["m"][lo:hi + 1, lo:hi + 1, :]
    assert np.isclose(grid["m"][idx].sum(), region.sum(), rtol=1e-12, atol=0)
    # node masks of the blocks wholly inside the complete region
    om_blocks = block_coords_of(okeys, d)
    gk = {tuple(c): m for c, m in zip((blocks - [I0 // 4, J0 // 4, 0]).tolist(), parts["masks"].tolist())}
    n_cmp = 0
    for c, m in zip(om_blocks.tolist(), omasks.tolist()):
        if 4 * c[0] >= lo and 4 * c[0] + 3 <= hi and 4 * c[1] >= lo and 4 * c[1] + 3 <= hi:
            assert gk.get(tuple(c)) == m, ("node mask", c)
            n_cmp += 1
    errs["blocks"] = n_cmp
    okset = {tuple(c) for c in om_blocks.tolist()}
    for c in gk:
        if 4 * c[0] >= lo and 4 * c[0] + 3 <= hi and 4 * c[1] >= lo and 4 * c[1] + 3 <= hi:
            assert c in okset, ("GPU block not in the oracle's active set", c)
    # particles whose 27 nodes are complete
    pos_in_sub = np.full(n, -1, np.int64)
    pos_in_sub[sel] = np.arange(len(sel))
    src = order                                                  # GPU output o holds input particle order[o]
    bsub = _base(sub["x"], dx)
    ok_sub = (bsub[0] >= lo) & (bsub[0] + 2 <= hi) & (bsub[1] >= lo) & (bsub[1] + 2 <= hi)
    o_sel = np.nonzero((pos_in_sub[src] >= 0) & ok_sub[np.maximum(pos_in_sub[src], 0)])[0]
    k_sel = pos_in_sub[src[o_sel]]
    ref = om.state_to_soa(out)
    # positions in window coordinates (the shift is exact in float64)
    x_gpu = sout["x"][:, o_sel].astype(np.float64)
    x_gpu[0] -= I0 * dx
    x_gpu[1] -= J0 * dx
    errs["x"] = assert_field("particle x", x_gpu, ref["x"][:, k_sel])
    for k in ("v", "C", "F"):
        errs[k] = assert_field(f"particle {k}", sout[k][:, o_sel], ref[k][:, k_sel])
    errs["tau"] = assert_field("particle tau", sout["tau"][:, o_sel], ref["tau"][:, k_sel], RTOL, atol=tau_floor(w))
    errs["particles"] = int(len(o_sel))
    print(errs)
    return errs


@pytest.mark.parametrize("steps_before", [10, 2500])
def test_landslide_full_size(steps_before):
    from paper_2605_28525_amd import mpm as M
    w = wl.landslide()
    n, d, dx = w.n, w.dim, w.dx
    print("CASE landslide full size", n, "after", steps_before, "steps", flush=True)
    sim = M.Simulation(w, block_capacity=1 << 18)
    try:
        sim.step(steps_before)
        M.mpm_autotune(sim.ctx, sim.a.view(), sim.b.view())
        parts = gpu_step_parts(sim)
    finally:
        sim.close()
    assert parts["status"][0] == 0, parts["status"]
    sin, sout = parts["state_in"], parts["state_out"]
    order = parts["order"].astype(np.int64)
    assert np.array_equal(np.sort(order), np.arange(n)), "order is not a permutation"
    assert np.array_equal(parts["ids_out"], parts["ids_in"][order]), "ids not carried"
    for f in ("x", "v", "C", "F", "tau"):
        assert np.isfinite(sout[f]).all(), f
    g1 = parts["grid_p2g"].reshape(-1, 4).astype(np.float64)
    g2 = parts["grid_upd"].reshape(-1, 4)
    m_tot = n * float(w.p_mass)
    assert abs(g1[:, 3].sum() - m_tot) <= 1e-5 * m_tot, (g1[:, 3].sum(), m_tot)
    v_in = sin["v"].astype(np.float64)
    mom = float(w.p_mass) * v_in.sum(axis=1)
    scale = float(w.p_mass) * np.abs(v_in).sum()
    assert np.all(np.abs(g1[:, :d].sum(axis=0) - mom) <= 1e-5 * scale), (g1[:, :d].sum(axis=0), mom)

    errs = check_window(w, parts, I0, J0, W)
    assert errs["particles"] > 100000 and errs["nodes"] > 10000 and errs["blocks"] > 100


def test_ensemble_full_size():
    """The 64-instance ensemble (about 19.5 M particles) in its benchmarked
    configuration (autotuned), one batched step after two: ids and instances
    carried, and four instances (the smallest, the largest and two others)
    against stand-alone runs from the same state (active sets bit-exact,
    fields at the parity tolerance)."""
    from paper_2605_28525_amd import mpm as M
    from test_gpu_ensemble import FIELDS, _by_id, _decode_ensemble_keys, _member_index, _one_step
    from oracle import sparse as osp
    ens = wl.ensemble()
    print("CASE ensemble full size", ens.n_instances, ens.n, flush=True)
    sizes = np.array([m.n for m in ens.members])
    pick = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 17, 42})
    midx = _member_index(ens)
    batch = M.Simulation(ens)
    try:
        batch.step(2)
        M.mpm_autotune(batch.ctx, batch.a.view(), batch.b.view())
        st = batch.a.to_arrays()
        ids = batch.a.ids().astype(np.int64)
        insts = batch.a.insts().astype(np.int64)
        bkeys, bmasks = _one_step(batch)
        binst, bblk = _decode_ensemble_keys(bkeys)
        out_ids = batch.b.ids()
        assert np.array_equal(np.sort(out_ids), np.arange(ens.n)), "ids lost"
        assert np.array_equal(np.bincount(batch.b.insts(), minlength=ens.n_instances), sizes), "instances lost"
        for i in pick:
            m = ens.members[i]
            sel = np.nonzero(insts == i)[0]
            order = np.argsort(midx[ids[sel]])
            sim = M.Simulation(m)
            try:
                sim.set_state({k: st[k][:, sel[order]] for k in FIELDS})
                skeys, smasks = _one_step(sim)
                sblk = osp.unpack_key(skeys, 3)
                got = {tuple(b): int(mk) for b, mk in zip(bblk[binst == i].tolist(), bmasks[binst == i])}
                ref = {tuple(b): int(mk) for b, mk in zip(sblk.tolist(), smasks)}
                assert got == ref, f"instance {i}: active sets differ ({len(got)} vs {len(ref)})"
                bo = _by_id(batch.b, ens.member_positions(i))
                so = _by_id(sim.b, np.arange(m.n))
                for k in FIELDS:
                    assert_field(f"inst {i} {k}", bo[k], so[k], RTOL, atol=tau_floor(m) if k == "tau" else 0.0)
                print("instance", i, m.n, "ok", flush=True)
            finally:
                sim.close()
    finally:
        batch.close()


def test_collapse_3d_full_size():
    """The 3D column collapse at full size (2,097,152 particles, 512 x 128 x 128
    cells): one step after 10 in the benchmarked configuration, checked by the
    whole-step properties (status, permutation and ids, finite outputs, grid
    mass and momentum) and against the FP64 oracle's step from the same state
    over the whole domain (active blocks and node masks bit-exact, every node
    and every particle at the parity tolerance; about 1.5 minutes of oracle
    time on the host)."""
    from paper_2605_28525_amd import mpm as M
    w = wl.collapse_3d()
    n, d = w.n, w.dim
    print("CASE collapse_3d full size", n, flush=True)
    sim = M.Simulation(w)
    try:
        sim.step(10)
        parts = gpu_step_parts(sim)
    finally:
        sim.close()
    assert parts["status"][0] == 0, parts["status"]
    order = parts["order"].astype(np.int64)
    assert np.array_equal(np.sort(order), np.arange(n))
    assert np.array_equal(parts["ids_out"], parts["ids_in"][order])
    for f in ("x", "v", "C", "F", "tau"):
        assert np.isfinite(parts["state_out"][f]).all(), f
    g1 = parts["grid_p2g"].reshape(-1, 4).astype(np.float64)
    m_tot = n * float(w.p_mass)
    assert abs(g1[:, 3].sum() - m_tot) <= 1e-5 * m_tot
    v_in = parts["state_in"]["v"].astype(np.float64)
    mom = float(w.p_mass) * v_in.sum(axis=1)
    assert np.all(np.abs(g1[:, :d].sum(axis=0) - mom) <= 1e-5 * float(w.p_mass) * np.abs(v_in).sum())
    print("oracle step of the whole collapse ...", flush=True)
    print(compare_step(w, parts), flush=True)


# window origin (block multiples) and width in coarse cells, and the least
# particles, nodes and blocks compared
COARSE_WINDOWS = {4: (20, 240, 24, (10000, 2000, 20)), 2: (40, 480, 32, (50000, 8000, 100))}


@pytest.mark.parametrize("h", [4, 2])
def test_landslide_coarse(h):
    """The landslide coarsened to dx = 4 m (312,480 particles, 512 x 512 x 64
    cells) and 2 m (2,480,000 particles, 1024 x 1024 x 128 cells), the
    resolution sweep of the bench: whole-step properties after 10 steps, the
    sparse and the dense grid giving the same positions after 10 steps
    (within 4 float32 ulps of the largest coordinate), and the next step of a
    window of the slide against the FP64 oracle, node by node and particle by
    particle (check_window)."""
    from paper_2605_28525_amd import mpm as M
    w = wl.landslide(h=h)
    n, d = w.n, w.dim
    print("CASE landslide coarse", h, n, flush=True)
    xs = {}
    for mode in (M.MPM_GRID_SPARSE, M.MPM_GRID_DENSE):
        sim = M.Simulation(w, grid_mode=mode)
        try:
            sim.step(10)
            rc, flags = sim.status()
            assert rc == 0, (mode, flags)
            x = sim.a.to_arrays()["x"].astype(np.float64)
            xb = np.empty_like(x)
            xb[:, sim.a.ids().astype(np.int64)] = x
            xs[mode] = xb
            if mode == M.MPM_GRID_SPARSE:
                parts = gpu_step_parts(sim)
        finally:
            sim.close()
    assert parts["status"][0] == 0, parts["status"]
    order = parts["order"].astype(np.int64)
    assert np.array_equal(np.sort(order), np.arange(n))
    assert np.array_equal(parts["ids_out"], parts["ids_in"][order])
    for f in ("x", "v", "C", "F", "tau"):
        assert np.isfinite(parts["state_out"][f]).all(), f
    g1 = parts["grid_p2g"].reshape(-1, 4).astype(np.float64)
    m_tot = n * float(w.p_mass)
    assert abs(g1[:, 3].sum() - m_tot) <= 1e-5 * m_tot
    v_in = parts["state_in"]["v"].astype(np.float64)
    mom = float(w.p_mass) * v_in.sum(axis=1)
    assert np.all(np.abs(g1[:, :d].sum(axis=0) - mom) <= 1e-5 * float(w.p_mass) * np.abs(v_in).sum())
    diff = float(np.max(np.abs(xs[M.MPM_GRID_SPARSE] - xs[M.MPM_GRID_DENSE])))
    ulp = float(np.spacing(np.float32(np.max(np.abs(xs[M.MPM_GRID_SPARSE])))))
    print("sparse - dense max |dx|", diff, "ulp", ulp, flush=True)
    assert diff <= 4 * ulp, (diff, ulp)
    # one step of a window of the coarse slide against the oracle (window in
    # coarse cells, inside the release footprint)
    i0, j0, width, need = COARSE_WINDOWS[h]
    errs = check_window(w, parts, i0, j0, width, h=h)
    assert errs["particles"] > need[0] and errs["nodes"] > need[1] and errs["blocks"] > need[2], errs
