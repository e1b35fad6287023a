"""Helpers for the GPU-vs-oracle parity tests (test infrastructure).

Protocol: the GPU and the FP64 oracle start every compared step from the same
float32 state (widened exactly to float64 for the oracle); the GPU runs its
four calls through the C ABI, the oracle runs the dense-grid definition, and
the results are compared

* active blocks and node masks: bit-exact as sets;
* grid mass, momentum (p = m v + dt f_int) and updated velocity: keyed by node
  coordinate;
* particle x, v, C, F, tau: keyed by particle id;

each float field normwise, max|a - b| <= RTOL * max|b| (RTOL = 1e-5), with an
absolute floor for the stress, TAU_ULPS u32 (2 mu + d lambda) with u32 = 2^-24:
float32 storage fixes the elastic strain only to about one float32 ulp, and
the stress inherits that absolute error.  The stress therefore misses the
1e-5 relative bar where strains are small (the 2D collapse: about 2e-5
normwise); the floor of a few ulps still catches a regression of a few times
that error.
"""
from __future__ import annotations

import numpy as np

from oracle import mpm as om
from oracle import sparse as osp

RTOL = 1e-5
TAU_ULPS = 4


def tau_floor(w) -> float:
    mu, lam = om.lame(w.E, w.nu)
    return TAU_ULPS * 2.0 ** -24 * (2 * mu + w.dim * lam)


def normwise(a: np.ndarray, b: np.ndarray) -> float:
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = np.max(np.abs(b)) if b.size else 0.0
    num = np.max(np.abs(a - b)) if b.size else 0.0
    return num / den if den > 0 else num


def assert_field(name, got, ref, rtol=RTOL, atol=0.0):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    err = np.max(np.abs(got - ref)) if ref.size else 0.0
    scale = np.max(np.abs(ref)) if ref.size else 0.0
    bound = max(rtol * scale, atol)
    assert err <= bound, f"{name}: max|diff| {err:.3e} > bound {bound:.3e} (max|ref| {scale:.3e})"
    return err / scale if scale > 0 else err


# ---------------------------------------------------------------------------
def gpu_step_parts(sim, sparse=True):
    """One GPU step on sim.a -> sim.b through the C ABI, capturing the active set
    and both grid states.  Leaves the advanced state in sim.b (not swapped)."""
    import torch
    from paper_2605_28525_amd import mpm as M
    ctx = sim.ctx
    a, b = sim.a.view(), sim.b.view()
    M.mpm_sparse_build(ctx, a)
    nb, nt = M.mpm_active_count(ctx)
    npb = 4 ** sim.w.dim
    out = {"nb": nb, "n_touched": nt}
    if sparse:
        keys = torch.zeros(nb, dtype=torch.int64, device="cuda")
        masks = torch.zeros(nb, dtype=torch.int64, device="cuda")
        M.mpm_get_active(ctx, keys, masks, nb)
        out["keys"] = keys.cpu().numpy().view(np.uint64)
        out["masks"] = masks.cpu().numpy().view(np.uint64)
    g = torch.zeros((nb, npb, 4), dtype=torch.float32, device="cuda")
    M.mpm_p2g(ctx, a)
    M.mpm_get_grid(ctx, g, nb)
    out["grid_p2g"] = g.cpu().numpy().copy()
    M.mpm_grid_update(ctx)
    M.mpm_get_grid(ctx, g, nb)
    out["grid_upd"] = g.cpu().numpy().copy()
    M.mpm_g2p(ctx, a, b)
    order = torch.zeros(sim.a.n, dtype=torch.int32, device="cuda")
    M.mpm_get_order(ctx, order, sim.a.n)
    out["order"] = order.cpu().numpy().view(np.uint32)
    rc, flags = M.mpm_get_status(ctx)
    out["status"] = (rc, flags)
    out["state_in"] = sim.a.to_arrays()
    out["ids_in"] = sim.a.ids()
    out["state_out"] = sim.b.to_arrays()
    out["ids_out"] = sim.b.ids()
    return out


def block_coords_of(keys, dim):
    return osp.unpack_key(keys, dim)


def grid_nodes(blocks: np.ndarray, dim: int) -> np.ndarray:
    """Node coordinates of every node of the given blocks, (nb, 4^d, d), l(n) order."""
    loc = np.array([[l & 3, (l >> 2) & 3, l >> 4][:dim] for l in range(4 ** dim)])
    return blocks[:, None, :] * 4 + loc[None, :, :]


def oracle_reference(w, state_soa: dict):
    p = om.Params.from_workload(w)
    st = om.state_from_soa(state_soa, w.dim)
    out, grid, vgrid = om.step(st, p, return_grid=True)
    keys, masks = osp.active_blocks_and_masks_by_cells(st["x"], p)
    return p, out, grid, vgrid, keys, masks


def compare_step(w, parts, sparse=True, check_particles=True):
    """Compare one captured GPU step with the oracle.  Returns a dict of the
    normwise errors."""
    d = w.dim
    p, out, grid, vgrid, okeys, omasks = oracle_reference(w, parts["state_in"])
    errs = {}
    nb = parts["nb"]
    if sparse:
        gk = parts["keys"]
        gm = parts["masks"]
        assert len(set(gk.tolist())) == nb, "duplicate block keys"
        got = dict(zip(gk.tolist(), gm.tolist()))
        ref = dict(zip(okeys.tolist(), omasks.tolist()))
        assert got.keys() == ref.keys(), f"active block sets differ: {len(got)} vs {len(ref)}"
        bad = [k for k in ref if got[k] != ref[k]]
        assert not bad, f"{len(bad)} blocks with different node masks"
        blocks = block_coords_of(gk, d)
    else:
        nblk = [(c + 1 + 3) // 4 for c in w.cells[:d]]
        lin = np.arange(nb)
        bx = lin % nblk[0]
        rest = lin // nblk[0]
        if d == 3:
            blocks = np.stack([bx, rest % nblk[1], rest // nblk[1]], axis=1)
        else:
            blocks = np.stack([bx, rest], axis=1)
    nodes = grid_nodes(blocks, d).reshape(-1, d)
    inside = np.all(nodes <= np.array(w.cells[:d]), axis=1)
    nodes = nodes[inside]
    idx = tuple(nodes.T)
    g1 = parts["grid_p2g"].reshape(-1, 4)[inside]
    g2 = parts["grid_upd"].reshape(-1, 4)[inside]
    # every oracle node with mass lies in a GPU block
    assert np.isclose(grid["m"][idx].sum(), grid["m"].sum(), rtol=1e-12, atol=0)
    pref = grid["mv"] + p.dt * grid["f_int"]
    errs["m"] = assert_field("grid m", g1[:, 3], grid["m"][idx])
    errs["p"] = assert_field("grid p", g1[:, :d], pref[idx])
    errs["v_grid"] = assert_field("grid v", g2[:, :d], vgrid[idx])
    assert np.array_equal(g2[:, 3], g1[:, 3])
    if not check_particles:
        return errs
    # particles: GPU output position i holds input particle order[i]
    order = parts["order"].astype(np.int64)
    so = parts["state_out"]
    ids_in, ids_out = parts["ids_in"], parts["ids_out"]
    assert np.array_equal(ids_out, ids_in[order]), "id not carried with the permutation"
    assert np.array_equal(np.sort(order), np.arange(len(order))), "order is not a permutation"
    n = len(order)
    ref_soa = om.state_to_soa(out)
    for k in ("x", "v", "C", "F"):
        errs[k] = assert_field(f"particle {k}", so[k], ref_soa[k][:, order])
    errs["tau"] = assert_field("particle tau", so["tau"], ref_soa["tau"][:, order], atol=tau_floor(w))
    # the stress error in units of the floor (<= 1 where the floor decides)
    errs["tau_floor_units"] = float(np.max(np.abs(so["tau"] - ref_soa["tau"][:, order]))) / tau_floor(w)
    return errs
