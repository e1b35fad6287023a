"""Batched ensembles, graph replay and the autotuner on the GPU.

The ensemble contract: instance i of a batch computes what the stand-alone
run of instance i computes.  Each compared step starts both sides from the
same float32 state; the active block sets (with node masks) must agree
bit-exactly and every particle field within the parity bar (normwise 1e-5,
stress with its float32 floor).  The batch is also checked directly against
the FP64 oracle, one instance at a time.
"""
import numpy as np
import pytest

from parity_util import RTOL, assert_field, oracle_reference, tau_floor
from oracle import mpm as om
from oracle import sparse as osp
from paper_2605_28525_amd import workloads as wl

pytestmark = pytest.mark.gpu

FIELDS = ("x", "v", "C", "F", "tau")


def _announce(*a):
    print("CASE", *a, flush=True)


def _decode_ensemble_keys(keys):
    """Ensemble block keys: instance in bits 57..62, 19-bit coordinates biased by 2^18."""
    k = keys.astype(np.uint64)
    m = np.uint64((1 << 19) - 1)
    inst = ((k >> np.uint64(57)) & np.uint64(63)).astype(np.int64)
    b = np.stack([((k >> np.uint64(38)) & m).astype(np.int64), ((k >> np.uint64(19)) & m).astype(np.int64),
                  (k & m).astype(np.int64)], axis=1) - (1 << 18)
    return inst, b


def _active(ctx, nb):
    import torch
    from paper_2605_28525_amd import mpm as M
    keys = torch.zeros(nb, dtype=torch.int64, device="cuda")
    masks = torch.zeros(nb, dtype=torch.int64, device="cuda")
    M.mpm_get_active(ctx, keys, masks, nb)
    return keys.cpu().numpy().view(np.uint64), masks.cpu().numpy().view(np.uint64)


def _one_step(sim):
    """Build + P2G + grid update + G2P of sim.a into sim.b; returns the active set."""
    from paper_2605_28525_amd import mpm as M
    a, b = sim.a.view(), sim.b.view()
    M.mpm_sparse_build(sim.ctx, a)
    nb, _ = M.mpm_active_count(sim.ctx)
    keys, masks = _active(sim.ctx, nb)
    M.mpm_p2g(sim.ctx, a)
    M.mpm_grid_update(sim.ctx)
    M.mpm_g2p(sim.ctx, a, b)
    rc, flags = M.mpm_get_status(sim.ctx)
    assert rc == 0, flags
    return keys, masks


def _by_id(ps, ids_wanted):
    """Fields of a ParticleSet at the positions holding the given ids."""
    st = ps.to_arrays()
    ids = ps.ids().astype(np.int64)
    pos = np.empty(ids.max() + 1, np.int64)
    pos[ids] = np.arange(len(ids))
    sel = pos[ids_wanted]
    return {k: st[k][:, sel] for k in FIELDS}


def _member_index(ens):
    """member_index[g] = position of combined particle g inside its member."""
    out = np.empty(ens.n, np.int64)
    for i in range(ens.n_instances):
        out[ens.member_positions(i)] = np.arange(ens.members[i].n)
    return out


def test_ensemble_matches_single_instance_runs():
    from paper_2605_28525_amd import mpm as M
    ens = wl.ensemble_small()
    _announce("ensemble vs single runs", ens.n_instances, [m.n for m in ens.members])
    midx = _member_index(ens)
    batch = M.Simulation(ens)
    singles = [M.Simulation(m) for m in ens.members]
    try:
        for step in range(4):
            st = batch.a.to_arrays()
            ids = batch.a.ids().astype(np.int64)
            insts = batch.a.insts().astype(np.int64)
            bkeys, bmasks = _one_step(batch)
            binst, bblk = _decode_ensemble_keys(bkeys)
            for i, (m, sim) in enumerate(zip(ens.members, singles)):
                sel = np.nonzero(insts == i)[0]
                order = np.argsort(midx[ids[sel]])
                sim.set_state({k: st[k][:, sel[order]] for k in FIELDS})
                skeys, smasks = _one_step(sim)
                sblk = osp.unpack_key(skeys, 3)
                got = {tuple(b): int(mk) for b, mk in zip(bblk[binst == i].tolist(), bmasks[binst == i])}
                ref = {tuple(b): int(mk) for b, mk in zip(sblk.tolist(), smasks)}
                assert got == ref, f"step {step} instance {i}: active sets differ ({len(got)} vs {len(ref)})"
                # batch output of member i, in member order, vs the single run's output (ids = member order)
                member_ids = ens.member_positions(i)
                bo = _by_id(batch.b, member_ids)
                so = _by_id(sim.b, np.arange(m.n))
                for k in FIELDS:
                    assert_field(f"step {step} inst {i} {k}", bo[k], so[k], RTOL,
                                 atol=tau_floor(m) if k == "tau" else 0.0)
            batch.a, batch.b = batch.b, batch.a
            assert np.array_equal(np.sort(batch.a.ids()), np.arange(ens.n)), "ids lost"
            assert np.array_equal(np.bincount(batch.a.insts(), minlength=ens.n_instances),
                                  [m.n for m in ens.members]), "instance ids not carried"
    finally:
        batch.close()
        for s in singles:
            s.close()


def test_ensemble_step_matches_oracle():
    """One batched step, then each instance against the FP64 dense-grid oracle
    run on that instance alone with its own material and dt."""
    import torch
    from paper_2605_28525_amd import mpm as M
    ens = wl.ensemble_small(seed=7, n_instances=5)
    for m in ens.members:
        wl.perturbed(m, seed=11, v_scale=0.05, C_scale=0.5, F_scale=1e-3, tau_scale=50.0)
    # rebuild the combined arrays from the perturbed members
    for k in FIELDS:
        arr = getattr(ens, k)
        for i, m in enumerate(ens.members):
            arr[:, ens.member_positions(i)] = getattr(m, k)
    _announce("ensemble vs oracle", [m.n for m in ens.members])
    batch = M.Simulation(ens)
    try:
        keys, masks = _one_step(batch)
        binst, bblk = _decode_ensemble_keys(keys)
        for i, m in enumerate(ens.members):
            p, out, grid, vgrid, okeys, omasks = oracle_reference(m, m.state())
            oblk = osp.unpack_key(okeys, 3)
            got = {tuple(b): int(mk) for b, mk in zip(bblk[binst == i].tolist(), masks[binst == i])}
            ref = {tuple(b): int(mk) for b, mk in zip(oblk.tolist(), omasks)}
            assert got == ref, f"instance {i}: active sets differ from the oracle"
            bo = _by_id(batch.b, ens.member_positions(i))
            ref_soa = om.state_to_soa(out)
            for k in FIELDS:
                assert_field(f"inst {i} {k}", bo[k], ref_soa[k], RTOL, atol=tau_floor(m) if k == "tau" else 0.0)
    finally:
        batch.close()


@pytest.mark.parametrize("kind", ["ensemble", "collapse_2d"])
def test_graph_replay_matches_eager(kind):
    """A captured two-step graph, replayed three times with eager work and host
    synchronisation in between; each replay starts from the eager state and
    must match two eager steps from it."""
    import torch
    from paper_2605_28525_amd import mpm as M
    w = wl.ensemble_small(seed=9) if kind == "ensemble" else wl.perturbed(wl.collapse_2d(), seed=3)
    _announce("graph replay", kind, w.n)
    g = M.Simulation(w)
    e = M.Simulation(w)
    try:
        M.mpm_graph_capture(g.ctx, g.a.view(), g.b.view(), 2)
        for rep in range(3):
            g.a.copy_(e.a)
            torch.cuda.synchronize()
            M.mpm_graph_launch(g.ctx, 1)
            e.step(2)
            torch.cuda.synchronize()
            assert g.status()[0] == 0 and e.status()[0] == 0
            ids = np.sort(e.a.ids().astype(np.int64))
            go, eo = _by_id(g.a, ids), _by_id(e.a, ids)
            for k in FIELDS:
                tf = tau_floor(w.members[0] if kind == "ensemble" else w)
                assert_field(f"replay {rep} {k}", go[k], eo[k], RTOL, atol=tf if k == "tau" else 0.0)
            if kind == "ensemble":
                assert np.array_equal(_by_id_inst(g.a, ids), _by_id_inst(e.a, ids))
        M.mpm_graph_release(g.ctx)
    finally:
        g.close()
        e.close()


def _by_id_inst(ps, ids_wanted):
    ids = ps.ids().astype(np.int64)
    pos = np.empty(ids.max() + 1, np.int64)
    pos[ids] = np.arange(len(ids))
    return ps.insts()[pos[ids_wanted]]


def test_autotune_leaves_input_and_steps_correctly():
    import torch
    from paper_2605_28525_amd import mpm as M
    ens = wl.ensemble_small(seed=13)
    _announce("autotune", ens.n)
    t = M.Simulation(ens)
    e = M.Simulation(ens)
    try:
        before = t.a.to_arrays()
        chunk, g2p_block, p2g_wg, g2p_wg = M.mpm_autotune(t.ctx, t.a.view(), t.b.view())
        assert (g2p_block, chunk) in ((64, 64), (64, 128), (128, 128), (128, 256), (256, 256), (256, 512),
                                      (256, 768))
        assert p2g_wg in (1024, 2048, 4096, 8192) and g2p_wg in (1024, 2048, 4096, 8192)
        after = t.a.to_arrays()
        for k in FIELDS:
            assert np.array_equal(before[k], after[k]), f"autotune changed input {k}"
        # b holds one step of a
        e.step(1)
        ids = np.arange(ens.n)
        to, eo = _by_id(t.b, ids), _by_id(e.a, ids)
        for k in FIELDS:
            assert_field(f"autotuned step {k}", to[k], eo[k], RTOL,
                         atol=tau_floor(ens.members[0]) if k == "tau" else 0.0)
        # and the tuned context keeps stepping like the default one
        t.step(3)
        e.step(3)
        assert t.status()[0] == 0
    finally:
        t.close()
        e.close()


def test_bad_instance_id_is_reported():
    import torch
    from paper_2605_28525_amd import mpm as M
    ens = wl.ensemble_small(seed=15, n_instances=3)
    _announce("bad instance id", ens.n)
    s = M.Simulation(ens)
    try:
        s.a.inst[5] = 3
        M.mpm_sparse_build(s.ctx, s.a.view())
        rc, flags = M.mpm_get_status(s.ctx)
        assert rc == M.MPM_ERR_DOMAIN and flags & M.MPM_FLAG_DOMAIN
    finally:
        s.close()


def test_g2p_launch_shapes_agree():
    """Every G2P launch shape the tuner may pick computes the same step: with
    one build and one grid, the three workgroup sizes give bit-identical
    particles; across work-item sizes (a new build and P2G each) the step
    agrees at the parity bar."""
    import torch
    from paper_2605_28525_amd import mpm as M
    w = wl.perturbed(wl.collapse_3d(seed=2, scale=2), seed=5)
    _announce("g2p launch shapes", w.n)
    sim = M.Simulation(w)
    try:
        a, b = sim.a.view(), sim.b.view()
        M.mpm_set_tuning(sim.ctx, 128, 128, 0, 0)
        M.mpm_sparse_build(sim.ctx, a)
        M.mpm_p2g(sim.ctx, a)
        M.mpm_grid_update(sim.ctx)
        outs = []
        for blk in (64, 128, 256):
            M.mpm_set_tuning(sim.ctx, 0, blk, 0, 0)
            sim.b.zero_()
            M.mpm_g2p(sim.ctx, a, b)
            assert M.mpm_get_status(sim.ctx)[0] == 0
            outs.append(sim.b.to_arrays())
        for o in outs[1:]:
            for k in FIELDS:
                assert np.array_equal(o[k], outs[0][k]), k
        ids = np.arange(w.n)
        ref = None
        for blk, chunk in ((256, 512), (64, 64), (64, 128), (128, 256), (256, 256), (256, 768)):
            M.mpm_set_tuning(sim.ctx, chunk, blk, 0, 0)
            M.mpm_step(sim.ctx, a, b, 1)
            assert M.mpm_get_status(sim.ctx)[0] == 0
            got = _by_id(sim.b, ids)
            if ref is None:
                ref = got
                continue
            for k in FIELDS:
                assert_field(f"shape {blk}/{chunk} {k}", got[k], ref[k], RTOL, atol=tau_floor(w) if k == "tau" else 0.0)
    finally:
        sim.close()
