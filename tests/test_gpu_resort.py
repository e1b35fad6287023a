"""GPU: the incremental re-sort (default after a build of the same particle
count) against the full radix sort (MPM_FLAG_FULL_SORT), and the particle
layout every build must produce.

Layout property, checked on the permutation mpm_g2p applies: each owner block's
particles occupy one contiguous range, and inside it the particles are stored
rank-major over the block's base cells (rank r lists, in ascending cell order,
the cells holding more than r particles; ranks from 32 on follow cell by cell).

Equivalence: two contexts step the same state; per step the active blocks and
node masks agree bit-exactly, the P2G grid and the advanced particles agree to
the parity tolerance (the two orders differ in how blocks are ordered and in the
order of the particles that changed block, which changes only the summation
order of float32 sums).
"""
import numpy as np
import pytest

from paper_2605_28525_amd import workloads as wl
from parity_util import RTOL, assert_field, gpu_step_parts, tau_floor

pytestmark = pytest.mark.gpu

IL_ROUNDS = 32


def _announce(*a):
    print("CASE", *a, flush=True)


def _owner_cell(x, dx, dim):
    """Owner block (tuple of arrays) and local base cell of each particle,
    base node floor(x * (1/dx) - 1/2) in float64 as the binning does."""
    s = x[:dim].astype(np.float64) * (1.0 / dx) - 0.5
    b = np.floor(s).astype(np.int64)
    owner = b >> 2
    loc = b & 3
    cell = loc[0] + 4 * loc[1] + (16 * loc[2] if dim == 3 else 0)
    return owner, cell


def check_layout(x_in, order, dx, dim):
    """x_in: input positions (dim, n); order[i] = input index written to position i."""
    owner, cell = _owner_cell(x_in[:, order], dx, dim)
    n = order.size
    assert np.array_equal(np.sort(order), np.arange(n, dtype=order.dtype)), "order is not a permutation"
    change = np.any(owner[:, 1:] != owner[:, :-1], axis=0)
    starts = np.concatenate([[0], np.nonzero(change)[0] + 1])
    ends = np.concatenate([starts[1:], [n]])
    ids = [tuple(owner[:, s]) for s in starts]
    assert len(set(ids)) == len(ids), "an owner block occupies more than one range"
    for s, e in zip(starts, ends):
        q = cell[s:e]
        counts = np.bincount(q, minlength=4 ** dim)
        expect = []
        for r in range(IL_ROUNDS):
            expect.extend(np.nonzero(counts > r)[0].tolist())
        for c in range(4 ** dim):
            expect.extend([c] * max(int(counts[c]) - IL_ROUNDS, 0))
        assert np.array_equal(q, np.asarray(expect)), f"block range {s}:{e} is not rank-major over its cells"


def _grid_by_key(parts):
    keys = parts["keys"]
    idx = np.argsort(keys)
    return keys[idx], parts["grid_p2g"][idx]


def compare_parts(w, a, b):
    ka, ma = np.sort(a["keys"]), a["masks"][np.argsort(a["keys"])]
    kb, mb = np.sort(b["keys"]), b["masks"][np.argsort(b["keys"])]
    assert np.array_equal(ka, kb), "active blocks differ"
    assert np.array_equal(ma, mb), "node masks differ"
    _, ga = _grid_by_key(a)
    _, gb = _grid_by_key(b)
    assert_field("grid m", ga[..., 3], gb[..., 3])
    assert_field("grid p", ga[..., :w.dim], gb[..., :w.dim])


def compare_states(w, sa, sb):
    ia, ib = np.argsort(sa.ids()), np.argsort(sb.ids())
    A, B = sa.to_arrays(), sb.to_arrays()
    for k in ("x", "v", "C", "F", "tau"):
        assert_field(k, A[k][:, ia], B[k][:, ib], RTOL, atol=tau_floor(w) if k == "tau" else 0.0)


def _pair(w):
    import torch
    from paper_2605_28525_amd import mpm as M
    assert torch.cuda.is_available()
    return M.Simulation(w), M.Simulation(w, flags=M.MPM_FLAG_FULL_SORT)


def _run_pair(w, steps, label):
    inc, full = _pair(w)
    for k in range(steps):
        x_in = inc.a.to_arrays()["x"]
        pi = gpu_step_parts(inc)
        pf = gpu_step_parts(full)
        assert pi["status"][0] == 0 and pf["status"][0] == 0, (label, k, pi["status"], pf["status"])
        check_layout(x_in, pi["order"], w.dx, w.dim)
        compare_parts(w, pi, pf)
        compare_states(w, inc.b, full.b)
        inc.a, inc.b = inc.b, inc.a
        full.a, full.b = full.b, full.a
    return inc, full


@pytest.mark.parametrize("name", ["collapse_2d", "landslide_crop", "tiny_3d"])
def test_incremental_matches_full_sort(name):
    w = {"collapse_2d": lambda: wl.perturbed(wl.collapse_2d(), seed=9, v_scale=0.5),
         "landslide_crop": wl.landslide_crop,
         "tiny_3d": lambda: wl.tiny_3d(n=64, ties=False)}[name]()
    _announce("resort vs full sort", name, w.n)
    inc, full = _run_pair(w, 6, name)
    inc.close()
    full.close()


@pytest.mark.parametrize("name", ["collapse_2d", "landslide_crop"])
def test_incremental_after_large_displacements(name):
    """Particles displaced by up to several blocks between two builds on the
    same context: most are movers, many into blocks without a previous slot."""
    w = {"collapse_2d": lambda: wl.perturbed(wl.collapse_2d(), seed=9, v_scale=0.5),
         "landslide_crop": wl.landslide_crop}[name]()
    _announce("resort after displacement", name, w.n)
    inc, full = _run_pair(w, 2, name)
    rng = np.random.default_rng(31)
    st = inc.a.to_arrays()
    ids = inc.a.ids()
    shift = rng.integers(-8, 9, size=(w.dim, w.n)) * (w.dx * rng.random((w.dim, w.n)))
    lo = 3.0 * w.dx
    hi = np.asarray(w.cells[:w.dim], np.float64)[:, None] * w.dx - 3.0 * w.dx
    st["x"] = np.clip(st["x"].astype(np.float64) + shift, lo, hi).astype(np.float32)
    # the same displaced state, in the incremental context's current order, on both
    inc.set_state(st, ids=ids)
    full.set_state(st, ids=ids)
    _run_pair_continue(w, inc, full, 2, name)
    inc.close()
    full.close()


def _run_pair_continue(w, inc, full, steps, label):
    for k in range(steps):
        x_in = inc.a.to_arrays()["x"]
        pi = gpu_step_parts(inc)
        pf = gpu_step_parts(full)
        assert pi["status"][0] == 0 and pf["status"][0] == 0, (label, k, pi["status"], pf["status"])
        check_layout(x_in, pi["order"], w.dx, w.dim)
        compare_parts(w, pi, pf)
        compare_states(w, inc.b, full.b)
        inc.a, inc.b = inc.b, inc.a
        full.a, full.b = full.b, full.a


def _dense_blocks():
    """A 3D cluster at 64 particles per cell (8^3 cells, 32,768 particles):
    4096 particles per owner block, more than the re-sort stages in LDS, and
    64 per cell, past the rank-major layout's 32 interleaved ranks."""
    w = wl.tiny_3d(n=48, ties=False)
    rng = np.random.default_rng(41)
    x = wl.stratified_cells((4, 4, 4), (12, 12, 12), w.dx, 4, rng)
    st = wl.rest_state(x)
    for k, a in st.items():
        setattr(w, k, a)
    w.ppc = 64
    w.p_vol0 = w.dx ** 3 / 64
    w.p_mass = 2000.0 * w.p_vol0
    return wl.perturbed(w, seed=43, v_scale=0.05, C_scale=0.2, F_scale=1e-3, tau_scale=50.0)


def test_incremental_dense_blocks():
    """Blocks of 4096 particles (placement without LDS staging) and cells of
    64 (ranks past the interleaved ones), before and after displacing every
    particle by up to a cell."""
    w = _dense_blocks()
    _announce("resort dense blocks", w.n)
    inc, full = _run_pair(w, 2, "dense_blocks")
    rng = np.random.default_rng(47)
    st = inc.a.to_arrays()
    ids = inc.a.ids()
    st["x"] = (st["x"].astype(np.float64) + rng.uniform(-1.0, 1.0, size=st["x"].shape) * w.dx).astype(np.float32)
    inc.set_state(st, ids=ids)
    full.set_state(st, ids=ids)
    _run_pair_continue(w, inc, full, 2, "dense_blocks displaced")
    inc.close()
    full.close()
