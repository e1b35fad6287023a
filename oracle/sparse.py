"""Active-node set and its block-level layout (test infrastructure only).

* Particle support S(p) and the active set A = union_p S(p) (Eqs. 4-5).  The
  support is taken as the full 3^d stencil from the base node, which contains
  the zero-weight node at exact half-cell ties (Methods 3.2 and Algorithm 6 visit
  "all nodes in the support" by enumerating that stencil).
* Blocks of B x B (x B) nodes with B = 4 (Methods 3.2, block-level
  construction); the block of node n is floor(n / B) per axis and its local
  index is l(n) = i_l + B (j_l + B k_l) with i_l = i - floor(i/B) B
  (Algorithms 1 and 5, final step).
* The packed key of Eq. 22 with m = 21 bits per coordinate and bias 2^20
  (Methods 3.3); in 2D the two coordinates fill the lower 2m bits.
* The sparsity ratio of Eq. 1 (Results 2.2).
"""
from __future__ import annotations

import numpy as np

from .mpm import base_node, stencil_offsets, check_domain

B = 4
KEY_BITS = 21
KEY_BIAS = 1 << 20


def stencil_nodes(x: np.ndarray, dx: float) -> np.ndarray:
    """All stencil nodes of every particle, (N, 3^d, d) int64."""
    b = base_node(x, dx)
    offs = np.array(stencil_offsets(x.shape[1]))
    return b[:, None, :] + offs[None, :, :]


def active_nodes(x: np.ndarray, p) -> np.ndarray:
    """A as sorted unique node indices (M, d), lexicographic order."""
    check_domain(base_node(x, p.dx), p)
    nodes = stencil_nodes(x, p.dx).reshape(-1, x.shape[1])
    return np.unique(nodes, axis=0)


def block_of(nodes: np.ndarray) -> np.ndarray:
    return np.floor_divide(nodes, B)


def local_index(nodes: np.ndarray) -> np.ndarray:
    """l(n) = (i - (i//B) B) + B ((j - (j//B) B) + B (k - (k//B) B))."""
    loc = nodes - np.floor_divide(nodes, B) * B
    out = loc[:, -1].copy()
    for a in range(nodes.shape[1] - 2, -1, -1):
        out = loc[:, a] + B * out
    return out


def block_masks(nodes: np.ndarray):
    """Active blocks (sorted, lexicographic) and, per block, the bit mask of its
    active nodes (bit l(n) set for every active node n of the block)."""
    blk = block_of(nodes)
    bits = np.left_shift(np.uint64(1), local_index(nodes).astype(np.uint64))
    ub, inv = np.unique(blk, axis=0, return_inverse=True)
    inv = inv.ravel()
    masks = np.zeros(len(ub), np.uint64)
    np.bitwise_or.at(masks, inv, bits)
    return ub, masks


def pack_key(coords: np.ndarray, m: int = KEY_BITS, bias: int = KEY_BIAS) -> np.ndarray:
    """Eq. 22: Key = ((i + b) << 2m) | ((j + b) << m) | (k + b) as uint64."""
    c = np.asarray(coords, np.int64) + bias
    if (c < 0).any() or (c >= (1 << m)).any():
        raise ValueError("coordinate outside the packable range")
    c = c.astype(np.uint64)
    d = c.shape[1]
    key = np.zeros(len(c), np.uint64)
    for a in range(d):
        key |= np.left_shift(c[:, a], np.uint64(m * (d - 1 - a)))
    return key


def unpack_key(key: np.ndarray, d: int, m: int = KEY_BITS, bias: int = KEY_BIAS) -> np.ndarray:
    key = np.asarray(key, np.uint64)
    mask = np.uint64((1 << m) - 1)
    out = np.empty((len(key), d), np.int64)
    for a in range(d):
        out[:, a] = (np.right_shift(key, np.uint64(m * (d - 1 - a))) & mask).astype(np.int64) - bias
    return out


def active_blocks_and_masks(x: np.ndarray, p):
    """(packed keys, node masks) of every active block, sorted by key."""
    ub, masks = block_masks(active_nodes(x, p))
    keys = pack_key(ub)
    order = np.argsort(keys, kind="stable")
    return keys[order], masks[order]


def active_blocks_and_masks_by_cells(x: np.ndarray, p):
    """The result of active_blocks_and_masks for large particle sets.  A depends
    only on the set of distinct base nodes, so those are found first (as linear
    node codes over the grid), then the union of their stencils."""
    b = base_node(x, p.dx)
    check_domain(b, p)
    shape = tuple(p.nodes)
    cells = np.unique(np.ravel_multi_index(tuple(b.T), shape))
    ub = np.stack(np.unravel_index(cells, shape), axis=1)
    offs = np.array(stencil_offsets(x.shape[1]))
    nodes = (ub[:, None, :] + offs[None, :, :]).reshape(-1, x.shape[1])
    codes = np.unique(np.ravel_multi_index(tuple(nodes.T), shape))
    blocks, masks = block_masks(np.stack(np.unravel_index(codes, shape), axis=1).astype(np.int64))
    keys = pack_key(blocks)
    order = np.argsort(keys, kind="stable")
    return keys[order], masks[order]


def n_active_nodes(x: np.ndarray, p) -> int:
    """n_active of Eq. 1 at one instant: the number of nodes in A."""
    return int(len(active_nodes(x, p)))


def sparsity_ratio(positions_over_time, p) -> float:
    """Eq. 1: r_active = min over t of n_dense / n_active(t), where n_dense is
    the number of nodes of the dense background grid (the potential domain,
    cells + 1 nodes per axis) and n_active(t) the number of active nodes at
    time t.  ``positions_over_time`` holds one (N, d) position array per
    sampled instant."""
    n_dense = int(np.prod(p.nodes))
    return float(min(n_dense / n_active_nodes(x, p) for x in positions_over_time))
