"""Sequential model of the hash-based block construction (test infrastructure only).

It follows Methods 3.3 and Algorithms 5-7: every particle enumerates its support
nodes, maps each to its block, packs the block key (Eq. 22), hashes it with a
64-bit mixer (Eq. 23), takes the initial slot h & (H - 1) (Eq. 24), and probes
linearly (Eq. 25) for at most ``n_probe`` slots.  A key seen for the first time
claims the empty slot and receives the next compact block index from a counter;
if that index is not below the block capacity, or no slot was found, the
overflow flag is raised and the table is rebuilt with doubled capacity
(Algorithm 7).  Run sequentially, the model is deterministic; it pins the
semantics (the final block set, overflow and rebuild), not the GPU's order.
"""
from __future__ import annotations

import numpy as np

from .sparse import stencil_nodes, block_of, pack_key

EMPTY = (1 << 64) - 1
MASK64 = (1 << 64) - 1


def mix64(z: int) -> int:
    """SplitMix64 output function (Steele, Lea and Flood 2014), one of the
    64-bit mixers the paper cites for Eq. 23."""
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9 & MASK64
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB & MASK64
    return z ^ (z >> 31)


class BlockHash:
    def __init__(self, H: int, block_capacity: int, n_probe: int | None = None):
        assert H & (H - 1) == 0
        self.H = H
        self.capacity = block_capacity
        self.n_probe = H if n_probe is None else n_probe
        self.reset()

    def reset(self):
        self.keys = [EMPTY] * self.H
        self.vals = [-1] * self.H
        self.active_block_keys = []
        self.count = 0
        self.overflow = False

    def insert(self, key: int):
        s = mix64(key) & (self.H - 1)
        for _ in range(self.n_probe):
            old = self.keys[s]
            if old == EMPTY:
                self.keys[s] = key
                phi = self.count
                self.count += 1
                if phi < self.capacity:
                    self.vals[s] = phi
                    self.active_block_keys.append(key)
                else:
                    self.overflow = True
                return
            if old == key:
                return
            s = (s + 1) & (self.H - 1)
        self.overflow = True

    def insert_particles(self, x: np.ndarray, dx: float):
        d = x.shape[1]
        nodes = stencil_nodes(x, dx)
        for p in range(nodes.shape[0]):
            keys = pack_key(block_of(nodes[p]))
            for k in keys:
                self.insert(int(k))


def build(x: np.ndarray, dx: float, H: int, block_capacity: int, n_probe: int | None = None):
    """Algorithm 5 with the rebuild loop of Algorithm 7 (H and the block capacity
    are doubled together).  Returns the table and the number of rebuilds."""
    t = BlockHash(H, block_capacity, n_probe)
    t.insert_particles(x, dx)
    rebuilds = 0
    while t.overflow:
        rebuilds += 1
        t = BlockHash(t.H * 2, t.capacity * 2, None if n_probe is None else n_probe)
        t.insert_particles(x, dx)
    return t, rebuilds
