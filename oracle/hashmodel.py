"""Model of the hash-based block construction (test infrastructure only).

What Methods 3.3 defines, written as sets rather than as a sequence of
insertions:

* the blocks to store are the distinct blocks of the nodes of every particle's
  support (the block-level layout of Methods 3.2, B = 4), each named by its
  packed 64-bit key (Eq. 22);
* a key's home slot is its 64-bit mix (Eq. 23) masked to the table size H, a
  power of two (Eq. 24); collisions continue to the next slot, cyclically
  (linear probing, Eq. 25);
* a construction overflows when the distinct keys outnumber the block
  capacity or the table, or when some key would have to probe more than
  ``n_probe`` slots; the remedy is to double the table and the capacity and
  build again until it fits.

With linear probing and no deletions the set of occupied slots does not depend
on the order of insertion, but which key ends up in which slot does.  The
model places the keys in ascending key order, one canonical choice; tests
compare only order-free results (the key set, the occupied slots, the
overflow decision with an unlimited probe length, the number of doublings).
"""
from __future__ import annotations

import numpy as np

from .sparse import stencil_nodes, block_of, pack_key

MASK64 = (1 << 64) - 1


def mix64(z: int) -> int:
    """SplitMix64 output function (Steele, Lea and Flood 2014), one of the
    64-bit mixers the paper cites for Eq. 23."""
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9 & MASK64
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB & MASK64
    return z ^ (z >> 31)


def block_keys(x: np.ndarray, dx: float) -> set:
    """Packed keys (Eq. 22) of the distinct blocks touched by the particles'
    supports."""
    d = x.shape[1]
    blocks = np.unique(block_of(stencil_nodes(x, dx).reshape(-1, d)), axis=0)
    return {int(k) for k in pack_key(blocks)}


def home_slot(key: int, H: int) -> int:
    """Eq. 24: s = h & (H - 1) with h the mixed key of Eq. 23."""
    return mix64(key) & (H - 1)


class HashModel:
    """The table that a set of keys occupies under linear probing."""

    def __init__(self, keys, H: int, block_capacity: int, n_probe: int | None = None):
        assert H > 0 and H & (H - 1) == 0
        self.H = H
        self.capacity = block_capacity
        self.n_probe = H if n_probe is None else n_probe
        self.keys = sorted(keys)
        self.slot = {}       # key -> slot
        self.probes = {}     # key -> slots examined to place it (1 = its home slot)
        occupied = set()
        for k in self.keys:
            if len(occupied) == H:
                break
            s, r = home_slot(k, H), 1
            while s in occupied:                 # Eq. 25
                s, r = (s + 1) & (H - 1), r + 1
            occupied.add(s)
            self.slot[k], self.probes[k] = s, r

    @property
    def overflow(self) -> bool:
        n = len(self.keys)
        return (n > self.capacity or n > self.H
                or any(r > self.n_probe for r in self.probes.values()))

    def compact_index(self) -> dict:
        """One compact index Phi per stored key, a bijection onto [0, n)
        (slot order: any bijection is a valid Phi)."""
        return {k: i for i, k in enumerate(sorted(self.slot, key=self.slot.get))}


def build(x: np.ndarray, dx: float, H: int, block_capacity: int, n_probe: int | None = None):
    """The construction with its rebuild rule (table and capacity doubled until
    nothing overflows).  Returns the final model and the number of doublings."""
    keys = block_keys(x, dx)
    t = HashModel(keys, H, block_capacity, n_probe)
    rebuilds = 0
    while t.overflow:
        rebuilds += 1
        t = HashModel(keys, t.H * 2, t.capacity * 2, n_probe)
    return t, rebuilds
