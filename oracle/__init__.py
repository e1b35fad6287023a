"""FP64 CPU reference of the explicit sparse-grid MPM step.

TEST INFRASTRUCTURE ONLY.  This package is the oracle against which the HIP
path is checked; only the test suite, the smoke check and the CPU-baseline leg
of the benchmark may import it.  It shares no code with the HIP path and the
HIP path never calls it.

Modules
-------
``mpm``           dense-grid explicit MPM step (P2G, grid update with boundary
                  conditions, G2P with APIC, Hencky elasticity and a
                  Drucker-Prager return map), all in float64.
``sparse``        the active-node set, its block-level layout, the local node
                  index, the packed 64-bit block key and the sparsity ratio.
``hashmodel``     the table a set of block keys occupies under linear probing,
                  with the overflow rule and the doubling rebuild, used to pin
                  the semantics of the hash-based construction.
"""
