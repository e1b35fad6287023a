"""Input generators: the landslide's resolution sweep keeps the same slide."""
import numpy as np

from paper_2605_28525_amd import workloads as wl


def test_landslide_coarse_geometry():
    w = wl.landslide(h=4)
    assert w.cells == (512, 512, 64) and w.dx == 4.0 and np.isclose(w.dt, 4e-3)
    # footprint 63 x 62 columns, 10 cells thick, 8 particles per cell
    assert w.n == 63 * 62 * 10 * 8
    x = w.x.astype(np.float64)
    i = np.floor(x[0] / w.dx).astype(np.int64)
    j = np.floor(x[1] / w.dx).astype(np.int64)
    # every particle lies above the terrain at the four corner nodes of its column
    corner = np.maximum(np.maximum(w.heightmap[i, j], w.heightmap[i + 1, j]),
                        np.maximum(w.heightmap[i, j + 1], w.heightmap[i + 1, j + 1]))
    assert np.all(x[2] >= corner)
    # the terrain is the full-resolution one sampled at every 4th node
    hm1, _ = wl.landslide_terrain((2048, 2048), 1.0, 2)
    assert np.array_equal(w.heightmap, hm1[::4, ::4])
    # the same mass of material per unit of footprint area
    assert np.isclose(w.p_mass * w.n / (63 * 62 * 16), 2000.0 * 40, rtol=0.01)
