"""The seeded and printed input models against what the paper states about
them (Sect. 4 and the scalability paragraph of Sect. 3.3): these generators
hold no method arithmetic, so these checks only pin the inputs."""
import numpy as np

import giem_synth as gs


def test_benchmark_model_matches_the_paper():
    m = gs.config_commemi3d3()
    # cubes of 25 m, Nx = 176, Ny = 224, Nz = 118 (Sect. 3.3)
    assert (m["nx"], m["ny"], m["nz"]) == (176, 224, 118)
    assert m["hx"] == m["hy"] == 25.0 and np.allclose(np.diff(m["z_edges"]), 25.0)
    # air, 1 km of 1e-3 S/m, 6.5 km of 1e-4 S/m, half-space 0.1 S/m (Sect. 4)
    assert np.allclose(m["d"], [0.0, 1000.0, 7500.0])
    assert np.allclose(m["sigma"], [0.0, 1e-3, 1e-4, 0.1])
    sb = m["sigma"][m["layer_of_cell"]].real[:, None, None] * np.ones(m["sigma_a"].shape)
    ratio = m["sigma_a"].real / sb
    first = m["layer_of_cell"] == 1
    # maximum contrast 1e4 in the first layer and 3.3e4 in the second (Sect. 4)
    assert np.isclose(ratio[first].max(), 1e4)
    assert np.isclose(ratio[~first].max(), 3.3333e4)
    # seven blocks; every block cell carries its printed conductivity and the
    # volumes match the printed corners
    assert len(m["boxes"]) == 7
    for (x0, x1, y0, y1, z0, z1, sg), blk in zip(m["boxes"], gs.COMMEMI3D3_BLOCKS):
        assert np.all(m["sigma_a"][z0:z1, y0:y1, x0:x1] == sg)
        vol = (x1 - x0) * (y1 - y0) * (z1 - z0) * 25.0 ** 3
        assert np.isclose(vol, 1e9 * (blk[3] - blk[0]) * (blk[4] - blk[1]) * (blk[5] - blk[2]))
    # elsewhere the background
    inside = np.zeros(m["sigma_a"].shape, bool)
    for (x0, x1, y0, y1, z0, z1, _) in m["boxes"]:
        inside[z0:z1, y0:y1, x0:x1] = True
    assert np.all(m["sigma_a"][~inside] == sb[~inside])
