"""Brick [min,max] at the volume's edges, bit-exact against the oracle.

Widths that are not a multiple of 16 voxels put the last quad of every row
past the row end (its bricks are loaded at the row end with the previous
brick's voxels masked); widths of 4 to 15 voxels have only such quads, and
widths below 4 take the voxel-at-a-time path; depths and heights that are
not a multiple of 4 cut the last brick layer.  Voxels are independent random
values, so a masked voxel that leaked into a brick, or a row that was missed,
changes its min or max.  Every volume goes through the brick pass, the
batched build (grouped and single launch) and the plain method's x pass
(occupancy from the voxels), u8 and 12-bit u16 (Sec. 3.1)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

# (z, y, x) voxels; several rows per volume, layers cut in z and y
EDGE_SHAPES = [(5, 7, 4), (6, 3, 5), (7, 9, 7), (3, 2, 15), (9, 6, 17), (5, 5, 20), (2, 3, 31),
               (7, 5, 33), (6, 9, 47), (3, 4, 61), (1, 1, 3), (2, 2, 2), (5, 11, 130), (3, 6, 515),
               (4, 4, 16), (8, 8, 64)]


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("dtype,levels", [(np.uint8, 256), (np.uint16, 4096)], ids=["u8", "u16"])
def test_edge_quads(orc, dtype, levels):
    import torch
    import paper_2407_21552_amd as pdm
    assert torch.cuda.is_available()
    rng = np.random.default_rng(31 if dtype == np.uint8 else 32)
    bounds = W.uniform_bounds(levels, 4)
    alpha = np.zeros(levels, np.float32)
    alpha[levels // 3: levels // 2] = 1.0
    vols = []
    for shape in EDGE_SHAPES:
        vol = rng.integers(0, levels, size=shape).astype(dtype)
        say(f"[case] edge quads {np.dtype(dtype).name} shape={shape}")
        v = pdm.Volume(pdm.to_device(vol), levels, bounds, voxel_dtype=dtype)
        v.build()
        d = torch.empty_like(v.dist)
        v.full_recompute(alpha, out=d)
        torch.cuda.synchronize()
        bmin, bmax = orc.bricks(vol)
        np.testing.assert_array_equal(pdm.from_device(v.bmin, dtype), bmin, err_msg=f"bmin {shape}")
        np.testing.assert_array_equal(pdm.from_device(v.bmax, dtype), bmax, err_msg=f"bmax {shape}")
        np.testing.assert_array_equal(pdm.from_device(v.pdms), orc.pdms(vol, bounds, levels),
                                      err_msg=f"pdms {shape}")
        np.testing.assert_array_equal(pdm.from_device(d), orc.full_recompute(vol, alpha, levels),
                                      err_msg=f"D {shape}")
        vols.append((vol, v))
    ws = torch.empty(pdm.batch_workspace_bytes(len(vols)), dtype=torch.uint8, device="cuda")
    for single in (0, 1):
        for _, v in vols:
            v.bmin.fill_(0)
            v.bmax.fill_(0)
            v.pdms.fill_(0)
        items = [(v.desc, v.volume, v.bmin, v.bmax, bounds, v.pdms) for _, v in vols]
        say(f"[case] batched build of the edge volumes, single_launch={single}")
        pdm.batch_build(items, ws, {"single_launch": single})
        torch.cuda.synchronize()
        assert pdm.batch_error(ws) == 0
        for vol, v in vols:
            bmin, bmax = orc.bricks(vol)
            np.testing.assert_array_equal(pdm.from_device(v.bmin, dtype), bmin, err_msg=f"batched bmin {vol.shape}")
            np.testing.assert_array_equal(pdm.from_device(v.bmax, dtype), bmax, err_msg=f"batched bmax {vol.shape}")
            np.testing.assert_array_equal(pdm.from_device(v.pdms), orc.pdms(vol, bounds, levels),
                                          err_msg=f"batched pdms {vol.shape}")
