"""GPU parity at the benchmark's full sizes, in the launch configuration the
benchmark times (one Volume, same calls, same stream).

CT-like 512x512x460 u16 (12-bit), 32 partitions: bricks, all 32 PDMs, D' for
all 200 TFs and D for 20 of them, each against the oracle element by element.

Tube tree 1024x1024x795 u8, 64 partitions: bricks in full; PDMs of 6 sampled
partitions (dense, sparse, empty); D' and D for 3 TFs, where the oracle's D'
is the distance transform of the union of the active POMs (the union
invariant, pinned separately); for all 200 TFs the active set against the
oracle and D' <= D element-wise (Sec. 3.1).
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def pdm():
    import torch
    import paper_2407_21552_amd as pkg
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    pkg._lib.lib()
    return pkg


@pytest.mark.timeout(300)
def test_ct_like_512x512x460_u16(pdm, orc):
    import torch
    cfg = W.config_info("c2")
    L, n = cfg["levels"], cfg["n"]
    say("[case] c2 generate")
    vol = W.make_volume("c2")
    bounds = W.uniform_bounds(L, n)
    alphas = W.make_tfs("c2")
    say("[case] c2 build on GPU")
    v = pdm.Volume(pdm.to_device(vol), L, bounds, voxel_dtype=np.uint16)
    v.build()
    torch.cuda.synchronize()
    v.check_range()
    bmin, bmax = orc.bricks(vol)
    np.testing.assert_array_equal(pdm.from_device(v.bmin, np.uint16), bmin)
    np.testing.assert_array_equal(pdm.from_device(v.bmax, np.uint16), bmax)
    say("[case] c2 oracle PDMs")
    want = orc.pdms(vol, bounds, L, brick_minmax=(bmin, bmax))
    np.testing.assert_array_equal(pdm.from_device(v.pdms), want)
    d = torch.empty_like(v.dist)
    for k, alpha in enumerate(alphas):
        mask = v.update_tf(alpha)
        torch.cuda.synchronize()
        dp, m = orc.tf_update(want, bounds, alpha, L)
        np.testing.assert_array_equal(mask, m)
        np.testing.assert_array_equal(pdm.from_device(v.dist), dp, err_msg=f"D' tf {k}")
        if k % 10 == 0:
            say(f"[case] c2 full recompute tf {k}")
            v.full_recompute(alpha, out=d)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(pdm.from_device(d), orc.full_recompute(vol, alpha, L),
                                          err_msg=f"D tf {k}")


@pytest.mark.timeout(400)
def test_tube_tree_1024x1024x795_u8(pdm, orc):
    import torch
    cfg = W.config_info("c3")
    L, n = cfg["levels"], cfg["n"]
    say("[case] c3 generate")
    vol = W.make_volume("c3")
    bounds = W.uniform_bounds(L, n)
    alphas = W.make_tfs("c3")
    say("[case] c3 build on GPU")
    v = pdm.Volume(pdm.to_device(vol), L, bounds)
    v.build()
    torch.cuda.synchronize()
    bmin, bmax = orc.bricks(vol)
    np.testing.assert_array_equal(pdm.from_device(v.bmin), bmin)
    np.testing.assert_array_equal(pdm.from_device(v.bmax), bmax)
    for p in (0, 1, 2, 15, 40, 63):
        say(f"[case] c3 PDM partition {p}")
        lo, hi = int(bounds[p]), int(bounds[p + 1]) - 1
        want = orc.dt(orc.pom_range(bmin, bmax, lo, hi))
        np.testing.assert_array_equal(pdm.from_device(v.pdms[p]), want, err_msg=f"PDM {p}")
    d = torch.empty_like(v.dist)
    for k, alpha in enumerate(alphas):
        mask = v.update_tf(alpha)
        v.full_recompute(alpha, out=d)
        torch.cuda.synchronize()
        m = orc.active(bounds, alpha, L)
        np.testing.assert_array_equal(mask, m)
        dp_gpu, d_gpu = pdm.from_device(v.dist), pdm.from_device(d)
        assert (dp_gpu <= d_gpu).all(), f"D' > D somewhere, tf {k}"
        if k in (0, 1, 2):
            say(f"[case] c3 oracle D', D for tf {k}")
            union = np.zeros(bmin.shape, np.uint8)
            for p in orc.active_list(m, n):
                union |= orc.pom_range(bmin, bmax, int(bounds[p]), int(bounds[p + 1]) - 1)
            np.testing.assert_array_equal(dp_gpu, orc.dt(union), err_msg=f"D' tf {k}")
            np.testing.assert_array_equal(d_gpu, orc.full_recompute(vol, alpha, L),
                                          err_msg=f"D tf {k}")
