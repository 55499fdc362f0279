"""GPU parity at the benchmark's full sizes, in the launch configuration the
benchmark times (one Volume, same calls, same stream).

CT-like 512x512x460 u16 (12-bit), 32 partitions: bricks, all 32 PDMs, D' for
all 200 TFs and D for 20 of them, each against the oracle element by element.

Both: the range table (max_level 8) and D' through it for every TF (c2:
the whole table against the oracle's definition; c3: 4 sampled table maps
against PDMs of the merged partitions built from scratch, and D' through the
table equal to the plain update's).

Tube tree 1024x1024x795 u8, 64 partitions: bricks and all 64 PDMs; the S
mask and D' for all 200 TFs; D from the volume and D from the cached brick
ranges for 20 of them (every tenth), each against the oracle element by
element, and D' <= D there (Sec. 3.1).

The batched workload of 48 volumes in the autotuner's launch shape: six
sampled volumes (largest and smallest of each dtype, two seeded) against
the oracle: bricks, every PDM, S and D' of its own TF.

A 2048x2048x1100 u8 volume (4.3 GiB, past 2^32 bytes) with 64 partitions
(4.3 GiB of PDMs): bricks in full, 3 sampled PDMs, and D' and D for one TF,
so that voxel and map offsets beyond 32 bits are exercised.
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
    say("[case] c2 range table")
    v.build_range_table(8)
    torch.cuda.synchronize()
    table = orc.range_table(want, 8)
    np.testing.assert_array_equal(pdm.from_device(v.table).reshape(table.shape), table)
    d = torch.empty_like(v.dist)
    dr = torch.empty_like(v.dist)
    for k, alpha in enumerate(alphas):
        mask = v.update_tf(alpha)
        mr = v.update_tf_ranges(alpha, out=dr)
        torch.cuda.synchronize()
        dp, m = orc.tf_update(want, bounds, alpha, L)
        np.testing.assert_array_equal(mask, m)
        np.testing.assert_array_equal(mr, m)
        np.testing.assert_array_equal(pdm.from_device(v.dist), dp, err_msg=f"D' tf {k}")
        np.testing.assert_array_equal(pdm.from_device(dr), dp, err_msg=f"D' via table, tf {k}")
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
    say("[case] c3 oracle PDMs, all 64")
    want = orc.pdms(vol, bounds, L, brick_minmax=(bmin, bmax))
    got = pdm.from_device(v.pdms)
    for p in range(n):
        np.testing.assert_array_equal(got[p], want[p], err_msg=f"PDM {p}")
    del got
    say("[case] c3 range table")
    v.build_range_table(8)
    torch.cuda.synchronize()
    # sampled table maps against the PDM of the merged partition built from
    # scratch (the union property), level k map p = partitions p .. p+2^k-1
    first = {1: 0}
    for k in range(2, 7):
        first[k] = first[k - 1] + n - (1 << (k - 1)) + 1
    for k, p in ((1, 0), (3, 5), (5, 20), (6, 0)):
        lo, hi = int(bounds[p]), int(bounds[p + (1 << k)]) - 1
        tw = orc.dt(orc.pom_range(bmin, bmax, lo, hi))
        np.testing.assert_array_equal(pdm.from_device(v.table[first[k] + p]), tw,
                                      err_msg=f"table level {k} map {p}")
    # the plain method's D (from the volume and from the cached brick
    # ranges) on every tenth TF: 20 of the 200
    d = torch.empty_like(v.dist)
    dc = torch.empty_like(v.dist)
    dr = torch.empty_like(v.dist)
    for k, alpha in enumerate(alphas):
        mask = v.update_tf(alpha)
        mr = v.update_tf_ranges(alpha, out=dr)
        full = k % 10 == 0
        if full:
            v.full_recompute(alpha, out=d)
            v.full_recompute_cached(alpha, out=dc)
        torch.cuda.synchronize()
        assert torch.equal(dr, v.dist), f"D' via table differs, tf {k}"
        np.testing.assert_array_equal(mr, mask)
        dp, m = orc.tf_update(want, bounds, alpha, L)
        np.testing.assert_array_equal(mask, m, err_msg=f"S tf {k}")
        dp_gpu = pdm.from_device(v.dist)
        np.testing.assert_array_equal(dp_gpu, dp, err_msg=f"D' tf {k}")
        if full:
            say(f"[case] c3 oracle D (volume and cached ranges) for tf {k}")
            d_gpu = pdm.from_device(d)
            np.testing.assert_array_equal(d_gpu, orc.full_recompute(vol, alpha, L),
                                          err_msg=f"D tf {k}")
            np.testing.assert_array_equal(pdm.from_device(dc),
                                          orc.dt(orc.plain_occ_range(bmin, bmax, alpha, L)),
                                          err_msg=f"D cached tf {k}")
            assert (dp_gpu <= d_gpu).all(), f"D' > D somewhere, tf {k}"


@pytest.mark.timeout(400)
def test_batched_48_volumes_sampled(pdm, orc):
    """The batched workload (48 volumes, dims 96-640 per axis, half u8 and
    half 12-bit u16, 16/32/64 partitions) built in the launch shape the
    autotuner picks for it and updated with a different TF per volume in one
    launch; six sampled volumes (the largest u8 and u16, the smallest of each,
    two more drawn from a seed) against the oracle: bricks, every PDM, the S
    mask and D'."""
    import torch
    specs = W.batch_specs()
    say(f"[case] batch of {len(specs)} volumes: generate and upload")
    vols, items = [], []
    for sp in specs:
        host = W.batch_volume(sp)
        bounds = W.uniform_bounds(sp["levels"], sp["n"])
        v = pdm.Volume(pdm.to_device(host), sp["levels"], bounds, voxel_dtype=sp["dtype"])
        vols.append((v, bounds, sp))
        items.append((v.desc, v.volume, v.bmin, v.bmax, bounds, v.pdms))
        del host
    ws = torch.empty(pdm.batch_workspace_bytes(len(items)), dtype=torch.uint8, device="cuda")
    config = dict(single_launch=0, rows_per_item=1, lines_mult=1, largest_first=1)
    say(f"[case] batch build, config {config}")
    pdm.batch_build(items, ws, config)
    rng = np.random.default_rng(48)
    alphas = [W.trapezoid_tf(sp["levels"], int(rng.integers(1, 5)), rng) for _, _, sp in vols]
    upd = [(v.desc, v.pdms, bounds, a, v.dist) for (v, bounds, _), a in zip(vols, alphas)]
    masks = pdm.batch_tf_update(upd)
    torch.cuda.synchronize()
    assert pdm.batch_error(ws) == 0
    size = [int(np.prod(sp["shape"])) for _, _, sp in vols]
    u8 = [k for k, (_, _, sp) in enumerate(vols) if sp["dtype"] == np.uint8]
    u16 = [k for k, (_, _, sp) in enumerate(vols) if sp["dtype"] == np.uint16]
    pick = {max(u8, key=size.__getitem__), max(u16, key=size.__getitem__),
            min(u8, key=size.__getitem__), min(u16, key=size.__getitem__)}
    rest = [k for k in range(len(vols)) if k not in pick]
    pick |= set(int(k) for k in rng.choice(rest, 2, replace=False))
    for k in sorted(pick):
        v, bounds, sp = vols[k]
        say(f"[case] batch volume {k}: {sp['shape']} {np.dtype(sp['dtype']).name} n={sp['n']}")
        host = W.batch_volume(sp)
        bmin, bmax = orc.bricks(host)
        np.testing.assert_array_equal(pdm.from_device(v.bmin, sp["dtype"]), bmin, err_msg=f"bmin {k}")
        np.testing.assert_array_equal(pdm.from_device(v.bmax, sp["dtype"]), bmax, err_msg=f"bmax {k}")
        want = orc.pdms(host, bounds, sp["levels"], brick_minmax=(bmin, bmax))
        np.testing.assert_array_equal(pdm.from_device(v.pdms), want, err_msg=f"PDMs {k}")
        dp, m = orc.tf_update(want, bounds, alphas[k], sp["levels"])
        np.testing.assert_array_equal(masks[k], m, err_msg=f"S {k}")
        np.testing.assert_array_equal(pdm.from_device(v.dist), dp, err_msg=f"D' {k}")


@pytest.mark.timeout(300)
def test_volume_over_4_gib_u8(pdm, orc):
    import torch
    shape = (1100, 2048, 2048)
    say(f"[case] volume over 4 GiB: generate {shape} u8")
    rng = np.random.default_rng(23)
    vol = np.zeros(shape, np.uint8)
    for _ in range(400):
        c = [int(rng.integers(0, d)) for d in shape]
        h = [int(rng.integers(2, 40)) for _ in shape]
        vol[max(0, c[0] - h[0]):c[0] + h[0], max(0, c[1] - h[1]):c[1] + h[1],
            max(0, c[2] - h[2]):c[2] + h[2]] = int(rng.integers(1, 256))
    assert vol.nbytes > 2 ** 32
    L, n = 256, 64
    bounds = W.uniform_bounds(L, n)
    say("[case] volume over 4 GiB: build on GPU")
    v = pdm.Volume(pdm.to_device(vol), L, bounds)
    assert v.pdm_bytes > 2 ** 32
    v.build()
    alpha = np.zeros(L, np.float32)
    alpha[100:140] = 0.5
    alpha[250] = 1.0
    mask = v.update_tf(alpha)
    d = torch.empty_like(v.dist)
    v.full_recompute(alpha, out=d)
    torch.cuda.synchronize()
    bmin, bmax = orc.bricks(vol)
    np.testing.assert_array_equal(pdm.from_device(v.bmin), bmin)
    np.testing.assert_array_equal(pdm.from_device(v.bmax), bmax)
    for p in (0, 17, 63):
        say(f"[case] volume over 4 GiB: PDM {p}")
        want = orc.dt(orc.pom_range(bmin, bmax, int(bounds[p]), int(bounds[p + 1]) - 1))
        np.testing.assert_array_equal(pdm.from_device(v.pdms[p]), want, err_msg=f"PDM {p}")
    m = orc.active(bounds, alpha, L)
    np.testing.assert_array_equal(mask, m)
    say("[case] volume over 4 GiB: D' and D")
    union = np.zeros(bmin.shape, np.uint8)
    for p in orc.active_list(m, n):
        union |= orc.pom_range(bmin, bmax, int(bounds[p]), int(bounds[p + 1]) - 1)
    np.testing.assert_array_equal(pdm.from_device(v.dist), orc.dt(union), err_msg="D'")
    np.testing.assert_array_equal(pdm.from_device(d), orc.full_recompute(vol, alpha, L),
                                  err_msg="D")
