"""GPU parity: every output of the HIP path against the CPU oracle, bit-exact.

Distances, brick summaries and active sets are integers, so the tolerance is
zero.  Inputs are seeded and synthetic (workloads), shaped to span several
work-groups and waves with ragged tails: dims not divisible by 4 or 16, rows
longer than one 256-brick wave segment, y/z lines longer than 256 bricks
(the 255 cap and the wide scan table), unaligned sizes for the vector paths.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pdm():
    import torch
    import paper_2407_21552_amd as pkg
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    pkg._lib.lib()
    return pkg


def say(*a):
    print(*a, flush=True)


def blocky(shape, dtype, levels, seed, keep=0.15, cell=3):
    """Piecewise-constant volume: many distinct brick intervals."""
    rng = np.random.default_rng(seed)
    cz, cy, cx = [(s + cell - 1) // cell for s in shape]
    cells = rng.integers(0, levels, size=(cz, cy, cx))
    cells = np.where(rng.random((cz, cy, cx)) < keep, cells, 0)
    v = np.repeat(np.repeat(np.repeat(cells, cell, 0), cell, 1), cell, 2)
    return np.ascontiguousarray(v[:shape[0], :shape[1], :shape[2]]).astype(dtype)


def run_all(pdm, orc, vol, levels, bounds, alphas, label):
    """Build on the GPU, apply every alpha both ways, compare everything."""
    import torch
    say(f"[case] {label}: shape={vol.shape} dtype={vol.dtype} L={levels} n={len(bounds) - 1}")
    v = pdm.Volume(pdm.to_device(vol), levels, bounds, voxel_dtype=vol.dtype)
    v.build()
    torch.cuda.synchronize()
    bmin, bmax = orc.bricks(vol)
    np.testing.assert_array_equal(pdm.from_device(v.bmin, vol.dtype), bmin)
    np.testing.assert_array_equal(pdm.from_device(v.bmax, vol.dtype), bmax)
    want = orc.pdms(vol, bounds, levels, brick_minmax=(bmin, bmax))
    np.testing.assert_array_equal(pdm.from_device(v.pdms), want)
    d = torch.empty_like(v.dist)
    dc = torch.empty_like(v.dist)
    for k, alpha in enumerate(alphas):
        mask = v.update_tf(alpha)
        # above 16384 levels the plain method takes the TF's runs of non-zero
        # opacity (a few for these TFs)
        v.full_recompute(alpha, out=d)
        v.full_recompute_cached(alpha, out=dc)
        torch.cuda.synchronize()
        dp, m = orc.tf_update(want, bounds, alpha, levels)
        np.testing.assert_array_equal(mask, m)
        np.testing.assert_array_equal(pdm.from_device(v.dist), dp, err_msg=f"D' tf {k}")
        np.testing.assert_array_equal(pdm.from_device(d), orc.full_recompute(vol, alpha, levels),
                                      err_msg=f"D tf {k}")
        # plain method from the cached brick ranges: occupancy of the
        # oracle's bricks under the TF, then its distance transform
        want_c = orc.dt(orc.plain_occ_range(bmin, bmax, alpha, levels))
        np.testing.assert_array_equal(pdm.from_device(dc), want_c, err_msg=f"D cached tf {k}")
    return v


def tfs(levels, count, seed, ramps=(1, 4)):
    rng = np.random.default_rng(seed)
    out = [W.trapezoid_tf(levels, int(rng.integers(ramps[0], ramps[1] + 1)), rng)
           for _ in range(count)]
    out.append(np.zeros(levels, np.float32))      # S empty
    out.append(np.ones(levels, np.float32))       # every intensity opaque
    # -0 is zero; a subnormal and a NaN are non-zero (bit-pattern test on the
    # host, IEEE comparison in the oracle)
    special = np.zeros(levels, np.float32)
    special[:levels // 3] = -0.0
    special[levels // 2] = np.float32(1e-42)
    special[-1] = np.nan
    out.append(special)
    return out


def test_config1_full(pdm, orc):
    cfg = W.config_info("c1")
    vol = W.make_volume("c1")
    alphas = W.make_tfs("c1") + tfs(256, 20, 77)
    run_all(pdm, orc, vol, 256, W.uniform_bounds(256, cfg["n"]), alphas, "c1 64^3 u8")


SHAPES = [
    # (shape zyx, dtype, levels, n, label)
    ((1, 1, 1), np.uint8, 256, 4, "single voxel"),
    ((3, 5, 7), np.uint8, 256, 8, "one partial brick per axis"),
    ((17, 9, 13), np.uint8, 256, 16, "ragged u8"),
    ((23, 18, 30), np.uint16, 4096, 32, "ragged u16 12-bit"),
    ((40, 36, 64), np.uint8, 256, 256, "one partition per level"),
    ((12, 20, 64), np.uint16, 65536, 7, "u16 full range, uneven partitions"),
    ((9, 14, 1030), np.uint8, 256, 8, "x rows over one wave segment"),
    ((6, 5, 1100), np.uint16, 4096, 5, "u16 x rows over one segment"),
    ((3, 1030, 6), np.uint8, 256, 3, "y lines over 256 bricks"),
    ((1100, 2, 3), np.uint8, 256, 2, "z lines over 256 bricks"),
    ((64, 64, 68), np.uint8, 256, 8, "x not a multiple of 16"),
    ((20, 24, 40), np.uint8, 256, 1, "one partition"),
]


@pytest.mark.parametrize("shape,dtype,levels,n,label", SHAPES, ids=[s[-1] for s in SHAPES])
def test_odd_shapes(pdm, orc, shape, dtype, levels, n, label):
    vol = blocky(shape, dtype, levels, seed=sum(shape) + n)
    bounds = W.uniform_bounds(levels, n)
    run_all(pdm, orc, vol, levels, bounds, tfs(levels, 6, sum(shape)), label)


def random_case(seed):
    """One seeded random case: shape, intensity type and levels, partition
    borders at random cut points, a piecewise-constant volume with noise."""
    rng = np.random.default_rng(10_000 + seed)
    kind = seed % 4
    spans = [(1, 9), (10, 70), (60, 300)]
    while True:
        shape = tuple(int(rng.integers(*spans[int(rng.integers(0, 3))])) for _ in range(3))
        if np.prod(shape) <= 2_500_000:
            break
    if kind in (0, 1):
        dtype, levels = np.uint8, int(rng.choice([256, 256, 100, 17]))
    else:
        dtype, levels = np.uint16, int(rng.choice([4096, 1000, 16384, 60000]))
    n = int(rng.integers(1, min(levels, 256) + 1))
    cuts = np.sort(rng.choice(np.arange(1, levels), size=n - 1, replace=False)) if n > 1 else []
    bounds = np.concatenate([[0], cuts, [levels]]).astype(np.int32)
    vol = blocky(shape, dtype, levels, seed=seed, keep=float(rng.uniform(0.02, 0.6)),
                 cell=int(rng.integers(1, 7)))
    noise = rng.integers(0, levels, size=shape)
    vol = np.where(rng.random(shape) < rng.uniform(0.0, 0.05), noise, vol).astype(dtype)
    return vol, levels, bounds


@pytest.mark.parametrize("seed", range(24))
def test_random_cases(pdm, orc, seed):
    """Seeded random shapes (1 to 300 voxels per axis), intensity types and
    level counts (u16 up to 60000 levels), partitions at random
    borders (1 to 256 of them), volumes of random density and granularity:
    bricks, every PDM, and D', D and D from the cached ranges for three
    random TFs plus the empty, all-opaque and special-value TFs; the same in
    the EXACT reading where its level limit allows."""
    vol, levels, bounds = random_case(seed)
    alphas = tfs(levels, 3, 500 + seed)
    run_all(pdm, orc, vol, levels, bounds, alphas, f"random case {seed}")
    if levels <= 16384:
        run_exact(pdm, orc, vol, levels, bounds, alphas, f"random case {seed}")


@pytest.mark.parametrize("seed", range(6))
def test_random_batches(pdm, orc, seed):
    """Seeded random batches of 3 to 12 volumes (random shapes up to 200
    voxels per axis, u8 and u16 with random level counts, 1 to 255
    partitions at random borders) built in one batched build with random
    launch knobs (grouped or single launch, alternating), then updated in one
    batched TF update: bricks, every PDM and every D' against the oracle."""
    import torch
    rng = np.random.default_rng(20_000 + seed)
    count = int(rng.integers(3, 13))
    vols, items, wants = [], [], []
    for k in range(count):
        vol, levels, bounds = random_case(100 * seed + k)
        vol = np.ascontiguousarray(vol[:200, :200, :200])  # at most 50 bricks per axis
        v = pdm.Volume(pdm.to_device(vol), levels, bounds, voxel_dtype=vol.dtype)
        vols.append((vol, v, bounds, levels))
        items.append((v.desc, v.volume, v.bmin, v.bmax, bounds, v.pdms))
    config = dict(rows_per_item=int(rng.choice([1, 2, 4])), lines_mult=int(rng.choice([1, 2, 4])),
                  largest_first=int(rng.integers(0, 2)), single_launch=seed % 2)
    ws = torch.empty(pdm.batch_workspace_bytes(count), dtype=torch.uint8, device="cuda")
    say(f"[case] random batch {seed}: {count} volumes, config {config}")
    pdm.batch_build(items, ws, config)
    torch.cuda.synchronize()
    assert pdm.batch_error(ws) == 0
    upd = []
    for k, (vol, v, bounds, levels) in enumerate(vols):
        bmin, bmax = orc.bricks(vol)
        np.testing.assert_array_equal(pdm.from_device(v.bmin, vol.dtype), bmin, err_msg=f"bmin {k}")
        np.testing.assert_array_equal(pdm.from_device(v.bmax, vol.dtype), bmax, err_msg=f"bmax {k}")
        want = orc.pdms(vol, bounds, levels, brick_minmax=(bmin, bmax))
        np.testing.assert_array_equal(pdm.from_device(v.pdms), want, err_msg=f"pdms {k}")
        alpha = W.trapezoid_tf(levels, int(rng.integers(1, 5)), rng)
        out = torch.empty(v.G, dtype=torch.uint8, device="cuda")
        upd.append((v.desc, v.pdms, bounds, alpha, out))
        wants.append(orc.tf_update(want, bounds, alpha, levels))
    masks = pdm.batch_tf_update(upd)
    torch.cuda.synchronize()
    for k, ((dp, m), it) in enumerate(zip(wants, upd)):
        np.testing.assert_array_equal(masks[k], m, err_msg=f"mask {k}")
        np.testing.assert_array_equal(pdm.from_device(it[4]).reshape(dp.shape), dp, err_msg=f"D' {k}")


def test_plain_method_full_16bit_range(pdm, orc):
    """16-bit volumes over all 65536 levels: the plain methods take the TF's
    runs of non-zero opacity (up to 512 of them) instead of the bitmap.  D and
    the cached D against the oracle for ramp TFs, a TF of exactly 512 runs
    spread over the range and one run at each end; 513 runs are refused."""
    import torch
    rng = np.random.default_rng(65536)
    L = 65536
    shape = (37, 45, 70)
    vol = blocky(shape, np.uint16, L, seed=65, keep=0.2, cell=2)
    vol = np.where(rng.random(shape) < 0.01, rng.integers(0, L, size=shape), vol).astype(np.uint16)
    bounds = W.uniform_bounds(L, 16)
    v = pdm.Volume(pdm.to_device(vol), L, bounds, voxel_dtype=np.uint16)
    v.build()
    bmin, bmax = orc.bricks(vol)
    alphas = tfs(L, 4, 66)
    many = np.zeros(L, np.float32)
    starts = np.sort(rng.choice(np.arange(0, L - 64, 64), size=pdm._lib.MAX_PLAIN_RUNS, replace=False))
    for a in starts:
        many[a:a + int(rng.integers(1, 40))] = 0.5      # runs separated by at least one zero level
    ends = np.zeros(L, np.float32)
    ends[:3] = 1.0
    ends[-2:] = 1.0
    alphas += [many, ends]
    d = torch.empty_like(v.dist)
    dc = torch.empty_like(v.dist)
    say(f"[case] plain method over 65536 levels: shape={shape}, {len(alphas)} TFs")
    for k, alpha in enumerate(alphas):
        v.full_recompute(alpha, out=d)
        v.full_recompute_cached(alpha, out=dc)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(pdm.from_device(d), orc.full_recompute(vol, alpha, L),
                                      err_msg=f"D tf {k}")
        np.testing.assert_array_equal(pdm.from_device(dc),
                                      orc.dt(orc.plain_occ_range(bmin, bmax, alpha, L)),
                                      err_msg=f"D cached tf {k}")
    too_many = many.copy()
    too_many[L - 2] = 0.5    # one more run, apart from the others (they start below L - 64)
    with pytest.raises(pdm.PdmError) as e:
        v.full_recompute(too_many, out=d)
    assert e.value.code == pdm._lib.PDM_E_UNSUPPORTED


def test_capped_lines_closed_form(pdm, orc):
    """A single occupied brick at one end of 1x1xN and Nx1x1 grids: the
    distance along the line is min(k, 255)."""
    import torch
    for shape in ((1, 1, 4 * 300), (4 * 300, 1, 1), (1, 4 * 300, 1)):
        say(f"[case] capped line {shape}")
        vol = np.zeros(shape, np.uint8)
        vol.reshape(-1)[0] = 200
        v = pdm.Volume(pdm.to_device(vol), 256, W.uniform_bounds(256, 2))
        v.build()
        alpha = np.zeros(256, np.float32)
        alpha[200] = 1.0
        v.update_tf(alpha)
        d = torch.empty_like(v.dist)
        v.full_recompute(alpha, out=d)
        torch.cuda.synchronize()
        want = np.minimum(np.arange(300), 255).astype(np.uint8)
        # partition 1 holds only the first brick; partition 0 holds every brick
        np.testing.assert_array_equal(pdm.from_device(v.pdms[1]).reshape(-1), want)
        assert (pdm.from_device(v.pdms[0]) == 0).all()
        np.testing.assert_array_equal(pdm.from_device(d).reshape(-1), want)
        # alpha non-zero only at 200: S = {1}, and D' = D
        np.testing.assert_array_equal(pdm.from_device(v.dist).reshape(-1), want)


def test_all_maps_long_lines_in_chunks(pdm, orc):
    """The all-maps y pass with lines of 200 bricks and 2^20 of them (256
    partitions of a 64x200x64 grid) takes the global-memory scan with 32-step
    chunks and a ragged last chunk (200 = 6*32 + 8); its z pass (64-brick
    lines) takes 16-step chunks.  Sampled PDMs against the oracle, and D' for
    three TFs against the oracle's plain method: with one partition per level
    the two are equal (Sec. 3.1)."""
    import torch
    vol = blocky((256, 800, 256), np.uint8, 256, seed=11, keep=0.02, cell=5)
    n = 256
    bounds = W.uniform_bounds(256, n)
    say(f"[case] all maps, 200-brick y lines: shape={vol.shape} n={n}")
    v = pdm.Volume(pdm.to_device(vol), 256, bounds)
    v.build()
    torch.cuda.synchronize()
    bmin, bmax = orc.bricks(vol)
    for p in (0, 1, 37, 128, 200, 255):
        want = orc.dt(orc.pom_range(bmin, bmax, int(bounds[p]), int(bounds[p + 1]) - 1))
        np.testing.assert_array_equal(pdm.from_device(v.pdms[p]), want, err_msg=f"PDM {p}")
    for k, alpha in enumerate(tfs(256, 3, 12)[:3]):
        v.update_tf(alpha)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(pdm.from_device(v.dist), orc.full_recompute(vol, alpha, 256),
                                      err_msg=f"D' tf {k}")


MANY_LINE_SHAPES = [
    # (voxel shape zyx, dtype, levels, n, label): all-partition y/z passes of
    # more than 2^18 lines of at most 256 bricks (the register-resident scan)
    ((244, 240, 180), np.uint8, 256, 100,
     "61x60x45 grid: tiles straddle rows and maps, partial last tiles"),
    ((160, 1024, 132), np.uint16, 4096, 256, "40x256x33 grid: 256-brick y lines, u16"),
    ((68, 66, 4000), np.uint8, 256, 32, "17x17x1000 grid: lines of 17 (one full chunk + 1)"),
    ((80, 1020, 256), np.uint8, 256, 256, "20x255x64 grid: 255-brick y lines, 256 partitions"),
    # the longest lines whose values are clamped to the line length (a table
    # of 255 rows); z lines of 20, most of them with every value above 20
    ((80, 1016, 256), np.uint8, 256, 256, "20x254x64 grid: 254-brick y lines, clamped"),
    ((8, 400, 1024), np.uint8, 256, 64, "2x100x256 grid: 2-brick z lines"),
]


@pytest.mark.parametrize("shape,dtype,levels,n,label", MANY_LINE_SHAPES,
                         ids=[s[-1].split(":")[0] for s in MANY_LINE_SHAPES])
def test_many_line_scans(pdm, orc, shape, dtype, levels, n, label):
    """Every PDM against the oracle where the y and z passes over all maps
    cover more than 2^18 lines of at most 256 bricks: ragged x (tiles of 64
    lines that cross rows and maps, lanes past the last line), line lengths
    at chunk borders, sparse occupancy (whole tiles at the cap) and dense."""
    import torch
    vol = blocky(shape, dtype, levels, seed=sum(shape) + n, keep=0.03, cell=4)
    # no voxel in the top quarter of the levels: those partitions' maps are
    # 255 everywhere, so whole tiles of their lines stay at the cap
    vol = (vol % (levels * 3 // 4)).astype(dtype)
    bounds = W.uniform_bounds(levels, n)
    v = pdm.Volume(pdm.to_device(vol), levels, bounds, voxel_dtype=dtype)
    say(f"[case] many-line scans {label}: shape={vol.shape} grid={(v.bz, v.by, v.bx)} n={n}")
    assert max(v.bx * v.bz, v.bx * v.by) * n > 4 * 1024 * 64
    v.build()
    torch.cuda.synchronize()
    bmin, bmax = orc.bricks(vol)
    want = orc.pdms(vol, bounds, levels, brick_minmax=(bmin, bmax))
    got = pdm.from_device(v.pdms)
    assert (want == 255).any() and (want == 0).any() and ((want > 0) & (want < 255)).any()
    for p in range(n):
        np.testing.assert_array_equal(got[p], want[p], err_msg=f"PDM {p}")


FEW_LINE_SHAPES = [
    # (voxel shape zyx, dtype, levels, n, label): y/z passes over few lines
    # (one map, or a few) of 17 to 256 bricks: two lanes per line
    ((132, 68, 180), np.uint8, 256, 4, "33x17x45 grid: lines of 17 and 33"),
    ((400, 1020, 148), np.uint8, 256, 3, "100x255x37 grid: lines of 255 and 100"),
    ((1024, 256, 80), np.uint16, 4096, 2, "256x64x20 grid: z lines of 256, u16"),
    ((516, 964, 36), np.uint8, 256, 5, "129x241x9 grid: lines of 241 and 129"),
    ((800, 192, 256), np.uint8, 256, 4, "200x48x64 grid: lines of 48 and 200"),
    # rows of 32 and 64 bricks: the tile passes through LDS slots
    ((128, 400, 128), np.uint8, 256, 3, "32x100x32 grid: LDS slots, lines of 100 and 32"),
    ((68, 68, 256), np.uint8, 256, 3, "17x17x64 grid: LDS slots, lines of 17"),
]


@pytest.mark.parametrize("shape,dtype,levels,n,label", FEW_LINE_SHAPES,
                         ids=[s[-1].split(":")[0] for s in FEW_LINE_SHAPES])
def test_few_line_scans(pdm, orc, shape, dtype, levels, n, label):
    """Passes over few lines of 17..256 bricks (a handful of PDMs, the plain
    method's one map and the cached-range one): every PDM, D' and both D
    against the oracle for a few TFs, with ragged line counts (the last pair
    tile partly past the last line) and an empty partition."""
    import torch
    vol = blocky(shape, dtype, levels, seed=sum(shape) + 7 * n, keep=0.02, cell=5)
    vol = (vol % (levels * 3 // 4)).astype(dtype)  # the top partition stays empty
    bounds = W.uniform_bounds(levels, n)
    say(f"[case] few-line scans {label}: shape={vol.shape} n={n}")
    run_all(pdm, orc, vol, levels, bounds, tfs(levels, 4, sum(shape)), label)


MAX_SHAPES = [
    # (shape zyx, dtype, levels, n, label): grids at the ABI's axis limits
    ((3, 5, 4 * 16384), np.uint8, 256, 16, "x at the limit: 16384 bricks, 64 wave segments"),
    ((4, 4 * 65535 - 2, 4), np.uint8, 256, 8, "y at the limit: 65535-brick lines"),
    ((4 * 65535 - 1, 3, 5), np.uint16, 4096, 4, "z at the limit: 65535-brick lines, u16"),
]


@pytest.mark.parametrize("shape,dtype,levels,n,label", MAX_SHAPES, ids=[s[-1] for s in MAX_SHAPES])
def test_grid_axis_limits(pdm, orc, shape, dtype, levels, n, label):
    """Every output at the largest grid axis the library accepts (16384 bricks
    along x, 65535 along y or z; one more is rejected, see the host tests):
    the segmented x pass at its 64-segment maximum, and y/z lines whose
    positions need the 16-bit scan table up to its last entry."""
    vol = blocky(shape, dtype, levels, seed=sum(shape) + n, keep=0.05, cell=7)
    run_all(pdm, orc, vol, levels, W.uniform_bounds(levels, n), tfs(levels, 3, 21), label)


def test_rhomin_partition(pdm, orc):
    vol = W.make_volume("c1")
    bounds = W.rhomin_bounds(256, 16, 2)
    run_all(pdm, orc, vol, 256, bounds, tfs(256, 8, 5), "rho_min partition")


@pytest.mark.parametrize("n", [16, 128, 256])
@pytest.mark.parametrize("kind", ["uniform", "rho_min"])
def test_partition_sweep_stag_beetle(pdm, orc, n, kind):
    """The partition sweep's corners on a small stag-beetle-shaped volume
    (background exactly at rho_min = 0): n from 16 to one partition per
    level, uniform or with the rho_min partition [0, 0]."""
    vol = W.stag_beetle_u8((62, 104, 104))
    bounds = W.uniform_bounds(256, n) if kind == "uniform" else W.rhomin_bounds(256, n, 0)
    alphas = tfs(256, 4, n)
    low = np.zeros(256, np.float32)
    low[1:40] = 0.5      # low intensities without rho_min itself
    alphas.append(low)
    run_all(pdm, orc, vol, 256, bounds, alphas, f"stag sweep {kind} n={n}")


RANGE_CASES = [((64, 64, 64), np.uint8, 256, 8), ((23, 18, 30), np.uint16, 4096, 32),
               ((40, 36, 64), np.uint8, 256, 256), ((17, 9, 13), np.uint8, 256, 19)]


@pytest.mark.parametrize("max_level", [1, 3, 8])
@pytest.mark.parametrize("shape,dtype,levels,n", RANGE_CASES,
                         ids=["c1-like", "ragged-u16", "256-partitions", "odd-n"])
def test_range_table_update(pdm, orc, shape, dtype, levels, n, max_level):
    """Range-table maps against the oracle's definition, and the TF update
    through the table against the oracle's D' (and the plain update): TFs
    with ramps, scattered opacities (many runs of S), none and all."""
    import torch
    vol = blocky(shape, dtype, levels, seed=sum(shape) + n + max_level)
    bounds = W.uniform_bounds(levels, n)
    say(f"[case] range table {shape} {np.dtype(dtype).name} n={n} max_level={max_level}")
    v = pdm.Volume(pdm.to_device(vol), levels, bounds, voxel_dtype=dtype)
    v.build()
    v.build_range_table(max_level)
    torch.cuda.synchronize()
    want_pd = orc.pdms(vol, bounds, levels)
    np.testing.assert_array_equal(pdm.from_device(v.pdms), want_pd)
    table = orc.range_table(want_pd, max_level)
    if len(table):
        np.testing.assert_array_equal(pdm.from_device(v.table).reshape(table.shape), table)
    else:
        assert v.table is None
    rng = np.random.default_rng(n)
    alphas = tfs(levels, 5, n + 1)
    for _ in range(6):
        a = np.zeros(levels, np.float32)
        a[rng.choice(levels, size=int(rng.integers(1, 40)), replace=False)] = 1.0
        alphas.append(a)
    plain = torch.empty_like(v.dist)
    for k, alpha in enumerate(alphas):
        m = v.update_tf_ranges(alpha)
        m2 = v.update_tf(alpha, out=plain)
        torch.cuda.synchronize()
        dp, want_m = orc.tf_update(want_pd, bounds, alpha, levels)
        np.testing.assert_array_equal(m, want_m)
        np.testing.assert_array_equal(m2, want_m)
        np.testing.assert_array_equal(pdm.from_device(v.dist), dp, err_msg=f"D' via table, tf {k}")
        assert torch.equal(v.dist.reshape(-1), plain.reshape(-1))


def test_range_table_exact_mode(pdm, orc):
    """The union property holds for the EXACT reading too (a voxel lies in
    the union of intervals when it lies in one of them): the table over
    EXACT PDMs gives the EXACT D'."""
    import torch
    vol = blocky((30, 26, 44), np.uint8, 256, seed=5)
    bounds = W.uniform_bounds(256, 16)
    say("[case] range table, EXACT reading")
    v = pdm.Volume(pdm.to_device(vol), 256, bounds, mode=pdm.EXACT)
    v.build()
    v.build_range_table(8)
    torch.cuda.synchronize()
    want = orc.pdms(vol, bounds, 256, mode=orc.EXACT)
    np.testing.assert_array_equal(pdm.from_device(v.pdms), want)
    table = orc.range_table(want, 8)
    np.testing.assert_array_equal(pdm.from_device(v.table).reshape(table.shape), table)
    for k, alpha in enumerate(tfs(256, 6, 3)):
        m = v.update_tf_ranges(alpha)
        torch.cuda.synchronize()
        dp, wm = orc.tf_update(want, bounds, alpha, 256)
        np.testing.assert_array_equal(m, wm)
        np.testing.assert_array_equal(pdm.from_device(v.dist), dp, err_msg=f"tf {k}")


def test_deterministic_and_no_out_of_bounds_writes(pdm, orc):
    """Outputs written into the middle of guarded buffers: guard bytes stay
    untouched and two runs give identical bytes."""
    import torch
    vol = blocky((37, 29, 45), np.uint8, 256, seed=9)
    bounds = W.uniform_bounds(256, 8)
    desc = pdm.volume_desc(vol.shape, np.uint8, 256)
    bz, by, bx, G = pdm.grid_of(desc)
    n = 8
    guard = 4096
    dvol = pdm.to_device(vol)

    def guarded(nbytes):
        t = torch.full((nbytes + 2 * guard,), 0xA5, dtype=torch.uint8, device="cuda")
        return t, t[guard:guard + nbytes]

    outs = []
    for rep in range(2):
        say(f"[case] guarded run {rep}")
        gmin, bmin = guarded(G)
        gmax, bmax = guarded(G)
        gp, pd = guarded(n * G)
        gd, dist = guarded(G)
        gf, full = guarded(G)
        pdm.build_bricks(desc, dvol, bmin, bmax)
        pdm.build_partitions(desc, bmin, bmax, bounds, pd)
        alpha = W.make_tfs("c1")[0]
        pdm.tf_update(desc, pd, bounds, alpha, dist)
        pdm.full_recompute(desc, dvol, alpha, full)
        torch.cuda.synchronize()
        for g in (gmin, gmax, gp, gd, gf):
            h = g.cpu().numpy()
            assert (h[:guard] == 0xA5).all() and (h[-guard:] == 0xA5).all()
        outs.append([t.cpu().numpy().copy() for t in (bmin, bmax, pd, dist, full)])
    for a, b in zip(*outs):
        np.testing.assert_array_equal(a, b)


def test_range_error_flag(pdm, orc):
    import torch
    vol = np.full((8, 8, 8), 100, np.uint16)
    v = pdm.Volume(pdm.to_device(vol), 4096, W.uniform_bounds(4096, 4), voxel_dtype=np.uint16)
    v.build()
    v.check_range()                                  # clean volume: no error
    vol[3, 5, 7] = 5000
    v2 = pdm.Volume(pdm.to_device(vol), 4096, W.uniform_bounds(4096, 4), voxel_dtype=np.uint16)
    v2.build()
    torch.cuda.synchronize()
    with pytest.raises(pdm.PdmError):
        v2.check_range()


def test_invalid_arguments_raise(pdm):
    import torch
    vol = torch.zeros((8, 8, 8), dtype=torch.uint8, device="cuda")
    with pytest.raises(pdm.PdmError):
        pdm.Volume(vol, 256, [0, 100, 100, 256]).build()
    v = pdm.Volume(vol, 256, W.uniform_bounds(256, 4))
    with pytest.raises(ValueError):
        v.update_tf(np.zeros(100, np.float32))
    with pytest.raises(ValueError):
        pdm.tf_update(v.desc, v.pdms[:2], v.bounds, np.zeros(256, np.float32), v.dist)


# ------------------------------------------------------- EXACT occupancy
def run_exact(pdm, orc, vol, levels, bounds, alphas, label):
    import torch
    say(f"[case] EXACT {label}: shape={vol.shape} dtype={vol.dtype} L={levels} n={len(bounds) - 1}")
    v = pdm.Volume(pdm.to_device(vol), levels, bounds, voxel_dtype=vol.dtype, mode=pdm.EXACT)
    v.build()
    torch.cuda.synchronize()
    want = orc.pdms(vol, bounds, levels, mode=orc.EXACT)
    np.testing.assert_array_equal(pdm.from_device(v.pdms), want)
    d = torch.empty_like(v.dist)
    for k, alpha in enumerate(alphas):
        mask = v.update_tf(alpha)
        v.full_recompute(alpha, out=d)
        torch.cuda.synchronize()
        dp, m = orc.tf_update(want, bounds, alpha, levels)
        np.testing.assert_array_equal(mask, m)
        np.testing.assert_array_equal(pdm.from_device(v.dist), dp, err_msg=f"D' tf {k}")
        np.testing.assert_array_equal(pdm.from_device(d),
                                      orc.full_recompute(vol, alpha, levels, mode=orc.EXACT),
                                      err_msg=f"D tf {k}")


EXACT_SHAPES = [
    ((1, 1, 1), np.uint8, 256, 4, "single voxel"),
    ((17, 9, 13), np.uint8, 256, 16, "ragged u8"),
    ((23, 18, 30), np.uint16, 4096, 32, "ragged u16 12-bit"),
    ((40, 36, 64), np.uint8, 256, 256, "one partition per level"),
    ((20, 24, 40), np.uint16, 4096, 100, "u16, 100 partitions"),
    ((9, 14, 1024), np.uint8, 256, 64, "x rows of 256 bricks"),
    ((3, 1030, 6), np.uint8, 256, 3, "y lines over 256 bricks"),
    ((64, 64, 68), np.uint8, 256, 8, "x not a multiple of 16"),
    # rows of 33-128 bricks packed 16 or 32 lanes per row, with a row count
    # (By*Bz) that is not a multiple of the rows per wave
    ((9, 11, 200), np.uint8, 256, 16, "50-brick rows, 16 lanes per row, u8"),
    ((10, 11, 198), np.uint16, 4096, 32, "50-brick rows, 16 lanes per row, u16"),
    ((17, 9, 500), np.uint8, 256, 32, "125-brick rows, 32 lanes per row, u8"),
    ((19, 10, 503), np.uint16, 4096, 64, "126-brick rows, 32 lanes per row, u16"),
]


@pytest.mark.parametrize("shape,dtype,levels,n,label", EXACT_SHAPES, ids=[s[-1] for s in EXACT_SHAPES])
def test_exact_shapes(pdm, orc, shape, dtype, levels, n, label):
    # noisier than `blocky`: bricks mix several intensities, so EXACT and
    # RANGE occupancy differ
    rng = np.random.default_rng(sum(shape) + n)
    vol = blocky(shape, dtype, levels, seed=sum(shape) + n)
    noise = rng.integers(0, levels, size=shape).astype(dtype)
    vol = np.where(rng.random(shape) < 0.05, noise, vol).astype(dtype)
    run_exact(pdm, orc, vol, levels, W.uniform_bounds(levels, n), tfs(levels, 5, sum(shape)), label)


def test_exact_config1_and_rhomin(pdm, orc):
    vol = W.make_volume("c1")
    run_exact(pdm, orc, vol, 256, W.uniform_bounds(256, 8), W.make_tfs("c1") + tfs(256, 10, 3), "c1")
    run_exact(pdm, orc, vol, 256, W.rhomin_bounds(256, 16, 2), tfs(256, 4, 4), "c1 rho_min")


def test_exact_within_range(pdm, orc):
    """EXACT occupancy is contained in RANGE occupancy, so EXACT distances are
    element-wise >= RANGE distances, for PDMs and for D."""
    import torch
    vol = W.make_volume("c1")
    bounds = W.uniform_bounds(256, 8)
    vr = pdm.Volume(pdm.to_device(vol), 256, bounds)
    ve = pdm.Volume(pdm.to_device(vol), 256, bounds, mode=pdm.EXACT)
    vr.build()
    ve.build()
    torch.cuda.synchronize()
    assert bool((ve.pdms >= vr.pdms).all().item())
    alpha = W.make_tfs("c1")[0]
    vr.full_recompute(alpha)
    ve.full_recompute(alpha)
    torch.cuda.synchronize()
    assert bool((ve.dist >= vr.dist).all().item())


# ----------------------------------------------------- batched TF update
def test_batch_tf_update_matches_oracle(pdm, orc):
    """Volumes of mixed dtypes, sizes (ragged, G not a multiple of 16),
    partition counts and TFs updated in one launch; every D' against the
    oracle, and against the single-volume call."""
    import torch
    rng = np.random.default_rng(31)
    specs = [((37, 29, 45), np.uint8, 256, 16), ((20, 24, 64), np.uint16, 4096, 32),
             ((9, 14, 30), np.uint8, 256, 64), ((64, 64, 64), np.uint8, 256, 8),
             ((5, 6, 7), np.uint16, 4096, 3), ((30, 30, 30), np.uint8, 256, 256)]
    vols, items, wants = [], [], []
    for k, (shape, dtype, L, n) in enumerate(specs):
        vol = blocky(shape, dtype, L, seed=100 + k)
        bounds = W.uniform_bounds(L, n)
        v = pdm.Volume(pdm.to_device(vol), L, bounds, voxel_dtype=dtype)
        v.build()
        alpha = W.trapezoid_tf(L, int(rng.integers(1, 4)), rng) if k != 4 else np.zeros(L, np.float32)
        # an odd offset into a larger buffer: unaligned chunks
        out = torch.full((v.G + 3,), 7, dtype=torch.uint8, device="cuda")[1:1 + v.G] if k == 2 \
            else torch.empty(v.G, dtype=torch.uint8, device="cuda")
        vols.append((v, out))
        items.append((v.desc, v.pdms, bounds, alpha, out))
        want_pd = orc.pdms(vol, bounds, L)
        wants.append(orc.tf_update(want_pd, bounds, alpha, L))
    say("[case] batch of 6 volumes")
    masks = pdm.batch_tf_update(items)
    torch.cuda.synchronize()
    for k, ((v, out), (dp, m)) in enumerate(zip(vols, wants)):
        np.testing.assert_array_equal(masks[k], m, err_msg=f"mask {k}")
        np.testing.assert_array_equal(pdm.from_device(out).reshape(dp.shape), dp, err_msg=f"D' {k}")
        single = torch.empty_like(v.dist)
        pdm.tf_update(v.desc, v.pdms, v.bounds, items[k][3], single)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(pdm.from_device(single).reshape(-1), pdm.from_device(out))
    # the prepared-volume path gives the same masks and maps
    outs2 = [torch.empty(v.G, dtype=torch.uint8, device="cuda") for v, _ in vols]
    masks2 = pdm.batch_tf_update_prepared(
        [(v.prepared, it[3], o) for (v, _), it, o in zip(vols, items, outs2)])
    torch.cuda.synchronize()
    np.testing.assert_array_equal(masks2, masks)
    for (v, out), o in zip(vols, outs2):
        assert torch.equal(o, out)


def _at_offset(t, off):
    """A copy of the uint8 device tensor `t` that starts `off` bytes into a
    larger buffer (a contiguous tensor whose base is not 16-byte aligned)."""
    import torch
    flat = t.reshape(-1)
    buf = torch.full((flat.numel() + off + 5,), 77, dtype=torch.uint8, device=t.device)
    view = buf[off:off + flat.numel()]
    view.copy_(flat)
    return buf, view


# G = 1, 15, 16, 17, 62 and 924 bricks (the chunk-per-lane path with its
# overlapping last chunk, and the byte path below 16 bricks)
COMBINE_SHAPES = [(1, 1, 1), (4, 4, 60), (4, 4, 64), (4, 4, 68), (4, 8, 124), (43, 27, 45)]


def test_combine_any_size_and_alignment(pdm, orc):
    """Every combine path (single update, update through range tables, range
    table levels, batched update) at sizes around the 16-byte chunk and with
    PDMs, tables and outputs at odd byte offsets, against the oracle."""
    import torch
    rng = np.random.default_rng(71)
    L, n, K = 256, 12, 3
    bounds = W.uniform_bounds(L, n)
    batch, wants = [], []
    for k, shape in enumerate(COMBINE_SHAPES):
        vol = blocky(shape, np.uint8, L, seed=300 + k, keep=0.4, cell=1)
        v = pdm.Volume(pdm.to_device(vol), L, bounds)
        v.build()
        G = v.G
        pd_stack = orc.pdms(vol, bounds, L)
        np.testing.assert_array_equal(pdm.from_device(v.pdms).reshape(pd_stack.shape), pd_stack)
        _, pdms_odd = _at_offset(v.pdms, 3 + k)
        maps = pdm.range_table_maps(n, K)
        tbuf = torch.full((maps * G + 7 + k,), 9, dtype=torch.uint8, device="cuda")
        table = tbuf[1 + k:1 + k + maps * G]
        say(f"[case] combine G={G} shape={shape}")
        pdm.build_range_table(v.desc, pdms_odd, n, K, table)
        want_table = orc.range_table(pd_stack, K)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(pdm.from_device(table).reshape(want_table.shape), want_table,
                                      err_msg=f"range table G={G}")
        for j in range(3):
            alpha = W.trapezoid_tf(L, int(rng.integers(1, 4)), rng)
            if j == 2:
                alpha = np.zeros(L, np.float32)   # empty S: 255 everywhere
            want, wm = orc.tf_update(pd_stack, bounds, alpha, L)
            obuf = torch.full((G + 9,), 5, dtype=torch.uint8, device="cuda")
            out = obuf[1 + j + k % 3:1 + j + k % 3 + G]
            m = pdm.tf_update(v.desc, pdms_odd, bounds, alpha, out)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(m, wm)
            np.testing.assert_array_equal(pdm.from_device(out).reshape(want.shape), want,
                                          err_msg=f"tf_update G={G} tf {j}")
            out.fill_(3)
            pdm.tf_update_ranges(v.desc, pdms_odd, table, bounds, K, alpha, out)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(pdm.from_device(out).reshape(want.shape), want,
                                          err_msg=f"tf_update_ranges G={G} tf {j}")
            # bytes around the output untouched
            lo = 1 + j + k % 3
            assert int(obuf[:lo].min()) == 5 and int(obuf[lo + G:].max()) == 5
        alpha = W.trapezoid_tf(L, 2, rng)
        ob, out = _at_offset(torch.zeros(G, dtype=torch.uint8, device="cuda"), 1 + 2 * k)
        batch.append((v, pdms_odd, alpha, out))
        wants.append(orc.tf_update(pd_stack, bounds, alpha, L))
    say("[case] batched combine over all sizes at odd offsets")
    masks = pdm.batch_tf_update([(v.desc, p, bounds, a, o) for v, p, a, o in batch])
    torch.cuda.synchronize()
    for k, ((v, _, _, out), (want, wm)) in enumerate(zip(batch, wants)):
        np.testing.assert_array_equal(masks[k], wm)
        np.testing.assert_array_equal(pdm.from_device(out).reshape(want.shape), want,
                                      err_msg=f"batched G={v.G}")


def test_combine_wide_ragged_unaligned(pdm, orc):
    """The two-chunks-per-lane combine (maps of 8 MiB and more) at a size that
    is not a multiple of 16 (G = 203*203*205 = 8,447,845) with the PDMs, the
    range table and the output at odd byte offsets; the maps are random bytes
    (the combine takes any maps), D' against the oracle's Eq. 1."""
    import torch
    from paper_2407_21552_amd import _lib
    rng = np.random.default_rng(88)
    L, n, K = 256, 16, 2
    desc = _lib.VolumeDesc(nx=812, ny=812, nz=820, dtype=1, levels=L, brick=4)
    G = pdm.grid_of(desc)[3]
    assert G == 203 * 203 * 205 and G % 16 == 5
    stack = rng.integers(0, 256, size=(n, G), dtype=np.uint8)
    _, pdms = _at_offset(pdm.to_device(stack), 7)
    maps = pdm.range_table_maps(n, K)
    tbuf = torch.empty(maps * G + 16, dtype=torch.uint8, device="cuda")
    table = tbuf[3:3 + maps * G]
    bounds = W.uniform_bounds(L, n)
    say(f"[case] wide combine G={G}")
    pdm.build_range_table(desc, pdms, n, K, table)
    want_table = orc.range_table(stack, K)
    torch.cuda.synchronize()
    assert torch.equal(table.cpu(), torch.from_numpy(want_table.reshape(-1)))
    del want_table
    obuf = torch.full((G + 20,), 5, dtype=torch.uint8, device="cuda")
    out = obuf[9:9 + G]
    for j in range(4):
        alpha = W.trapezoid_tf(L, j + 1, rng) if j < 3 else np.ones(L, np.float32)
        want, wm = orc.tf_update(stack, bounds, alpha, L)
        out.fill_(1)
        m = pdm.tf_update(desc, pdms, bounds, alpha, out)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(m, wm)
        assert torch.equal(out.cpu(), torch.from_numpy(want.reshape(-1))), f"tf_update tf {j}"
        out.fill_(2)
        pdm.tf_update_ranges(desc, pdms, table, bounds, K, alpha, out)
        torch.cuda.synchronize()
        assert torch.equal(out.cpu(), torch.from_numpy(want.reshape(-1))), f"ranges tf {j}"
        assert int(obuf[:9].min()) == 5 and int(obuf[9 + G:].max()) == 5


def test_batch_range_update(pdm, orc):
    """Updates through range tables of many requests in one call: volumes of
    sizes around the 16-byte chunk (and below it), u8 and u16, different n
    and max_level, PDMs, tables and outputs at odd byte offsets, an empty S;
    then a batch whose covers exceed one launch's map list (256 partitions
    with every other one active: covers of 128 maps, six requests), which the
    call splits.  Every D' and S mask against the oracle and the single
    call."""
    import torch
    rng = np.random.default_rng(77)
    cases = [(shape, np.uint8, 256, 12, 3) for shape in COMBINE_SHAPES] + \
            [((20, 24, 64), np.uint16, 4096, 32, 4), ((30, 30, 30), np.uint8, 256, 64, 0)]
    vols, items, wants = [], [], []
    for k, (shape, dtype, L, n, K) in enumerate(cases):
        vol = blocky(shape, dtype, L, seed=500 + k, keep=0.4, cell=1)
        bounds = W.uniform_bounds(L, n)
        v = pdm.Volume(pdm.to_device(vol), L, bounds, voxel_dtype=dtype)
        v.build()
        G = v.G
        pd_stack = orc.pdms(vol, bounds, L)
        _, pdms = _at_offset(v.pdms, 1 + k)
        maps = pdm.range_table_maps(n, K)
        table = None
        if maps:
            tbuf = torch.empty(maps * G + 8, dtype=torch.uint8, device="cuda")
            table = tbuf[3:3 + maps * G]
            pdm.build_range_table(v.desc, pdms, n, K, table)
        alpha = np.zeros(L, np.float32) if k == 2 else W.trapezoid_tf(L, int(rng.integers(1, 5)), rng)
        _, out = _at_offset(torch.zeros(G, dtype=torch.uint8, device="cuda"), 2 + k)
        vols.append((v, pdms, table, n, K, out))
        items.append((v.desc, pdms, table, bounds, K, alpha, out))
        wants.append(orc.tf_update(pd_stack, bounds, alpha, L))
    say(f"[case] batched range-table update, {len(items)} requests")
    masks = pdm.batch_tf_update_ranges(items)
    torch.cuda.synchronize()
    for k, ((v, pdms, table, n, K, out), (want, wm), it) in enumerate(zip(vols, wants, items)):
        np.testing.assert_array_equal(masks[k], wm, err_msg=f"mask {k}")
        np.testing.assert_array_equal(pdm.from_device(out).reshape(want.shape), want, err_msg=f"D' {k}")
        single = torch.empty(v.G, dtype=torch.uint8, device="cuda")
        pdm.tf_update_ranges(v.desc, pdms, table, it[3], K, it[5], single)
        torch.cuda.synchronize()
        assert torch.equal(single, out), f"single call {k}"
    # covers longer than one launch's map list: the call splits the batch
    shape, L, n, K = (37, 29, 45), 256, 256, 4
    vol = blocky(shape, np.uint8, L, seed=600, keep=0.6, cell=1)
    bounds = W.uniform_bounds(L, n)
    v = pdm.Volume(pdm.to_device(vol), L, bounds)
    v.build()
    pd_stack = orc.pdms(vol, bounds, L)
    table = torch.empty(pdm.range_table_maps(n, K) * v.G, dtype=torch.uint8, device="cuda")
    pdm.build_range_table(v.desc, v.pdms, n, K, table)
    items, wants = [], []
    for j in range(6):
        alpha = np.zeros(L, np.float32)
        alpha[j % 2::2] = 0.5                     # every other partition: 128 runs of one
        if j == 5:
            alpha[100:180] = 1.0                  # one long run among them
        out = torch.empty(v.G, dtype=torch.uint8, device="cuda")
        items.append((v.desc, v.pdms, table, bounds, K, alpha, out))
        wants.append(orc.tf_update(pd_stack, bounds, alpha, L))
    covers = [len(pdm.range_cover(n, K, w[1])) for w in wants]
    assert sum(covers) > 640 and max(covers) == 128
    say(f"[case] batched range-table update over two launches, covers {covers}")
    masks = pdm.batch_tf_update_ranges(items)
    torch.cuda.synchronize()
    for k, (it, (want, wm)) in enumerate(zip(items, wants)):
        np.testing.assert_array_equal(masks[k], wm)
        np.testing.assert_array_equal(pdm.from_device(it[6]).reshape(want.shape), want,
                                      err_msg=f"split batch D' {k}")


# ------------------------------------------------------ batched build
@pytest.mark.parametrize("config", [None, dict(rows_per_item=1, lines_mult=4, largest_first=1),
                                    dict(rows_per_item=7, lines_mult=1),
                                    dict(rows_per_item=256, lines_mult=16, largest_first=1),
                                    dict(single_launch=1),
                                    dict(single_launch=1, rows_per_item=1, lines_mult=2,
                                         largest_first=1)],
                         ids=["default", "one-row-long-chunks", "seven-rows", "whole-slices",
                              "single-launch", "single-launch-one-row"])
def test_batch_build_matches_single_volume_and_oracle(pdm, orc, config):
    """Bricks and PDMs of volumes of mixed dtypes, ragged sizes and partition
    counts, including grid axes of 1 and of the 256-brick maximum, built by
    the three grouped launches or by the single cooperative launch; each
    against the oracle and the single-volume calls."""
    import torch
    specs = [((37, 29, 45), np.uint8, 256, 16), ((20, 24, 64), np.uint16, 4096, 32),
             ((9, 14, 30), np.uint8, 256, 64), ((64, 64, 64), np.uint8, 256, 8),
             ((5, 6, 7), np.uint16, 4096, 3), ((1, 1, 1), np.uint8, 256, 2),
             ((30, 31, 33), np.uint8, 256, 200), ((3, 9, 1021), np.uint8, 256, 5),
             ((1021, 5, 6), np.uint16, 4096, 4)]
    vols, items = [], []
    for k, (shape, dtype, L, n) in enumerate(specs):
        vol = blocky(shape, dtype, L, seed=200 + k)
        bounds = W.uniform_bounds(L, n)
        v = pdm.Volume(pdm.to_device(vol), L, bounds, voxel_dtype=dtype)
        vols.append((vol, v, bounds, L))
        items.append((v.desc, v.volume, v.bmin, v.bmax, bounds, v.pdms))
    ws = torch.empty(pdm.batch_workspace_bytes(len(items)), dtype=torch.uint8, device="cuda")
    say(f"[case] batch build of {len(items)} volumes, config {config}")
    pdm.batch_build(items, ws, config)
    torch.cuda.synchronize()
    assert pdm.batch_error(ws) == 0
    for k, (vol, v, bounds, L) in enumerate(vols):
        bmin, bmax = orc.bricks(vol)
        np.testing.assert_array_equal(pdm.from_device(v.bmin, vol.dtype), bmin, err_msg=f"bmin {k}")
        np.testing.assert_array_equal(pdm.from_device(v.bmax, vol.dtype), bmax, err_msg=f"bmax {k}")
        np.testing.assert_array_equal(pdm.from_device(v.pdms), orc.pdms(vol, bounds, L),
                                      err_msg=f"pdms {k}")
        single = pdm.Volume(v.volume, L, bounds, voxel_dtype=vol.dtype)
        single.build()
        torch.cuda.synchronize()
        assert torch.equal(single.pdms, v.pdms) and torch.equal(single.bmax, v.bmax), k
