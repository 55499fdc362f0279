"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Nothing here re-types the oracle's own formulas: every check comes from an
independent route (brute force on tiny grids, scipy's chessboard transform,
closed forms, numpy reshapes, the paper's Fig. 2 example and its stated
properties D' <= D and D' = D when no partition is split; Sec. 3.1).
"""
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st
from scipy import ndimage

import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------- helpers
def brute_dt(occ: np.ndarray, cap: int = 255) -> np.ndarray:
    """Nearest occupied brick by exhaustive search, L-infinity, clamped."""
    occ = occ.astype(bool)
    pts = np.argwhere(occ)
    out = np.full(occ.shape, cap, np.int64)
    if len(pts) == 0:
        return out.astype(np.uint8)
    allc = np.argwhere(np.ones(occ.shape, bool))
    best = np.full(len(allc), 1 << 30, np.int64)
    for s in range(0, len(pts), 512):
        d = np.abs(allc[:, None, :] - pts[None, s:s + 512, :]).max(axis=2)
        best = np.minimum(best, d.min(axis=1))
    return np.minimum(best, cap).reshape(occ.shape).astype(np.uint8)


def scipy_dt(occ: np.ndarray) -> np.ndarray:
    if not occ.any():
        return np.full(occ.shape, 255, np.uint8)
    d = ndimage.distance_transform_cdt((occ == 0).astype(np.uint8), metric="chessboard")
    return np.minimum(d, 255).astype(np.uint8)


def numpy_bricks(vol: np.ndarray, b: int = 4):
    """Brick min/max by edge padding and a reshape (padding with copies of the
    border voxels leaves every brick's min and max unchanged)."""
    nz, ny, nx = vol.shape
    pz, py, px = (-nz) % b, (-ny) % b, (-nx) % b
    v = np.pad(vol, ((0, pz), (0, py), (0, px)), mode="edge")
    Bz, By, Bx = v.shape[0] // b, v.shape[1] // b, v.shape[2] // b
    r = v.reshape(Bz, b, By, b, Bx, b)
    return r.min(axis=(1, 3, 5)), r.max(axis=(1, 3, 5))


def rand_vol(rng, shape, dtype, levels):
    return rng.integers(0, levels, size=shape).astype(dtype)


# ------------------------------------------------------------- P1 bricks
@pytest.mark.parametrize("shape,dtype,levels", [
    ((17, 9, 13), np.uint8, 256), ((4, 4, 4), np.uint8, 256), ((1, 1, 1), np.uint16, 4096),
    ((23, 5, 31), np.uint16, 4096), ((8, 12, 3), np.uint16, 65536), ((3, 2, 7), np.uint8, 256)])
def test_bricks_match_numpy_reshape(orc, shape, dtype, levels):
    rng = np.random.default_rng(11)
    vol = rand_vol(rng, shape, dtype, levels)
    bmin, bmax = orc.bricks(vol)
    rmin, rmax = numpy_bricks(vol)
    assert bmin.dtype == dtype and bmax.dtype == dtype
    np.testing.assert_array_equal(bmin, rmin)
    np.testing.assert_array_equal(bmax, rmax)


def test_partial_bricks_are_not_zero_padded(orc):
    # Every voxel 100: every brick, partial ones included, is [100,100].
    vol = np.full((9, 6, 7), 100, np.uint8)
    bmin, bmax = orc.bricks(vol)
    assert bmin.shape == (3, 2, 2)
    assert (bmin == 100).all() and (bmax == 100).all()


# --------------------------------------------------------- P2/P3 distance
@settings(max_examples=60, deadline=None)
@given(st.integers(1, 12), st.integers(1, 12), st.integers(1, 12),
       st.floats(0.0, 0.3), st.integers(0, 2**31 - 1))
def test_dt_matches_brute_force(orc, bz, by, bx, density, seed):
    rng = np.random.default_rng(seed)
    occ = (rng.random((bz, by, bx)) < density).astype(np.uint8)
    np.testing.assert_array_equal(orc.dt(occ), brute_dt(occ))


@pytest.mark.parametrize("shape,density", [((40, 37, 29), 0.001), ((16, 64, 50), 0.02),
                                            ((5, 300, 3), 0.004), ((33, 33, 33), 0.3)])
def test_dt_matches_scipy_chessboard(orc, shape, density):
    rng = np.random.default_rng(7)
    occ = (rng.random(shape) < density).astype(np.uint8)
    np.testing.assert_array_equal(orc.dt(occ), scipy_dt(occ))


def test_dt_tube_shaped_occupancy_matches_scipy(orc):
    # thin oblique lines: many distinct distances along every axis
    occ = np.zeros((30, 40, 50), np.uint8)
    for t in range(40):
        occ[min(29, t * 3 // 4), t, (t * 5) % 50] = 1
    np.testing.assert_array_equal(orc.dt(occ), scipy_dt(occ))


# ---------------------------------------------------------- P4 closed forms
def test_dt_single_occupied_brick(orc):
    shape = (9, 11, 13)
    c = (2, 7, 4)
    occ = np.zeros(shape, np.uint8)
    occ[c] = 1
    z, y, x = np.indices(shape)
    want = np.maximum(np.maximum(abs(z - c[0]), abs(y - c[1])), abs(x - c[2]))
    np.testing.assert_array_equal(orc.dt(occ), want.astype(np.uint8))


def test_dt_all_and_none(orc):
    assert (orc.dt(np.ones((5, 6, 7), np.uint8)) == 0).all()
    assert (orc.dt(np.zeros((5, 6, 7), np.uint8)) == 255).all()


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_dt_long_line_hits_the_cap(orc, axis):
    shape = [1, 1, 1]
    shape[axis] = 300
    occ = np.zeros(shape, np.uint8)
    occ.reshape(-1)[0] = 1
    want = np.minimum(np.arange(300), 255).astype(np.uint8).reshape(shape)
    np.testing.assert_array_equal(orc.dt(occ), want)


def test_dt_cap_in_two_axes(orc):
    occ = np.zeros((1, 280, 270), np.uint8)
    occ[0, 0, 0] = 1
    y, x = np.indices((280, 270))
    want = np.minimum(np.maximum(y, x), 255).astype(np.uint8)[None]
    np.testing.assert_array_equal(orc.dt(occ), want)


# ------------------------------------------------------------ P5 union
@settings(max_examples=30, deadline=None)
@given(st.integers(1, 10), st.integers(1, 10), st.integers(1, 10), st.integers(0, 2**31 - 1))
def test_dt_of_union_is_min_of_dts(orc, bz, by, bx, seed):
    rng = np.random.default_rng(seed)
    a = (rng.random((bz, by, bx)) < 0.1).astype(np.uint8)
    b = (rng.random((bz, by, bx)) < 0.1).astype(np.uint8)
    np.testing.assert_array_equal(orc.dt(a | b), np.minimum(orc.dt(a), orc.dt(b)))


# ------------------------------------------------ partitions / POMs / D'
def _case(seed=5, shape=(29, 22, 18), dtype=np.uint8, levels=256, n=8):
    rng = np.random.default_rng(seed)
    # blocky volume: constant 3^3 cells of random values, plus a background
    vol = np.zeros(shape, dtype)
    cz, cy, cx = [(s + 2) // 3 for s in shape]
    cells = rng.integers(0, levels, size=(cz, cy, cx))
    keep = rng.random((cz, cy, cx)) < 0.15
    cells = np.where(keep, cells, 0)
    vol[:] = np.repeat(np.repeat(np.repeat(cells, 3, 0), 3, 1), 3, 2)[:shape[0], :shape[1], :shape[2]]
    return vol, W.uniform_bounds(levels, n), levels


def test_pom_range_by_brute_force(orc):
    vol, bounds, L = _case()
    bmin, bmax = orc.bricks(vol)
    for p in range(len(bounds) - 1):
        lo, hi = int(bounds[p]), int(bounds[p + 1]) - 1
        occ = orc.pom_range(bmin, bmax, lo, hi)
        # a brick's interval meets [lo,hi] iff some integer of [lo,hi] lies in it
        want = np.zeros_like(occ)
        for v in range(lo, hi + 1):
            want |= ((bmin <= v) & (v <= bmax)).astype(np.uint8)
        np.testing.assert_array_equal(occ, want)


def test_pom_exact_by_voxel_scan(orc):
    vol, bounds, L = _case(shape=(13, 10, 9))
    for p in range(len(bounds) - 1):
        lo, hi = int(bounds[p]), int(bounds[p + 1]) - 1
        inside = ((vol >= lo) & (vol <= hi)).astype(np.uint8)
        _, want = numpy_bricks(inside)       # max over a brick = "any voxel"
        np.testing.assert_array_equal(orc.pom_exact(vol, lo, hi), want)


def test_exact_occupancy_within_range_occupancy(orc):
    vol, bounds, L = _case(seed=9)
    bmin, bmax = orc.bricks(vol)
    dr = orc.pdms(vol, bounds, L, mode=orc.RANGE)
    de = orc.pdms(vol, bounds, L, mode=orc.EXACT)
    for p in range(len(bounds) - 1):
        lo, hi = int(bounds[p]), int(bounds[p + 1]) - 1
        assert (orc.pom_exact(vol, lo, hi) <= orc.pom_range(bmin, bmax, lo, hi)).all()
    assert (dr <= de).all()


def test_pdms_are_dt_of_brute_force_poms(orc):
    vol, bounds, L = _case(seed=3, shape=(21, 17, 15), n=4)
    pd = orc.pdms(vol, bounds, L)
    assert pd.shape == (4,) + orc.grid(vol.shape)
    bmin, bmax = numpy_bricks(vol)
    for p in range(4):
        lo, hi = int(bounds[p]), int(bounds[p + 1]) - 1
        pom = ((bmin <= hi) & (bmax >= lo)).astype(np.uint8)
        np.testing.assert_array_equal(pd[p], brute_dt(pom))


def test_memory_is_n_times_bricks(orc):
    # Sec. 5: n * volumesize / b^3 bytes, with ceil for partial bricks
    vol = np.zeros((18, 9, 5), np.uint8)
    pd = orc.pdms(vol, W.uniform_bounds(256, 16), 256)
    assert pd.nbytes == 16 * 5 * 3 * 2


def _load_fig2():
    kv = {}
    for line in open(os.path.join(GOLD, "fig2_active_sets.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, *vals = line.split()
        kv[k] = [int(v) for v in vals]
    return kv


def test_fig2_active_sets(orc):
    g = _load_fig2()
    L = g["levels"][0]
    bounds = np.array(g["bounds"], np.int32)
    want = sorted(s - 1 for s in g["s_1based"])
    for key in ("tf_a", "tf_b"):
        alpha = np.array(g[key], np.float32) * 0.5
        m = orc.active(bounds, alpha, L)
        assert orc.active_list(m, len(bounds) - 1) == want


def test_fig2_dprime_same_for_both_and_equal_to_d_for_tf_a(orc):
    g = _load_fig2()
    L = g["levels"][0]
    bounds = np.array(g["bounds"], np.int32)
    rng = np.random.default_rng(2)
    vol = rng.integers(0, L, size=(20, 24, 28)).astype(np.uint8)
    vol[rng.random(vol.shape) < 0.9] = 0
    pd = orc.pdms(vol, bounds, L)
    a = np.array(g["tf_a"], np.float32)
    b = np.array(g["tf_b"], np.float32)
    da, _ = orc.tf_update(pd, bounds, a, L)
    db, _ = orc.tf_update(pd, bounds, b, L)
    np.testing.assert_array_equal(da, db)
    # TF_A is non-zero on the whole of each active partition: D' = D.
    for mode in (orc.RANGE, orc.EXACT):
        pdm = orc.pdms(vol, bounds, L, mode=mode)
        dpa, _ = orc.tf_update(pdm, bounds, a, L)
        np.testing.assert_array_equal(dpa, orc.full_recompute(vol, a, L, mode=mode))
        dpb, _ = orc.tf_update(pdm, bounds, b, L)
        assert (dpb <= orc.full_recompute(vol, b, L, mode=mode)).all()


def test_active_set_edges(orc):
    bounds = W.uniform_bounds(256, 8)
    a = np.zeros(256, np.float32)
    assert orc.active_list(orc.active(bounds, a, 256), 8) == []
    a[31] = 1e-30            # last intensity of partition 0
    a[32] = -0.5             # first of partition 1 (non-zero counts, sign does not)
    a[255] = np.nan          # NaN is not equal to zero
    assert orc.active_list(orc.active(bounds, a, 256), 8) == [0, 1, 7]
    # all 256 partitions of width 1
    b1 = W.uniform_bounds(256, 256)
    a = np.zeros(256, np.float32)
    a[[0, 63, 64, 200, 255]] = 1
    assert orc.active_list(orc.active(b1, a, 256), 256) == [0, 63, 64, 200, 255]


def test_invalid_bounds_rejected(orc):
    assert orc.check_bounds([0, 128, 256], 256)
    assert not orc.check_bounds([0, 128, 128, 256], 256)
    assert not orc.check_bounds([1, 128, 256], 256)
    assert not orc.check_bounds([0, 128, 255], 256)
    assert not orc.check_bounds([0, 256], 4096)


# --------------------------------------------------- P6/P7/P9 D' versus D
def test_dprime_below_d_and_equal_when_unsplit(orc):
    vol = W.make_volume("c1")
    L, n = 256, 8
    bounds = W.uniform_bounds(L, n)
    pd = orc.pdms(vol, bounds, L)
    rng = np.random.default_rng(4)
    for k in range(12):
        alpha = W.trapezoid_tf(L, int(rng.integers(1, 4)), rng)
        dp, m = orc.tf_update(pd, bounds, alpha, L)
        d = orc.full_recompute(vol, alpha, L)
        assert (dp <= d).all()
        # the unsplit TF: non-zero on every intensity of each active partition
        full = np.zeros(L, np.float32)
        for p in orc.active_list(m, n):
            full[bounds[p]:bounds[p + 1]] = 1.0
        np.testing.assert_array_equal(orc.tf_update(pd, bounds, full, L)[0],
                                      orc.full_recompute(vol, full, L))


def test_one_partition_per_level_gives_d(orc):
    vol = W.make_volume("c1")[:40, :36, :44]
    L = 256
    bounds = W.uniform_bounds(L, 256)
    pd = orc.pdms(vol, bounds, L)
    rng = np.random.default_rng(8)
    for _ in range(3):
        alpha = W.trapezoid_tf(L, 2, rng)
        np.testing.assert_array_equal(orc.tf_update(pd, bounds, alpha, L)[0],
                                      orc.full_recompute(vol, alpha, L))


def test_empty_and_opaque_transfer_functions(orc):
    vol = W.make_volume("c1")
    L = 256
    bounds = W.uniform_bounds(L, 8)
    pd = orc.pdms(vol, bounds, L)
    zero = np.zeros(L, np.float32)
    assert (orc.tf_update(pd, bounds, zero, L)[0] == 255).all()
    assert (orc.full_recompute(vol, zero, L) == 255).all()
    # every intensity non-transparent: every brick holds a voxel -> all 0
    one = np.ones(L, np.float32)
    assert (orc.tf_update(pd, bounds, one, L)[0] == 0).all()
    assert (orc.full_recompute(vol, one, L) == 0).all()
    assert (orc.full_recompute(vol, one, L, mode=orc.EXACT) == 0).all()


def test_plain_occupancy_range_by_scan(orc):
    rng = np.random.default_rng(12)
    vol = rng.integers(0, 4096, size=(10, 9, 11)).astype(np.uint16)
    vol[rng.random(vol.shape) < 0.7] = 3
    bmin, bmax = orc.bricks(vol)
    alpha = W.trapezoid_tf(4096, 2, rng)
    occ = orc.plain_occ_range(bmin, bmax, alpha, 4096)
    nz = alpha != 0
    want = np.array([nz[a:b + 1].any() for a, b in zip(bmin.ravel(), bmax.ravel())],
                    np.uint8).reshape(occ.shape)
    np.testing.assert_array_equal(occ, want)
    # EXACT: "any voxel maps to non-zero", by a numpy gather
    _, want_e = numpy_bricks(nz[vol].astype(np.uint8))
    np.testing.assert_array_equal(orc.plain_occ_exact(vol, alpha, 4096), want_e)


def test_voxel_beyond_levels_is_an_error(orc):
    vol = np.full((4, 4, 4), 300, np.uint16)
    with pytest.raises(ValueError):
        orc.full_recompute(vol, np.ones(256, np.float32), 256)


# ------------------------------------------------------ P11 determinism
def test_thread_count_does_not_change_results(orc):
    vol, bounds, L = _case(seed=21, shape=(40, 33, 36))
    t0 = orc.threads()
    try:
        orc.set_threads(1)
        a = orc.pdms(vol, bounds, L)
        orc.set_threads(max(2, t0))
        b = orc.pdms(vol, bounds, L)
    finally:
        orc.set_threads(t0)
    np.testing.assert_array_equal(a, b)


def _union_pdm(orc, vol, levels, lo, hi):
    """PDM of the single partition [lo, hi] built from scratch: bounds that
    tile [0, levels) with [lo, hi] as one partition."""
    cuts = sorted({0, lo, hi + 1, levels})
    k = cuts.index(lo)
    return orc.pdms(vol, np.array(cuts, np.int32), levels)[k]


@pytest.mark.parametrize("n,max_level", [(8, 3), (8, 1), (12, 8), (5, 2)])
def test_range_table_maps_are_union_pdms(orc, n, max_level):
    """Range-table map T_k[p] equals the PDM of the union of partitions
    p .. p+2^k-1 computed from scratch (a fresh POM of the merged interval
    and its distance transform), not only the min of the parts."""
    rng = np.random.default_rng(n + max_level)
    vol = np.zeros((20, 24, 28), np.uint8)
    for _ in range(30):
        z, y, x = rng.integers(0, 20), rng.integers(0, 24), rng.integers(0, 28)
        vol[z, y, x] = rng.integers(1, 256)
    bounds = W.uniform_bounds(256, n)
    stack = orc.pdms(vol, bounds, 256)
    table = orc.range_table(stack, max_level)
    j = 0
    k = 1
    while k <= max_level and (1 << k) <= n:
        for p in range(n - (1 << k) + 1):
            want = _union_pdm(orc, vol, 256, int(bounds[p]), int(bounds[p + (1 << k)]) - 1)
            np.testing.assert_array_equal(table[j], want, err_msg=f"k={k} p={p}")
            j += 1
        k += 1
    assert j == len(table)
