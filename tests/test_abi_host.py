"""The C ABI on the host: the library loads, exports every function the header
declares, and rejects invalid arguments before any device work (so these run
without a GPU).  Also checks the host-side active set (step 1 of the update,
Sec. 3.1) against the oracle."""
import ctypes

import numpy as np
import pytest

import workloads as W
from paper_2407_21552_amd import _lib as L


@pytest.fixture(scope="module")
def lib():
    return L.lib()


def test_exports_every_declared_symbol(lib):
    names = L.header_symbols()
    assert {"pdm_build_bricks", "pdm_build_partitions", "pdm_tf_update",
            "pdm_full_recompute"} <= set(names)
    for name in names:
        assert hasattr(lib, name), name
    assert "gfx950" in L.version()


def test_status_strings(lib):
    assert L.status_string(0) == "ok"
    for c in (-1, -2, -3, -4):
        assert L.status_string(c) not in ("ok", "unknown status")
    assert L.status_string(7) == "unknown status"


def desc(nx=64, ny=64, nz=64, dtype=1, levels=256, brick=4):
    return L.VolumeDesc(nx, ny, nz, dtype, levels, brick)


@pytest.mark.parametrize("shape,grid", [((64, 64, 64), (16, 16, 16, 4096)),
                                        ((795, 1024, 1024), (199, 256, 256, 13041664)),
                                        ((460, 512, 512), (115, 128, 128, 1884160)),
                                        ((1, 1, 1), (1, 1, 1, 1)), ((5, 6, 9), (2, 2, 3, 12))])
def test_grid_of(shape, grid):
    assert L.grid_of(L.volume_desc(shape, np.uint8, 256)) == grid


@pytest.mark.parametrize("kw,code", [
    (dict(nx=0), L.PDM_E_INVAL), (dict(ny=-3), L.PDM_E_INVAL), (dict(dtype=3), L.PDM_E_INVAL),
    (dict(levels=0), L.PDM_E_INVAL), (dict(levels=257), L.PDM_E_INVAL),
    (dict(dtype=2, levels=65537), L.PDM_E_INVAL), (dict(brick=0), L.PDM_E_INVAL),
    (dict(brick=8), L.PDM_E_UNSUPPORTED), (dict(nx=4 * 16385), L.PDM_E_UNSUPPORTED),
    (dict(nz=4 * 65536), L.PDM_E_UNSUPPORTED)])
def test_grid_of_rejects(kw, code):
    with pytest.raises(L.PdmError) as e:
        L.grid_of(desc(**kw))
    assert e.value.code == code


NULL = ctypes.c_void_p(0)
FAKE = ctypes.c_void_p(0x10000)  # never dereferenced: validation fails first


def _b(arr):
    a = np.ascontiguousarray(arr, np.int32)
    return a, ctypes.c_void_p(a.ctypes.data)


def test_null_pointers_rejected(lib):
    d = desc()
    bnd, pb = _b(W.uniform_bounds(256, 8))
    alpha = np.zeros(256, np.float32)
    pa = ctypes.c_void_p(alpha.ctypes.data)
    r = ctypes.byref
    assert lib.pdm_build_bricks(r(d), NULL, FAKE, FAKE, NULL, NULL) == L.PDM_E_INVAL
    assert lib.pdm_build_bricks(r(d), FAKE, NULL, FAKE, NULL, NULL) == L.PDM_E_INVAL
    assert lib.pdm_build_partitions(r(d), FAKE, FAKE, pb, 8, NULL, NULL) == L.PDM_E_INVAL
    assert lib.pdm_build_partitions(r(d), FAKE, FAKE, NULL, 8, FAKE, NULL) == L.PDM_E_INVAL
    assert lib.pdm_tf_update(r(d), NULL, pb, 8, pa, FAKE, NULL, NULL) == L.PDM_E_INVAL
    assert lib.pdm_tf_update(r(d), FAKE, pb, 8, NULL, FAKE, NULL, NULL) == L.PDM_E_INVAL
    assert lib.pdm_full_recompute(r(d), FAKE, pa, NULL, NULL) == L.PDM_E_INVAL
    assert lib.pdm_full_recompute(r(d), FAKE, NULL, FAKE, NULL) == L.PDM_E_INVAL
    assert lib.pdm_full_recompute_cached(r(d), NULL, FAKE, pa, FAKE, NULL) == L.PDM_E_INVAL
    assert lib.pdm_full_recompute_cached(r(d), FAKE, NULL, pa, FAKE, NULL) == L.PDM_E_INVAL
    assert lib.pdm_full_recompute_cached(r(d), FAKE, FAKE, NULL, FAKE, NULL) == L.PDM_E_INVAL
    assert lib.pdm_full_recompute_cached(r(d), FAKE, FAKE, pa, NULL, NULL) == L.PDM_E_INVAL
    assert lib.pdm_plain_cached_distance_x(r(d), NULL, FAKE, pa, FAKE, NULL) == L.PDM_E_INVAL
    assert lib.pdm_distance_yz(r(d), NULL, 1, NULL) == L.PDM_E_INVAL
    assert lib.pdm_distance_yz(r(d), FAKE, 0, NULL) == L.PDM_E_INVAL
    assert lib.pdm_distance_yz(r(d), FAKE, 257, NULL) == L.PDM_E_INVAL
    assert lib.pdm_build_bricks(None, FAKE, FAKE, FAKE, NULL, NULL) == L.PDM_E_INVAL
    assert lib.pdm_grid_of(r(d), None) == L.PDM_E_INVAL


@pytest.mark.parametrize("bounds,n", [
    ([0, 128, 128, 256], 3), ([1, 128, 256], 2), ([0, 128, 255], 2), ([0, 300], 1),
    ([0, 256], 0), (list(range(0, 258)), 257)])
def test_bad_bounds_rejected_before_launch(lib, bounds, n):
    d = desc()
    bnd, pb = _b(bounds)
    alpha = np.ones(256, np.float32)
    pa = ctypes.c_void_p(alpha.ctypes.data)
    r = ctypes.byref
    assert lib.pdm_build_partitions(r(d), FAKE, FAKE, pb, n, FAKE, NULL) == L.PDM_E_INVAL
    assert lib.pdm_pom_distance_x(r(d), FAKE, FAKE, pb, n, FAKE, NULL) == L.PDM_E_INVAL
    assert lib.pdm_tf_update(r(d), FAKE, pb, n, pa, FAKE, NULL, NULL) == L.PDM_E_INVAL
    m = np.zeros(4, np.uint64)
    assert lib.pdm_active_set(pb, n, pa, 256, ctypes.c_void_p(m.ctypes.data)) == L.PDM_E_INVAL


def test_plain_limits_match_the_header():
    import re
    text = open(L.HEADER).read()
    defs = dict(re.findall(r"#define (PDM_\w+) (\d+)", text))
    assert int(defs["PDM_MAX_PLAIN_RUNS"]) == L.MAX_PLAIN_RUNS
    assert int(defs["PDM_MAX_PLAIN_BITMAP_LEVELS"]) == L.MAX_PLAIN_BITMAP_LEVELS


def test_plain_method_rejects_too_many_runs(lib):
    # above 16384 levels the non-zero opacity levels travel as runs: more
    # than PDM_MAX_PLAIN_RUNS of them is refused before any device call
    for levels in (16385, 65536):
        d = desc(dtype=2, levels=levels)
        alpha = np.zeros(levels, np.float32)
        alpha[: 2 * (L.MAX_PLAIN_RUNS + 1) : 2] = 1.0   # one run more than accepted
        assert lib.pdm_full_recompute(ctypes.byref(d), FAKE, ctypes.c_void_p(alpha.ctypes.data),
                                      FAKE, NULL) == L.PDM_E_UNSUPPORTED
        assert lib.pdm_full_recompute_cached(ctypes.byref(d), FAKE, FAKE,
                                             ctypes.c_void_p(alpha.ctypes.data), FAKE,
                                             NULL) == L.PDM_E_UNSUPPORTED
    # 16-bit volumes of more than 65536 levels do not exist
    d = desc(dtype=2, levels=65537)
    alpha = np.ones(65537, np.float32)
    assert lib.pdm_full_recompute(ctypes.byref(d), FAKE, ctypes.c_void_p(alpha.ctypes.data),
                                  FAKE, NULL) != L.PDM_OK


def test_active_set_matches_oracle(orc):
    rng = np.random.default_rng(3)
    for L_, n in ((256, 8), (256, 64), (4096, 32), (256, 256), (8, 4), (4096, 1)):
        bounds = W.uniform_bounds(L_, n)
        for _ in range(20):
            alpha = W.trapezoid_tf(L_, int(rng.integers(1, 5)), rng) if L_ >= 32 else \
                (rng.random(L_) < 0.4).astype(np.float32)
            np.testing.assert_array_equal(L.active_set(bounds, alpha, L_),
                                          orc.active(bounds, alpha, L_))
    # non-uniform borders, NaN and negative opacities
    bounds = W.rhomin_bounds(256, 32, 3)
    a = np.zeros(256, np.float32)
    a[2] = np.nan
    a[200] = -1.0
    np.testing.assert_array_equal(L.active_set(bounds, a, 256), orc.active(bounds, a, 256))
    assert L.mask_to_list(L.active_set(bounds, a, 256), 32) == \
        orc.active_list(orc.active(bounds, a, 256), 32)
    # -0 is zero (its partition stays out); a subnormal and a NaN in the last
    # entry of a partition are non-zero; 4096 levels in 64 partitions
    bounds = W.uniform_bounds(4096, 64)
    a = np.zeros(4096, np.float32)
    a[0:64] = -0.0
    a[64 + 17] = np.float32(1e-42)
    a[2 * 64 - 1] = np.nan
    a[4095] = np.float32(-1e-45)
    m = L.active_set(bounds, a, 4096)
    np.testing.assert_array_equal(m, orc.active(bounds, a, 4096))
    assert L.mask_to_list(m, 64) == [1, 63]


def test_opacity_table_marshalling():
    a = np.linspace(0, 1, 256, dtype=np.float32)
    b, p = L._opacity_table(a, 256, "alpha")
    assert b is a and p == a.ctypes.data
    ro = a.copy()
    ro.flags.writeable = False
    b, p = L._opacity_table(ro, 256, "alpha")
    assert b is ro and p == ro.ctypes.data
    b, p = L._opacity_table(a.astype(np.float64), 256, "alpha")   # converted copy
    assert b.dtype == np.float32 and p == b.ctypes.data
    np.testing.assert_array_equal(b, a)
    wide = np.zeros((256, 2), np.float32)
    b, p = L._opacity_table(wide[:, 0], 256, "alpha")             # strided: copied
    assert b.flags.c_contiguous and p == b.ctypes.data
    with pytest.raises(ValueError):
        L._opacity_table(a[:255], 256, "alpha")


def test_binding_rejects_wrong_alpha_length():
    with pytest.raises(ValueError):
        L.active_set(W.uniform_bounds(256, 8), np.zeros(255, np.float32), 256)


def test_exact_calls_reject_unsupported_sizes(lib):
    r = ctypes.byref
    bnd, pb = _b(W.uniform_bounds(256, 8))
    wide = desc(nx=4 * 257)                       # 257 bricks along x
    assert lib.pdm_build_partitions_exact(r(wide), FAKE, pb, 8, FAKE, NULL) == L.PDM_E_UNSUPPORTED
    big = desc(dtype=2, levels=16385)
    bnd2, pb2 = _b(W.uniform_bounds(16385, 8))
    assert lib.pdm_build_partitions_exact(r(big), FAKE, pb2, 8, FAKE, NULL) == L.PDM_E_UNSUPPORTED
    alpha = np.ones(16385, np.float32)
    assert lib.pdm_full_recompute_exact(r(big), FAKE, ctypes.c_void_p(alpha.ctypes.data), FAKE,
                                        NULL) == L.PDM_E_UNSUPPORTED
    assert lib.pdm_build_partitions_exact(r(desc()), NULL, pb, 8, FAKE, NULL) == L.PDM_E_INVAL
    assert lib.pdm_full_recompute_exact(r(desc()), FAKE, NULL, FAKE, NULL) == L.PDM_E_INVAL


def test_batch_update_validates_every_item(lib):
    d = desc()
    bnd, pb = _b(W.uniform_bounds(256, 8))
    alpha = np.ones(256, np.float32)
    good = L.BatchUpdate(ctypes.pointer(d), FAKE, pb, 8, ctypes.c_void_p(alpha.ctypes.data), FAKE)
    bad_bounds_arr, pbad = _b([0, 100, 100, 256])
    bad = L.BatchUpdate(ctypes.pointer(d), FAKE, pbad, 3, ctypes.c_void_p(alpha.ctypes.data), FAKE)
    arr = (L.BatchUpdate * 2)(good, bad)
    assert lib.pdm_batch_tf_update(arr, 2, NULL, NULL) == L.PDM_E_INVAL
    assert lib.pdm_batch_tf_update(arr, 0, NULL, NULL) == L.PDM_E_INVAL
    assert lib.pdm_batch_tf_update(arr, 49, NULL, NULL) == L.PDM_E_INVAL
    assert lib.pdm_batch_tf_update(None, 1, NULL, NULL) == L.PDM_E_INVAL
    nod = L.BatchUpdate(ctypes.pointer(d), NULL, pb, 8, ctypes.c_void_p(alpha.ctypes.data), FAKE)
    assert lib.pdm_batch_tf_update((L.BatchUpdate * 1)(nod), 1, NULL, NULL) == L.PDM_E_INVAL


def test_batch_build_validation(lib):
    d = desc()
    bnd, pb = _b(W.uniform_bounds(256, 8))
    good = L.BatchVolume(ctypes.pointer(d), FAKE, FAKE, FAKE, pb, 8, FAKE)
    arr = (L.BatchVolume * 1)(good)
    need = lib.pdm_batch_workspace_bytes(1)
    assert need > 0 and lib.pdm_batch_workspace_bytes(0) == 0 and lib.pdm_batch_workspace_bytes(49) == 0
    assert lib.pdm_batch_build(arr, 1, NULL, need, None, NULL) == L.PDM_E_INVAL
    assert lib.pdm_batch_build(arr, 1, FAKE, need - 1, None, NULL) == L.PDM_E_INVAL
    assert lib.pdm_batch_build(arr, 0, FAKE, need, None, NULL) == L.PDM_E_INVAL
    big = desc(nx=4 * 257)
    arr2 = (L.BatchVolume * 1)(L.BatchVolume(ctypes.pointer(big), FAKE, FAKE, FAKE, pb, 8, FAKE))
    assert lib.pdm_batch_build(arr2, 1, FAKE, need, None, NULL) == L.PDM_E_UNSUPPORTED
    bad_cfg = ctypes.pointer(L.BatchConfig(0, 17, 0, 0))
    assert lib.pdm_batch_build(arr, 1, FAKE, need, bad_cfg, NULL) == L.PDM_E_INVAL
    bad_rows = ctypes.pointer(L.BatchConfig(257, 1, 0, 0))
    assert lib.pdm_batch_build(arr, 1, FAKE, need, bad_rows, NULL) == L.PDM_E_INVAL
    bad_mode = ctypes.pointer(L.BatchConfig(0, 1, 0, 2))
    assert lib.pdm_batch_build(arr, 1, FAKE, need, bad_mode, NULL) == L.PDM_E_INVAL

    # the allocation-free variant validates the same way, before any HIP call
    assert lib.pdm_batch_build_noalloc(arr, 0, None, NULL, NULL) == L.PDM_E_INVAL
    assert lib.pdm_batch_build_noalloc(arr, 49, None, NULL, NULL) == L.PDM_E_INVAL
    assert lib.pdm_batch_build_noalloc(None, 1, None, NULL, NULL) == L.PDM_E_INVAL
    assert lib.pdm_batch_build_noalloc(arr2, 1, None, NULL, NULL) == L.PDM_E_UNSUPPORTED
    assert lib.pdm_batch_build_noalloc(arr, 1, bad_cfg, NULL, NULL) == L.PDM_E_INVAL
    nulls = (L.BatchVolume * 1)(L.BatchVolume(ctypes.pointer(d), FAKE, NULL, FAKE, pb, 8, FAKE))
    assert lib.pdm_batch_build_noalloc(nulls, 1, None, NULL, NULL) == L.PDM_E_INVAL


def _level_first(n, k):
    return sum(n - (1 << j) + 1 for j in range(1, k))


def _expand(n, K, idx):
    """Partitions covered by map index idx (PDM or range-table map)."""
    if idx < n:
        return {idx}
    t = idx - n
    for k in range(1, K + 1):
        cnt = n - (1 << k) + 1
        if t < cnt:
            return set(range(t, t + (1 << k)))
        t -= cnt
    raise AssertionError(f"index {idx} beyond the table")


def _runs(bits):
    runs, a = [], None
    for p, b in enumerate(bits + [False]):
        if b and a is None:
            a = p
        if not b and a is not None:
            runs.append((a, p - 1))
            a = None
    return runs


@pytest.mark.parametrize("n", [1, 2, 3, 8, 17, 64, 200, 256])
@pytest.mark.parametrize("max_level", [0, 1, 3, 8])
def test_range_cover_is_exact(n, max_level):
    """The maps chosen for an active set cover exactly S (no partition
    outside S), take no more maps than |S|, and at most two per run while
    runs fit the table; the table size is the sum of its levels."""
    rng = np.random.default_rng(n * 31 + max_level)
    K = 0
    while K < max_level and (2 << K) <= n:
        K += 1
    assert L.range_table_maps(n, max_level) == _level_first(n, K + 1)
    masks = []
    for dens in (0.0, 0.05, 0.3, 0.7, 0.95, 1.0):
        for _ in range(12):
            masks.append(rng.random(n) < dens)
    for a, b in ((0, n - 1), (n // 3, n // 2), (n - 1, n - 1)):  # single runs
        bits = np.zeros(n, bool)
        bits[a:b + 1] = True
        masks.append(bits)
    for bits in masks:
        m = np.zeros(4, np.uint64)
        for p in np.nonzero(bits)[0]:
            m[p >> 6] |= np.uint64(1) << np.uint64(p & 63)
        cov = L.range_cover(n, max_level, m)
        got = set()
        for idx in cov:
            part = _expand(n, K, idx)
            assert part <= set(np.nonzero(bits)[0].tolist()), (idx, part)
            got |= part
        assert got == set(np.nonzero(bits)[0].tolist())
        assert len(cov) <= int(bits.sum())
        runs = _runs(bits.tolist())
        if all(b - a + 1 <= (2 << K) for a, b in runs):
            assert len(cov) <= 2 * len(runs)


def test_range_calls_validate(lib):
    r = ctypes.byref
    d = desc()
    bnd, pb = _b(W.uniform_bounds(256, 8))
    alpha = np.ones(256, np.float32)
    pa = ctypes.c_void_p(alpha.ctypes.data)
    assert L.lib().pdm_range_table_maps(0, 3) == -1 and L.lib().pdm_range_table_maps(257, 3) == -1
    assert L.lib().pdm_range_table_maps(8, -1) == -1
    assert lib.pdm_build_range_table(r(d), NULL, 8, 3, FAKE, NULL) == L.PDM_E_INVAL
    assert lib.pdm_build_range_table(r(d), FAKE, 8, 3, NULL, NULL) == L.PDM_E_INVAL
    assert lib.pdm_build_range_table(r(d), FAKE, 8, 0, NULL, NULL) == L.PDM_OK  # K = 0: nothing to do
    assert lib.pdm_tf_update_ranges(r(d), FAKE, NULL, pb, 8, 3, pa, FAKE, NULL, NULL) == L.PDM_E_INVAL
    assert lib.pdm_tf_update_ranges(r(d), FAKE, FAKE, pb, 8, -1, pa, FAKE, NULL, NULL) == L.PDM_E_INVAL
    bad, pbad = _b([0, 100, 100, 256])
    assert lib.pdm_tf_update_ranges(r(d), FAKE, FAKE, pbad, 3, 3, pa, FAKE, NULL, NULL) == L.PDM_E_INVAL
    m = np.zeros(4, np.uint64)
    out = np.zeros(256, np.int32)
    cnt = ctypes.c_int32(0)
    assert lib.pdm_range_cover(8, 3, None, ctypes.c_void_p(out.ctypes.data), r(cnt)) == L.PDM_E_INVAL
    assert lib.pdm_range_cover(0, 3, ctypes.c_void_p(m.ctypes.data), ctypes.c_void_p(out.ctypes.data),
                               r(cnt)) == L.PDM_E_INVAL


def test_batch_range_update_validates_before_launch(lib):
    """Every request of a batched range-table update is checked before any
    launch: a bad request anywhere in the batch fails the whole call with no
    device work (the fake pointers are never dereferenced)."""
    d = desc()
    bnd, pb = _b(W.uniform_bounds(256, 8))
    alpha = np.ones(256, np.float32)
    pa = ctypes.c_void_p(alpha.ctypes.data)

    def item(**kw):
        it = L.BatchRangeUpdate()
        it.v = ctypes.pointer(d)
        it.d_pdms, it.d_table, it.h_bounds = FAKE, FAKE, pb
        it.n, it.max_level, it.h_alpha, it.d_dist = 8, 3, pa, FAKE
        for k, v in kw.items():
            setattr(it, k, v)
        return it

    def call(items, count=None):
        arr = (L.BatchRangeUpdate * max(1, len(items)))(*items)
        return lib.pdm_batch_tf_update_ranges(arr, len(items) if count is None else count, NULL, NULL)

    assert lib.pdm_batch_tf_update_ranges(None, 1, NULL, NULL) == L.PDM_E_INVAL
    assert call([item()], count=0) == L.PDM_E_INVAL
    assert call([item()] * 49) == L.PDM_E_INVAL
    bad, pbad = _b([0, 100, 100, 256])
    for broken in (dict(d_pdms=None), dict(d_dist=None), dict(h_alpha=None), dict(max_level=-1),
                   dict(d_table=None), dict(h_bounds=pbad, n=3), dict(n=0)):
        assert call([item(), item(**broken)]) == L.PDM_E_INVAL, broken
    # no table is needed when the level count is 0 (validation passes; the
    # call would then launch, so it is not made here)
    assert L.range_table_maps(8, 0) == 0
