"""ctypes binding of libpdm (include/pdm.h): argument marshalling only.

Every step of the path runs inside libpdm (host validation, the active set,
the kernels).  This module checks that torch tensors have the dtype, size,
device and layout the C ABI documents, passes their device pointers and
torch's current HIP stream, and raises PdmError on a non-zero status.  It
fails loudly when libpdm.so is missing: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import re
import struct

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpdm.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "pdm.h")

PDM_OK, PDM_E_INVAL, PDM_E_RANGE, PDM_E_UNSUPPORTED, PDM_E_DEVICE = 0, -1, -2, -3, -4
PDM_U8, PDM_U16 = 1, 2
BRICK = 4
DIST_CAP = 255
MAX_PARTITIONS = 256
MAX_PLAIN_BITMAP_LEVELS = 16384  # above: the non-zero opacity levels go as runs
MAX_PLAIN_RUNS = 512             # runs accepted above MAX_PLAIN_BITMAP_LEVELS levels


class PdmError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {status_string(code)} ({code})")


class VolumeDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("levels", ctypes.c_int32), ("brick", ctypes.c_int32)]


class BatchUpdate(ctypes.Structure):
    _fields_ = [("v", ctypes.POINTER(VolumeDesc)), ("d_pdms", ctypes.c_void_p),
                ("h_bounds", ctypes.c_void_p), ("n", ctypes.c_int32),
                ("h_alpha", ctypes.c_void_p), ("d_dist", ctypes.c_void_p)]


class BatchRangeUpdate(ctypes.Structure):
    _fields_ = [("v", ctypes.POINTER(VolumeDesc)), ("d_pdms", ctypes.c_void_p),
                ("d_table", ctypes.c_void_p), ("h_bounds", ctypes.c_void_p),
                ("n", ctypes.c_int32), ("max_level", ctypes.c_int32),
                ("h_alpha", ctypes.c_void_p), ("d_dist", ctypes.c_void_p)]


BATCH_MAX = 48


class BatchVolume(ctypes.Structure):
    _fields_ = [("v", ctypes.POINTER(VolumeDesc)), ("d_volume", ctypes.c_void_p),
                ("d_bmin", ctypes.c_void_p), ("d_bmax", ctypes.c_void_p),
                ("h_bounds", ctypes.c_void_p), ("n", ctypes.c_int32),
                ("d_pdms", ctypes.c_void_p)]


class BatchConfig(ctypes.Structure):
    _fields_ = [("rows_per_item", ctypes.c_int32), ("lines_mult", ctypes.c_int32),
                ("largest_first", ctypes.c_int32), ("single_launch", ctypes.c_int32)]


class GridDesc(ctypes.Structure):
    _fields_ = [("bx", ctypes.c_int32), ("by", ctypes.c_int32), ("bz", ctypes.c_int32),
                ("count", ctypes.c_int64)]


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libpdm.so; raises ImportError if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, st = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int
        V = ctypes.POINTER(VolumeDesc)
        L.pdm_grid_of.argtypes = [V, ctypes.POINTER(GridDesc)]
        L.pdm_active_set.argtypes = [P, i32, P, i32, P]
        L.pdm_build_bricks.argtypes = [V, P, P, P, P, P]
        L.pdm_build_partitions.argtypes = [V, P, P, P, i32, P, P]
        L.pdm_tf_update.argtypes = [V, P, P, i32, P, P, P, P]
        L.pdm_full_recompute.argtypes = [V, P, P, P, P]
        L.pdm_full_recompute_cached.argtypes = [V, P, P, P, P, P]
        L.pdm_plain_cached_distance_x.argtypes = [V, P, P, P, P, P]
        L.pdm_pom_distance_x.argtypes = [V, P, P, P, i32, P, P]
        L.pdm_plain_distance_x.argtypes = [V, P, P, P, P]
        L.pdm_distance_yz.argtypes = [V, P, i32, P]
        L.pdm_build_partitions_exact.argtypes = [V, P, P, i32, P, P]
        L.pdm_pom_exact_distance_x.argtypes = [V, P, P, i32, P, P]
        L.pdm_full_recompute_exact.argtypes = [V, P, P, P, P]
        L.pdm_plain_exact_distance_x.argtypes = [V, P, P, P, P]
        L.pdm_batch_tf_update.argtypes = [ctypes.POINTER(BatchUpdate), i32, P, P]
        L.pdm_batch_tf_update_ranges.argtypes = [ctypes.POINTER(BatchRangeUpdate), i32, P, P]
        L.pdm_batch_workspace_bytes.argtypes = [i32]
        L.pdm_batch_workspace_bytes.restype = ctypes.c_size_t
        L.pdm_batch_build.argtypes = [ctypes.POINTER(BatchVolume), i32, P, ctypes.c_size_t,
                                      ctypes.POINTER(BatchConfig), P]
        L.pdm_batch_build_noalloc.argtypes = [ctypes.POINTER(BatchVolume), i32,
                                              ctypes.POINTER(BatchConfig), P, P]
        for name in ("pdm_grid_of", "pdm_active_set", "pdm_build_bricks", "pdm_build_partitions",
                     "pdm_tf_update", "pdm_full_recompute", "pdm_pom_distance_x",
                     "pdm_full_recompute_cached", "pdm_plain_cached_distance_x",
                     "pdm_plain_distance_x", "pdm_distance_yz", "pdm_build_partitions_exact",
                     "pdm_pom_exact_distance_x", "pdm_full_recompute_exact",
                     "pdm_plain_exact_distance_x", "pdm_batch_tf_update", "pdm_batch_build",
                     "pdm_batch_build_noalloc",
                     "pdm_build_range_table", "pdm_range_cover", "pdm_tf_update_ranges",
                     "pdm_batch_tf_update_ranges"):
            getattr(L, name).restype = st
        L.pdm_range_table_maps.argtypes = [i32, i32]
        L.pdm_range_table_maps.restype = ctypes.c_int64
        L.pdm_build_range_table.argtypes = [V, P, i32, i32, P, P]
        L.pdm_range_cover.argtypes = [i32, i32, P, P, P]
        L.pdm_tf_update_ranges.argtypes = [V, P, P, P, i32, i32, P, P, P, P]
        L.pdm_status_string.argtypes = [st]
        L.pdm_status_string.restype = ctypes.c_char_p
        L.pdm_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def header_symbols() -> list:
    """Names of the functions include/pdm.h declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pdm_[a-z_]+)\s*\(", text)))


def status_string(code: int) -> str:
    return lib().pdm_status_string(int(code)).decode()


def version() -> str:
    return lib().pdm_version().decode()


def _check(code: int, what: str) -> None:
    if code != PDM_OK:
        raise PdmError(code, what)


# ------------------------------------------------------------- descriptors
def volume_desc(shape_zyx, dtype, levels: int, brick: int = BRICK) -> VolumeDesc:
    nz, ny, nx = (int(s) for s in shape_zyx)
    code = {1: PDM_U8, 2: PDM_U16}[np.dtype(_np_dtype(dtype)).itemsize]
    return VolumeDesc(nx, ny, nz, code, int(levels), int(brick))


def _np_dtype(dtype):
    try:
        import torch
        if isinstance(dtype, torch.dtype):
            return {torch.uint8: np.uint8, torch.uint16: np.uint16, torch.int16: np.uint16}[dtype]
    except ImportError:
        pass
    return np.dtype(dtype)


def grid_of(desc: VolumeDesc):
    """(Bz, By, Bx, G) of a volume descriptor."""
    g = GridDesc()
    _check(lib().pdm_grid_of(ctypes.byref(desc), ctypes.byref(g)), "pdm_grid_of")
    return g.bz, g.by, g.bx, g.count


def _bounds(bounds) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(bounds, dtype=np.int32))


def _alpha(alpha, levels: int) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(alpha, dtype=np.float32))
    if a.ndim != 1 or a.size != levels:
        raise ValueError(f"alpha must hold {levels} float32 entries, got shape {a.shape}")
    return a


def _np_ptr(a: np.ndarray) -> ctypes.c_void_p:
    return ctypes.c_void_p(a.ctypes.data)


def active_set(bounds, alpha, levels: int) -> np.ndarray:
    """Step 1 of the TF update: the 4-word uint64 mask of S (host only)."""
    b = _bounds(bounds)
    a = _alpha(alpha, levels)
    m = np.zeros(4, np.uint64)
    _check(lib().pdm_active_set(_np_ptr(b), len(b) - 1, _np_ptr(a), int(levels), _np_ptr(m)),
           "pdm_active_set")
    return m


def mask_to_list(mask, n: int):
    return [p for p in range(n) if (int(mask[p >> 6]) >> (p & 63)) & 1]


# ------------------------------------------------------------ tensor checks
def _dev_ptr(t, nbytes: int, what: str) -> ctypes.c_void_p:
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what}: expected a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{what}: tensor must be on a GPU")
    if not t.is_contiguous():
        raise ValueError(f"{what}: tensor must be contiguous")
    if t.numel() * t.element_size() != nbytes:
        raise ValueError(f"{what}: expected {nbytes} bytes, got {t.numel() * t.element_size()}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream) -> ctypes.c_void_p:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _vox_bytes(desc: VolumeDesc) -> int:
    return desc.nx * desc.ny * desc.nz * desc.dtype


# ------------------------------------------------------------- entry points
def build_bricks(desc, volume, bmin, bmax, range_err=None, stream=None) -> None:
    G = grid_of(desc)[3]
    err = ctypes.c_void_p(0) if range_err is None else _dev_ptr(range_err, 4, "range_err")
    _check(lib().pdm_build_bricks(ctypes.byref(desc), _dev_ptr(volume, _vox_bytes(desc), "volume"),
                                  _dev_ptr(bmin, G * desc.dtype, "bmin"),
                                  _dev_ptr(bmax, G * desc.dtype, "bmax"), err, _stream(stream)),
           "pdm_build_bricks")


def build_partitions(desc, bmin, bmax, bounds, pdms, stream=None) -> None:
    G = grid_of(desc)[3]
    b = _bounds(bounds)
    n = len(b) - 1
    _check(lib().pdm_build_partitions(ctypes.byref(desc), _dev_ptr(bmin, G * desc.dtype, "bmin"),
                                      _dev_ptr(bmax, G * desc.dtype, "bmax"), _np_ptr(b), n,
                                      _dev_ptr(pdms, n * G, "pdms"), _stream(stream)),
           "pdm_build_partitions")


def pom_distance_x(desc, bmin, bmax, bounds, pdms, stream=None) -> None:
    G = grid_of(desc)[3]
    b = _bounds(bounds)
    n = len(b) - 1
    _check(lib().pdm_pom_distance_x(ctypes.byref(desc), _dev_ptr(bmin, G * desc.dtype, "bmin"),
                                    _dev_ptr(bmax, G * desc.dtype, "bmax"), _np_ptr(b), n,
                                    _dev_ptr(pdms, n * G, "pdms"), _stream(stream)),
           "pdm_pom_distance_x")


def distance_yz(desc, maps, count: int, stream=None) -> None:
    G = grid_of(desc)[3]
    _check(lib().pdm_distance_yz(ctypes.byref(desc), _dev_ptr(maps, count * G, "maps"), int(count),
                                 _stream(stream)), "pdm_distance_yz")


def tf_update(desc, pdms, bounds, alpha, dist, stream=None) -> np.ndarray:
    """D' into `dist`; returns the S mask."""
    G = grid_of(desc)[3]
    b = _bounds(bounds)
    n = len(b) - 1
    a = _alpha(alpha, desc.levels)
    m = np.zeros(4, np.uint64)
    _check(lib().pdm_tf_update(ctypes.byref(desc), _dev_ptr(pdms, n * G, "pdms"), _np_ptr(b), n,
                               _np_ptr(a), _dev_ptr(dist, G, "dist"), _np_ptr(m), _stream(stream)),
           "pdm_tf_update")
    return m


# ------------------------------------------------------------- range tables
def range_table_maps(n: int, max_level: int) -> int:
    """Maps in the range table of n partitions with levels 1..min(max_level,
    floor(log2 n))."""
    r = int(lib().pdm_range_table_maps(int(n), int(max_level)))
    if r < 0:
        raise ValueError(f"range table: n={n} must be in 1..256 and max_level={max_level} >= 0")
    return r


def build_range_table(desc, pdms, n: int, max_level: int, table, stream=None) -> None:
    """Levels 1..K of the range table of `pdms` into `table` (a uint8 device
    tensor of range_table_maps(n, max_level) * G bytes; None when that is 0)."""
    G = grid_of(desc)[3]
    maps = range_table_maps(n, max_level)
    tp = _dev_ptr(table, maps * G, "table") if maps > 0 else ctypes.c_void_p(0)
    _check(lib().pdm_build_range_table(ctypes.byref(desc), _dev_ptr(pdms, n * G, "pdms"), int(n),
                                       int(max_level), tp, _stream(stream)),
           "pdm_build_range_table")


def range_cover(n: int, max_level: int, mask) -> list:
    """Map indices combined for the S mask (i < n: PDM i, else table map i - n)."""
    m = np.ascontiguousarray(np.asarray(mask, dtype=np.uint64))
    if m.shape != (4,):
        raise ValueError("mask must hold 4 uint64 words")
    out = np.zeros(256, np.int32)
    cnt = ctypes.c_int32(0)
    _check(lib().pdm_range_cover(int(n), int(max_level), _np_ptr(m), _np_ptr(out), ctypes.byref(cnt)),
           "pdm_range_cover")
    return [int(x) for x in out[:cnt.value]]


def tf_update_ranges(desc, pdms, table, bounds, max_level: int, alpha, dist, stream=None) -> np.ndarray:
    """tf_update through the range table; returns the S mask."""
    G = grid_of(desc)[3]
    b = _bounds(bounds)
    n = len(b) - 1
    a = _alpha(alpha, desc.levels)
    maps = range_table_maps(n, max_level)
    tp = _dev_ptr(table, maps * G, "table") if maps > 0 else ctypes.c_void_p(0)
    m = np.zeros(4, np.uint64)
    _check(lib().pdm_tf_update_ranges(ctypes.byref(desc), _dev_ptr(pdms, n * G, "pdms"), tp,
                                      _np_ptr(b), n, int(max_level), _np_ptr(a),
                                      _dev_ptr(dist, G, "dist"), _np_ptr(m), _stream(stream)),
           "pdm_tf_update_ranges")
    return m


def full_recompute(desc, volume, alpha, dist, stream=None) -> None:
    G = grid_of(desc)[3]
    a = _alpha(alpha, desc.levels)
    _check(lib().pdm_full_recompute(ctypes.byref(desc), _dev_ptr(volume, _vox_bytes(desc), "volume"),
                                    _np_ptr(a), _dev_ptr(dist, G, "dist"), _stream(stream)),
           "pdm_full_recompute")


def full_recompute_cached(desc, bmin, bmax, alpha, dist, stream=None) -> None:
    """Plain method from the cached brick [min, max] (pdm_build_bricks'
    output): the same D as full_recompute without reading the volume."""
    G = grid_of(desc)[3]
    a = _alpha(alpha, desc.levels)
    _check(lib().pdm_full_recompute_cached(ctypes.byref(desc), _dev_ptr(bmin, G * desc.dtype, "bmin"),
                                           _dev_ptr(bmax, G * desc.dtype, "bmax"), _np_ptr(a),
                                           _dev_ptr(dist, G, "dist"), _stream(stream)),
           "pdm_full_recompute_cached")


def plain_cached_distance_x(desc, bmin, bmax, alpha, dist, stream=None) -> None:
    G = grid_of(desc)[3]
    a = _alpha(alpha, desc.levels)
    _check(lib().pdm_plain_cached_distance_x(ctypes.byref(desc),
                                             _dev_ptr(bmin, G * desc.dtype, "bmin"),
                                             _dev_ptr(bmax, G * desc.dtype, "bmax"), _np_ptr(a),
                                             _dev_ptr(dist, G, "dist"), _stream(stream)),
           "pdm_plain_cached_distance_x")


def plain_distance_x(desc, volume, alpha, dist, stream=None) -> None:
    G = grid_of(desc)[3]
    a = _alpha(alpha, desc.levels)
    _check(lib().pdm_plain_distance_x(ctypes.byref(desc),
                                      _dev_ptr(volume, _vox_bytes(desc), "volume"), _np_ptr(a),
                                      _dev_ptr(dist, G, "dist"), _stream(stream)),
           "pdm_plain_distance_x")


# ------------------------------------------------------- EXACT occupancy
def build_partitions_exact(desc, volume, bounds, pdms, stream=None) -> None:
    """PDMs with EXACT POMs (a voxel of the brick in the partition), from the volume."""
    G = grid_of(desc)[3]
    b = _bounds(bounds)
    n = len(b) - 1
    _check(lib().pdm_build_partitions_exact(ctypes.byref(desc),
                                            _dev_ptr(volume, _vox_bytes(desc), "volume"),
                                            _np_ptr(b), n, _dev_ptr(pdms, n * G, "pdms"),
                                            _stream(stream)), "pdm_build_partitions_exact")


def pom_exact_distance_x(desc, volume, bounds, pdms, stream=None) -> None:
    G = grid_of(desc)[3]
    b = _bounds(bounds)
    n = len(b) - 1
    _check(lib().pdm_pom_exact_distance_x(ctypes.byref(desc),
                                          _dev_ptr(volume, _vox_bytes(desc), "volume"),
                                          _np_ptr(b), n, _dev_ptr(pdms, n * G, "pdms"),
                                          _stream(stream)), "pdm_pom_exact_distance_x")


def full_recompute_exact(desc, volume, alpha, dist, stream=None) -> None:
    """Plain method with EXACT occupancy (a voxel of the brick has alpha != 0)."""
    G = grid_of(desc)[3]
    a = _alpha(alpha, desc.levels)
    _check(lib().pdm_full_recompute_exact(ctypes.byref(desc),
                                          _dev_ptr(volume, _vox_bytes(desc), "volume"),
                                          _np_ptr(a), _dev_ptr(dist, G, "dist"), _stream(stream)),
           "pdm_full_recompute_exact")


def plain_exact_distance_x(desc, volume, alpha, dist, stream=None) -> None:
    G = grid_of(desc)[3]
    a = _alpha(alpha, desc.levels)
    _check(lib().pdm_plain_exact_distance_x(ctypes.byref(desc),
                                            _dev_ptr(volume, _vox_bytes(desc), "volume"),
                                            _np_ptr(a), _dev_ptr(dist, G, "dist"),
                                            _stream(stream)), "pdm_plain_exact_distance_x")


# ------------------------------------------------------------ batched update
def batch_tf_update(items, stream=None) -> np.ndarray:
    """TF updates of several volumes in one launch.  items: sequence of
    (desc, pdms, bounds, alpha, dist).  Returns the S masks, shape (count, 4)."""
    count = len(items)
    if not 1 <= count <= BATCH_MAX:
        raise ValueError(f"a batch holds 1..{BATCH_MAX} volumes, got {count}")
    arr = (BatchUpdate * count)()
    keep = []
    for k, (desc, pdms, bounds, alpha, dist) in enumerate(items):
        G = grid_of(desc)[3]
        b = _bounds(bounds)
        n = len(b) - 1
        a = _alpha(alpha, desc.levels)
        keep += [desc, b, a]
        arr[k].v = ctypes.pointer(desc)
        arr[k].d_pdms = _dev_ptr(pdms, n * G, "pdms")
        arr[k].h_bounds = _np_ptr(b)
        arr[k].n = n
        arr[k].h_alpha = _np_ptr(a)
        arr[k].d_dist = _dev_ptr(dist, G, "dist")
    masks = np.zeros((count, 4), np.uint64)
    _check(lib().pdm_batch_tf_update(arr, count, _np_ptr(masks), _stream(stream)),
           "pdm_batch_tf_update")
    del keep
    return masks


# Rows of pdm_batch_update packed without ctypes objects: the fixed part of a
# prepared volume (descriptor, PDMs, borders, n) once, the two per-call
# pointers (opacity table, output map) per launch.
_BATCH_FIXED = struct.Struct("<QQQi4x")
_BATCH_PTRS = struct.Struct("<QQ")
assert (BatchUpdate.v.offset, BatchUpdate.d_pdms.offset, BatchUpdate.h_bounds.offset,
        BatchUpdate.n.offset, BatchUpdate.h_alpha.offset, BatchUpdate.d_dist.offset,
        ctypes.sizeof(BatchUpdate)) == (0, 8, 16, 24, 32, 40, _BATCH_FIXED.size + _BATCH_PTRS.size)
# the same for pdm_batch_range_update: descriptor, PDMs, table, borders, n,
# max_level fixed; opacity table and output per launch
_RANGE_FIXED = struct.Struct("<QQQQii")
assert (BatchRangeUpdate.v.offset, BatchRangeUpdate.d_pdms.offset, BatchRangeUpdate.d_table.offset,
        BatchRangeUpdate.h_bounds.offset, BatchRangeUpdate.n.offset, BatchRangeUpdate.max_level.offset,
        BatchRangeUpdate.h_alpha.offset, BatchRangeUpdate.d_dist.offset,
        ctypes.sizeof(BatchRangeUpdate)) == (0, 8, 16, 24, 32, 36, 40, 48,
                                             _RANGE_FIXED.size + _BATCH_PTRS.size)
_F32 = np.dtype(np.float32)


class PreparedVolume:
    """The fixed part of a resident volume's batched-update item (descriptor,
    PDMs, partition borders), checked once so that a launch only adds the
    opacity tables and output maps.  The PDM tensor must stay alive and
    unchanged in place while the object is used."""
    __slots__ = ("desc", "levels", "G", "n", "bounds", "pdms", "fixed", "packed", "table",
                 "max_level", "table_ptr", "packed_ranges")

    def __init__(self, desc, pdms, bounds, table=None, max_level: int = 0):
        self.desc = desc
        self.levels = int(desc.levels)
        self.G = grid_of(desc)[3]
        self.bounds = _bounds(bounds)
        self.n = len(self.bounds) - 1
        if not 1 <= self.n <= 256:
            raise ValueError(f"1..256 partitions, got {self.n}")
        _dev_ptr(pdms, self.n * self.G, "pdms")
        self.pdms = pdms
        self.fixed = (ctypes.addressof(desc), pdms.data_ptr(), self.bounds.ctypes.data, self.n)
        self.packed = _BATCH_FIXED.pack(*self.fixed)
        # optional range table (for tf_update_ranges_prepared)
        self.max_level = int(max_level)
        maps = range_table_maps(self.n, self.max_level)
        self.table = table
        self.table_ptr = _dev_ptr(table, maps * self.G, "table") if maps > 0 else ctypes.c_void_p(0)
        self.packed_ranges = _RANGE_FIXED.pack(self.fixed[0], self.fixed[1], self.table_ptr.value or 0,
                                               self.fixed[2], self.n, self.max_level)


def _opacity_table(alpha, levels: int, what: str):
    """(array, host address) of `alpha` as C-contiguous float32 of `levels`
    entries; an array that already is one is used in place."""
    a = alpha
    if type(a) is not np.ndarray or a.dtype is not _F32 or not a.flags.c_contiguous:
        a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    if a.shape != (levels,):
        raise ValueError(f"{what} must hold {levels} float32 entries, got shape {a.shape}")
    if a.flags.writeable:  # the buffer protocol is the cheap route to the address
        return a, ctypes.addressof(ctypes.c_char.from_buffer(a))
    return a, a.ctypes.data


def batch_tf_update_prepared(entries, stream=None) -> np.ndarray:
    """batch_tf_update over prepared volumes.  entries: sequence of
    (PreparedVolume, alpha, dist): alpha holds the volume's `levels` opacities
    (float32), dist is a contiguous device tensor of G bytes.  Returns the S
    masks, shape (count, 4)."""
    count = len(entries)
    if not 1 <= count <= BATCH_MAX:
        raise ValueError(f"a batch holds 1..{BATCH_MAX} volumes, got {count}")
    rows, keep = [], []
    for k, (pv, alpha, dist) in enumerate(entries):
        a, ap = _opacity_table(alpha, pv.levels, f"alpha {k}")
        keep.append(a)
        if dist.nbytes != pv.G or not dist.is_cuda or not dist.is_contiguous():
            raise ValueError(f"dist {k}: expected a contiguous device tensor of {pv.G} bytes")
        rows.append(pv.packed + _BATCH_PTRS.pack(ap, dist.data_ptr()))
    arr = (BatchUpdate * count).from_buffer_copy(b"".join(rows))
    masks = np.zeros((count, 4), np.uint64)
    _check(lib().pdm_batch_tf_update(arr, count, _np_ptr(masks), _stream(stream)),
           "pdm_batch_tf_update")
    del keep
    return masks


def tf_update_ranges_prepared(pv, alpha, dist, stream=None) -> np.ndarray:
    """tf_update_ranges for a PreparedVolume that holds a range table;
    returns the S mask."""
    a, ap = _opacity_table(alpha, pv.levels, "alpha")
    if dist.nbytes != pv.G or not dist.is_cuda or not dist.is_contiguous():
        raise ValueError(f"dist: expected a contiguous device tensor of {pv.G} bytes")
    m = np.zeros(4, np.uint64)
    _, pd, b, n = pv.fixed
    _check(lib().pdm_tf_update_ranges(ctypes.byref(pv.desc), ctypes.c_void_p(pd), pv.table_ptr,
                                      ctypes.c_void_p(b), n, pv.max_level, ctypes.c_void_p(ap),
                                      ctypes.c_void_p(dist.data_ptr()), _np_ptr(m), _stream(stream)),
           "pdm_tf_update_ranges")
    return m


def batch_tf_update_ranges(items, stream=None) -> np.ndarray:
    """TF updates through range tables of several volumes in one launch (more
    when the covers' map lists need it).  items: sequence of (desc, pdms,
    table, bounds, max_level, alpha, dist); table may be None when the level
    count is 0.  Returns the S masks, shape (count, 4)."""
    count = len(items)
    if not 1 <= count <= BATCH_MAX:
        raise ValueError(f"a batch holds 1..{BATCH_MAX} volumes, got {count}")
    arr = (BatchRangeUpdate * count)()
    keep = []
    for k, (desc, pdms, table, bounds, max_level, alpha, dist) in enumerate(items):
        G = grid_of(desc)[3]
        b = _bounds(bounds)
        n = len(b) - 1
        a = _alpha(alpha, desc.levels)
        maps = range_table_maps(n, max_level)
        keep += [desc, b, a]
        arr[k].v = ctypes.pointer(desc)
        arr[k].d_pdms = _dev_ptr(pdms, n * G, "pdms")
        arr[k].d_table = _dev_ptr(table, maps * G, "table") if maps > 0 else None
        arr[k].h_bounds = _np_ptr(b)
        arr[k].n = n
        arr[k].max_level = int(max_level)
        arr[k].h_alpha = _np_ptr(a)
        arr[k].d_dist = _dev_ptr(dist, G, "dist")
    masks = np.zeros((count, 4), np.uint64)
    _check(lib().pdm_batch_tf_update_ranges(arr, count, _np_ptr(masks), _stream(stream)),
           "pdm_batch_tf_update_ranges")
    del keep
    return masks


def batch_tf_update_ranges_prepared(entries, stream=None) -> np.ndarray:
    """batch_tf_update_ranges over prepared volumes that hold range tables.
    entries: sequence of (PreparedVolume, alpha, dist).  Returns the S masks,
    shape (count, 4)."""
    count = len(entries)
    if not 1 <= count <= BATCH_MAX:
        raise ValueError(f"a batch holds 1..{BATCH_MAX} volumes, got {count}")
    rows, keep = [], []
    for k, (pv, alpha, dist) in enumerate(entries):
        a, ap = _opacity_table(alpha, pv.levels, f"alpha {k}")
        keep.append(a)
        if dist.nbytes != pv.G or not dist.is_cuda or not dist.is_contiguous():
            raise ValueError(f"dist {k}: expected a contiguous device tensor of {pv.G} bytes")
        rows.append(pv.packed_ranges + _BATCH_PTRS.pack(ap, dist.data_ptr()))
    arr = (BatchRangeUpdate * count).from_buffer_copy(b"".join(rows))
    masks = np.zeros((count, 4), np.uint64)
    _check(lib().pdm_batch_tf_update_ranges(arr, count, _np_ptr(masks), _stream(stream)),
           "pdm_batch_tf_update_ranges")
    del keep
    return masks


# ------------------------------------------------------------- batched build
def batch_workspace_bytes(count: int) -> int:
    return int(lib().pdm_batch_workspace_bytes(int(count)))


def _batch_volumes(items):
    """pdm_batch_volume rows for (desc, volume, bmin, bmax, bounds, pdms)
    items, and the host objects they point to (keep them alive)."""
    count = len(items)
    if not 1 <= count <= BATCH_MAX:
        raise ValueError(f"a batch holds 1..{BATCH_MAX} volumes, got {count}")
    arr = (BatchVolume * count)()
    keep = []
    for k, (desc, volume, bmin, bmax, bounds, pdms) in enumerate(items):
        G = grid_of(desc)[3]
        b = _bounds(bounds)
        n = len(b) - 1
        keep += [desc, b]
        arr[k].v = ctypes.pointer(desc)
        arr[k].d_volume = _dev_ptr(volume, _vox_bytes(desc), "volume")
        arr[k].d_bmin = _dev_ptr(bmin, G * desc.dtype, "bmin")
        arr[k].d_bmax = _dev_ptr(bmax, G * desc.dtype, "bmax")
        arr[k].h_bounds = _np_ptr(b)
        arr[k].n = n
        arr[k].d_pdms = _dev_ptr(pdms, n * G, "pdms")
    return arr, keep


def _batch_config(config):
    if config is None:
        return None
    return ctypes.pointer(BatchConfig(int(config.get("rows_per_item", 0)),
                                      int(config.get("lines_mult", 0)),
                                      int(config.get("largest_first", 0)),
                                      int(config.get("single_launch", 0))))


def batch_build(items, workspace, config=None, stream=None) -> None:
    """Bricks and PDMs of several volumes in three grouped launches.
    items: sequence of (desc, volume, bmin, bmax, bounds, pdms); workspace: a
    uint8 device tensor of batch_workspace_bytes(len(items)) bytes or more
    (it receives the descriptors; keep it until the stream has passed);
    config: None or dict(rows_per_item=, lines_mult=, largest_first=,
    single_launch=)."""
    arr, keep = _batch_volumes(items)
    count = len(items)
    need = batch_workspace_bytes(count)
    ws_bytes = workspace.numel() * workspace.element_size()
    if ws_bytes < need:
        raise ValueError(f"workspace holds {ws_bytes} bytes, needs {need}")
    _check(lib().pdm_batch_build(arr, count, _dev_ptr(workspace, ws_bytes, "workspace"),
                                 ws_bytes, _batch_config(config), _stream(stream)),
           "pdm_batch_build")
    del keep


def batch_build_noalloc(items, config=None, error=None, stream=None) -> None:
    """batch_build without a workspace: the library's static device array
    holds the descriptors and barrier state, nothing is allocated.  Calls on
    one device must not overlap in time.  error: None or a device tensor of
    4 bytes that receives the build's error word."""
    arr, keep = _batch_volumes(items)
    err = ctypes.c_void_p(0) if error is None else _dev_ptr(error, 4, "error")
    _check(lib().pdm_batch_build_noalloc(arr, len(items), _batch_config(config), err,
                                         _stream(stream)), "pdm_batch_build_noalloc")
    del keep


def batch_error(workspace) -> int:
    """The error word of a batch-build workspace (synchronises with the
    device): non-zero means a single-launch barrier wait gave up."""
    import torch
    return int(workspace[0:4].view(torch.int32).item())
