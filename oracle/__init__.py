"""CPU oracle for partitioned distance maps -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct C implementation (``pdm_oracle.c``) of what
the GPU library computes, wrapped with ctypes for numpy arrays.  Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import this
package.  It shares no code with the HIP library and never imports it.

Paper: arXiv 2407.21552, Sec. 3.1 (POMs, PDMs, the two update steps, Eq. 1),
Sec. 3.2 (uint8 clamp at 255), Sec. 2/4.2 (the plain method of Deakin and
Knackstedt: occupancy and distance map recomputed per transfer function).

Occupancy has two readings (see each function): RANGE (mode 0) tests the
brick's [min,max] interval, EXACT (mode 1) tests the brick's voxels.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pdm_oracle.c")
# PDM_ORACLE_LIB names a prebuilt oracle to load instead (the sanitizer test
# builds one with -fsanitize=address,undefined and runs the pins against it)
_LIB = os.environ.get("PDM_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
FLAGS = ["-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared"]
SANITIZE_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                  "-fno-sanitize-recover=undefined"]

RANGE = 0
EXACT = 1
CAP = 255


def build(force: bool = True, out: str = None, sanitize: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP) into ``oracle/liboracle.so`` (or
    `out`); with `sanitize`, instrumented for AddressSanitizer and
    UndefinedBehaviorSanitizer."""
    target = out or _LIB
    if force or not os.path.exists(target):
        tmp = target + ".tmp"
        flags = FLAGS + (SANITIZE_FLAGS if sanitize else [])
        subprocess.run(["gcc"] + flags + [_SRC, "-o", tmp], check=True)
        os.replace(tmp, target)
    return target


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if "PDM_ORACLE_LIB" not in os.environ and (
                not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int, ctypes.c_int64
        L.oracle_threads.restype = i32
        L.oracle_set_threads.argtypes = [i32]
        L.oracle_grid.argtypes = [i32, i32, i32, i32, P, P, P]
        L.oracle_bricks.argtypes = [P, i32, i32, i32, i32, i32, P, P]
        L.oracle_check_bounds.argtypes = [P, i32, i32]
        L.oracle_check_bounds.restype = i32
        L.oracle_pom_range.argtypes = [P, P, i64, i32, i32, P]
        L.oracle_pom_exact.argtypes = [P, i32, i32, i32, i32, i32, i32, i32, P]
        L.oracle_dt.argtypes = [P, i32, i32, i32, P]
        L.oracle_pdms.argtypes = [P, i32, i32, i32, i32, i32, P, P, P, i32, i32, i32, P]
        L.oracle_pdms.restype = i32
        L.oracle_active.argtypes = [P, i32, P, i32, P]
        L.oracle_active.restype = i32
        L.oracle_combine.argtypes = [P, i32, i64, P, P]
        L.oracle_plain_occ_range.argtypes = [P, P, i64, P, i32, P]
        L.oracle_plain_occ_range.restype = i32
        L.oracle_plain_occ_exact.argtypes = [P, i32, i32, i32, i32, i32, P, i32, P]
        L.oracle_plain_occ_exact.restype = i32
        L.oracle_full_recompute.argtypes = [P, i32, i32, i32, i32, i32, P, i32, i32, P]
        L.oracle_full_recompute.restype = i32
        _lib = L
    return _lib


def _p(a: np.ndarray) -> ctypes.c_void_p:
    assert a.flags["C_CONTIGUOUS"]
    return ctypes.c_void_p(a.ctypes.data)


def threads() -> int:
    return int(lib().oracle_threads())


def set_threads(t: int) -> None:
    lib().oracle_set_threads(int(t))


def grid(shape_zyx, b: int = 4):
    """Brick grid (Bz, By, Bx) of a volume of shape (nz, ny, nx) (Sec. 3.1)."""
    nz, ny, nx = shape_zyx
    out = [ctypes.c_int(), ctypes.c_int(), ctypes.c_int()]
    lib().oracle_grid(nx, ny, nz, b, *[ctypes.byref(o) for o in out])
    bx, by, bz = (o.value for o in out)
    return bz, by, bx


def _vol(vol: np.ndarray):
    assert vol.ndim == 3 and vol.dtype in (np.uint8, np.uint16)
    return np.ascontiguousarray(vol), vol.dtype.itemsize


def bricks(vol: np.ndarray, b: int = 4):
    """Per-brick (min, max) over in-volume voxels, as arrays of the volume's dtype."""
    vol, s = _vol(vol)
    g = grid(vol.shape, b)
    bmin = np.empty(g, np.uint16)
    bmax = np.empty(g, np.uint16)
    nz, ny, nx = vol.shape
    lib().oracle_bricks(_p(vol), s, nx, ny, nz, b, _p(bmin), _p(bmax))
    return bmin.astype(vol.dtype), bmax.astype(vol.dtype)


def check_bounds(bounds, levels: int) -> bool:
    b = np.ascontiguousarray(bounds, dtype=np.int32)
    return lib().oracle_check_bounds(_p(b), len(b) - 1, levels) == 0


def pom_range(bmin, bmax, lo: int, hi: int) -> np.ndarray:
    bmin = np.ascontiguousarray(bmin, np.uint16)
    bmax = np.ascontiguousarray(bmax, np.uint16)
    occ = np.empty(bmin.shape, np.uint8)
    lib().oracle_pom_range(_p(bmin), _p(bmax), bmin.size, lo, hi, _p(occ))
    return occ


def pom_exact(vol: np.ndarray, lo: int, hi: int, b: int = 4) -> np.ndarray:
    vol, s = _vol(vol)
    occ = np.empty(grid(vol.shape, b), np.uint8)
    nz, ny, nx = vol.shape
    lib().oracle_pom_exact(_p(vol), s, nx, ny, nz, b, lo, hi, _p(occ))
    return occ


def dt(occ: np.ndarray) -> np.ndarray:
    """Clamped chessboard distance transform of an occupancy grid (Bz, By, Bx)."""
    occ = np.ascontiguousarray(occ, dtype=np.uint8)
    bz, by, bx = occ.shape
    out = np.empty_like(occ)
    lib().oracle_dt(_p(occ), bx, by, bz, _p(out))
    return out


def pdms(vol, bounds, levels: int, mode: int = RANGE, b: int = 4, brick_minmax=None) -> np.ndarray:
    """All partitioned distance maps, shape (n, Bz, By, Bx), uint8."""
    vol, s = _vol(vol)
    bnd = np.ascontiguousarray(bounds, dtype=np.int32)
    n = len(bnd) - 1
    if brick_minmax is None:
        bmin, bmax = bricks(vol, b)
    else:
        bmin, bmax = brick_minmax
    bmin = np.ascontiguousarray(bmin, np.uint16)
    bmax = np.ascontiguousarray(bmax, np.uint16)
    g = grid(vol.shape, b)
    out = np.empty((n,) + g, np.uint8)
    nz, ny, nx = vol.shape
    rc = lib().oracle_pdms(_p(vol), s, nx, ny, nz, b, _p(bmin), _p(bmax), _p(bnd), n,
                           levels, mode, _p(out))
    if rc != 0:
        raise ValueError("invalid partition bounds")
    return out


def active(bounds, alpha, levels: int) -> np.ndarray:
    """S as a 4-word uint64 mask (bit p set when partition p is active)."""
    bnd = np.ascontiguousarray(bounds, dtype=np.int32)
    a = np.ascontiguousarray(alpha, dtype=np.float32)
    assert a.size >= levels
    m = np.zeros(4, np.uint64)
    if lib().oracle_active(_p(bnd), len(bnd) - 1, _p(a), levels, _p(m)) != 0:
        raise ValueError("invalid partition bounds")
    return m


def active_list(mask: np.ndarray, n: int):
    return [p for p in range(n) if (int(mask[p >> 6]) >> (p & 63)) & 1]


def combine(pdm_stack: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """Eq. 1: element-wise minimum of the PDMs selected by the mask."""
    pdm_stack = np.ascontiguousarray(pdm_stack, np.uint8)
    n = pdm_stack.shape[0]
    out = np.empty(pdm_stack.shape[1:], np.uint8)
    m = np.ascontiguousarray(mask, np.uint64)
    lib().oracle_combine(_p(pdm_stack), n, out.size, _p(m), _p(out))
    return out


def tf_update(pdm_stack, bounds, alpha, levels: int):
    """Both update steps: returns (D', S mask)."""
    m = active(bounds, alpha, levels)
    return combine(pdm_stack, m), m


def range_table(pdm_stack, max_level: int) -> np.ndarray:
    """The range-table maps, level after level (k = 1 .. K, K = min(max_level,
    floor(log2 n))): map T_k[p] is the element-wise min of PDMs p .. p+2^k-1,
    the distance map of the union of those partitions (the distance to a
    union is the min of the distances; Sec. 3.1).  Written from that
    definition, one np.min per map."""
    n = pdm_stack.shape[0]
    out = []
    k = 1
    while k <= max_level and (1 << k) <= n:
        w = 1 << k
        for p in range(n - w + 1):
            out.append(pdm_stack[p:p + w].min(axis=0))
        k += 1
    if not out:
        return np.zeros((0,) + pdm_stack.shape[1:], np.uint8)
    return np.stack(out)


def plain_occ_range(bmin, bmax, alpha, levels: int) -> np.ndarray:
    bmin = np.ascontiguousarray(bmin, np.uint16)
    bmax = np.ascontiguousarray(bmax, np.uint16)
    a = np.ascontiguousarray(alpha, dtype=np.float32)
    occ = np.empty(bmin.shape, np.uint8)
    if lib().oracle_plain_occ_range(_p(bmin), _p(bmax), bmin.size, _p(a), levels, _p(occ)):
        raise ValueError("a voxel is not below the number of levels")
    return occ


def plain_occ_exact(vol, alpha, levels: int, b: int = 4) -> np.ndarray:
    vol, s = _vol(vol)
    a = np.ascontiguousarray(alpha, dtype=np.float32)
    occ = np.empty(grid(vol.shape, b), np.uint8)
    nz, ny, nx = vol.shape
    if lib().oracle_plain_occ_exact(_p(vol), s, nx, ny, nz, b, _p(a), levels, _p(occ)):
        raise ValueError("a voxel is not below the number of levels")
    return occ


def full_recompute(vol, alpha, levels: int, mode: int = RANGE, b: int = 4) -> np.ndarray:
    """Plain method: distance map D recomputed from the raw volume."""
    vol, s = _vol(vol)
    a = np.ascontiguousarray(alpha, dtype=np.float32)
    out = np.empty(grid(vol.shape, b), np.uint8)
    nz, ny, nx = vol.shape
    if lib().oracle_full_recompute(_p(vol), s, nx, ny, nz, b, _p(a), levels, mode, _p(out)):
        raise ValueError("a voxel is not below the number of levels")
    return out
