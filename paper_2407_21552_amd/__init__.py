"""Partitioned distance maps on MI355X (gfx950): a HIP library behind a C ABI.

Paper: "Accelerating Transfer Function Update for Distance Map based Volume
Rendering" (arXiv 2407.21552).  The C ABI is ``include/pdm.h``; ``_lib`` is
its ctypes binding; ``Volume`` keeps one volume's device buffers together:

    vol = Volume(t_volume_on_gpu, levels=256, bounds=uniform_bounds(256, 64))
    vol.build()                      # brick [min,max] + PDMs (one-time init)
    mask = vol.update_tf(alpha)      # D' (Eq. 1) into vol.dist
    vol.full_recompute(alpha, out)   # plain method, D

PyTorch is used for device memory and streams only.
"""
from __future__ import annotations

import numpy as np

from . import _lib
from ._lib import (BATCH_MAX, BRICK, DIST_CAP, MAX_PARTITIONS, PdmError, PreparedVolume,
                   active_set, batch_build, batch_build_noalloc, batch_error, batch_tf_update,
                   batch_tf_update_prepared, batch_workspace_bytes, build_bricks, build_range_table, range_cover,
                   range_table_maps, tf_update_ranges, tf_update_ranges_prepared,
                   batch_tf_update_ranges, batch_tf_update_ranges_prepared,
                   build_partitions, build_partitions_exact, distance_yz, full_recompute,
                   full_recompute_cached, full_recompute_exact, plain_cached_distance_x, grid_of, mask_to_list, plain_distance_x,
                   plain_exact_distance_x, pom_distance_x, pom_exact_distance_x, tf_update,
                   volume_desc)

__all__ = ["Volume", "PdmError", "PreparedVolume", "active_set", "batch_build",
           "batch_build_noalloc", "batch_error",
           "batch_tf_update", "batch_tf_update_prepared", "batch_workspace_bytes", "BATCH_MAX",
           "build_bricks", "build_partitions", "build_range_table", "range_cover",
           "range_table_maps", "tf_update_ranges", "tf_update_ranges_prepared",
           "batch_tf_update_ranges", "batch_tf_update_ranges_prepared",
           "build_partitions_exact", "distance_yz", "full_recompute", "full_recompute_cached",
           "full_recompute_exact", "plain_cached_distance_x",
           "grid_of", "mask_to_list", "plain_distance_x", "plain_exact_distance_x",
           "pom_distance_x", "pom_exact_distance_x", "tf_update", "volume_desc", "BRICK",
           "DIST_CAP", "MAX_PARTITIONS", "to_device", "from_device", "RANGE", "EXACT"]

RANGE = "range"  # occupancy from the brick's [min, max] interval
EXACT = "exact"  # occupancy from the brick's voxels (Sec. 3.1 wording)


def to_device(arr: np.ndarray, device="cuda"):
    """Copy a uint8/uint16 numpy array to the GPU (uint16 travels as int16
    bits; the library only sees bytes)."""
    import torch
    a = np.ascontiguousarray(arr)
    if a.dtype == np.uint16:
        a = a.view(np.int16)
    return torch.from_numpy(a).to(device)


def from_device(t, dtype=None) -> np.ndarray:
    a = t.detach().cpu().numpy()
    if dtype is not None and np.dtype(dtype) == np.uint16:
        a = a.view(np.uint16)
    return a


class Volume:
    """One volume resident on the GPU with its bricks, PDMs and output map.

    t_volume: contiguous (nz, ny, nx) tensor of uint8, or int16 holding the
    bits of uint16 intensities (dtype given by `voxel_dtype`).  `mode` selects
    the occupancy reading of both the PDMs and the plain method: RANGE (brick
    [min, max]) or EXACT (brick voxels)."""

    def __init__(self, t_volume, levels: int, bounds, voxel_dtype=None, mode: str = RANGE):
        import torch
        if mode not in (RANGE, EXACT):
            raise ValueError(f"mode must be {RANGE!r} or {EXACT!r}")
        self.mode = mode
        if voxel_dtype is None:
            voxel_dtype = np.uint8 if t_volume.dtype == torch.uint8 else np.uint16
        self.voxel_dtype = np.dtype(voxel_dtype)
        self.volume = t_volume
        self.levels = int(levels)
        self.bounds = np.ascontiguousarray(bounds, dtype=np.int32)
        self.n = len(self.bounds) - 1
        self.desc = volume_desc(t_volume.shape, self.voxel_dtype, levels)
        self.bz, self.by, self.bx, self.G = grid_of(self.desc)
        tdt = torch.uint8 if self.voxel_dtype.itemsize == 1 else torch.int16
        dev = t_volume.device
        self.bmin = torch.empty((self.bz, self.by, self.bx), dtype=tdt, device=dev)
        self.bmax = torch.empty_like(self.bmin)
        self.pdms = torch.empty((self.n, self.bz, self.by, self.bx), dtype=torch.uint8, device=dev)
        self.dist = torch.empty((self.bz, self.by, self.bx), dtype=torch.uint8, device=dev)
        self.range_err = torch.zeros(1, dtype=torch.int32, device=dev)

    @property
    def pdm_bytes(self) -> int:
        return self.n * self.G

    def build(self, stream=None) -> None:
        """One-time initialisation: brick [min,max], then every PDM."""
        build_bricks(self.desc, self.volume, self.bmin, self.bmax, self.range_err, stream)
        if self.mode == EXACT:
            build_partitions_exact(self.desc, self.volume, self.bounds, self.pdms, stream)
        else:
            build_partitions(self.desc, self.bmin, self.bmax, self.bounds, self.pdms, stream)

    def build_range_table(self, max_level: int = 8, stream=None) -> None:
        """Allocate and build the range table over this volume's PDMs (call
        after build()); update_tf_ranges then reads the covering maps."""
        import torch
        self.range_level = int(max_level)
        maps = range_table_maps(self.n, self.range_level)
        self.table = (torch.empty((maps, self.bz, self.by, self.bx), dtype=torch.uint8,
                                  device=self.pdms.device) if maps > 0 else None)
        build_range_table(self.desc, self.pdms, self.n, self.range_level, self.table, stream)
        self._prepared = None

    def update_tf_ranges(self, alpha, out=None, stream=None) -> np.ndarray:
        """update_tf through the range table (same D' and S mask)."""
        return tf_update_ranges(self.desc, self.pdms, self.table, self.bounds, self.range_level,
                                alpha, self.dist if out is None else out, stream)

    @property
    def prepared(self) -> PreparedVolume:
        """This volume's fixed update fields (built once; with the range table
        when build_range_table has run)."""
        if getattr(self, "_prepared", None) is None:
            self._prepared = PreparedVolume(self.desc, self.pdms, self.bounds,
                                            getattr(self, "table", None),
                                            getattr(self, "range_level", 0))
        return self._prepared

    def check_range(self) -> None:
        """Synchronises; raises PdmError if some voxel was >= levels."""
        if int(self.range_err.item()) != 0:
            raise PdmError(_lib.PDM_E_RANGE, "volume holds a voxel >= levels")

    def update_tf(self, alpha, out=None, stream=None) -> np.ndarray:
        """D' for a new opacity table; returns the S mask."""
        return tf_update(self.desc, self.pdms, self.bounds, alpha,
                         self.dist if out is None else out, stream)

    def full_recompute(self, alpha, out=None, stream=None) -> None:
        """Plain method: D from the raw volume."""
        fn = full_recompute_exact if self.mode == EXACT else full_recompute
        fn(self.desc, self.volume, alpha, self.dist if out is None else out, stream)

    def full_recompute_cached(self, alpha, out=None, stream=None) -> None:
        """Plain method from the cached brick [min, max] (RANGE reading; call
        after build()): the same D as full_recompute."""
        if self.mode != RANGE:
            raise ValueError("the cached-range plain method exists in the RANGE reading only")
        full_recompute_cached(self.desc, self.bmin, self.bmax, alpha,
                              self.dist if out is None else out, stream)
