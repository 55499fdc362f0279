"""The allocation-free batched build (pdm_batch_build_noalloc) against the
batched build with a caller workspace (pdm_batch_build), bit-exact.

Two calls in a row share the library's static scratch array, the second
with fewer and smaller volumes, in both launch kinds (three grouped
launches, one cooperative launch); the second call must not see anything
left over from the first.
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


def blocky(shape, dtype, levels, seed, keep=0.15, cell=3):
    rng = np.random.default_rng(seed)
    cz, cy, cx = [(s + cell - 1) // cell for s in shape]
    cells = rng.integers(0, levels, size=(cz, cy, cx))
    cells = np.where(rng.random((cz, cy, cx)) < keep, cells, 0)
    v = np.repeat(np.repeat(np.repeat(cells, cell, 0), cell, 1), cell, 2)
    return np.ascontiguousarray(v[:shape[0], :shape[1], :shape[2]]).astype(dtype)


def _volumes(pdm, specs, seed):
    out = []
    for k, (shape, dtype, L, n) in enumerate(specs):
        vol = blocky(shape, dtype, L, seed=seed + k)
        bounds = W.uniform_bounds(L, n)
        a = pdm.Volume(pdm.to_device(vol), L, bounds, voxel_dtype=dtype)
        b = pdm.Volume(a.volume, L, bounds, voxel_dtype=dtype)
        out.append((a, b, bounds))
    return out


def _items(vols, which):
    return [(v.desc, v.volume, v.bmin, v.bmax, bounds, v.pdms)
            for (v, bounds) in ((t[which], t[2]) for t in vols)]


FIRST = [((37, 29, 45), np.uint8, 256, 16), ((20, 24, 64), np.uint16, 4096, 32),
         ((30, 31, 33), np.uint8, 256, 200), ((3, 9, 1021), np.uint8, 256, 5),
         ((1021, 5, 6), np.uint16, 4096, 4), ((64, 64, 64), np.uint8, 256, 64)]
SECOND = [((9, 14, 30), np.uint8, 256, 8), ((5, 6, 7), np.uint16, 4096, 3)]


@pytest.mark.parametrize("config", [None, dict(single_launch=1, lines_mult=2, largest_first=1)],
                         ids=["grouped", "single-launch"])
def test_noalloc_build_equals_workspace_build(pdm, config):
    import torch
    for call, (specs, seed) in enumerate([(FIRST, 900), (SECOND, 950)]):
        print(f"[case] no-alloc batch build, call {call}, {len(specs)} volumes, config {config}",
              flush=True)
        vols = _volumes(pdm, specs, seed)
        # poison the outputs so that anything left unwritten shows
        for a, b, _ in vols:
            for t in (a.pdms, b.pdms):
                t.fill_(0x5A)
        ws = torch.empty(pdm.batch_workspace_bytes(len(specs)), dtype=torch.uint8, device="cuda")
        err = torch.full((1,), 7, dtype=torch.int32, device="cuda")
        pdm.batch_build(_items(vols, 1), ws, config)
        pdm.batch_build_noalloc(_items(vols, 0), config, error=err)
        torch.cuda.synchronize()
        assert pdm.batch_error(ws) == 0
        assert int(err.item()) == 0
        for k, (a, b, _) in enumerate(vols):
            assert torch.equal(a.bmin, b.bmin), f"call {call} volume {k}: bmin"
            assert torch.equal(a.bmax, b.bmax), f"call {call} volume {k}: bmax"
            assert torch.equal(a.pdms, b.pdms), f"call {call} volume {k}: PDMs"


def test_noalloc_rejects_more_volumes_than_the_scratch_holds(pdm):
    import torch
    vols = _volumes(pdm, [((5, 6, 7), np.uint8, 256, 2)], 990)
    items = _items(vols, 0) * (pdm.BATCH_MAX + 1)
    with pytest.raises(ValueError):
        pdm.batch_build_noalloc(items)
    # through the C ABI directly: PDM_E_INVAL, nothing launched
    arr, keep = pdm._lib._batch_volumes(items[:1])
    rc = pdm._lib.lib().pdm_batch_build_noalloc(arr, pdm.BATCH_MAX + 1, None, None, None)
    assert rc == pdm._lib.PDM_E_INVAL
    torch.cuda.synchronize()
