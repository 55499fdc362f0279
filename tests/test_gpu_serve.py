"""The server on the GPU: every result of a served Poisson stream (batched
with other volumes' requests, overlapping admissions and evictions) equals
the same update run alone, byte for byte; with the batched update of the
active PDMs and with updates through range tables.  A second case gives each
volume a pool of two output maps for streams of many requests per volume, so
maps are reused while launches overlap; each result is copied to the host
as the server retires its request and must still equal the update alone."""
import collections

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("range_level", [None, 6], ids=["batched", "range-tables"])
def test_served_results_equal_alone(orc, range_level):
    import torch
    import paper_2407_21552_amd as pdm
    from paper_2407_21552_amd.serve import GpuExecutor, Server, VolumeSpec, requests_from
    assert torch.cuda.is_available()
    rng = np.random.default_rng(7)
    specs = [((37, 29, 45), np.uint8, 256, 16), ((20, 24, 64), np.uint16, 4096, 32),
             ((64, 64, 64), np.uint8, 256, 64), ((30, 31, 33), np.uint8, 256, 8),
             ((9, 14, 30), np.uint16, 4096, 16), ((48, 40, 36), np.uint8, 256, 32)]
    vols, cat = {}, {}
    for k, (shape, dtype, L, n) in enumerate(specs):
        v = rng.integers(0, L, size=shape).astype(dtype)
        v[rng.random(shape) < 0.85] = 0
        vols[k] = v
        cat[k] = VolumeSpec(k, shape, dtype, L, W.uniform_bounds(L, n), lambda v=v: v)
    sched = requests_from(W.poisson_requests(5000.0, 0.06, list(cat), {k: cat[k].levels for k in cat},
                                             seed=11))
    per_vol = collections.Counter(r.vol_id for r in sched)
    ex = GpuExecutor(outputs_per_volume=max(per_vol.values()) + 1, range_level=range_level)
    srv = Server(ex, cat, budget_bytes=10**10, max_slots=4)   # 6 volumes, 4 slots: evictions
    print(f"[case] serving {len(sched)} requests over {len(cat)} volumes, range_level {range_level}",
          flush=True)
    srv.run(sched, timeout=60)
    torch.cuda.synchronize()
    rep = srv.report()
    print(rep, flush=True)
    assert rep["completed"] == len(sched) and rep["rejected"] == 0
    assert rep["evictions"] > 0 and rep["mean_batch"] > 1
    alone = {}
    for k, spec in cat.items():
        a = pdm.Volume(pdm.to_device(vols[k]), spec.levels, spec.bounds, voxel_dtype=spec.dtype)
        a.build()
        alone[k] = a
    out = None
    for r in srv.completed:
        a = alone[r.vol_id]
        out = torch.empty_like(a.dist)
        pdm.tf_update(a.desc, a.pdms, a.bounds, r.alpha, out)
        assert torch.equal(out.reshape(-1), r.result.reshape(-1)), f"request {r.req_id}"
    torch.cuda.synchronize()
    # and a few against the oracle
    for r in srv.completed[:5]:
        spec = cat[r.vol_id]
        want = orc.tf_update(orc.pdms(vols[r.vol_id], spec.bounds, spec.levels), spec.bounds,
                             r.alpha, spec.levels)[0]
        np.testing.assert_array_equal(pdm.from_device(r.result).reshape(want.shape), want)


@pytest.mark.parametrize("range_level", [None, 6], ids=["batched", "range-tables"])
def test_served_results_with_small_output_pool(orc, range_level):
    import torch
    import paper_2407_21552_amd as pdm
    from paper_2407_21552_amd.serve import GpuExecutor, Server, VolumeSpec, requests_from
    assert torch.cuda.is_available()
    rng = np.random.default_rng(17)
    specs = [((64, 64, 64), np.uint8, 256, 64), ((20, 24, 64), np.uint16, 4096, 32),
             ((48, 40, 36), np.uint8, 256, 32)]
    vols, cat = {}, {}
    for k, (shape, dtype, L, n) in enumerate(specs):
        v = rng.integers(0, L, size=shape).astype(dtype)
        v[rng.random(shape) < 0.85] = 0
        vols[k] = v
        cat[k] = VolumeSpec(k, shape, dtype, L, W.uniform_bounds(L, n), lambda v=v: v)
    sched = requests_from(W.poisson_requests(20000.0, 0.05, list(cat),
                                             {k: cat[k].levels for k in cat}, seed=19))
    per_vol = collections.Counter(r.vol_id for r in sched)
    assert min(per_vol.values()) > 20
    captured = {}
    ex = GpuExecutor(outputs_per_volume=2, range_level=range_level)
    srv = Server(ex, cat, budget_bytes=10**10, max_slots=3,
                 on_complete=lambda r: captured.__setitem__(r.req_id, r.result.cpu()))
    print(f"[case] serving {len(sched)} requests over {len(cat)} volumes with 2 outputs each, "
          f"range_level {range_level}", flush=True)
    srv.run(sched, timeout=60)
    torch.cuda.synchronize()
    rep = srv.report()
    print(rep, flush=True)
    assert rep["completed"] == len(sched) and rep["rejected"] == 0
    assert len(captured) == len(sched)
    alone = {}
    for k, spec in cat.items():
        a = pdm.Volume(pdm.to_device(vols[k]), spec.levels, spec.bounds, voxel_dtype=spec.dtype)
        a.build()
        alone[k] = a
    for r in srv.completed:
        a = alone[r.vol_id]
        out = torch.empty_like(a.dist)
        pdm.tf_update(a.desc, a.pdms, a.bounds, r.alpha, out)
        assert torch.equal(out.reshape(-1).cpu(), captured[r.req_id].reshape(-1)), f"request {r.req_id}"
