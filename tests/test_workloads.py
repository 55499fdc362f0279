"""Seeded input generators: determinism and the stated value distributions."""
import numpy as np
import pytest

import workloads as W


def test_same_seed_same_bytes():
    a = W.make_volume("c1")
    b = W.make_volume("c1")
    assert a.dtype == np.uint8 and a.shape == (64, 64, 64)
    assert a.tobytes() == b.tobytes()
    t1 = W.make_tfs("c2", 3)
    t2 = W.make_tfs("c2", 3)
    for x, y in zip(t1, t2):
        assert x.dtype == np.float32 and x.shape == (4096,)
        assert x.tobytes() == y.tobytes()


def test_small_shapes_of_large_configs():
    v2 = W.make_volume("c2", shape=(20, 64, 48))
    assert v2.dtype == np.uint16 and v2.max() <= 4095
    assert (v2 == 4095).mean() > 0.03                     # salt noise
    v3 = W.make_volume("c3", shape=(60, 128, 96))
    assert v3.dtype == np.uint8 and v3.max() <= 255


def test_large_volume_is_mostly_empty():
    v3 = W.make_volume("c3")
    assert v3.shape == (795, 1024, 1024)
    assert (v3 < 10).mean() >= 0.9                        # 90% of voxels below 10


def test_tf_nonzero_set_is_open_interval():
    rng = np.random.default_rng(0)
    for L in (256, 4096):
        for _ in range(50):
            a = W.trapezoid_tf(L, 1, rng)
            nz = np.nonzero(a)[0]
            assert len(nz) >= 1
            assert (np.diff(nz) == 1).all()                # one contiguous run
            assert L // 32 - 1 <= len(nz) <= L // 4 - 1
            assert a.max() <= 1.0 and a.min() >= 0.0


def test_uniform_and_rhomin_bounds():
    b = W.uniform_bounds(4096, 32)
    assert b[0] == 0 and b[-1] == 4096 and (np.diff(b) == 128).all()
    r = W.rhomin_bounds(256, 32, 0)
    assert r[0] == 0 and r[1] == 1 and r[-1] == 256 and (np.diff(r) > 0).all()
    assert len(r) == 33


def test_stag_beetle_volume():
    a = W.stag_beetle_u8((62, 104, 104))
    b = W.stag_beetle_u8((62, 104, 104))
    assert a.dtype == np.uint8 and a.shape == (62, 104, 104)
    assert a.tobytes() == b.tobytes()
    zero = a == 0
    assert zero.mean() > 0.8                               # heavy rho_min mass
    assert (a > 120).mean() > 0.005                        # bright shell, mandibles, legs
    # the body is connected around the centre and the border is background
    assert a[31, 52, 52] > 0 and a[:, :, 0].max() <= 24
    assert W.stag_tfs(3)[0].shape == (256,)


@pytest.mark.parametrize("L,n,rho", [(256, 16, 0), (256, 256, 0), (4096, 128, 7), (256, 2, 0)])
def test_rhomin_bounds_tile_the_range(L, n, rho):
    r = W.rhomin_bounds(L, n, rho)
    assert len(r) == n + 1 and r[0] == 0 and r[1] == rho + 1 and r[-1] == L
    assert (np.diff(r) > 0).all()
    sizes = np.diff(r[1:])
    assert sizes.max() - sizes.min() <= 1                  # the rest split evenly
