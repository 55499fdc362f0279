"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws inputs: volumes, opacity tables and partition tables.
It holds none of the method's arithmetic (no brick reduction, occupancy,
distance or combine step), so the GPU library and the CPU oracle can both be
fed from it without sharing code.

The paper's datasets (manix 512x512x460, stag beetle 832x832x494, kingsnake
1024x1024x795; Table 1) and its transfer functions TF1-TF6 are not available;
these generators stand in for them with the same shapes and bit depths and
CT-like value distributions.  All randomness comes from
``numpy.random.default_rng(seed)`` (PCG64).

Volumes are numpy arrays of shape (nz, ny, nx), x fastest.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_CHUNK = 16  # z-slices per independently seeded noise chunk


def _chunk_map(fn, nz: int, seed: int, salt: int):
    """Run fn(z0, z1, rng) over z-chunks in threads.  Chunk i draws from its
    own generator, spawned from SeedSequence((seed, salt)), so the result does
    not depend on the thread count."""
    starts = list(range(0, nz, _CHUNK))
    seqs = np.random.SeedSequence((seed, salt)).spawn(len(starts))
    jobs = [(z0, min(nz, z0 + _CHUNK), np.random.default_rng(s)) for z0, s in zip(starts, seqs)]
    workers = max(1, min(8, os.cpu_count() or 1))
    with ThreadPoolExecutor(workers) as ex:
        list(ex.map(lambda j: fn(*j), jobs))

__all__ = [
    "CONFIGS", "ellipsoids_u8", "ct_like_u16", "tube_tree_u8", "make_volume",
    "trapezoid_tf", "make_tfs", "uniform_bounds", "rhomin_bounds", "config_info",
    "batch_specs", "batch_volume", "poisson_requests", "stag_beetle_u8", "STAG", "stag_tfs",
]

# name -> (shape (nz,ny,nx), dtype, levels L, partitions n, volume seed,
#          TF count, TF ramps (lo,hi), TF seed base)
CONFIGS = {
    "c1": dict(shape=(64, 64, 64), dtype=np.uint8, levels=256, n=8, seed=1,
               tfs=1, ramps=(2, 2), tf_seed=101),
    "c2": dict(shape=(460, 512, 512), dtype=np.uint16, levels=4096, n=32, seed=2,
               tfs=200, ramps=(1, 4), tf_seed=2000),
    "c3": dict(shape=(795, 1024, 1024), dtype=np.uint8, levels=256, n=64, seed=3,
               tfs=200, ramps=(1, 3), tf_seed=3000),
}


def config_info(name: str) -> dict:
    return dict(CONFIGS[name])


def _ellipsoid_fill(vol, center, semi, value):
    """Write `value` into the voxels of a solid axis-aligned ellipsoid."""
    nz, ny, nx = vol.shape
    cz, cy, cx = center
    az, ay, ax = semi
    z0, z1 = max(0, int(np.floor(cz - az))), min(nz, int(np.ceil(cz + az)) + 1)
    y0, y1 = max(0, int(np.floor(cy - ay))), min(ny, int(np.ceil(cy + ay)) + 1)
    x0, x1 = max(0, int(np.floor(cx - ax))), min(nx, int(np.ceil(cx + ax)) + 1)
    if z0 >= z1 or y0 >= y1 or x0 >= x1:
        return
    z = ((np.arange(z0, z1, dtype=np.float64) - cz) / az) ** 2
    y = ((np.arange(y0, y1, dtype=np.float64) - cy) / ay) ** 2
    x = ((np.arange(x0, x1, dtype=np.float64) - cx) / ax) ** 2
    inside = (z[:, None, None] + y[None, :, None] + x[None, None, :]) <= 1.0
    sub = vol[z0:z1, y0:y1, x0:x1]
    sub[inside] = value


def ellipsoids_u8(shape=(64, 64, 64), seed=1, count=6, semi=(4, 20), value=(30, 250),
                  sigma=3.0) -> np.ndarray:
    """Background 0, `count` solid ellipsoids (later ones overwrite earlier
    ones), Gaussian noise, rint, clip to [0,255]."""
    rng = np.random.default_rng(seed)
    vol = np.zeros(shape, np.float32)
    for _ in range(count):
        c = [rng.uniform(0, s) for s in shape]
        a = [int(rng.integers(semi[0], semi[1] + 1)) for _ in range(3)]
        v = int(rng.integers(value[0], value[1] + 1))
        _ellipsoid_fill(vol, c, a, v)
    if int(np.prod(shape)) <= (1 << 22):
        vol += rng.normal(0.0, sigma, size=shape).astype(np.float32)
        return np.clip(np.rint(vol), 0, 255).astype(np.uint8)
    out = np.empty(shape, np.uint8)

    def fill(z0, z1, r):
        sl = vol[z0:z1] + np.float32(sigma) * r.standard_normal(size=vol[z0:z1].shape,
                                                                  dtype=np.float32)
        out[z0:z1] = np.clip(np.rint(sl), 0, 255).astype(np.uint8)

    _chunk_map(fill, shape[0], seed, 2)
    return out


def ct_like_u16(shape=(460, 512, 512), seed=2, levels=4096, bones=20, salt=0.05) -> np.ndarray:
    """CT-like 12-bit volume in uint16: air rint(|N(0,8)|), a soft-tissue
    cylinder along z (radius 0.45 of the width, N(1000,40)), `bones` constant
    ellipsoids in 1800..3000 inside it, then salt noise (probability `salt`,
    value levels-1), clipped to [0, levels-1]."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    out = np.empty(shape, np.uint16)
    cy, cx = (ny - 1) / 2.0, (nx - 1) / 2.0
    rad = 0.45 * min(nx, ny)
    yy = (np.arange(ny, dtype=np.float32) - cy)[:, None]
    xx = (np.arange(nx, dtype=np.float32) - cx)[None, :]
    disk = (yy * yy + xx * xx) <= rad * rad
    # bone ellipsoids: centres inside the cylinder
    ells = []
    for _ in range(bones):
        r = rad * np.sqrt(rng.uniform(0, 0.8))
        th = rng.uniform(0, 2 * np.pi)
        c = (rng.uniform(0, nz), cy + r * np.sin(th), cx + r * np.cos(th))
        a = tuple(int(rng.integers(8, 61)) for _ in range(3))
        v = int(rng.integers(1800, 3001))
        ells.append((c, a, v))
    def fill(z0, z1, r):
        sl = np.abs(r.normal(0.0, 8.0, size=(z1 - z0, ny, nx)).astype(np.float32))
        tissue = r.normal(1000.0, 40.0, size=(z1 - z0, ny, nx)).astype(np.float32)
        sl = np.where(disk[None], tissue, sl)
        for (c, a, v) in ells:
            _ellipsoid_fill_slab(sl, z0, c, a, float(v))
        s = r.random(size=(z1 - z0, ny, nx), dtype=np.float32) < salt
        sl[s] = levels - 1
        out[z0:z1] = np.clip(np.rint(sl), 0, levels - 1).astype(np.uint16)

    _chunk_map(fill, nz, seed, 1)
    return out


def _ellipsoid_fill_slab(slab, z_off, center, semi, value):
    cz, cy, cx = center
    view_center = (cz - z_off, cy, cx)
    _ellipsoid_fill(slab, view_center, semi, value)


def _capsule_fill(vol, p0, p1, radius, value):
    """Write `value` into voxels within `radius` of segment p0-p1 (z,y,x order),
    clipped to the volume.  Works slice by slice on the slice's bounding box."""
    nz, ny, nx = vol.shape
    p0 = np.asarray(p0, np.float64)
    p1 = np.asarray(p1, np.float64)
    d = p1 - p0
    L2 = float(d @ d)
    zlo = max(0, int(np.floor(min(p0[0], p1[0]) - radius)))
    zhi = min(nz - 1, int(np.ceil(max(p0[0], p1[0]) + radius)))
    for z in range(zlo, zhi + 1):
        # segment parameters whose z lies within `radius` of this slice
        if abs(d[0]) > 1e-9:
            ta = (z - radius - p0[0]) / d[0]
            tb = (z + radius - p0[0]) / d[0]
            t0, t1 = max(0.0, min(ta, tb)), min(1.0, max(ta, tb))
        else:
            if abs(z - p0[0]) > radius:
                continue
            t0, t1 = 0.0, 1.0
        if t0 > t1:
            continue
        qa, qb = p0 + t0 * d, p0 + t1 * d
        y0 = max(0, int(np.floor(min(qa[1], qb[1]) - radius)))
        y1 = min(ny - 1, int(np.ceil(max(qa[1], qb[1]) + radius)))
        x0 = max(0, int(np.floor(min(qa[2], qb[2]) - radius)))
        x1 = min(nx - 1, int(np.ceil(max(qa[2], qb[2]) + radius)))
        if y0 > y1 or x0 > x1:
            continue
        ys = np.arange(y0, y1 + 1, dtype=np.float64)[:, None]
        xs = np.arange(x0, x1 + 1, dtype=np.float64)[None, :]
        rz, ry, rx = z - p0[0], ys - p0[1], xs - p0[2]
        t = (rz * d[0] + ry * d[1] + rx * d[2]) / L2 if L2 > 0 else np.zeros_like(ry + rx)
        t = np.clip(t, 0.0, 1.0)
        ez, ey, ex = rz - t * d[0], ry - t * d[1], rx - t * d[2]
        inside = (ez * ez + ey * ey + ex * ex) <= radius * radius
        sub = vol[z, y0:y1 + 1, x0:x1 + 1]
        sub[inside] = value


def tube_tree_u8(shape=(795, 1024, 1024), seed=3, tubes=40, length=(80, 400), radius=(2, 12),
                 value=(60, 240), sigma=2.0) -> np.ndarray:
    """Mostly empty uint8 volume holding a random tree of capsule tubes.  The
    first tube starts at a random interior point, every later one at a random
    point of an earlier tube; directions are uniform on the sphere.  Noise
    N(0, sigma) is added everywhere, then rint and clip to [0,255]."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    base = np.zeros(shape, np.uint8)
    segs = []
    for t in range(tubes):
        if t == 0:
            start = np.array([rng.uniform(0.25, 0.75) * s for s in shape])
        else:
            a, b = segs[int(rng.integers(0, len(segs)))]
            start = a + rng.uniform(0, 1) * (b - a)
        v = rng.normal(size=3)
        v /= np.linalg.norm(v)
        ln = rng.uniform(length[0], length[1])
        end = start + ln * v
        end = np.clip(end, 0, np.array(shape, np.float64) - 1)
        r = rng.uniform(radius[0], radius[1])
        val = int(rng.integers(value[0], value[1] + 1))
        segs.append((start, end))
        _capsule_fill(base, start, end, r, val)
    out = np.empty(shape, np.uint8)

    def fill(z0, z1, r):
        noise = r.standard_normal(size=(z1 - z0, ny, nx), dtype=np.float32)
        sl = base[z0:z1].astype(np.float32) + np.float32(sigma) * noise
        out[z0:z1] = np.clip(np.rint(sl), 0, 255).astype(np.uint8)

    _chunk_map(fill, nz, seed, 1)
    return out


def stag_beetle_u8(shape=(494, 832, 832), seed=7, sigma=6.0, speckle=2e-4) -> np.ndarray:
    """A stag-beetle-shaped uint8 volume whose background is exactly the
    minimum intensity 0, so most voxels sit at rho_min (the case the rho_min
    partition targets).  The beetle lies along y: head, thorax and abdomen
    are ellipsoids with a bright shell (170..230) around a darker interior
    (40..90); two curved mandibles (190..240), six two-segment legs
    (150..210) and two antennae are capsules.  Object voxels get N(0, sigma)
    noise and are clipped to [1, 255]; background voxels stay 0 except a
    sparse speckle (probability `speckle`, values 1..24)."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    base = np.zeros(shape, np.uint8)
    cz, cx = nz / 2.0, nx / 2.0
    parts = [(0.64, (0.30, 0.22, 0.21)), (0.42, (0.24, 0.10, 0.18)), (0.30, (0.19, 0.07, 0.14))]
    for fy, (sz, sy, sx) in parts:
        c = (cz, fy * ny, cx)
        semi = (sz * nz, sy * ny, sx * nx)
        _ellipsoid_fill(base, c, semi, int(rng.integers(170, 231)))
        _ellipsoid_fill(base, c, tuple(0.85 * a for a in semi), int(rng.integers(40, 91)))
    head_y = (0.30 - 0.07) * ny
    for side in (-1.0, 1.0):
        # mandible: three segments curving outwards then inwards
        p = np.array([cz, head_y + 0.02 * ny, cx + side * 0.06 * nx])
        val = int(rng.integers(190, 241))
        for dy, dx in ((-0.08, 0.05), (-0.07, 0.02), (-0.05, -0.04)):
            q = p + np.array([rng.uniform(-0.02, 0.02) * nz, dy * ny, side * dx * nx])
            _capsule_fill(base, p, q, rng.uniform(0.008, 0.012) * nx, val)
            p = q
        # antenna
        a0 = np.array([cz - 0.05 * nz, head_y + 0.03 * ny, cx + side * 0.08 * nx])
        a1 = a0 + np.array([-0.05 * nz, -0.10 * ny, side * 0.12 * nx])
        _capsule_fill(base, a0, a1, 0.003 * nx + 1.0, int(rng.integers(150, 211)))
        for fy in (0.40, 0.52, 0.66):
            # leg: from the body's side outwards and down, then back
            l0 = np.array([cz + 0.05 * nz, fy * ny, cx + side * 0.12 * nx])
            l1 = l0 + np.array([0.15 * nz, rng.uniform(-0.06, 0.06) * ny, side * 0.18 * nx])
            l2 = l1 + np.array([0.12 * nz, rng.uniform(-0.08, 0.08) * ny, side * 0.08 * nx])
            val = int(rng.integers(150, 211))
            rad = rng.uniform(0.004, 0.007) * nx + 1.0
            _capsule_fill(base, l0, np.clip(l1, 0, np.array(shape) - 1), rad, val)
            _capsule_fill(base, np.clip(l1, 0, np.array(shape) - 1), np.clip(l2, 0, np.array(shape) - 1),
                          0.8 * rad, val)
    out = np.empty(shape, np.uint8)

    def fill(z0, z1, r):
        b = base[z0:z1]
        obj = b > 0
        noisy = np.clip(np.rint(b.astype(np.float32)
                                + np.float32(sigma) * r.standard_normal(size=b.shape, dtype=np.float32)),
                        1, 255).astype(np.uint8)
        sl = np.where(obj, noisy, np.uint8(0))
        spk = (~obj) & (r.random(size=b.shape, dtype=np.float32) < speckle)
        sl[spk] = r.integers(1, 25, size=int(spk.sum()), dtype=np.uint8)
        out[z0:z1] = sl

    _chunk_map(fill, nz, seed, 3)
    return out


STAG = dict(shape=(494, 832, 832), dtype=np.uint8, levels=256, seed=7, rho_min=0,
            tfs=50, ramps=(1, 3), tf_seed=7000)


def stag_tfs(count: int = 50):
    """TFs for the stag-beetle volume: TF k from seed tf_seed + k, U{ramps}
    trapezoids."""
    out = []
    for k in range(count):
        rng = np.random.default_rng(STAG["tf_seed"] + k)
        r = int(rng.integers(STAG["ramps"][0], STAG["ramps"][1] + 1))
        out.append(trapezoid_tf(STAG["levels"], r, rng))
    return out


def make_volume(name: str, shape=None) -> np.ndarray:
    """The volume of a named configuration (optionally with another shape)."""
    c = CONFIGS[name]
    shp = tuple(shape) if shape is not None else c["shape"]
    if name == "c1":
        return ellipsoids_u8(shp, c["seed"])
    if name == "c2":
        return ct_like_u16(shp, c["seed"], c["levels"])
    if name == "c3":
        vol = tube_tree_u8(shp, c["seed"])
        return vol
    raise KeyError(name)


def batch_specs(count: int = 48, seed: int = 4, dims=(96, 640), parts=(16, 32, 64)):
    """The batched workload: `count` volumes with dims drawn from U{dims} per
    axis, the first half uint8 (ellipsoid recipe of the 64^3 volume, semi-axes
    scaled with the volume) and the second half 12-bit in uint16 (CT recipe),
    partition counts drawn from `parts`.  Returns a list of dicts with shape,
    dtype, levels, n and seed (volumes are made by batch_volume)."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        shape = tuple(int(rng.integers(dims[0], dims[1] + 1)) for _ in range(3))
        u8 = k < count // 2
        out.append(dict(shape=shape, dtype=np.uint8 if u8 else np.uint16,
                        levels=256 if u8 else 4096, n=int(rng.choice(parts)),
                        seed=10_000 * seed + k))
    return out


def batch_volume(spec: dict) -> np.ndarray:
    """The volume of one batch_specs entry."""
    shape = spec["shape"]
    if spec["dtype"] == np.uint8:
        scale = min(shape) / 64.0
        return ellipsoids_u8(shape, spec["seed"], semi=(max(1, int(4 * scale)), max(2, int(20 * scale))))
    return ct_like_u16(shape, spec["seed"], spec["levels"])


def trapezoid_tf(levels: int, ramps: int, rng: np.random.Generator) -> np.ndarray:
    """A 1-D opacity table of `levels` float32 entries made of `ramps` trapezoids
    combined by max, zero elsewhere.  Each trapezoid has integer corners
    a < b <= c < d with support width d-a drawn from U{L/32 .. L/4} and a
    height drawn from U(0.05, 1]; it rises linearly on (a,b), is flat on [b,c]
    and falls linearly on (c,d), so it is non-zero exactly on the open
    interval (a,d)."""
    L = levels
    alpha = np.zeros(L, np.float32)
    x = np.arange(L, dtype=np.float64)
    for _ in range(ramps):
        w = int(rng.integers(max(2, L // 32), max(3, L // 4) + 1))
        a = int(rng.integers(0, L - w))
        d = a + w
        b = a + int(rng.integers(1, w))          # a < b <= d-1
        c = int(rng.integers(b, d))              # b <= c <= d-1
        h = 1.0 - rng.uniform(0.0, 0.95)         # (0.05, 1]
        y = np.zeros(L)
        up = (x > a) & (x < b)
        y[up] = h * (x[up] - a) / (b - a)
        y[(x >= b) & (x <= c)] = h
        dn = (x > c) & (x < d)
        y[dn] = h * (d - x[dn]) / (d - c)
        alpha = np.maximum(alpha, y.astype(np.float32))
    return alpha


def make_tfs(name: str, count=None):
    """The transfer-function sequence of a configuration: TF k is drawn from
    seed tf_seed + k with U{ramps} trapezoids."""
    c = CONFIGS[name]
    k_count = c["tfs"] if count is None else count
    out = []
    for k in range(k_count):
        rng = np.random.default_rng(c["tf_seed"] + k)
        r = int(rng.integers(c["ramps"][0], c["ramps"][1] + 1))
        out.append(trapezoid_tf(c["levels"], r, rng))
    return out


def poisson_requests(rate_hz: float, seconds: float, vol_ids, levels_of, ramps=(1, 4), seed: int = 5,
                     tf_pool: int = 0, window=None):
    """A Poisson stream of TF-change requests: exponential inter-arrival gaps
    of mean 1/rate_hz over [0, seconds), each with a uniformly random volume id
    and a random trapezoid TF of U{ramps} ramps.  With `tf_pool` > 0 each
    volume draws its TFs from a pool of that many (the arrays are shared, so
    long high-rate streams stay small in host memory).  With window=(size,
    period_s) the id is drawn from `size` consecutive entries of vol_ids
    (wrapping around) that start at entry floor(t / period_s): the working
    set drifts by one volume per period, so a catalog larger than the
    server's slots sees a new volume, and an eviction, every period.
    Returns a list of (arrival seconds, volume id, opacity table)."""
    rng = np.random.default_rng(seed)
    vol_ids = list(vol_ids)
    pools = {}
    if tf_pool > 0:
        for v in vol_ids:
            pools[v] = [trapezoid_tf(levels_of[v], int(rng.integers(ramps[0], ramps[1] + 1)), rng)
                        for _ in range(tf_pool)]
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= seconds:
            break
        if window is None:
            v = vol_ids[int(rng.integers(0, len(vol_ids)))]
        else:
            size, period = window
            v = vol_ids[(int(t // period) + int(rng.integers(0, size))) % len(vol_ids)]
        if tf_pool > 0:
            alpha = pools[v][int(rng.integers(0, tf_pool))]
        else:
            alpha = trapezoid_tf(levels_of[v], int(rng.integers(ramps[0], ramps[1] + 1)), rng)
        out.append((t, v, alpha))
    return out


def uniform_bounds(levels: int, n: int) -> np.ndarray:
    """Partition table of n equal partitions over [0, L-1] (Sec. 3.1):
    bounds[p] = floor(p*L/n); partition p is [bounds[p], bounds[p+1]-1]."""
    return np.array([(p * levels) // n for p in range(n + 1)], np.int32)


def rhomin_bounds(levels: int, n: int, rho_min: int) -> np.ndarray:
    """A partition of its own for the intensities [0, rho_min] (Sec. 3.1 and
    Fig. 4), the rest [rho_min+1, L-1] split into n-1 equal partitions."""
    rest = levels - (rho_min + 1)
    assert n >= 2 and rest >= n - 1
    tail = [rho_min + 1 + (q * rest) // (n - 1) for q in range(n)]
    return np.array([0] + tail, np.int32)
