// pdm_kernels.hip -- gfx950 kernels for partitioned distance maps.
//
// Paper: arXiv 2407.21552.  Sec. 3.1 defines the brick reduction (b = 4), the
// partitioned occupancy maps (POMs), the partitioned distance maps (PDMs,
// chessboard distance in bricks) and the update D' = min over p in S of PDM_p
// (Eq. 1); Sec. 3.2 stores distances as uint8 clamped at 255; Sec. 2 and 4.2
// describe the plain method (occupancy and distance map recomputed per TF).
//
// Everything here is integer byte work bound by HBM bandwidth or by the
// per-line scans; there is no dense contraction, so no MFMA.
//
// Kernels
//   k_bricks        volume -> per-brick [min,max]; one lane per 4 bricks in x
//                   (16 voxels = one 16-byte load per voxel row for u8).
//   k_pom_x         [min,max] -> for every partition, the POM and the distance
//                   to the nearest occupied brick along x (wave ballots).
//   k_plain_x       volume + TF -> occupancy and x distance (plain method).
//   k_plain_cached_x cached [min,max] + TF -> occupancy and x distance (the
//                   plain method without reading the volume).
//   k_dist_lines    x distances -> full chessboard distances: 1-D max-min
//                   pass along y or z, one lane per line, linear-time scan,
//                   the line in registers (many lines: all maps of a grid);
//                   on lines under 255 bricks the values are clamped to the
//                   line length and the table sized to it.
//   k_dist_pairs    the same pass with two lanes per line (forward and
//                   backward halves at once; few lines: one map).
//   k_dist_global   the same pass on global memory (lines over 256 bricks,
//                   or offsets past 31 bits).
//   k_dist_axis, k_dist_split  the same pass with lines staged in LDS (lines
//                   of at most 16 bricks).
//   k_combine       min over a list of G-byte maps (the active PDMs, or the
//                   range-table maps covering them), 16 bytes per lane.
//   k_range_level   one level of the range table: min of two maps.
//   k_batch_combine the TF updates of up to 48 volumes in one launch.
//   k_batch_combine_maps  the same through range tables (a map list each).
//   k_batch_rows, k_batch_scan, k_batch_single
//                   batched build of up to 48 volumes: grouped launches per
//                   phase, or one cooperative launch with grid barriers.
//   k_pom_exact_x   EXACT reading: per-brick partition masks from the voxels,
//                   then the x distances of every partition.
//   k_plain_exact_x EXACT reading of the plain method's occupancy.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <mutex>

#include "pdm_launch.h"

namespace pdm {

constexpr int kWave = 64;
constexpr int kSegBricks = 4 * kWave;  // bricks of one x segment handled by a wave
constexpr int kNone = 1 << 20;         // "no occupied brick": farther than any cap

typedef unsigned short us2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pk_min16(uint32_t a, uint32_t b) {
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_min(__builtin_bit_cast(us2, a),
                                                                  __builtin_bit_cast(us2, b)));
}
__device__ __forceinline__ uint32_t pk_max16(uint32_t a, uint32_t b) {
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(us2, a),
                                                                  __builtin_bit_cast(us2, b)));
}
// bytes 0 and 2 of w in the two 16-bit halves
__device__ __forceinline__ uint32_t even_bytes(uint32_t w) { return w & 0x00FF00FFu; }
// bytes 1 and 3 of w in the two 16-bit halves
__device__ __forceinline__ uint32_t odd_bytes(uint32_t w) {
    return __builtin_amdgcn_perm(0u, w, 0x0c030c01u);
}
__device__ __forceinline__ uint32_t lo16(uint32_t w) { return w & 0xFFFFu; }
__device__ __forceinline__ uint32_t hi16(uint32_t w) { return w >> 16; }
__device__ __forceinline__ uint32_t umin(uint32_t a, uint32_t b) { return a < b ? a : b; }
__device__ __forceinline__ uint32_t umax(uint32_t a, uint32_t b) { return a > b ? a : b; }

// ---------------------------------------------------------------------------
// Brick [min,max] of the 4 bricks x = 4q..4q+3 of brick row (bz, by):
// voxels x in [16q, 16q+16), y in [4by, 4by+4), z in [4bz, 4bz+4), clipped to
// the volume.  Results for bricks outside the grid are unspecified.
// ---------------------------------------------------------------------------
// 16 bytes from any byte address: one vector load (the hardware serves
// unaligned vector loads), so voxel rows of any width and offset stream in
// 16-byte pieces.
__device__ __forceinline__ uint4 load16(const void* p) {
    uint4 w;
    __builtin_memcpy(&w, p, 16);
    return w;
}

// Pointers typed in the global address space.  Kernel arguments are known to
// be global; pointers read from a descriptor are not, and would compile to
// flat accesses, which also count against the LDS wait counter and so stall
// the LDS-paced scan loops.  The batched kernels cast their descriptor
// pointers to these types; the helpers below take either kind.
#define PDM_GLB __attribute__((address_space(1)))

__device__ __forceinline__ uint4 load16(const PDM_GLB void* p) {
    uint4 w;
    __builtin_memcpy(&w, p, 16);
    return w;
}

// 16 bytes from any byte address, non-temporal: voxels are streamed once per
// pass and the volume does not fit in the caches, so they should not evict
// what does.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef u32x4 u32x4_u __attribute__((aligned(1)));

__device__ __forceinline__ u32x4 load16_nt(const void* p) {
    return __builtin_nontemporal_load(reinterpret_cast<const u32x4_u*>(p));
}
__device__ __forceinline__ u32x4 load16_nt(const PDM_GLB void* p) {
    return __builtin_nontemporal_load(reinterpret_cast<const PDM_GLB u32x4_u*>(p));
}

template <typename T>
struct QuadMinMax {
    uint32_t mn[4], mx[4];
};

// 4 and 8 bytes from any byte address (one load each; see load16).
template <typename VP>
__device__ __forceinline__ uint32_t load4(VP p) {
    uint32_t w;
    __builtin_memcpy(&w, p, 4);
    return w;
}
template <typename VP>
__device__ __forceinline__ uint2 load8(VP p) {
    uint2 w;
    __builtin_memcpy(&w, p, 8);
    return w;
}

// The quad's 16 voxel rows, x in [x0, x0 + 16) inside the row: row i is
// (z0 + i/4, y0 + i%4).  With CLAMP (a brick layer cut by the volume's end
// in z or y) rows past the volume repeat its last row, which never changes a
// brick's min or max; every load is issued before the first use.
template <typename T, bool CLAMP, typename VP>
__device__ __forceinline__ QuadMinMax<T> quad_whole_rows(VP __restrict__ vol, int nx, int ny,
                                                         int z0, int y0, int zn, int yn, int x0) {
    QuadMinMax<T> r;
    const int64_t base = ((int64_t)z0 * ny + y0) * nx + x0;
    auto off = [&](int i) -> int64_t {
        const int zz = CLAMP ? min(i >> 2, zn - 1) : (i >> 2);
        const int yy = CLAMP ? min(i & 3, yn - 1) : (i & 3);
        return base + ((int64_t)zz * ny + yy) * nx;
    };
    if constexpr (sizeof(T) == 1) {
        u32x4 w[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) w[i] = load16_nt(vol + off(i));
        // even/odd byte lanes held as packed u16 pairs, one pair per brick
        uint32_t mnE[4], mnO[4], mxE[4], mxO[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) { mnE[k] = mnO[k] = 0xFFFFFFFFu; mxE[k] = mxO[k] = 0u; }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const uint32_t ws[4] = {w[i].x, w[i].y, w[i].z, w[i].w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t e = even_bytes(ws[k]), o = odd_bytes(ws[k]);
                mnE[k] = pk_min16(mnE[k], e);
                mnO[k] = pk_min16(mnO[k], o);
                mxE[k] = pk_max16(mxE[k], e);
                mxO[k] = pk_max16(mxO[k], o);
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t a = pk_min16(mnE[k], mnO[k]);
            const uint32_t b = pk_max16(mxE[k], mxO[k]);
            r.mn[k] = umin(lo16(a), hi16(a));
            r.mx[k] = umax(lo16(b), hi16(b));
        }
    } else {
        // u16: 32 bytes per row; two rounds of 8 rows (16 loads each)
        uint32_t mn[4], mx[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) { mn[k] = 0xFFFFFFFFu; mx[k] = 0u; }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            u32x4 w[16];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int64_t o = off(8 * h + i);
                w[2 * i] = load16_nt(vol + o);
                w[2 * i + 1] = load16_nt(vol + o + 8);
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const uint32_t ws[8] = {w[2 * i].x, w[2 * i].y, w[2 * i].z, w[2 * i].w,
                                        w[2 * i + 1].x, w[2 * i + 1].y, w[2 * i + 1].z, w[2 * i + 1].w};
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    mn[k] = pk_min16(mn[k], pk_min16(ws[2 * k], ws[2 * k + 1]));
                    mx[k] = pk_max16(mx[k], pk_max16(ws[2 * k], ws[2 * k + 1]));
                }
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            r.mn[k] = umin(lo16(mn[k]), hi16(mn[k]));
            r.mx[k] = umax(lo16(mx[k]), hi16(mx[k]));
        }
    }
    return r;
}

// The quad's rows when its 16 voxels run past the row end (nx >= 4): brick
// k's 4 voxels are loaded at min(x0 + 4k, nx - 4), so every load stays in
// the row; when that start is pulled back, its first voxels belong to the
// brick before and are masked out (to the maximum value for the min, to 0
// for the max).  Bricks wholly past the row end get unspecified results.
// Rows past the volume repeat its last row, as above.
template <typename T, typename VP>
__device__ __forceinline__ QuadMinMax<T> quad_ragged_rows(VP __restrict__ vol, int nx, int ny,
                                                          int z0, int y0, int zn, int yn, int x0) {
    QuadMinMax<T> r;
    const int64_t base = ((int64_t)z0 * ny + y0) * nx;
    int pos[4];
    uint32_t mlo[4], mhi[4];  // voxels of the brick before: bits set in the loaded words
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int x = x0 + 4 * k;
        pos[k] = min(x, nx - 4);
        const int lead = min(x - pos[k], 3);
        const uint64_t m = lead ? (~0ull >> (64 - 8 * (int)sizeof(T) * lead)) : 0ull;
        mlo[k] = (uint32_t)m;
        mhi[k] = (uint32_t)(m >> 32);
    }
    // one brick (its 16 row loads in flight) at a time: few registers, so the
    // callers keep the occupancy their whole-quad path sets
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        uint32_t mnA = 0xFFFFFFFFu, mnB = 0xFFFFFFFFu, mxA = 0u, mxB = 0u;
        typename std::conditional<sizeof(T) == 1, uint32_t, uint2>::type w[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int64_t row = base + ((int64_t)min(i >> 2, zn - 1) * ny + min(i & 3, yn - 1)) * nx;
            if constexpr (sizeof(T) == 1)
                w[i] = load4(vol + row + pos[k]);
            else
                w[i] = load8(vol + row + pos[k]);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            if constexpr (sizeof(T) == 1) {
                const uint32_t lo = w[i] | mlo[k], hi = w[i] & ~mlo[k];
                mnA = pk_min16(mnA, even_bytes(lo));
                mnB = pk_min16(mnB, odd_bytes(lo));
                mxA = pk_max16(mxA, even_bytes(hi));
                mxB = pk_max16(mxB, odd_bytes(hi));
            } else {
                mnA = pk_min16(mnA, pk_min16(w[i].x | mlo[k], w[i].y | mhi[k]));
                mxA = pk_max16(mxA, pk_max16(w[i].x & ~mlo[k], w[i].y & ~mhi[k]));
            }
        }
        const uint32_t a = pk_min16(mnA, mnB);
        const uint32_t b = pk_max16(mxA, mxB);
        r.mn[k] = umin(lo16(a), hi16(a));
        r.mx[k] = umax(lo16(b), hi16(b));
        __builtin_amdgcn_sched_barrier(0);  // the next brick's loads stay below
    }
    return r;
}

// The quad's rows one at a time (a brick layer cut in z or y): few registers.
template <typename T, typename VP>
__device__ __forceinline__ QuadMinMax<T> quad_rows_looped(VP __restrict__ vol, int nx, int ny,
                                                          int z0, int y0, int zn, int yn, int x0) {
    QuadMinMax<T> r;
    if constexpr (sizeof(T) == 1) {
        // even/odd byte lanes held as packed u16 pairs, one pair per brick
        uint32_t mnE[4], mnO[4], mxE[4], mxO[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) { mnE[k] = mnO[k] = 0xFFFFFFFFu; mxE[k] = mxO[k] = 0u; }
        for (int zz = 0; zz < zn; ++zz) {
#pragma unroll
            for (int yy = 0; yy < 4; ++yy) {
                if (yy < yn) {
                    const int64_t off = ((int64_t)(z0 + zz) * ny + (y0 + yy)) * nx + x0;
                    const uint4 w = load16(vol + off);
                    const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const uint32_t e = even_bytes(ws[k]), o = odd_bytes(ws[k]);
                        mnE[k] = pk_min16(mnE[k], e);
                        mnO[k] = pk_min16(mnO[k], o);
                        mxE[k] = pk_max16(mxE[k], e);
                        mxO[k] = pk_max16(mxO[k], o);
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t a = pk_min16(mnE[k], mnO[k]);
            const uint32_t b = pk_max16(mxE[k], mxO[k]);
            r.mn[k] = umin(lo16(a), hi16(a));
            r.mx[k] = umax(lo16(b), hi16(b));
        }
    } else {
        // u16: each 32-bit word holds 2 voxels; 2 words per brick row
        uint32_t mn[4], mx[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) { mn[k] = 0xFFFFFFFFu; mx[k] = 0u; }
        for (int zz = 0; zz < zn; ++zz) {
#pragma unroll
            for (int yy = 0; yy < 4; ++yy) {
                if (yy < yn) {
                    const int64_t off = ((int64_t)(z0 + zz) * ny + (y0 + yy)) * nx + x0;
                    const uint4 a = load16(vol + off), b = load16(vol + off + 8);
                    const uint32_t ws[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        mn[k] = pk_min16(mn[k], pk_min16(ws[2 * k], ws[2 * k + 1]));
                        mx[k] = pk_max16(mx[k], pk_max16(ws[2 * k], ws[2 * k + 1]));
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            r.mn[k] = umin(lo16(mn[k]), hi16(mn[k]));
            r.mx[k] = umax(lo16(mx[k]), hi16(mx[k]));
        }
    }
    return r;
}

// Brick [min,max] of the quad.  FAST_EDGES: quads at the volume's edges (a
// brick layer cut in z or y, 16 voxels that run past the row end) take the
// unrolled paths above; otherwise compact looped ones, for a caller whose
// register budget must stay that of the whole-quad path (with the unrolled
// edge paths inlined, the compiler schedules the plain x pass for 190
// registers instead of 97, which halves its occupancy on whole rows).
template <typename T, bool FAST_EDGES = true, typename VP>
__device__ __forceinline__ QuadMinMax<T> quad_minmax(VP __restrict__ vol, int nx, int ny, int nz,
                                                     int q, int by, int bz) {
    const int x0 = 16 * q;
    const int z0 = 4 * bz, y0 = 4 * by;
    const int zn = min(4, nz - z0), yn = min(4, ny - y0);
    if (x0 + 16 <= nx) {
        if (zn == 4 && yn == 4) return quad_whole_rows<T, false>(vol, nx, ny, z0, y0, zn, yn, x0);
        if constexpr (FAST_EDGES)
            return quad_whole_rows<T, true>(vol, nx, ny, z0, y0, zn, yn, x0);
        else
            return quad_rows_looped<T>(vol, nx, ny, z0, y0, zn, yn, x0);
    }
    if constexpr (FAST_EDGES) {
        if (nx >= 4) return quad_ragged_rows<T>(vol, nx, ny, z0, y0, zn, yn, x0);
    }
    // one voxel at a time (rows of fewer than 4 voxels; or ragged rows when
    // not FAST_EDGES)
    QuadMinMax<T> r;
#pragma unroll
    for (int k = 0; k < 4; ++k) { r.mn[k] = 0xFFFFFFFFu; r.mx[k] = 0u; }
    const int xn = min(16, nx - x0);
    for (int zz = 0; zz < zn; ++zz)
        for (int yy = 0; yy < yn; ++yy) {
            const int64_t off = ((int64_t)(z0 + zz) * ny + (y0 + yy)) * nx + x0;
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int xx = 0; xx < 4; ++xx)
                    if (4 * k + xx < xn) {
                        const uint32_t val = vol[off + 4 * k + xx];
                        r.mn[k] = umin(r.mn[k], val);
                        r.mx[k] = umax(r.mx[k], val);
                    }
        }
    return r;
}

// The [min,max] of 4 bricks, one store each at any alignment (one vector
// store: the hardware serves unaligned vector accesses, as in load16).
template <typename T, typename P>
__device__ __forceinline__ void store_bricks4(P mn, P mx, const QuadMinMax<T>& r) {
    if constexpr (sizeof(T) == 1) {
        const uint32_t a = r.mn[0] | (r.mn[1] << 8) | (r.mn[2] << 16) | (r.mn[3] << 24);
        const uint32_t b = r.mx[0] | (r.mx[1] << 8) | (r.mx[2] << 16) | (r.mx[3] << 24);
        __builtin_memcpy(mn, &a, 4);
        __builtin_memcpy(mx, &b, 4);
    } else {
        const uint2 a = make_uint2(r.mn[0] | (r.mn[1] << 16), r.mn[2] | (r.mn[3] << 16));
        const uint2 b = make_uint2(r.mx[0] | (r.mx[1] << 16), r.mx[2] | (r.mx[3] << 16));
        __builtin_memcpy(mn, &a, 8);
        __builtin_memcpy(mx, &b, 8);
    }
}

// ---------------------------------------------------------------------------
// k_bricks: one lane per 4 bricks along x.  Grid covers Qx*By*Bz lanes,
// Qx = ceil(Bx/4), quad index fastest so neighbouring lanes read neighbouring
// 16-byte chunks of the same voxel rows.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_bricks(const T* __restrict__ vol, int nx, int ny, int nz,
                                                int Bx, int By, int Bz, int Qx, T* __restrict__ bmin,
                                                T* __restrict__ bmax, int levels,
                                                int32_t* __restrict__ range_err) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)Qx * By * Bz;
    if (t >= total) return;
    const int q = (int)(t % Qx);
    const int64_t row = t / Qx;
    const int by = (int)(row % By), bz = (int)(row / By);
    const QuadMinMax<T> r = quad_minmax<T>(vol, nx, ny, nz, q, by, bz);
    const int64_t base = row * Bx + 4 * q;
    const int nb = min(4, Bx - 4 * q);
    if (range_err != nullptr) {
        uint32_t m = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (k < nb) m = umax(m, r.mx[k]);
        if (m >= (uint32_t)levels) *range_err = 1;
    }
    if (nb == 4) {
        store_bricks4<T>(bmin + base, bmax + base, r);
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (k < nb) {
                bmin[base + k] = (T)r.mn[k];
                bmax[base + k] = (T)r.mx[k];
            }
    }
}

// ---------------------------------------------------------------------------
// Distances along x inside one wave.  Lane L holds the occupancy nibble `o`
// of bricks xs+4L .. xs+4L+3 (bit k = brick xs+4L+k).  prev_last is the last
// occupied brick left of the segment and next_first the first one right of it
// (absolute x, or -kNone / +kNone).  Returns the 4 clamped distances packed
// into bytes.  Must be called by the whole wave.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t x_distances(uint32_t o, int lane, int xs, int prev_last,
                                                int next_first) {
    const uint64_t any = __ballot(o != 0u);
    // no occupied brick in the segment or beyond it: every distance is capped
    if (any == 0ull && prev_last == -kNone && next_first == kNone) return 0xFFFFFFFFu;
    const int hik = o ? 31 - __clz(o) : 0;
    const int lok = o ? __ffs(o) - 1 : 0;
    const uint64_t below = any & ((1ull << lane) - 1ull);
    const uint64_t above = (lane == kWave - 1) ? 0ull : (any & (~0ull << (lane + 1)));
    const int src_l = below ? 63 - __clzll((long long)below) : lane;
    const int src_r = above ? __ffsll((unsigned long long)above) - 1 : lane;
    const int hi_l = __shfl(hik, src_l, kWave);
    const int lo_r = __shfl(lok, src_r, kWave);
    const int left_lane = below ? xs + 4 * src_l + hi_l : prev_last;
    const int right_lane = above ? xs + 4 * src_r + lo_r : next_first;
    uint32_t packed = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int x = xs + 4 * lane + k;
        const uint32_t ml = o & ((2u << k) - 1u);
        const uint32_t mr = o & (0xFu & ~((1u << k) - 1u));
        const int lp = ml ? xs + 4 * lane + (31 - __clz(ml)) : left_lane;
        const int rp = mr ? xs + 4 * lane + (__ffs(mr) - 1) : right_lane;
        int d = min(x - lp, rp - x);
        d = min(d, 255);
        packed |= (uint32_t)d << (8 * k);
    }
    return packed;
}

// Distances along x for short rows packed into one wave: lane L holds the
// occupancy nibble of bricks 4r .. 4r+3 (r = L mod W) of the wave's row
// floor(L / W), W a power of two from 1 to 64; a row has at most 4W bricks
// and nothing outside it counts.  Returns the 4 clamped distances packed into
// bytes.  Must be called by the whole wave.
__device__ __forceinline__ uint32_t x_distances_rows(uint32_t o, int lane, int W) {
    const uint64_t any = __ballot(o != 0u);
    if (any == 0ull) return 0xFFFFFFFFu;  // no occupied brick in these rows
    const int base = lane & ~(W - 1);
    const uint64_t seg = W >= kWave ? ~0ull : (((1ull << W) - 1ull) << base);
    const uint64_t mine = any & seg;
    const uint64_t below = mine & ((1ull << lane) - 1ull);
    const uint64_t above = (lane == kWave - 1) ? 0ull : (mine & (~0ull << (lane + 1)));
    const int hik = o ? 31 - __clz(o) : 0;
    const int lok = o ? __ffs(o) - 1 : 0;
    const int src_l = below ? 63 - __clzll((long long)below) : lane;
    const int src_r = above ? __ffsll((unsigned long long)above) - 1 : lane;
    const int hi_l = __shfl(hik, src_l, kWave);
    const int lo_r = __shfl(lok, src_r, kWave);
    const int r = lane - base;
    const int left_lane = below ? 4 * (src_l - base) + hi_l : -kNone;
    const int right_lane = above ? 4 * (src_r - base) + lo_r : kNone;
    uint32_t packed = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int x = 4 * r + k;
        const uint32_t ml = o & ((2u << k) - 1u);
        const uint32_t mr = o & (0xFu & ~((1u << k) - 1u));
        const int lp = ml ? 4 * r + (31 - __clz(ml)) : left_lane;
        const int rp = mr ? 4 * r + (__ffs(mr) - 1) : right_lane;
        int d = min(x - lp, rp - x);
        d = min(d, 255);
        packed |= (uint32_t)d << (8 * k);
    }
    return packed;
}

// Position of the first / last occupied brick of a segment (wave-uniform).
__device__ __forceinline__ int seg_first(uint32_t o, int xs) {
    const uint64_t any = __ballot(o != 0u);
    const int lok = o ? __ffs(o) - 1 : 0;
    const int src = any ? __ffsll((unsigned long long)any) - 1 : 0;
    const int v = __shfl(lok, src, kWave);
    return any ? xs + 4 * src + v : kNone;
}
__device__ __forceinline__ int seg_last(uint32_t o, int xs) {
    const uint64_t any = __ballot(o != 0u);
    const int hik = o ? 31 - __clz(o) : 0;
    const int src = any ? 63 - __clzll((long long)any) : 0;
    const int v = __shfl(hik, src, kWave);
    return any ? xs + 4 * src + v : -kNone;
}

__device__ __forceinline__ void store_u32(uint8_t* p, uint32_t v) {
    *reinterpret_cast<uint32_t*>(p) = v;
}
__device__ __forceinline__ void store_u32(PDM_GLB uint8_t* p, uint32_t v) {
    *reinterpret_cast<PDM_GLB uint32_t*>(p) = v;
}

template <typename DP>
__device__ __forceinline__ void store_quad(DP __restrict__ dst, int64_t idx, int nb,
                                           uint32_t packed, bool vec) {
    if (nb == 4) {
        // four bytes at any alignment: one store (the hardware serves
        // unaligned vector accesses, as for load16)
        if (vec)
            store_u32(dst + idx, packed);
        else
            __builtin_memcpy(dst + idx, &packed, 4);
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (k < nb) dst[idx + k] = (uint8_t)(packed >> (8 * k));
    }
}

// The smallest brick minimum and the largest brick maximum over the wave's
// lanes (wave-uniform; lanes without bricks hold min = ~0, max = 0).  A
// partition [lo, hi] with hi < wmin or lo > wmax holds none of the wave's
// bricks, so every distance of its rows is the cap and no x pass is needed.
__device__ __forceinline__ void wave_value_range(const uint32_t (&mn)[4], const uint32_t (&mx)[4],
                                                 uint32_t& wmin, uint32_t& wmax) {
    uint32_t a = umin(umin(mn[0], mn[1]), umin(mn[2], mn[3]));
    uint32_t b = umax(umax(mx[0], mx[1]), umax(mx[2], mx[3]));
#pragma unroll
    for (int o = kWave / 2; o >= 1; o >>= 1) {
        a = umin(a, (uint32_t)__shfl_xor((int)a, o, kWave));
        b = umax(b, (uint32_t)__shfl_xor((int)b, o, kWave));
    }
    wmin = __builtin_amdgcn_readfirstlane(a);
    wmax = __builtin_amdgcn_readfirstlane(b);
}

// ---------------------------------------------------------------------------
// k_pom_x: one wave per brick row (bz, by); 4 waves per work-group.  For
// every partition p: POM nibble from [min,max] (RANGE reading) and the x
// distances, written to pdms[p*G + row*Bx + x].  Rows of at most 128 bricks
// are packed 64/W to a wave (W < 64 lanes per row, the power of two with
// 4W >= Bx), so narrow grids keep every lane busy.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_pom_x(const T* __restrict__ bmin,
                                               const T* __restrict__ bmax, int Bx, int64_t rows,
                                               Bounds bounds, int n, uint8_t* __restrict__ pdms,
                                               int64_t G, int store_vec, int W) {
    const int lane = threadIdx.x & (kWave - 1);
    if (W < kWave) {
        const int per = kWave / W;
        const int64_t row0 = ((int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave)) * per;
        if (row0 >= rows) return;  // wave-uniform
        const int64_t row = row0 + lane / W;
        const int q = lane & (W - 1);
        const int nb = row < rows ? max(0, min(4, Bx - 4 * q)) : 0;
        const int64_t rbase = row * Bx + 4 * q;
        uint32_t mn[4], mx[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            mn[k] = k < nb ? (uint32_t)bmin[rbase + k] : 0xFFFFFFFFu;
            mx[k] = k < nb ? (uint32_t)bmax[rbase + k] : 0u;
        }
        uint32_t wmin, wmax;
        wave_value_range(mn, mx, wmin, wmax);
        for (int p = 0; p < n; ++p) {
            const uint32_t lo = (uint32_t)bounds.b[p], hi = (uint32_t)bounds.b[p + 1] - 1u;
            uint32_t packed = 0xFFFFFFFFu;
            if (hi >= wmin && lo <= wmax) {
                uint32_t o = 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) o |= (mn[k] <= hi && mx[k] >= lo) ? (1u << k) : 0u;
                packed = x_distances_rows(o, lane, W);
            }
            if (nb > 0) store_quad(pdms + (int64_t)p * G, rbase, nb, packed, store_vec);
        }
        return;
    }
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
    if (row >= rows) return;  // wave-uniform
    const int nseg = (Bx + kSegBricks - 1) / kSegBricks;
    const int64_t rbase = row * Bx;
    if (nseg == 1) {
        uint32_t mn[4], mx[4];
        const int nb = max(0, min(4, Bx - 4 * lane));
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            mn[k] = k < nb ? (uint32_t)bmin[rbase + 4 * lane + k] : 0xFFFFFFFFu;
            mx[k] = k < nb ? (uint32_t)bmax[rbase + 4 * lane + k] : 0u;
        }
        uint32_t wmin, wmax;
        wave_value_range(mn, mx, wmin, wmax);
        for (int p = 0; p < n; ++p) {
            const uint32_t lo = (uint32_t)bounds.b[p], hi = (uint32_t)bounds.b[p + 1] - 1u;
            uint32_t packed = 0xFFFFFFFFu;
            if (hi >= wmin && lo <= wmax) {
                uint32_t o = 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) o |= (mn[k] <= hi && mx[k] >= lo) ? (1u << k) : 0u;
                packed = x_distances(o, lane, 0, -kNone, kNone);
            }
            if (nb > 0) store_quad(pdms + (int64_t)p * G, rbase + 4 * lane, nb, packed, store_vec);
        }
        return;
    }
    // long rows: segments of 256 bricks; only the neighbouring segments can
    // hold a brick within the cap
    auto nibble = [&](int seg, uint32_t lo, uint32_t hi) -> uint32_t {
        const int x = seg * kSegBricks + 4 * lane;
        uint32_t o = 0;
        for (int k = 0; k < 4; ++k)
            if (x + k < Bx) {
                const uint32_t a = bmin[rbase + x + k], b = bmax[rbase + x + k];
                o |= (a <= hi && b >= lo) ? (1u << k) : 0u;
            }
        return o;
    };
    for (int p = 0; p < n; ++p) {
        const uint32_t lo = (uint32_t)bounds.b[p], hi = (uint32_t)bounds.b[p + 1] - 1u;
        int prev_last = -kNone;
        uint32_t cur = nibble(0, lo, hi);
        for (int s = 0; s < nseg; ++s) {
            const int xs = s * kSegBricks;
            const uint32_t nxt = (s + 1 < nseg) ? nibble(s + 1, lo, hi) : 0u;
            const int next_first = (s + 1 < nseg) ? seg_first(nxt, xs + kSegBricks) : kNone;
            const uint32_t packed = x_distances(cur, lane, xs, prev_last, next_first);
            const int nb = max(0, min(4, Bx - xs - 4 * lane));
            if (nb > 0) store_quad(pdms + (int64_t)p * G, rbase + xs + 4 * lane, nb, packed, store_vec);
            prev_last = seg_last(cur, xs);
            cur = nxt;
        }
    }
}

// ---------------------------------------------------------------------------
// Plain method, phase 1.  One wave per brick row; each lane reduces its 4
// bricks from the volume, tests [min,max] against the non-zero opacity bitmap
// and the wave computes x distances.  The bitmap test uses per-word prefix
// counts in LDS: any set bit in [lo,hi].
// ---------------------------------------------------------------------------
constexpr int kMaxSegs = PDM_PLAIN_MAX_SEGS;

__device__ __forceinline__ bool any_bit(const uint32_t* __restrict__ words,
                                        const uint16_t* __restrict__ pre, uint32_t lo, uint32_t hi) {
    const uint32_t wl = lo >> 5, wh = hi >> 5;
    const uint32_t ml = ~0u << (lo & 31u);
    const uint32_t mh = (hi & 31u) == 31u ? ~0u : ((2u << (hi & 31u)) - 1u);
    if (wl == wh) return (words[wl] & ml & mh) != 0u;
    if ((words[wl] & ml) != 0u || (words[wh] & mh) != 0u) return true;
    return pre[wh] != pre[wl + 1];
}

// Whether [lo, hi] meets one of the nruns maximal runs of non-zero levels,
// runs[j] = first | last << 16 in increasing order: the first run whose last
// level is >= lo decides (binary search).
__device__ __forceinline__ bool any_run(const uint32_t* __restrict__ runs, int nruns, uint32_t lo,
                                        uint32_t hi) {
    int l = 0, h = nruns;
    while (l < h) {
        const int mid = (l + h) >> 1;
        if ((runs[mid] >> 16) < lo)
            l = mid + 1;
        else
            h = mid;
    }
    return l < nruns && (runs[l] & 0xFFFFu) <= hi;
}

// The plain method's occupancy test of one brick [lo, hi]: the bitmap, or
// with RUNS the run list (levels above the bitmap's 16384).
template <bool RUNS>
__device__ __forceinline__ bool any_alpha(const uint32_t* __restrict__ words,
                                          const uint16_t* __restrict__ pre, int nwords, uint32_t lo,
                                          uint32_t hi) {
    if constexpr (RUNS)
        return any_run(words, nwords, lo, hi);
    else
        return any_bit(words, pre, lo, hi);
}

template <typename T, bool RUNS>
__global__ void __launch_bounds__(256) k_plain_x(const T* __restrict__ vol, int nx, int ny, int nz,
                                                 int Bx, int By, int64_t rows, AlphaBits bits,
                                                 int nwords, int levels, uint8_t* __restrict__ dist,
                                                 int store_vec) {
    __shared__ uint32_t s_words[PDM_ALPHA_WORDS];
    __shared__ uint16_t s_pre[PDM_ALPHA_WORDS + 1];
    __shared__ uint8_t s_nib[4][kMaxSegs][kWave];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x / kWave) + wv;
    const bool live = row < rows;  // wave-uniform
    const int by = live ? (int)(row % By) : 0, bz = live ? (int)(row / By) : 0;
    // the first segment's voxels are requested before the bitmap set-up, so
    // the loads are in flight while the block fills LDS
    QuadMinMax<T> r0;
    if (live && 4 * lane < Bx) r0 = quad_minmax<T, false>(vol, nx, ny, nz, lane, by, bz);
    for (int i = threadIdx.x; i < nwords; i += blockDim.x) s_words[i] = bits.w[i];
    for (int i = threadIdx.x; i <= nwords; i += blockDim.x) s_pre[i] = bits.pre[i];
    __syncthreads();
    if (!live) return;  // after the only barrier
    const int nseg = (Bx + kSegBricks - 1) / kSegBricks;
    const int64_t rbase = row * Bx;
    // voxels >= levels break the precondition; clamping keeps the bitmap
    // lookups inside the table
    const uint32_t top = (uint32_t)levels - 1u;
    for (int s = 0; s < nseg; ++s) {
        const int q = s * kWave + lane;  // quad index within the row
        uint32_t o = 0;
        if (4 * q < Bx) {
            const QuadMinMax<T> r = s == 0 ? r0 : quad_minmax<T, false>(vol, nx, ny, nz, q, by, bz);
            const int nb = min(4, Bx - 4 * q);
            for (int k = 0; k < 4; ++k)
                if (k < nb && any_alpha<RUNS>(s_words, s_pre, nwords, umin(r.mn[k], top), umin(r.mx[k], top)))
                    o |= 1u << k;
        }
        s_nib[wv][s][lane] = (uint8_t)o;
    }
    // the wave reads back only its own entries (written by its own lanes)
    __builtin_amdgcn_wave_barrier();
    for (int s = 0; s < nseg; ++s) {
        const int xs = s * kSegBricks;
        const uint32_t cur = s_nib[wv][s][lane];
        const int prev_last = s > 0 ? seg_last(s_nib[wv][s - 1][lane], xs - kSegBricks) : -kNone;
        const int next_first = s + 1 < nseg ? seg_first(s_nib[wv][s + 1][lane], xs + kSegBricks) : kNone;
        const uint32_t packed = x_distances(cur, lane, xs, prev_last, next_first);
        const int nb = max(0, min(4, Bx - xs - 4 * lane));
        if (nb > 0) store_quad(dist, rbase + xs + 4 * lane, nb, packed, store_vec);
    }
}

// ---------------------------------------------------------------------------
// Plain method from the cached brick [min,max] (the volume is not read): the
// same occupancy test as k_plain_x on bmin/bmax, then the x distances.
// Rows of up to 256 bricks: W lanes per row (the power of two with 4W >= Bx),
// so one wave pass covers 64/W rows, and a wave takes kCachedPasses passes
// with the loads of all of them issued first (4 bricks per lane, one vector
// load each for bmin and bmax when rows and pointers allow).  Longer rows:
// one wave per row in 256-brick segments.
// ---------------------------------------------------------------------------
constexpr int kCachedPasses = 4;

template <typename T>
struct Quad {
    T v[4];
};

// Bricks x0 .. x0+3 of a row (nb of them inside it; the rest get `fill`).
template <typename T>
__device__ __forceinline__ Quad<T> load_quad(const T* __restrict__ p, int64_t idx, int nb, bool vec,
                                             T fill) {
    Quad<T> q;
    if (vec && nb == 4) {
        if constexpr (sizeof(T) == 1) {
            const uint32_t w = *reinterpret_cast<const uint32_t*>(p + idx);
#pragma unroll
            for (int k = 0; k < 4; ++k) q.v[k] = (T)(w >> (8 * k));
        } else {
            const uint2 w = *reinterpret_cast<const uint2*>(p + idx);
            q.v[0] = (T)w.x;
            q.v[1] = (T)(w.x >> 16);
            q.v[2] = (T)w.y;
            q.v[3] = (T)(w.y >> 16);
        }
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) q.v[k] = k < nb ? p[idx + k] : fill;
    }
    return q;
}

template <typename T, bool RUNS>
__global__ void __launch_bounds__(256) k_plain_cached_x(const T* __restrict__ bmin,
                                                        const T* __restrict__ bmax, int Bx,
                                                        int64_t rows, AlphaBits bits, int nwords,
                                                        int levels, uint8_t* __restrict__ dist,
                                                        int store_vec, int W, int load_vec) {
    __shared__ uint32_t s_words[PDM_ALPHA_WORDS];
    __shared__ uint16_t s_pre[PDM_ALPHA_WORDS + 1];
    for (int i = threadIdx.x; i < nwords; i += blockDim.x) s_words[i] = bits.w[i];
    for (int i = threadIdx.x; i <= nwords; i += blockDim.x) s_pre[i] = bits.pre[i];
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t top = (uint32_t)levels - 1u;
    auto nibble = [&](const Quad<T>& a, const Quad<T>& b, int nb) -> uint32_t {
        uint32_t o = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (k < nb && any_alpha<RUNS>(s_words, s_pre, nwords, umin((uint32_t)a.v[k], top),
                                          umin((uint32_t)b.v[k], top)))
                o |= 1u << k;
        return o;
    };
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
    if (W <= kWave && Bx <= kSegBricks) {
        const int per = kWave / W;  // rows per wave pass
        const int64_t row0 = wave * per * kCachedPasses;
        if (row0 >= rows) return;  // wave-uniform
        const int q = lane & (W - 1);
        Quad<T> mn[kCachedPasses], mx[kCachedPasses];
        int nb[kCachedPasses];
#pragma unroll
        for (int j = 0; j < kCachedPasses; ++j) {
            const int64_t row = row0 + (int64_t)j * per + lane / W;
            nb[j] = row < rows ? max(0, min(4, Bx - 4 * q)) : 0;
            const int64_t idx = row * Bx + 4 * q;
            mn[j] = load_quad<T>(bmin, idx, nb[j], load_vec, (T)0);
            mx[j] = load_quad<T>(bmax, idx, nb[j], load_vec, (T)0);
        }
#pragma unroll
        for (int j = 0; j < kCachedPasses; ++j) {
            const int64_t row = row0 + (int64_t)j * per + lane / W;
            const uint32_t packed = x_distances_rows(nibble(mn[j], mx[j], nb[j]), lane, W);
            if (nb[j] > 0) store_quad(dist, row * Bx + 4 * q, nb[j], packed, store_vec);
        }
        return;
    }
    const int64_t row = wave;
    if (row >= rows) return;  // wave-uniform
    const int nseg = (Bx + kSegBricks - 1) / kSegBricks;
    const int64_t rbase = row * Bx;
    auto seg_nibble = [&](int seg) -> uint32_t {
        const int x = seg * kSegBricks + 4 * lane;
        const int nb = max(0, min(4, Bx - x));
        return nibble(load_quad<T>(bmin, rbase + x, nb, false, (T)0),
                      load_quad<T>(bmax, rbase + x, nb, false, (T)0), nb);
    };
    int prev_last = -kNone;
    uint32_t cur = seg_nibble(0);
    for (int s = 0; s < nseg; ++s) {
        const int xs = s * kSegBricks;
        const uint32_t nxt = (s + 1 < nseg) ? seg_nibble(s + 1) : 0u;
        const int next_first = (s + 1 < nseg) ? seg_first(nxt, xs + kSegBricks) : kNone;
        const uint32_t packed = x_distances(cur, lane, xs, prev_last, next_first);
        const int nb = max(0, min(4, Bx - xs - 4 * lane));
        if (nb > 0) store_quad(dist, rbase + xs + 4 * lane, nb, packed, store_vec);
        prev_last = seg_last(cur, xs);
        cur = nxt;
    }
}

// ---------------------------------------------------------------------------
// EXACT occupancy (a brick is occupied when one of its voxels qualifies, the
// literal POM wording of Sec. 3.1), for the PDM build and the plain method.
// ---------------------------------------------------------------------------

// Calls f(k, value) for every voxel of the 4 bricks x = 4q..4q+3 of brick row
// (bz, by) that lies inside the volume (k = brick within the quad).
template <typename T, typename F>
__device__ __forceinline__ void quad_voxels(const T* __restrict__ vol, int nx, int ny, int nz, int q,
                                            int by, int bz, F f) {
    const int x0 = 16 * q;
    const int z0 = 4 * bz, y0 = 4 * by;
    const int zn = min(4, nz - z0), yn = min(4, ny - y0);
    if (x0 + 16 <= nx) {
        for (int zz = 0; zz < zn; ++zz) {
#pragma unroll
            for (int yy = 0; yy < 4; ++yy) {
                if (yy < yn) {
                    const int64_t off = ((int64_t)(z0 + zz) * ny + (y0 + yy)) * nx + x0;
                    if constexpr (sizeof(T) == 1) {
                        const uint4 w = load16(vol + off);
                        const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
                        for (int k = 0; k < 4; ++k)
#pragma unroll
                            for (int b = 0; b < 4; ++b) f(k, (ws[k] >> (8 * b)) & 0xFFu);
                    } else {
                        const uint4 a = load16(vol + off), c = load16(vol + off + 8);
                        const uint32_t ws[8] = {a.x, a.y, a.z, a.w, c.x, c.y, c.z, c.w};
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            f(k, lo16(ws[2 * k]));
                            f(k, hi16(ws[2 * k]));
                            f(k, lo16(ws[2 * k + 1]));
                            f(k, hi16(ws[2 * k + 1]));
                        }
                    }
                }
            }
        }
    } else {
        const int xn = min(16, nx - x0);
        for (int zz = 0; zz < zn; ++zz)
            for (int yy = 0; yy < yn; ++yy) {
                const int64_t off = ((int64_t)(z0 + zz) * ny + (y0 + yy)) * nx + x0;
#pragma unroll
                for (int k = 0; k < 4; ++k)
#pragma unroll
                    for (int xx = 0; xx < 4; ++xx)
                        if (4 * k + xx < xn) f(k, (uint32_t)vol[off + 4 * k + xx]);
            }
    }
}

// k_pom_exact_x: one wave per brick row (Bx <= 256).  Each lane marks, for
// its 4 bricks, which partitions hold one of their voxels (NW = ceil(n/32)
// mask words per brick, from an LDS table intensity -> partition), then the
// wave computes every partition's x distances from those masks.  Reads the
// volume once and writes n*G bytes.  Rows of at most 128 bricks are packed
// 64/W to a wave (W lanes per row), as in k_pom_x.
template <typename T, int NW, bool PACK>
__global__ void __launch_bounds__(256) k_pom_exact_x(const T* __restrict__ vol, int nx, int ny,
                                                     int nz, int Bx, int By, int64_t rows,
                                                     Bounds bounds, int n, int levels,
                                                     uint8_t* __restrict__ pdms, int64_t G,
                                                     int store_vec, int W) {
    __shared__ uint8_t s_part[PDM_EXACT_MAX_LEVELS];
    // partition p paints its intensities [bounds[p], bounds[p+1])
    for (int p = threadIdx.x; p < n; p += blockDim.x)
        for (int v = bounds.b[p]; v < bounds.b[p + 1]; ++v) s_part[v] = (uint8_t)p;
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1);
    // PACK (W < 64): rows of at most 128 bricks, 64/W to a wave (W lanes per row)
    if (!PACK) W = kWave;
    const int per = kWave / W;
    const int64_t row0 = ((int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave)) * per;
    if (row0 >= rows) return;  // wave-uniform, after the barrier
    const int64_t row = row0 + lane / W;
    const int q = lane & (W - 1);  // quad index within the row
    const bool row_ok = row < rows;
    const int by = row_ok ? (int)(row % By) : 0, bz = row_ok ? (int)(row / By) : 0;
    const int64_t rbase = row * Bx;
    uint32_t mk[4][NW];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int w = 0; w < NW; ++w) mk[k][w] = 0u;
    const uint32_t top = (uint32_t)levels - 1u;  // voxels >= levels break the precondition
    if (row_ok && 4 * q < Bx) {
        quad_voxels<T>(vol, nx, ny, nz, q, by, bz, [&](int k, uint32_t val) {
            const uint32_t pid = s_part[umin(val, top)];
            const uint32_t bit = 1u << (pid & 31u);
#pragma unroll
            for (int w = 0; w < NW; ++w) mk[k][w] |= ((pid >> 5) == (uint32_t)w) ? bit : 0u;
        });
    }
    const int nb = row_ok ? max(0, min(4, Bx - 4 * q)) : 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const int pend = min(32, n - 32 * w);
        for (int b = 0; b < pend; ++b) {
            uint32_t o = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) o |= ((mk[k][w] >> b) & 1u) << k;
            uint32_t packed;
            if constexpr (PACK)
                packed = x_distances_rows(o, lane, W);
            else
                packed = x_distances(o, lane, 0, -kNone, kNone);
            if (nb > 0)
                store_quad(pdms + (int64_t)(32 * w + b) * G, rbase + 4 * q, nb, packed, store_vec);
        }
    }
}

// k_plain_exact_x: the plain method's occupancy in the EXACT reading (some
// voxel of the brick has alpha != 0, looked up in the LDS bitmap) and its x
// distances; long rows in 256-brick segments as in k_plain_x.
template <typename T>
__global__ void __launch_bounds__(256) k_plain_exact_x(const T* __restrict__ vol, int nx, int ny,
                                                       int nz, int Bx, int By, int64_t rows,
                                                       AlphaBits bits, int nwords, int levels,
                                                       uint8_t* __restrict__ dist,
                                                       int store_vec) {
    __shared__ uint32_t s_words[PDM_ALPHA_WORDS];
    __shared__ uint8_t s_nib[4][kMaxSegs][kWave];
    for (int i = threadIdx.x; i < nwords; i += blockDim.x) s_words[i] = bits.w[i];
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x / kWave) + wv;
    if (row >= rows) return;  // wave-uniform, after the barrier
    const int by = (int)(row % By), bz = (int)(row / By);
    const int nseg = (Bx + kSegBricks - 1) / kSegBricks;
    const int64_t rbase = row * Bx;
    const uint32_t top = (uint32_t)levels - 1u;
    for (int s = 0; s < nseg; ++s) {
        const int q = s * kWave + lane;
        uint32_t o = 0;
        if (4 * q < Bx) {
            quad_voxels<T>(vol, nx, ny, nz, q, by, bz, [&](int k, uint32_t val) {
                const uint32_t v = umin(val, top);
                o |= ((s_words[v >> 5] >> (v & 31u)) & 1u) << k;
            });
        }
        s_nib[wv][s][lane] = (uint8_t)o;
    }
    __builtin_amdgcn_wave_barrier();
    for (int s = 0; s < nseg; ++s) {
        const int xs = s * kSegBricks;
        const uint32_t cur = s_nib[wv][s][lane];
        const int prev_last = s > 0 ? seg_last(s_nib[wv][s - 1][lane], xs - kSegBricks) : -kNone;
        const int next_first = s + 1 < nseg ? seg_first(s_nib[wv][s + 1][lane], xs + kSegBricks) : kNone;
        const uint32_t packed = x_distances(cur, lane, xs, prev_last, next_first);
        const int nb = max(0, min(4, Bx - xs - 4 * lane));
        if (nb > 0) store_quad(dist, rbase + xs + 4 * lane, nb, packed, store_vec);
    }
}

// ---------------------------------------------------------------------------
// k_dist_axis: 1-D max-min pass g(i) = min_j max(|i-j|, f(j)), in place, for
// lines along y (stride Bx) or z (stride Bx*By), one lane per line.
//
// The pass is a forward one-sided pass F(i) = min_{j<=i} max(i-j, f(j))
// followed by the same pass backwards over F, which yields g exactly (a
// candidate j > i reaches i only through the backward pass, j <= i through
// the forward one).  The one-sided pass runs in one sweep: keep v = F(i-1)
// and a witness W with max(i-1-W, f(W)) <= v.  Then F(i) is min(f(i), X)
// with X = v if i-W <= v, else v+1.  In the second case the next witness is
// the latest position holding exactly v+1, looked up in a per-lane table
// last[w] = latest position with value w.  The exact rule would keep the
// later of that entry and W; taking the entry alone changes no later
// decision, because when it is the earlier one, W itself was already too far
// for v+1 at the next position, so both choices advance again there.  An
// empty entry (0) behaves the same way.
//
// With that rule the witness after each step is always last[F(i)], read
// after the step's own write last[f(i)] = i: a new minimum (f(i) <= X) makes
// i the witness, and last[f(i)] = i was just written; an advance takes
// last[v+1], which the write did not touch (f(i) > v+1); otherwise v and W
// stay, and last[v] was not touched either (f(i) > v).  So a step is one
// table write, X = min(v+1, max(v, i-W)), F(i) = min(f(i), X) and one table
// read W = last[F(i)]: no selects between witness candidates.
//
// Tables: rows for the values 0..255 (F(i) <= 255 from the first step on) of
// kPitch entries, lane-major inside a row; the odd dword pitch (17) spreads
// lanes that look up different values over the LDS banks.
// ---------------------------------------------------------------------------
constexpr int kScanLanes = 64;
constexpr int kPitch = 68;      // entries per table row (>= kScanLanes)
constexpr int kRows = 256;
constexpr int kMaxLine = 256;   // longest line staged in LDS
// Passes over at most this many lines use the LDS-staged kernel: they cannot
// fill the chip's 1024 SIMDs with more than a few waves each, so per-wave
// latency matters more than occupancy.
constexpr int64_t kStagedMaxLines = 4 * 1024 * kScanLanes;
// Steps per chunk of the global-memory scans, which serve lines of more than
// 256 bricks and passes whose offsets exceed the register kernels' 31 bits
// (values loaded into registers before their steps run).  Measured over all
// maps of a grid, 32 against 16: 3% faster for lines of 199 to 256 bricks
// over more than 2^20 lines, 5-10% slower for shorter lines or fewer lines.
// Lines shorter than a chunk run step by step.
constexpr int kLongChunk = 32;
constexpr int kLongChunkLine = 192;
constexpr int64_t kLongChunkLines = 1 << 20;

template <typename P>
__device__ __forceinline__ void clear_table(P* tbl) {
    constexpr int kBytes = ((kRows * kPitch * (int)sizeof(P)) + 15) & ~15;
    uint4* t4 = reinterpret_cast<uint4*>(tbl);
    for (int i = threadIdx.x; i < kBytes / 16; i += kScanLanes) t4[i] = make_uint4(0, 0, 0, 0);
}

// Clears the first n16 16-byte pieces of a table (one wave).
__device__ __forceinline__ void clear_rows(uint8_t* tbl, int n16) {
    uint4* t4 = reinterpret_cast<uint4*>(tbl);
    for (int i = threadIdx.x; i < n16; i += kScanLanes) t4[i] = make_uint4(0, 0, 0, 0);
}

// One step of the one-sided pass at position i with input fi.  State:
// v = F(i-1) and its witness W = last[v]; the first step of a pass starts
// from v above every value (511), so it takes F = f(0) with witness 0.
// Table offsets are 32-bit: v stays below 2^8 after the unsigned min with
// the 8-bit input, so rows times kPitch plus the lane stays far below 2^24.
#define PDM_SCAN_STEP(i_, fi_, out_)                                              \
    {                                                                             \
        const int i__ = (i_), fi__ = (fi_);                                       \
        tbl[__umul24((unsigned)fi__, (unsigned)kPitch) + (unsigned)lane] = (P)i__; \
        const unsigned X__ = umin((unsigned)v + 1u, umax((unsigned)v, (unsigned)(i__ - W))); \
        v = (int)umin((unsigned)fi__, X__);                                       \
        W = (int)tbl[__umul24((unsigned)v, (unsigned)kPitch) + (unsigned)lane];   \
        out_ = v;                                                                 \
    }

// The one-sided pass over one line held in an LDS column: col[k * cs] for
// k = 0..m-1 in the pass's direction (cs may be negative), overwritten in
// place with the result.  Values are read CH at a time into registers before
// their steps run.
template <typename P, int CH>
__device__ __forceinline__ void one_sided_lds(uint8_t* col, int cs, int m, P* __restrict__ tbl) {
    const int lane = threadIdx.x;
    // F(0) = f(0); its table entry (position 0) equals the cleared value
    int v = col[0];
    int W = 0;
    int c = 1;
    for (; c + CH <= m; c += CH) {
        int f[CH];
#pragma unroll
        for (int k = 0; k < CH; ++k) f[k] = col[(c + k) * cs];
        int pc = c;  // the position in a vector register: one add per step
        __asm__ volatile("" : "+v"(pc));
#pragma unroll
        for (int k = 0; k < CH; ++k) PDM_SCAN_STEP(pc + k, f[k], f[k]);
#pragma unroll
        for (int k = 0; k < CH; ++k) col[(c + k) * cs] = (uint8_t)f[k];
    }
    for (; c < m; ++c) {
        int out;
        PDM_SCAN_STEP(c, (int)col[c * cs], out);
        col[c * cs] = (uint8_t)out;
    }
}

// The same pass over a line in global memory, p[k * step] (lines longer
// than the LDS tile); `active` false lanes only keep the wave in step.
template <typename P, int CH, typename BP>
__device__ __forceinline__ void one_sided_global(BP p, int64_t step, int m, bool active,
                                                 P* __restrict__ tbl) {
    const int lane = threadIdx.x;
    int v = active ? (int)p[0] : 0;
    int W = 0;
    int c = 1;
    for (; c + CH <= m; c += CH) {
        int f[CH];
#pragma unroll
        for (int k = 0; k < CH; ++k) f[k] = active ? (int)p[(int64_t)(c + k) * step] : 0;
        int pc = c;  // the position in a vector register: one add per step
        __asm__ volatile("" : "+v"(pc));
#pragma unroll
        for (int k = 0; k < CH; ++k) PDM_SCAN_STEP(pc + k, f[k], f[k]);
        if (active) {
#pragma unroll
            for (int k = 0; k < CH; ++k) p[(int64_t)(c + k) * step] = (uint8_t)f[k];
        }
    }
    for (; c < m; ++c) {
        const int fi = active ? (int)p[(int64_t)c * step] : 0;
        int out;
        PDM_SCAN_STEP(c, fi, out);
        if (active) p[(int64_t)c * step] = (uint8_t)out;
    }
}

// The one-sided pass over steps [ib, ie) of a line held in an LDS column
// col[k * cs], with the scan state carried in and out (the split pass below
// runs it in phases).  Values are clamped at vmax before their step; with
// `track` the raw values read are folded into raw_min.
template <int CH>
__device__ __forceinline__ void one_sided_lds_range(uint8_t* col, int cs, int ib, int ie, int vmax,
                                                    bool track, uint8_t* __restrict__ tbl, int& v,
                                                    int& W, int& raw_min) {
    using P = uint8_t;  // table entry type of PDM_SCAN_STEP
    const int lane = threadIdx.x;
    int c = ib;
    for (; c + CH <= ie; c += CH) {
        int f[CH];
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            const int r = col[(c + k) * cs];
            if (track) raw_min = min(raw_min, r);
            f[k] = (int)umin((unsigned)r, (unsigned)vmax);
        }
        int pc = c;  // the position in a vector register: one add per step
        __asm__ volatile("" : "+v"(pc));
#pragma unroll
        for (int k = 0; k < CH; ++k) PDM_SCAN_STEP(pc + k, f[k], f[k]);
#pragma unroll
        for (int k = 0; k < CH; ++k) col[(c + k) * cs] = (uint8_t)f[k];
    }
    for (; c < ie; ++c) {
        const int r = col[c * cs];
        if (track) raw_min = min(raw_min, r);
        int out;
        PDM_SCAN_STEP(c, (int)umin((unsigned)r, (unsigned)vmax), out);
        col[c * cs] = (uint8_t)out;
    }
}

// Work-groups are handed to the 8 XCDs round-robin (work-group b runs on XCD
// b % 8).  xcd_item maps work-group b to a work item so that runs of kXcdRun
// consecutive items land on one XCD at about the same time: neighbouring
// 64-line tiles of a row share 128-byte cache lines, and under one L2 the
// second tile finds the line the first one fetched.  The grid is rounded up
// to a multiple of kXcds * kXcdRun; work-groups past the last item return.
constexpr int kXcds = 8;
constexpr int kXcdRun = 4;
constexpr int64_t kXcdSpan = (int64_t)kXcds * kXcdRun;

__device__ __forceinline__ int64_t xcd_item(int64_t b) {
    const int64_t r = b % kXcdSpan;
    return (b - r) + (r % kXcds) * kXcdRun + r / kXcds;
}

// Line l of a pass: x fastest, then the other in-grid axis (`inner` values
// with step `plane`), then the grid index.
__device__ __forceinline__ int64_t line_offset(int64_t l, int Bx, int inner, int64_t plane,
                                               int64_t G) {
    const int64_t r = l / Bx;
    return (r / inner) * G + (r % inner) * plane + l % Bx;
}

// ---------------------------------------------------------------------------
// k_dist_lines: both one-sided passes of 64 lines (one per lane) with the
// whole line held in registers, for passes over many lines (all partitions
// of a grid): each byte is read once and written once, and the backward pass
// reads the forward pass's results from registers instead of global memory.
//
// The 64 lines of a work-group are addressed through a buffer resource at
// the first line's offset: every lane keeps its line's 32-bit offset in a
// vector register and a position's offset (p * stride) is a scalar, so a
// load or store costs no vector address arithmetic.  The host checks that
// every offset fits in 31 bits.  Lanes past the last line repeat it and
// write the same bytes as its own lane.
//
// The line is held as 4 bytes per register, positions in chunks of 16 under
// wave-uniform branches (register indices must be compile-time constants,
// so every chunk and step is unrolled).  Positions from m up to the end of
// the last chunk repeat the line's last value: a repeated value never lowers
// the result at a real position (position m-1 offers the same value at a
// smaller distance), so both passes run over whole chunks.  Stores of those
// positions go to position m-1 before its own store, which comes later in
// the backward pass and is the one that stays (program order of one lane's
// stores to one address).
//
// A tile whose every byte is 255 (no occupied brick anywhere near its
// lines) is left as it is: the result equals the input.
// ---------------------------------------------------------------------------
constexpr int kLineWords = kMaxLine / 4;  // registers holding a line of up to 256 bytes
constexpr int kLineChunk = 16;           // positions per wave-uniform branch
constexpr int kLineChunks = kMaxLine / kLineChunk;
constexpr int kBufferFlags = 0x00020000;  // raw buffer, 32-bit data format (gfx9 family)

__device__ __forceinline__ int line_byte(uint32_t w, int k) {
    return (int)__builtin_amdgcn_ubfe(w, 8u * (unsigned)k, 8u);
}

// Bytes of LDS, addressed by 32-bit LDS offsets.
typedef __attribute__((address_space(3))) uint8_t lds_u8;

// A lane's column of a table: the table's LDS offset plus the lane, kept
// opaque in a register, so that an entry's address is one multiply-add of
// the row.  (For a table in dynamic LDS the compiler otherwise adds the
// table's base on every access, one more instruction on the scan's chain.)
__device__ __forceinline__ lds_u8* lane_column(uint8_t* tbl, int lane) {
    uint32_t a = (uint32_t)(uintptr_t)(lds_u8*)tbl + (uint32_t)lane;
    __asm__ volatile("" : "+v"(a));
    return (lds_u8*)(uintptr_t)a;
}

// The table of a pass over lines of m bricks: values are clamped at
// s = min(m, 255), so rows 0..s.
__host__ __device__ constexpr int scan_rows(int m) { return (m < 255 ? m : 255) + 1; }
__host__ __device__ constexpr int scan_table_bytes(int m) { return (scan_rows(m) * kPitch + 15) & ~15; }

// The two-sided pass of one line per lane, the line in registers: lane's
// line at byte offsets voff + p * stride (p < m <= 256) from `base`, all
// offsets below 2^31.  `tbl` holds scan_table_bytes(m) bytes with CLAMP,
// else scan_table_bytes(255).  Called by the whole wave; returns early (all
// lanes) when every byte of the wave's lines is 255.
//
// With CLAMP, values are clamped at s = min(m, 255) on the way in, so the
// table needs s + 1 rows, not 256, and more waves fit a compute unit on short
// lines (without it the table has all 256 rows).  For m < 255 (s = m): two
// positions of one line are less than m apart, so a term max(|i-j|, f(j))
// with f(j) >= s is f(j), while every term with f(j) < s is below s.  Where
// the line holds a value below s, the clamped result is therefore below s and
// exact; where every value is at least s, the result is the line's minimum
// everywhere (and the clamped pass gives s).  The backward pass's stores take
// max(result, fix) with fix = that minimum on such lines, 0 on the others.
// For m >= 255 (s = 255) the clamp changes no value.
template <bool CLAMP>
__device__ __forceinline__ void scan_lines_regs(uint8_t* base, int voff, int stride, int m,
                                                uint8_t* __restrict__ tbl_mem) {
    using P = uint8_t;  // table entry type of PDM_SCAN_STEP
    // PDM_SCAN_STEP's table and lane: this lane's column, lane offset 0
    lds_u8* const tbl = lane_column(tbl_mem, threadIdx.x & (kScanLanes - 1));
    constexpr int lane = 0;
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(base, (short)0, 0x7FFFFFFF, kBufferFlags);
    const int last = m - 1;
    const int nch = (m + kLineChunk - 1) / kLineChunk;  // chunks holding the line
    uint32_t w[kLineWords];
    uint32_t all = 0xFFFFFFFFu;
#pragma unroll
    for (int c = 0; c < kLineChunks; ++c) {
        if (c < nch) {
            // the chunk's scalar offsets are computed here, not all at once
            // ahead of the loop (256 of them would spill)
            int st = stride, lst = last;
            __asm__ volatile("" : "+s"(st), "+s"(lst));
#pragma unroll
            for (int j = 0; j < kLineChunk / 4; ++j) {
                uint32_t b[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int pos = min(kLineChunk * c + 4 * j + k, lst);
                    b[k] = __builtin_amdgcn_raw_buffer_load_b8(rs, voff, pos * st, 0);
                }
                const uint32_t word = b[0] | (b[1] << 8) | (b[2] << 16) | (b[3] << 24);
                w[4 * c + j] = word;
                all &= word;
            }
        }
    }
    if (__ballot(all != 0xFFFFFFFFu) == 0ull) return;  // every byte 255: nothing changes
    const unsigned s = CLAMP ? (unsigned)min(m, 255) : 255u;
    const int table16 = scan_table_bytes(CLAMP ? m : 255) / 16;
    clear_rows(tbl_mem, table16);
    __syncthreads();  // work-groups of the callers are one wave
    // forward pass; the first step starts from "no candidate yet" (v above
    // every value), so it takes f(0) with witness 0 like every later one
    int v = 511, W = 0;
    unsigned lmin = 255;
#pragma unroll
    for (int c = 0; c < kLineChunks; ++c) {
        if (c < nch) {
            int pc = kLineChunk * c;  // the position in a vector register: one add per step
            __asm__ volatile("" : "+v"(pc));
#pragma unroll
            for (int j = 0; j < kLineChunk / 4; ++j) {
                uint32_t acc = 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int q = 4 * j + k;
                    const unsigned raw = (unsigned)line_byte(w[4 * c + j], k);
                    if (CLAMP) lmin = umin(lmin, raw);
                    int out;
                    PDM_SCAN_STEP(pc + q, CLAMP ? (int)umin(raw, s) : (int)raw, out);
                    acc |= (uint32_t)out << (8 * k);
                }
                w[4 * c + j] = acc;
            }
        }
    }
    __syncthreads();
    clear_rows(tbl_mem, table16);
    __syncthreads();
    const int fix = CLAMP && lmin >= s ? (int)lmin : 0;
    // backward pass from the end of the last chunk, positions counted from it
    const int pend = kLineChunk * nch - 1;
    v = 511;
    W = 0;
#pragma unroll
    for (int c = kLineChunks - 1; c >= 0; --c) {
        if (c < nch) {
            int pc = pend - kLineChunk * c;  // backward position of this chunk's first byte
            __asm__ volatile("" : "+v"(pc));
            int st = stride, lst = last;
            __asm__ volatile("" : "+s"(st), "+s"(lst));
#pragma unroll
            for (int q = kLineChunk - 1; q >= 0; --q) {
                const int fi = line_byte(w[4 * c + q / 4], q % 4);
                int out;
                PDM_SCAN_STEP(pc - q, fi, out);
                const int pos = min(kLineChunk * c + q, lst);
                __builtin_amdgcn_raw_buffer_store_b8((uint8_t)(CLAMP ? max(out, fix) : out), rs, voff,
                                                     pos * st, 0);
            }
        }
    }
}

template <bool CLAMP>
__global__ void __launch_bounds__(kScanLanes) k_dist_lines(uint8_t* __restrict__ maps, int64_t lines,
                                                           int Bx, int inner, int64_t plane,
                                                           int stride, int m, int64_t G) {
    // with CLAMP the table is the launch's dynamic LDS (scan_table_bytes(m))
    extern __shared__ __align__(16) uint8_t dyn_tbl[];
    __shared__ __align__(16) uint8_t full_tbl[CLAMP ? 16 : scan_table_bytes(255)];
    uint8_t* tbl = CLAMP ? dyn_tbl : full_tbl;
    const int64_t l0 = xcd_item(blockIdx.x) * kScanLanes;
    if (l0 >= lines) return;
    const int64_t l = min(l0 + (int64_t)threadIdx.x, lines - 1);
    const int64_t base = line_offset(l0, Bx, inner, plane, G);
    const int voff = (int)(line_offset(l, Bx, inner, plane, G) - base);
    scan_lines_regs<CLAMP>(maps + base, voff, stride, m, tbl);
}

// ---------------------------------------------------------------------------
// k_dist_pairs: the two-sided pass with two lanes per line, the line held in
// registers, for passes over few lines (one map), where the chain of steps
// of one wave sets the time.  Lanes L and L + 32 take line L of the
// work-group's 32: the lower lane runs the forward one-sided pass and the
// upper lane the backward one, each first over its half of the (padded)
// line, then -- after the two lanes swap halves -- over the half the other
// lane has finished.  A one-sided pass over the other direction's results
// gives the two-sided result, so each lane ends holding the final values of
// one half: half the chain of a one-lane pass, with no LDS tile.
//
// Both lanes of a pair run the same instructions on the same register
// indices: the upper lane holds its line reversed (register r, byte k =
// position pend - 4r - k, pend = 16*NCH - 1 the end of the padded line), so
// step s of either lane is byte s%4 of register s/4.  NCH, the chunks of 16
// positions the line spans, is a template argument because the swap
// pairs registers r and 4*NCH-1-r.  Padding repeats the line's last value,
// as in k_dist_lines.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t byte_reverse(uint32_t w) {
    return __builtin_amdgcn_perm(w, w, 0x00010203u);
}

// Steps 4*R0 .. 4*R1-1 of one lane over registers R0 .. R1-1 of its line,
// each output written over its input byte.  The step index lives in a
// vector register, reset every 16 steps (one add per step).
template <int R0, int R1, int NW>
__device__ __forceinline__ void pairs_phase(uint32_t (&w)[NW], uint8_t* __restrict__ tbl, int lane,
                                            int& v, int& W) {
    using P = uint8_t;  // table entry type of PDM_SCAN_STEP
    int pc = 0;
    int pbase = 0;
#pragma unroll
    for (int r = R0; r < R1; ++r) {
        if (r == R0 || r % 4 == 0) {
            pbase = 4 * r;
            pc = pbase;
            __asm__ volatile("" : "+v"(pc));
        }
        uint32_t acc = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            int out;
            PDM_SCAN_STEP(pc + (4 * r - pbase) + k, line_byte(w[r], k), out);
            acc |= (uint32_t)out << (8 * k);
        }
        w[r] = acc;
    }
}

template <int NCH>
__global__ void __launch_bounds__(kScanLanes) k_dist_pairs(uint8_t* __restrict__ maps, int64_t lines,
                                                           int Bx, int inner, int64_t plane,
                                                           int stride, int m, int64_t G, int wide) {
    constexpr int NW = 4 * NCH;          // registers per line
    constexpr int H = 8 * NCH;           // steps per phase (half the padded line)
    constexpr int KS = (16 * NCH + 31) / 32;  // staging rounds of 32 positions
    // the table; before and after the passes also the staging tile [pos][32]
    __shared__ __align__(16) uint8_t tbl[(kRows * kPitch + 15) & ~15];
    static_assert(32 * kMaxLine <= (int)sizeof(tbl), "the staging tile fits in the table's space");
    const int lane = threadIdx.x;
    const bool upper = lane >= 32;
    const int li = lane & 31;
    const int64_t l0 = xcd_item(blockIdx.x) * 32;
    if (l0 >= lines) return;
    const int64_t l = min(l0 + (int64_t)li, lines - 1);
    const int64_t base = line_offset(l0, Bx, inner, plane, G);
    const int voff = (int)(line_offset(l, Bx, inner, plane, G) - base);
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(maps + base, (short)0, 0x7FFFFFFF, kBufferFlags);
    const int last = m - 1;
    uint32_t w[NW];
    uint32_t all = 0xFFFFFFFFu;
    // wide: the tile passes through LDS in slots of 32 bytes (one position of
    // the 32 lines): slot s < H holds position s, slot H + s position pend - s,
    // so each lane reads only its half, already in its own step order, from
    // slot (upper ? H : 0) + s
    const int half_base = li + (upper ? 32 * H : 0);
    if (wide) {
        // the 32 lines are x0 .. x0+31 of one row and rows are 16-byte
        // aligned: load the tile in 16-byte pieces (two per position, all in
        // flight at once; rows past the line repeat row m-1), store them to
        // their slots, then each lane gathers its half column
        const int q = lane & 1;
        uint4 piece[KS];
#pragma unroll
        for (int k = 0; k < KS; ++k)
            piece[k] = *reinterpret_cast<const uint4*>(
                maps + base + (int64_t)min((lane >> 1) + 32 * k, last) * stride + 16 * q);
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const int r = (lane >> 1) + 32 * k;
            const int slot = r < H ? r : 3 * H - 1 - r;
            if (r < 2 * H) *reinterpret_cast<uint4*>(&tbl[slot * 32 + 16 * q]) = piece[k];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < NW / 2; ++r) {
            uint32_t b[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) b[k] = tbl[half_base + (4 * r + k) * 32];
            w[r] = b[0] | (b[1] << 8) | (b[2] << 16) | (b[3] << 24);
            all &= w[r];
        }
        __syncthreads();  // the tile is read: its space becomes the table
    } else {
#pragma unroll
        for (int r = 0; r < NW; ++r) {
            uint32_t b[4];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                b[k] = __builtin_amdgcn_raw_buffer_load_b8(rs, voff, min(4 * r + k, last) * stride, 0);
            w[r] = b[0] | (b[1] << 8) | (b[2] << 16) | (b[3] << 24);
            all &= w[r];
        }
        // the upper lane's half in backward order
#pragma unroll
        for (int j = 0; j < NW / 2; ++j) w[j] = upper ? byte_reverse(w[NW - 1 - j]) : w[j];
    }
    if (__ballot(all != 0xFFFFFFFFu) == 0ull) return;  // every byte 255: nothing changes
    clear_table<uint8_t>(tbl);
    __syncthreads();
    int v = 511, W = 0;
    // phase 1: steps 0 .. H-1 (registers 0 .. NW/2-1) over the lane's own half
    pairs_phase<0, NW / 2>(w, tbl, lane, v, W);
    // swap halves: register r (r >= NW/2) takes the other lane's register
    // NW-1-r, reversed into this lane's order
#pragma unroll
    for (int r = NW / 2; r < NW; ++r)
        w[r] = byte_reverse((uint32_t)__shfl_xor((int)w[NW - 1 - r], 32, kScanLanes));
    // phase 2: steps H .. 2H-1 (registers NW/2 .. NW-1) over the other lane's results
    pairs_phase<NW / 2, NW>(w, tbl, lane, v, W);
    // the lower lane holds positions H .. pend in order (step H + s is
    // position H + s); the upper lane positions H-1 .. 0 (step H + s is
    // position H - 1 - s)
    if (wide) {
        // back through the slots: step H + s of either lane goes to slot
        // (upper ? H : 0) + s, which holds position H + s (lower) or
        // H - 1 - s (upper); rows leave in 16-byte pieces, positions of the
        // padding are never stored
        __syncthreads();  // every lane is done with the table
#pragma unroll
        for (int r = NW / 2; r < NW; ++r)
#pragma unroll
            for (int k = 0; k < 4; ++k)
                tbl[half_base + (4 * (r - NW / 2) + k) * 32] = (uint8_t)(w[r] >> (8 * k));
        __syncthreads();
        const int q = lane & 1;
        uint4 piece[KS];
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const int r = min((lane >> 1) + 32 * k, 2 * H - 1);
            const int slot = r >= H ? r - H : 2 * H - 1 - r;
            piece[k] = *reinterpret_cast<const uint4*>(&tbl[slot * 32 + 16 * q]);
        }
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const int r = (lane >> 1) + 32 * k;
            if (r < m) *reinterpret_cast<uint4*>(maps + base + (int64_t)r * stride + 16 * q) = piece[k];
        }
        return;
    }
#pragma unroll
    for (int j = 0; j < NW / 2; ++j) w[j] = byte_reverse(w[NW - 1 - j]);
    if (upper) {
        // positions 0 .. H-1: all inside the line (m > 16*(NCH-1) >= H for NCH >= 2)
#pragma unroll
        for (int r = 0; r < NW / 2; ++r)
#pragma unroll
            for (int k = 0; k < 4; ++k)
                __builtin_amdgcn_raw_buffer_store_b8((uint8_t)(w[r] >> (8 * k)), rs, voff,
                                                     (4 * r + k) * stride, 0);
    } else {
        // positions H .. pend, last first: stores of padded positions go to
        // position m-1 before its own store
#pragma unroll
        for (int r = NW - 1; r >= NW / 2; --r)
#pragma unroll
            for (int k = 3; k >= 0; --k)
                __builtin_amdgcn_raw_buffer_store_b8((uint8_t)(w[r] >> (8 * k)), rs, voff,
                                                     min(4 * r + k, last) * stride, 0);
    }
}

#undef PDM_SCAN_STEP

// Lines of at most kMaxLine bricks.  One wave per work-group handles 64
// lines, staged into LDS ([pos][lane], 64 bytes per position) so that no
// step waits on global memory.  With `wide` set (the 64 lines are
// x0..x0+63 of one row and rows are 16-byte aligned) the staging moves 16
// bytes per lane per instruction, 16 positions per wave instruction;
// otherwise one byte per lane.
__global__ void __launch_bounds__(kScanLanes) k_dist_axis(uint8_t* __restrict__ maps, int64_t lines,
                                                          int Bx, int inner, int64_t plane,
                                                          int64_t stride, int m, int64_t G,
                                                          int wide) {
    __shared__ __align__(16) uint8_t tbl[(kRows * kPitch + 15) & ~15];
    __shared__ __align__(16) uint8_t tile[kMaxLine * kScanLanes];
    const int lane = threadIdx.x;
    const int64_t l0 = xcd_item(blockIdx.x) * kScanLanes;
    if (l0 >= lines) return;
    const int64_t l = l0 + lane;
    const bool active = l < lines;
    const int q = lane & 3;  // 16-byte quarter of a 64-byte row
    if (wide) {
        const uint8_t* base = maps + line_offset(l0, Bx, inner, plane, G);
        for (int r = lane >> 2; r < m; r += 16)
            *reinterpret_cast<uint4*>(&tile[r * kScanLanes + 16 * q]) =
                *reinterpret_cast<const uint4*>(base + (int64_t)r * stride + 16 * q);
    } else {
        const uint8_t* line = maps + (active ? line_offset(l, Bx, inner, plane, G) : 0);
        for (int r = 0; r < m; ++r)
            tile[r * kScanLanes + lane] = active ? line[(int64_t)r * stride] : (uint8_t)0;
    }
    clear_table<uint8_t>(tbl);
    __syncthreads();
    one_sided_lds<uint8_t, 16>(&tile[lane], kScanLanes, m, tbl);
    __syncthreads();
    clear_table<uint8_t>(tbl);
    __syncthreads();
    one_sided_lds<uint8_t, 16>(&tile[(m - 1) * kScanLanes + lane], -kScanLanes, m, tbl);
    __syncthreads();
    if (wide) {
        uint8_t* base = maps + line_offset(l0, Bx, inner, plane, G);
        for (int r = lane >> 2; r < m; r += 16)
            *reinterpret_cast<uint4*>(base + (int64_t)r * stride + 16 * q) =
                *reinterpret_cast<const uint4*>(&tile[r * kScanLanes + 16 * q]);
    } else if (active) {
        uint8_t* line = maps + line_offset(l, Bx, inner, plane, G);
        for (int r = 0; r < m; ++r) line[(int64_t)r * stride] = tile[r * kScanLanes + lane];
    }
}

// Split pass, 32 lines per wave: lanes 0-31 run the forward one-sided pass
// of lines 0-31 and lanes 32-63 the backward pass of the same lines at the
// same time, each first over its half of the line (phase 1), then over the
// half the other lane has finished (phase 2).  A one-sided pass over the
// other direction's results gives the two-sided result, so [h, m) ends
// with the values the forward lane wrote in phase 2 and [0, h) with the
// backward lane's: both two-sided.  Halves never touch the same position in
// the same step; for odd m the backward lane's last phase-1 step and the
// forward lane's first phase-2 step (both at position h) run one after the
// other.  Values are clamped at vmax = min(m, 255) (table rows vmax + 3): a
// pass over min(f, m) gives min(g, m), and a result of m means every value
// of the line is >= m, where the two-sided result is the line's minimum.
// The chain is half that of k_dist_axis for 1.5x its LDS per line; the
// launcher takes it when every work-group fits at once.
__global__ void __launch_bounds__(kScanLanes) k_dist_split(uint8_t* __restrict__ maps, int64_t lines,
                                                           int Bx, int inner, int64_t plane,
                                                           int64_t stride, int m, int64_t G,
                                                           int rows, int wide) {
    extern __shared__ __align__(16) uint8_t smem[];
    uint8_t* tbl = smem;
    uint8_t* tile = smem + ((rows * kPitch + 15) & ~15);  // [pos][32]
    const int lane = threadIdx.x;
    const int half = lane >> 5, li = lane & 31;
    const int64_t l0 = xcd_item(blockIdx.x) * 32;
    if (l0 >= lines) return;
    const int64_t l = l0 + li;
    const bool active = l < lines;
    if (wide) {
        // 32 lines = x0..x0+31 of one row: two 16-byte pieces per position
        const uint8_t* base = maps + line_offset(l0, Bx, inner, plane, G);
        const int q = lane & 1;
        for (int r = lane >> 1; r < m; r += 32)
            *reinterpret_cast<uint4*>(&tile[r * 32 + 16 * q]) =
                *reinterpret_cast<const uint4*>(base + (int64_t)r * stride + 16 * q);
    } else {
        const uint8_t* line = maps + (active ? line_offset(l, Bx, inner, plane, G) : 0);
        for (int r = half; r < m; r += 2) tile[r * 32 + li] = active ? line[(int64_t)r * stride] : (uint8_t)0;
    }
    {
        const int bytes = ((rows * kPitch + 15) & ~15) / 16;
        uint4* t4 = reinterpret_cast<uint4*>(tbl);
        for (int i = lane; i < bytes; i += kScanLanes) t4[i] = make_uint4(0, 0, 0, 0);
    }
    __syncthreads();
    const int vmax = min(m, 255);
    const int h = m / 2;
    uint8_t* col = half == 0 ? &tile[li] : &tile[(m - 1) * 32 + li];
    const int cs = half == 0 ? 32 : -32;
    int raw_min = col[0];
    int v = min(raw_min, vmax);
    int W = 0;
    // phase 1: forward lanes steps [1, h), backward lanes [1, m - h)
    one_sided_lds_range<16>(col, cs, 1, h, vmax, true, tbl, v, W, raw_min);
    if (m - h > h && half == 1)
        one_sided_lds_range<1>(col, cs, h, h + 1, vmax, true, tbl, v, W, raw_min);
    __builtin_amdgcn_wave_barrier();
    const int lmin = min(raw_min, __shfl_xor(raw_min, 32, kScanLanes));
    // phase 2: forward lanes steps [h, m), backward lanes [m - h, m)
    if (m - h > h && half == 0)
        one_sided_lds_range<1>(col, cs, h, h + 1, vmax, false, tbl, v, W, raw_min);
    __builtin_amdgcn_wave_barrier();
    one_sided_lds_range<16>(col, cs, m - h, m, vmax, false, tbl, v, W, raw_min);
    // every value of the line >= vmax: the two-sided result is the minimum
    if (lmin >= vmax) {
        const int n = half == 0 ? m - h : h;  // this lane's phase-2 positions
        for (int k = 0; k < n; ++k) col[(m - 1 - k) * cs] = (uint8_t)lmin;
    }
    __syncthreads();
    if (wide) {
        uint8_t* base = maps + line_offset(l0, Bx, inner, plane, G);
        const int q = lane & 1;
        for (int r = lane >> 1; r < m; r += 32)
            *reinterpret_cast<uint4*>(base + (int64_t)r * stride + 16 * q) =
                *reinterpret_cast<const uint4*>(&tile[r * 32 + 16 * q]);
    } else if (active) {
        uint8_t* line = maps + line_offset(l, Bx, inner, plane, G);
        for (int r = half; r < m; r += 2) line[(int64_t)r * stride] = tile[r * 32 + li];
    }
}

// The scan on global memory directly, one lane per line, 64 lanes per
// work-group and only the table in LDS (17.4 KB with 8-bit entries), so up to
// nine waves share a compute unit: the choice when the passes cover many
// lines (all partitions at once) and occupancy hides the memory latency.
// P = uint16_t serves lines longer than 256 bricks (positions beyond 255).
template <typename P, int CH>
__global__ void __launch_bounds__(kScanLanes) k_dist_global(uint8_t* __restrict__ maps,
                                                            int64_t lines, int Bx, int inner,
                                                            int64_t plane, int64_t stride, int m,
                                                            int64_t G) {
    __shared__ __align__(16) P tbl[((kRows * kPitch * sizeof(P) + 15) & ~15) / sizeof(P)];
    const int64_t l0 = xcd_item(blockIdx.x) * kScanLanes;
    if (l0 >= lines) return;
    const int64_t l = l0 + threadIdx.x;
    const bool active = l < lines;
    uint8_t* line = maps + (active ? line_offset(l, Bx, inner, plane, G) : 0);
    clear_table<P>(tbl);
    __syncthreads();
    one_sided_global<P, CH>(line, stride, m, active, tbl);
    __syncthreads();
    clear_table<P>(tbl);
    __syncthreads();
    one_sided_global<P, CH>(line + (int64_t)(m - 1) * stride, -stride, m, active, tbl);
}

// ---------------------------------------------------------------------------
// k_combine: D'[c] = min over the listed maps of map[c] (the active
// partitions' PDMs, or range-table maps covering them).
// A map of G >= 16 bytes is cut into ceil(G/16) chunks of 16 bytes; chunk c
// starts at min(16c, G - 16), so the last chunk ends at G and overlaps its
// neighbour, whose lane writes the same bytes there.  Chunks are loaded and
// stored at any byte alignment (the hardware serves unaligned vector
// accesses), so every size and every base pointer take the chunked path.
// CHUNKS = chunks per lane:
//   2  large maps: chunks t and t + nthr, maps two at a time (four 16-byte
//      non-temporal loads in flight; every load instruction of a wave covers
//      1 KiB of one stream).  Measured best on runs of consecutive PDMs.
//   1  small maps (too few chunks to give every CU several work-groups with
//      two per lane): one chunk per lane, maps four at a time.
//   0  maps of fewer than 16 bytes: one byte per lane.
// The running minimum is kept as even/odd byte pairs in packed u16 lanes.
// An empty list writes 255.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void min_bytes16(uint32_t (&e)[4], uint32_t (&o)[4], const u32x4 w) {
    e[0] = pk_min16(e[0], even_bytes(w.x));
    o[0] = pk_min16(o[0], odd_bytes(w.x));
    e[1] = pk_min16(e[1], even_bytes(w.y));
    o[1] = pk_min16(o[1], odd_bytes(w.y));
    e[2] = pk_min16(e[2], even_bytes(w.z));
    o[2] = pk_min16(o[2], odd_bytes(w.z));
    e[3] = pk_min16(e[3], even_bytes(w.w));
    o[3] = pk_min16(o[3], odd_bytes(w.w));
}

__device__ __forceinline__ int64_t chunk_off(int64_t c, int64_t G) {
    return 16 * c < G - 16 ? 16 * c : G - 16;
}

__device__ __forceinline__ void store16_u(PDM_GLB uint8_t* p, const u32x4 v) {
    *reinterpret_cast<PDM_GLB u32x4_u*>(p) = v;
}

typedef const PDM_GLB uint8_t* MapPtr;

// Minimum of one 16-byte chunk over the maps added so far.
struct ChunkMin {
    uint32_t e[4], o[4];

    __device__ __forceinline__ ChunkMin() {
#pragma unroll
        for (int k = 0; k < 4; ++k) e[k] = o[k] = 0x00FF00FFu;
    }
    __device__ __forceinline__ void add(const u32x4 w) { min_bytes16(e, o, w); }
    // N maps: every load issued before the first minimum
    template <int N>
    __device__ __forceinline__ void add(const MapPtr (&m)[N], int64_t off) {
        u32x4 w[N];
#pragma unroll
        for (int i = 0; i < N; ++i) w[i] = load16_nt(m[i] + off);
#pragma unroll
        for (int i = 0; i < N; ++i) min_bytes16(e, o, w[i]);
    }
    __device__ __forceinline__ void store(PDM_GLB uint8_t* out, int64_t off) const {
        u32x4 r;
        r.x = e[0] | (o[0] << 8);
        r.y = e[1] | (o[1] << 8);
        r.z = e[2] | (o[2] << 8);
        r.w = e[3] | (o[3] << 8);
        store16_u(out + off, r);
    }
};

template <typename T>
__device__ __forceinline__ const PDM_GLB T* glb(const T* p) {
    return (const PDM_GLB T*)p;
}
template <typename T>
__device__ __forceinline__ PDM_GLB T* glb(T* p) {
    return (PDM_GLB T*)p;
}

template <int CHUNKS>
__global__ void __launch_bounds__(256) k_combine(MapList maps, int64_t G, uint8_t* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int cnt = maps.count;
    if constexpr (CHUNKS == 2) {
        const int64_t nch = (G + 15) / 16;
        const int64_t nthr = (int64_t)gridDim.x * blockDim.x;
        const int64_t i0 = t, i1 = t + nthr;
        if (i0 >= nch) return;
        const bool two = i1 < nch;
        const int64_t o0 = chunk_off(i0, G), o1 = two ? chunk_off(i1, G) : o0;
        ChunkMin c0, c1;
        int j = 0;
        for (; j + 2 <= cnt; j += 2) {
            const MapPtr pa = glb(maps.src[j]), pb = glb(maps.src[j + 1]);
            const u32x4 a0 = load16_nt(pa + o0), a1 = load16_nt(pa + o1);
            const u32x4 b0 = load16_nt(pb + o0), b1 = load16_nt(pb + o1);
            c0.add(a0);
            c1.add(a1);
            c0.add(b0);
            c1.add(b1);
        }
        if (j < cnt) {
            const MapPtr pa = glb(maps.src[j]);
            const u32x4 a0 = load16_nt(pa + o0), a1 = load16_nt(pa + o1);
            c0.add(a0);
            c1.add(a1);
        }
        c0.store(glb(out), o0);
        if (two) c1.store(glb(out), o1);
    } else if constexpr (CHUNKS == 1) {
        if (t >= (G + 15) / 16) return;
        const int64_t off = chunk_off(t, G);
        ChunkMin acc;
        int j = 0;
        for (; j + 4 <= cnt; j += 4) {
            const MapPtr m[4] = {glb(maps.src[j]), glb(maps.src[j + 1]), glb(maps.src[j + 2]),
                                 glb(maps.src[j + 3])};
            acc.add(m, off);
        }
        if (cnt - j == 3) {
            const MapPtr m[3] = {glb(maps.src[j]), glb(maps.src[j + 1]), glb(maps.src[j + 2])};
            acc.add(m, off);
        } else if (cnt - j == 2) {
            const MapPtr m[2] = {glb(maps.src[j]), glb(maps.src[j + 1])};
            acc.add(m, off);
        } else if (cnt - j == 1) {
            const MapPtr m[1] = {glb(maps.src[j])};
            acc.add(m, off);
        }
        acc.store(glb(out), off);
    } else {
        if (t >= G) return;
        uint32_t m = 255u;
        for (int j = 0; j < cnt; ++j) m = umin(m, (uint32_t)maps.src[j][t]);
        out[t] = (uint8_t)m;
    }
}

// ---------------------------------------------------------------------------
// k_range_level: one level of the range table, dst[p] = min(src[p], src[p+h])
// element-wise over maps of G bytes, i.e. over the flat `total` bytes of the
// destination maps.  VEC = 16 cuts the flat range into 16-byte chunks as
// k_combine does (total >= 16, any alignment); VEC = 1 otherwise.
// ---------------------------------------------------------------------------
template <int VEC>
__global__ void __launch_bounds__(256) k_range_level(const uint8_t* __restrict__ src, int64_t h,
                                                     uint8_t* __restrict__ dst, int64_t total,
                                                     int64_t G) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if constexpr (VEC == 16) {
        if (t >= (total + 15) / 16) return;
        const int64_t off = chunk_off(t, total);
        const MapPtr m[2] = {glb(src), glb(src) + h * G};
        ChunkMin acc;
        acc.add(m, off);
        acc.store(glb(dst), off);
    } else {
        if (t >= total) return;
        dst[t] = (uint8_t)umin((uint32_t)src[t], (uint32_t)src[t + h * G]);
    }
}

// ---------------------------------------------------------------------------
// k_batch_combine: the TF update of many volumes in one launch.  Each volume
// has its own PDM stack, output map and active set (a 256-bit mask); blocks
// are assigned to volumes by the prefix counts in first_block (a binary
// search), so every work-group serves one volume and its control values are
// uniform.  Within a volume the work is that of k_combine for small maps
// (batched volumes are mostly small): one 16-byte chunk per lane at any size
// and alignment, the active PDMs taken four at a time; volumes of fewer than
// 16 bricks take a byte path.
// ---------------------------------------------------------------------------
// The set bits of a 256-bit mask in increasing order: the current word and
// its index are kept (in scalar registers: the mask is uniform), the next
// word is read from the argument when one runs out.
struct BitWalk {
    const uint64_t* words;
    uint64_t cur;
    int w;

    __device__ __forceinline__ explicit BitWalk(const uint64_t* m) : words(m), cur(m[0]), w(0) {}
    // next set bit, or -1 when none is left
    __device__ __forceinline__ int next() {
        while (cur == 0) {
            if (++w == 4) return -1;
            cur = words[w];
        }
        const int p = 64 * w + (__ffsll((unsigned long long)cur) - 1);
        cur &= cur - 1;
        return p;
    }
};

__global__ void __launch_bounds__(256) k_batch_combine(BatchArgs a) {
    int lo = 0, hi = a.count - 1;  // last volume with first_block <= blockIdx.x
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((int64_t)blockIdx.x >= a.it[mid].first_block) lo = mid;
        else hi = mid - 1;
    }
    const BatchItem& it = a.it[lo];
    const PDM_GLB uint8_t* pdms = glb(it.pdms);
    PDM_GLB uint8_t* out = glb(it.out);
    const int64_t G = it.G;
    const int64_t t = ((int64_t)blockIdx.x - it.first_block) * blockDim.x + threadIdx.x;
    BitWalk bits(it.mask);
    if (G >= 16) {
        if (t >= (G + 15) / 16) return;
        const int64_t off = chunk_off(t, G);
        ChunkMin acc;
        for (;;) {  // four active PDMs per step, then the last one to three
            const int p0 = bits.next();
            if (p0 < 0) break;
            const int p1 = bits.next();
            const int p2 = p1 < 0 ? -1 : bits.next();
            const int p3 = p2 < 0 ? -1 : bits.next();
            if (p3 >= 0) {
                const MapPtr m[4] = {pdms + (int64_t)p0 * G, pdms + (int64_t)p1 * G,
                                     pdms + (int64_t)p2 * G, pdms + (int64_t)p3 * G};
                acc.add(m, off);
                continue;
            }
            if (p2 >= 0) {
                const MapPtr m[3] = {pdms + (int64_t)p0 * G, pdms + (int64_t)p1 * G,
                                     pdms + (int64_t)p2 * G};
                acc.add(m, off);
            } else if (p1 >= 0) {
                const MapPtr m[2] = {pdms + (int64_t)p0 * G, pdms + (int64_t)p1 * G};
                acc.add(m, off);
            } else {
                const MapPtr m[1] = {pdms + (int64_t)p0 * G};
                acc.add(m, off);
            }
            break;
        }
        acc.store(out, off);
    } else {
        if (t >= G) return;
        uint32_t v = 255u;
        for (int p = bits.next(); p >= 0; p = bits.next()) v = umin(v, (uint32_t)pdms[(int64_t)p * G + t]);
        out[t] = (uint8_t)v;
    }
}

// ---------------------------------------------------------------------------
// k_batch_combine_maps: the updates of many requests through range tables in
// one launch.  Each request lists the maps of its cover (PDMs or table maps
// of its own volume); work-groups find their request by binary search as in
// k_batch_combine, and a lane min-combines one 16-byte chunk of the listed
// maps, four at a time (an empty list writes 255); requests of fewer than 16
// bricks take a byte path.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_batch_combine_maps(BatchMapsArgs a) {
    int lo = 0, hi = a.count - 1;  // last request with first_block <= blockIdx.x
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((int64_t)blockIdx.x >= a.it[mid].first_block) lo = mid;
        else hi = mid - 1;
    }
    const MapsItem& it = a.it[lo];
    const PDM_GLB uint8_t* pdms = glb(it.pdms);
    const PDM_GLB uint8_t* table = glb(it.table);
    PDM_GLB uint8_t* out = glb(it.out);
    const int64_t G = it.G;
    const int n = it.n, cnt = it.map_count, first = it.map_first;
    const int64_t t = ((int64_t)blockIdx.x - it.first_block) * blockDim.x + threadIdx.x;
    // indices read as 32-bit words at uniform addresses: scalar loads through
    // the scalar cache (a 16-bit read would be a vector load per lane from
    // the argument buffer)
    const uint32_t* ix32 = reinterpret_cast<const uint32_t*>(a.idx);
    auto map = [&](int j) -> MapPtr {
        const int k = first + j;
        const uint32_t w = ix32[k >> 1];
        const int q = (int)((k & 1) ? (w >> 16) : (w & 0xFFFFu));
        return q < n ? pdms + (int64_t)q * G : table + (int64_t)(q - n) * G;
    };
    if (G >= 16) {
        if (t >= (G + 15) / 16) return;
        const int64_t off = chunk_off(t, G);
        ChunkMin acc;
        int j = 0;
        for (; j + 4 <= cnt; j += 4) {
            const MapPtr m[4] = {map(j), map(j + 1), map(j + 2), map(j + 3)};
            acc.add(m, off);
        }
        if (cnt - j == 3) {
            const MapPtr m[3] = {map(j), map(j + 1), map(j + 2)};
            acc.add(m, off);
        } else if (cnt - j == 2) {
            const MapPtr m[2] = {map(j), map(j + 1)};
            acc.add(m, off);
        } else if (cnt - j == 1) {
            const MapPtr m[1] = {map(j)};
            acc.add(m, off);
        }
        acc.store(out, off);
    } else {
        if (t >= G) return;
        uint32_t v = 255u;
        for (int j = 0; j < cnt; ++j) v = umin(v, (uint32_t)map(j)[t]);
        out[t] = (uint8_t)v;
    }
}

// ---------------------------------------------------------------------------
// Batched build: the one-time initialisation of many volumes in three
// grouped launches, each covering every volume of the batch:
//   rows  item (volume, z slice, group of brick rows): brick [min,max] of the
//         rows, then every partition's POM row and x distances (bricks and
//         POM x fused: the volume is read once);
//   y     item (volume, z slice, chunk of 64*lines_mult lines (p, x));
//   z     item (volume, y row, chunk of 64*lines_mult lines (p, x)).
// Launch boundaries order the phases, so no work-group waits on another.
// The items of a phase are numbered volume by volume in descriptor order
// (first[ph] is the running prefix).  Work-groups are handed to the XCDs
// round-robin; xcd_item maps them so that runs of kXcdRun consecutive items
// land on one XCD.
// ---------------------------------------------------------------------------
// The volume holding item t of phase ph: the last descriptor whose first
// item is <= t (volumes with no items in the phase share the next one's
// first and are skipped by taking the last).
__device__ __forceinline__ int batch_volume_of(const BatchVol* __restrict__ vols, int count, int ph,
                                               int64_t t) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (vols[mid].first[ph] <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// First phase for brick rows [by0, by1) of z slice bz.  A row of Bx <= 256
// bricks takes W = row_lanes lanes (4 bricks each, W the power of two >=
// Bx/4), so one wave pass covers 64/W rows.
template <typename T>
__device__ __forceinline__ void batch_rows(const BatchVol& d, int bz, int by0, int by1) {
    const int lane = threadIdx.x;
    const PDM_GLB T* vol = (const PDM_GLB T*)d.vol;
    PDM_GLB T* bmin = (PDM_GLB T*)d.bmin;
    PDM_GLB T* bmax = (PDM_GLB T*)d.bmax;
    PDM_GLB uint8_t* pdms = (PDM_GLB uint8_t*)d.pdms;
    // descriptor fields in registers: the map stores below could alias the
    // descriptor as far as the compiler knows, which would reload them per
    // partition
    const int W = d.row_lanes;
    const int n = d.n, Bx = d.Bx, By = d.By;
    const int64_t G = d.G;
    const bool vec = d.store_vec != 0;
    const PDM_GLB int32_t* bounds = (const PDM_GLB int32_t*)d.bounds;
    const int q = lane & (W - 1);
    const int per = kWave / W;
    const int nb_row = max(0, min(4, Bx - 4 * q));
    for (int row0 = by0; row0 < by1; row0 += per) {
        const int by = row0 + lane / W;
        const int nb = by < by1 ? nb_row : 0;
        const int64_t rbase = ((int64_t)bz * By + by) * Bx + 4 * q;
        uint32_t mn[4] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu};
        uint32_t mx[4] = {0u, 0u, 0u, 0u};
        if (nb > 0) {
            const QuadMinMax<T> r = quad_minmax<T>(vol, d.nx, d.ny, d.nz, q, by, bz);
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (k < nb) {
                    mn[k] = r.mn[k];
                    mx[k] = r.mx[k];
                }
            if (nb == 4) {
                store_bricks4<T>(bmin + rbase, bmax + rbase, r);
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (k < nb) {
                        bmin[rbase + k] = (T)r.mn[k];
                        bmax[rbase + k] = (T)r.mx[k];
                    }
            }
        }
        uint32_t wmin, wmax;
        wave_value_range(mn, mx, wmin, wmax);
        uint32_t lo = (uint32_t)bounds[0];
        for (int p = 0; p < n; ++p) {
            const uint32_t next = (uint32_t)bounds[p + 1], hi = next - 1u;
            uint32_t packed = 0xFFFFFFFFu;
            if (hi >= wmin && lo <= wmax) {
                uint32_t o = 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) o |= (mn[k] <= hi && mx[k] >= lo) ? (1u << k) : 0u;
                packed = x_distances_rows(o, lane, W);
            }
            if (nb > 0) store_quad(pdms + (int64_t)p * G, rbase, nb, packed, vec);
            lo = next;
        }
    }
}

__device__ __forceinline__ void batch_rows_item(const BatchVol* __restrict__ vols, int count,
                                                int64_t t) {
    const BatchVol& d = vols[batch_volume_of(vols, count, 0, t)];
    const int64_t local = t - d.first[0];
    const int bz = (int)(local / d.row_groups);
    const int by0 = (int)(local % d.row_groups) * d.rows;
    const int by1 = min(d.By, by0 + d.rows);
    if (d.bytes == 1)
        batch_rows<uint8_t>(d, bz, by0, by1);
    else
        batch_rows<uint16_t>(d, bz, by0, by1);
}

// ph 1: y passes, ph 2: z passes of one item (64*lines_mult lines).
__device__ __forceinline__ void batch_scan_item(const BatchVol* __restrict__ vols, int count, int ph,
                                                int64_t t, int lines_mult, uint8_t* tbl) {
    const int lane = threadIdx.x;
    const BatchVol& d = vols[batch_volume_of(vols, count, ph, t)];
    const int64_t local = t - d.first[ph];
    const int outer = (int)(local / d.chunks);  // z slice (phase 1) or y row (phase 2)
    const int m = ph == 1 ? d.By : d.Bz;
    if (m <= 1) return;  // a line of one brick is unchanged
    const int stride = ph == 1 ? d.Bx : d.Bx * d.By;  // <= 2^16: axes of at most 256 bricks
    const int64_t plane = ph == 1 ? (int64_t)outer * d.Bx * d.By : (int64_t)outer * d.Bx;
    const int64_t nlines = (int64_t)d.n * d.Bx;
    // offset of line (p, x) of this slice or row
    auto offset = [&](int64_t line) { return (line / d.Bx) * d.G + plane + line % d.Bx; };
    for (int j = 0; j < lines_mult; ++j) {
        // (p, x) lines of this slice or row, 64 per pass of the wave; lanes
        // past the last line repeat it
        const int64_t g0 = ((local % d.chunks) * lines_mult + j) * kWave;
        if (g0 >= nlines) break;  // wave-uniform
        const int64_t line = min(g0 + (int64_t)lane, nlines - 1);
        const int64_t off0 = offset(g0);
        // at most 64 lines apart: below 64 maps of at most 2^24 bricks
        scan_lines_regs<true>((uint8_t*)d.pdms + off0, (int)(offset(line) - off0), stride, m, tbl);
    }
}

__global__ void __launch_bounds__(kWave) k_batch_rows(const BatchVol* __restrict__ vols, int count,
                                                      int64_t total) {
    const int64_t t = xcd_item(blockIdx.x);
    if (t < total) batch_rows_item(vols, count, t);
}

__global__ void __launch_bounds__(kWave) k_batch_scan(const BatchVol* __restrict__ vols, int count,
                                                      int ph, int64_t total, int lines_mult) {
    extern __shared__ __align__(16) uint8_t tbl[];  // scan_table_bytes of the longest line
    const int64_t t = xcd_item(blockIdx.x);
    if (t < total) batch_scan_item(vols, count, ph, t, lines_mult, tbl);
}

// ---------------------------------------------------------------------------
// Single-launch variant: one cooperative launch whose work-groups are all
// resident take the three phases in turn, with a grid-wide barrier between
// phases.  Within a phase each work-group takes items from the phase's
// ticket counter until none is left (items differ in cost, so a static share
// would leave work-groups idle); with lines_mult >= 2 the 64-line groups of
// one item are neighbours in x and share cache lines in the same L2.
//
// Barrier: arrivals are counted cumulatively, so barrier k is complete when
// the count reaches (k + 1) * gridDim.x; the work-group that makes it so
// advances the generation word, the others poll it.  Stores before the
// barrier are released at agent scope before the arrival, and acquired after
// it.  Every control value is wave-uniform (readfirstlane) and lane-0 atomics
// sit in plain if-blocks, so the compiler cannot move the arrival past the
// wait.  A wait is bounded by wall-clock time (the 100 MHz real-time
// counter): past the limit, or once another work-group has failed, the
// work-group sets the error word and returns, so every wave exits.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lane0_fetch_add(uint32_t* cnt, uint32_t add) {
    uint32_t r = 0;
    if (threadIdx.x == 0)
        r = __hip_atomic_fetch_add(cnt, add, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return __builtin_amdgcn_readfirstlane(r);
}

__device__ __forceinline__ uint32_t lane0_load(uint32_t* p) {
    uint32_t r = 0;
    if (threadIdx.x == 0) r = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return __builtin_amdgcn_readfirstlane(r);
}

__device__ __forceinline__ bool grid_barrier(BatchSync* st, uint32_t k, uint64_t limit_ticks) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const uint32_t arrivals = (k + 1u) * gridDim.x;
    const uint32_t before = lane0_fetch_add(&st->arrive, 1u);
    bool ok = true;
    if (before + 1u == arrivals) {
        if (threadIdx.x == 0)
            __hip_atomic_store(&st->generation, k + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
        uint32_t naps = 1;
        while (lane0_load(&st->generation) <= k) {
            if (__builtin_amdgcn_s_memrealtime() - t0 > limit_ticks || lane0_load(&st->error) != 0u) {
                ok = false;
                break;
            }
            for (uint32_t i = 0; i < naps; ++i) __builtin_amdgcn_s_sleep(127);
            naps = naps < 8u ? naps + 1u : 8u;
        }
    }
    if (!ok && threadIdx.x == 0) __hip_atomic_fetch_or(&st->error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return ok;
}

__global__ void __launch_bounds__(kWave) k_batch_single(const BatchVol* __restrict__ vols, int count,
                                                        int64_t total0, int64_t total1,
                                                        int64_t total2, int lines_mult,
                                                        BatchSync* st, uint64_t limit_ticks) {
    extern __shared__ __align__(16) uint8_t tbl[];  // scan_table_bytes of the longest line
    for (;;) {
        const int64_t t = lane0_fetch_add(&st->ticket[0][0], 1u);
        if (t >= total0) break;
        batch_rows_item(vols, count, t);
    }
    if (!grid_barrier(st, 0u, limit_ticks)) return;
    for (;;) {
        const int64_t t = lane0_fetch_add(&st->ticket[1][0], 1u);
        if (t >= total1) break;
        batch_scan_item(vols, count, 1, t, lines_mult, tbl);
    }
    if (!grid_barrier(st, 1u, limit_ticks)) return;
    for (;;) {
        const int64_t t = lane0_fetch_add(&st->ticket[2][0], 1u);
        if (t >= total2) break;
        batch_scan_item(vols, count, 2, t, lines_mult, tbl);
    }
}

// Copies descriptor bytes carried in kernel arguments to device memory; run
// before the batched build kernels on the same stream.
struct UploadChunk {
    int32_t bytes;
    int32_t pad[3];
    uint4 data[220];  // 3520 bytes
};

__global__ void __launch_bounds__(256) k_upload(uint8_t* __restrict__ dst, UploadChunk c) {
    for (int i = threadIdx.x; i < c.bytes / 16; i += blockDim.x)
        reinterpret_cast<uint4*>(dst)[i] = c.data[i];
}

__global__ void __launch_bounds__(256) k_zero(uint32_t* __restrict__ p, int words) {
    for (int i = threadIdx.x; i < words; i += blockDim.x) p[i] = 0u;
}

__global__ void __launch_bounds__(64) k_copy_word(const uint32_t* __restrict__ src,
                                                  uint32_t* __restrict__ dst) {
    if (threadIdx.x == 0) *dst = *src;
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free batched build: the barrier state and the
// descriptors of up to PDM_BATCH_MAX_ITEMS volumes, laid out as the caller's
// workspace of the other entry point (57,600 bytes).  Each device holds its
// own copy for the life of the process.  In host code `scratch` only names
// the symbol: its device address comes from hipGetSymbolAddress, looked up
// once per device with that device current and kept here.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = sizeof(BatchSync) + (size_t)PDM_BATCH_MAX_ITEMS * sizeof(BatchVol);
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kScratchDevices = 64;
static std::mutex g_scratch_mu;
static uint8_t* g_scratch_ptr[kScratchDevices];

hipError_t batch_scratch(int dev, uint8_t** ptr, size_t* bytes) {
    if (dev < 0 || dev >= kScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (p == nullptr) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = static_cast<uint8_t*>(p);
    }
    *ptr = g_scratch_ptr[dev];
    *bytes = kScratchBytes;
    return hipSuccess;
}

hipError_t launch_copy_word(const uint32_t* src, uint32_t* dst, hipStream_t s) {
    k_copy_word<<<1, 64, 0, s>>>(src, dst);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Launchers (host side).  Shapes are validated by the caller.
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(int64_t threads, int tpb) {
    return (unsigned)((threads + tpb - 1) / tpb);
}

hipError_t launch_bricks(const BrickArgs& a, hipStream_t s) {
    const int Qx = (a.Bx + 3) / 4;
    const int64_t thr = (int64_t)Qx * a.By * a.Bz;
    const unsigned nb = blocks_for(thr, 256);
    if (a.bytes == 1)
        k_bricks<uint8_t><<<nb, 256, 0, s>>>((const uint8_t*)a.vol, a.nx, a.ny, a.nz, a.Bx, a.By,
                                             a.Bz, Qx, (uint8_t*)a.bmin, (uint8_t*)a.bmax,
                                             a.levels, a.range_err);
    else
        k_bricks<uint16_t><<<nb, 256, 0, s>>>((const uint16_t*)a.vol, a.nx, a.ny, a.nz, a.Bx,
                                              a.By, a.Bz, Qx, (uint16_t*)a.bmin,
                                              (uint16_t*)a.bmax, a.levels, a.range_err);
    return hipGetLastError();
}

hipError_t launch_pom_x(const PomArgs& a, const Bounds& b, hipStream_t s) {
    const int64_t rows = (int64_t)a.By * a.Bz;
    int W = 1;  // lanes per row: the power of two with 4W >= Bx, at most a wave
    while (W < kWave && 4 * W < a.Bx) W *= 2;
    const unsigned nb = blocks_for(rows, 4 * (kWave / W));
    if (a.bytes == 1)
        k_pom_x<uint8_t><<<nb, 256, 0, s>>>((const uint8_t*)a.bmin, (const uint8_t*)a.bmax, a.Bx,
                                            rows, b, a.n, a.pdms, a.G, a.store_vec, W);
    else
        k_pom_x<uint16_t><<<nb, 256, 0, s>>>((const uint16_t*)a.bmin, (const uint16_t*)a.bmax,
                                             a.Bx, rows, b, a.n, a.pdms, a.G, a.store_vec, W);
    return hipGetLastError();
}

hipError_t launch_plain_x(const PlainArgs& a, const AlphaBits& bits, hipStream_t s) {
    const int64_t rows = (int64_t)a.By * a.Bz;
    const unsigned nb = blocks_for(rows, 4);
    // run lists only above 16384 levels, so only for 16-bit volumes
    if (a.bytes == 1)
        k_plain_x<uint8_t, false><<<nb, 256, 0, s>>>((const uint8_t*)a.vol, a.nx, a.ny, a.nz, a.Bx,
                                                     a.By, rows, bits, a.nwords, a.levels, a.dist,
                                                     a.store_vec);
    else if (!a.runs)
        k_plain_x<uint16_t, false><<<nb, 256, 0, s>>>((const uint16_t*)a.vol, a.nx, a.ny, a.nz, a.Bx,
                                                      a.By, rows, bits, a.nwords, a.levels, a.dist,
                                                      a.store_vec);
    else
        k_plain_x<uint16_t, true><<<nb, 256, 0, s>>>((const uint16_t*)a.vol, a.nx, a.ny, a.nz, a.Bx,
                                                     a.By, rows, bits, a.nwords, a.levels, a.dist,
                                                     a.store_vec);
    return hipGetLastError();
}

hipError_t launch_plain_cached_x(const CachedArgs& a, const AlphaBits& bits, hipStream_t s) {
    const int64_t rows = (int64_t)a.By * a.Bz;
    int W = 1;  // lanes per row: the power of two with 4W >= Bx, at most a wave
    while (W < kWave && 4 * W < a.Bx) W *= 2;
    // rows per wave: kCachedPasses passes of 64/W rows up to 256 bricks, else one
    const int64_t per_wave = a.Bx <= kSegBricks ? (int64_t)kCachedPasses * (kWave / W) : 1;
    const int64_t waves = (rows + per_wave - 1) / per_wave;
    const int64_t blocks = (waves + 3) / 4;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    if (a.bytes == 1)
        k_plain_cached_x<uint8_t, false><<<(unsigned)blocks, 256, 0, s>>>(
            (const uint8_t*)a.bmin, (const uint8_t*)a.bmax, a.Bx, rows, bits, a.nwords, a.levels,
            a.dist, a.store_vec, W, a.load_vec);
    else if (!a.runs)
        k_plain_cached_x<uint16_t, false><<<(unsigned)blocks, 256, 0, s>>>(
            (const uint16_t*)a.bmin, (const uint16_t*)a.bmax, a.Bx, rows, bits, a.nwords, a.levels,
            a.dist, a.store_vec, W, a.load_vec);
    else
        k_plain_cached_x<uint16_t, true><<<(unsigned)blocks, 256, 0, s>>>(
            (const uint16_t*)a.bmin, (const uint16_t*)a.bmax, a.Bx, rows, bits, a.nwords, a.levels,
            a.dist, a.store_vec, W, a.load_vec);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_pom_exact_t(const PomExactArgs& a, const Bounds& b, hipStream_t s) {
    const int64_t rows = (int64_t)a.By * a.Bz;
    int W = 1;  // lanes per row: the power of two with 4W >= Bx, at most a wave
    while (W < kWave && 4 * W < a.Bx) W *= 2;
    const unsigned nb = blocks_for(rows, 4 * (kWave / W));
    const int nw = (a.n + 31) / 32;
#define PDM_LAUNCH_EXACT(NW)                                                                   \
    do {                                                                                       \
        if (W < kWave)                                                                         \
            k_pom_exact_x<T, NW, true><<<nb, 256, 0, s>>>((const T*)a.vol, a.nx, a.ny, a.nz,     \
                                                          a.Bx, a.By, rows, b, a.n, a.levels,    \
                                                          a.pdms, a.G, a.store_vec, W);          \
        else                                                                                   \
            k_pom_exact_x<T, NW, false><<<nb, 256, 0, s>>>((const T*)a.vol, a.nx, a.ny, a.nz,    \
                                                           a.Bx, a.By, rows, b, a.n, a.levels,   \
                                                           a.pdms, a.G, a.store_vec, W);         \
    } while (0)
    if (nw == 1)
        PDM_LAUNCH_EXACT(1);
    else if (nw == 2)
        PDM_LAUNCH_EXACT(2);
    else if (nw <= 4)
        PDM_LAUNCH_EXACT(4);
    else
        PDM_LAUNCH_EXACT(8);
#undef PDM_LAUNCH_EXACT
    return hipGetLastError();
}

hipError_t launch_pom_exact_x(const PomExactArgs& a, const Bounds& b, hipStream_t s) {
    return a.bytes == 1 ? launch_pom_exact_t<uint8_t>(a, b, s) : launch_pom_exact_t<uint16_t>(a, b, s);
}

hipError_t launch_plain_exact_x(const PlainArgs& a, const AlphaBits& bits, hipStream_t s) {
    const int64_t rows = (int64_t)a.By * a.Bz;
    const unsigned nb = blocks_for(rows, 4);
    if (a.bytes == 1)
        k_plain_exact_x<uint8_t><<<nb, 256, 0, s>>>((const uint8_t*)a.vol, a.nx, a.ny, a.nz, a.Bx,
                                                    a.By, rows, bits, a.nwords, a.levels, a.dist,
                                                    a.store_vec);
    else
        k_plain_exact_x<uint16_t><<<nb, 256, 0, s>>>((const uint16_t*)a.vol, a.nx, a.ny, a.nz, a.Bx,
                                                     a.By, rows, bits, a.nwords, a.levels, a.dist,
                                                     a.store_vec);
    return hipGetLastError();
}

// Line geometry of a pass along y (axis 1) or z (axis 2) over `count` grids.
struct AxisLines {
    int64_t lines, plane, stride;
    int inner, m;
};

static AxisLines axis_lines(int count, int Bx, int By, int Bz, int axis) {
    AxisLines a;
    if (axis == 1) {  // along y: lines (g, z, x)
        a.lines = (int64_t)count * Bx * Bz;
        a.inner = Bz;
        a.plane = (int64_t)Bx * By;
        a.stride = Bx;
        a.m = By;
    } else {  // along z: lines (g, y, x)
        a.lines = (int64_t)count * Bx * By;
        a.inner = By;
        a.plane = Bx;
        a.stride = (int64_t)Bx * By;
        a.m = Bz;
    }
    return a;
}

// Whether k_dist_lines can address a tile of 64 lines with 31-bit offsets
// from the tile's first line: the largest distance between two lines of one
// tile plus the whole extent of a line.
static bool lines_fit_32(const AxisLines& a, int Bx, int64_t G) {
    // consecutive lines differ by 1 within a row; a tile that leaves a row
    // jumps by at most one map (G) plus one plane step per row it crosses
    const int64_t span = (int64_t)kScanLanes + G + a.plane * (int64_t)(kScanLanes / Bx + 2);
    return a.stride <= INT32_MAX && span + (int64_t)(a.m - 1) * a.stride < (int64_t)INT32_MAX;
}

static hipError_t launch_axis(uint8_t* maps, int count, int Bx, int By, int Bz, int axis,
                              hipStream_t s) {
    const AxisLines a = axis_lines(count, Bx, By, Bz, axis);
    const int64_t G = (int64_t)Bx * By * Bz;
    const int64_t tiles = (a.lines + kScanLanes - 1) / kScanLanes;
    const int64_t blocks = (tiles + kXcdSpan - 1) / kXcdSpan * kXcdSpan;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    if (a.m > kMaxLine) {
        k_dist_global<uint16_t, kLongChunk><<<(unsigned)blocks, kScanLanes, 0, s>>>(
            maps, a.lines, Bx, a.inner, a.plane, a.stride, a.m, G);
    } else if (a.lines <= kStagedMaxLines && a.m > kLineChunk && lines_fit_32(a, Bx, G)) {
        const int64_t ptiles = (a.lines + 31) / 32;
        const int64_t pblocks = (ptiles + kXcdSpan - 1) / kXcdSpan * kXcdSpan;
        if (pblocks > INT32_MAX) return hipErrorInvalidValue;
        const int nch = (a.m + kLineChunk - 1) / kLineChunk;
        // 16-byte staging: groups of 32 lines never straddle a row, rows and
        // the map base are 16-byte aligned
        const int wide = Bx % 32 == 0 && a.stride % 16 == 0 && ((uintptr_t)maps & 15) == 0;
        switch (nch) {
#define PDM_PAIRS_CASE(N)                                                                    \
    case N:                                                                                  \
        k_dist_pairs<N><<<(unsigned)pblocks, kScanLanes, 0, s>>>(maps, a.lines, Bx, a.inner, \
                                                                 a.plane, (int)a.stride, a.m, G, \
                                                                 wide);                      \
        break;
            PDM_PAIRS_CASE(2) PDM_PAIRS_CASE(3) PDM_PAIRS_CASE(4) PDM_PAIRS_CASE(5)
            PDM_PAIRS_CASE(6) PDM_PAIRS_CASE(7) PDM_PAIRS_CASE(8) PDM_PAIRS_CASE(9)
            PDM_PAIRS_CASE(10) PDM_PAIRS_CASE(11) PDM_PAIRS_CASE(12) PDM_PAIRS_CASE(13)
            PDM_PAIRS_CASE(14) PDM_PAIRS_CASE(15) PDM_PAIRS_CASE(16)
#undef PDM_PAIRS_CASE
            default: return hipErrorInvalidValue;
        }
    } else if (a.lines > kStagedMaxLines && lines_fit_32(a, Bx, G)) {
        // values clamped to the line length where that shortens the table
        // (more waves per compute unit: 3.6% faster over all 64 maps of the
        // 1024x1024x795 volume, whose z lines are 199 bricks, and 18% on a
        // 128x128x115 grid); lines of 255 and 256 keep all rows, unclamped
        if (scan_rows(a.m) < kRows)
            k_dist_lines<true><<<(unsigned)blocks, kScanLanes, (size_t)scan_table_bytes(a.m), s>>>(
                maps, a.lines, Bx, a.inner, a.plane, (int)a.stride, a.m, G);
        else
            k_dist_lines<false><<<(unsigned)blocks, kScanLanes, 0, s>>>(
                maps, a.lines, Bx, a.inner, a.plane, (int)a.stride, a.m, G);
    } else if (a.lines > kStagedMaxLines) {
        if (a.m >= kLongChunkLine && a.lines >= kLongChunkLines)
            k_dist_global<uint8_t, kLongChunk><<<(unsigned)blocks, kScanLanes, 0, s>>>(
                maps, a.lines, Bx, a.inner, a.plane, a.stride, a.m, G);
        else
            k_dist_global<uint8_t, 16><<<(unsigned)blocks, kScanLanes, 0, s>>>(
                maps, a.lines, Bx, a.inner, a.plane, a.stride, a.m, G);
    } else {
        // the split pass when every one of its work-groups is resident at once
        // (one round of half-length chains); otherwise 64 lines per wave
        const int rows = min(a.m, 255) + 3;
        const size_t lds = (size_t)((rows * kPitch + 15) & ~15) + (size_t)32 * a.m;
        const int64_t split_tiles = (a.lines + 31) / 32;
        const int64_t split_blocks = (split_tiles + kXcdSpan - 1) / kXcdSpan * kXcdSpan;
        int dev = 0, cus = 0, per_cu = 0;
        bool split = hipGetDevice(&dev) == hipSuccess &&
                     hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
                     hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_dist_split, kScanLanes,
                                                                  lds) == hipSuccess &&
                     (int64_t)per_cu * cus >= split_tiles && split_blocks <= INT32_MAX;
        if (split) {
            const int wide = Bx % 32 == 0 && a.stride % 16 == 0 && ((uintptr_t)maps & 15) == 0;
            k_dist_split<<<(unsigned)split_blocks, kScanLanes, lds, s>>>(
                maps, a.lines, Bx, a.inner, a.plane, a.stride, a.m, G, rows, wide);
        } else {
            // 16-byte staging: groups of 64 lines never straddle a row, rows
            // and the map base are 16-byte aligned
            const int wide = Bx % kScanLanes == 0 && a.stride % 16 == 0 && ((uintptr_t)maps & 15) == 0;
            k_dist_axis<<<(unsigned)blocks, kScanLanes, 0, s>>>(maps, a.lines, Bx, a.inner, a.plane,
                                                                a.stride, a.m, G, wide);
        }
    }
    return hipGetLastError();
}

hipError_t launch_distance_yz(uint8_t* maps, int count, int Bx, int By, int Bz, hipStream_t s) {
    for (int axis = 1; axis <= 2; ++axis) {
        const int m = axis == 1 ? By : Bz;
        if (m == 1) continue;  // a line of one brick is unchanged
        const hipError_t e = launch_axis(maps, count, Bx, By, Bz, axis, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Two chunks per lane from this many chunks on: 256 CUs x 4 work-groups of
// 256 lanes x 2 chunks (maps of 8 MiB and more).
constexpr int64_t kCombineWideChunks = 256LL * 4 * 256 * 2;

hipError_t launch_combine(const MapList& maps, int64_t G, uint8_t* out, hipStream_t s) {
    const int64_t nch = (G + 15) / 16;
    if (G < 16)
        k_combine<0><<<blocks_for(G, 256), 256, 0, s>>>(maps, G, out);
    else if (nch >= kCombineWideChunks)
        k_combine<2><<<blocks_for((nch + 1) / 2, 256), 256, 0, s>>>(maps, G, out);
    else
        k_combine<1><<<blocks_for(nch, 256), 256, 0, s>>>(maps, G, out);
    return hipGetLastError();
}

hipError_t launch_range_level(const uint8_t* src, int64_t h, uint8_t* dst, int64_t count, int64_t G,
                              hipStream_t s) {
    const int64_t total = count * G;
    if (total >= 16) {
        const int64_t blocks = ((total + 15) / 16 + 255) / 256;
        if (blocks > INT32_MAX) return hipErrorInvalidValue;
        k_range_level<16><<<(unsigned)blocks, 256, 0, s>>>(src, h, dst, total, G);
    } else {
        const int64_t blocks = (total + 255) / 256;
        if (blocks > INT32_MAX) return hipErrorInvalidValue;
        k_range_level<1><<<(unsigned)blocks, 256, 0, s>>>(src, h, dst, total, G);
    }
    return hipGetLastError();
}

hipError_t launch_batch_combine(BatchArgs& a, hipStream_t s) {
    int64_t blocks = 0;
    for (int k = 0; k < a.count; ++k) {
        const int64_t G = a.it[k].G;
        a.it[k].first_block = blocks;
        blocks += G >= 16 ? ((G + 15) / 16 + 255) / 256 : 1;
    }
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    k_batch_combine<<<(unsigned)blocks, 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_batch_maps(BatchMapsArgs& a, hipStream_t s) {
    int64_t blocks = 0;
    for (int k = 0; k < a.count; ++k) {
        const int64_t G = a.it[k].G;
        a.it[k].first_block = blocks;
        blocks += G >= 16 ? ((G + 15) / 16 + 255) / 256 : 1;
    }
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    k_batch_combine_maps<<<(unsigned)blocks, 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_batch_build(const BatchVol* h_vols, int count, BatchVol* d_vols,
                              BatchSync* d_sync, const int64_t totals[3], int lines_mult,
                              int single, hipStream_t s) {
    static_assert(sizeof(BatchVol) % 16 == 0, "descriptor size");
    static_assert(sizeof(BatchSync) % 16 == 0, "sync size");
    const uint8_t* src = reinterpret_cast<const uint8_t*>(h_vols);
    const int64_t bytes = (int64_t)count * (int64_t)sizeof(BatchVol);
    UploadChunk c;
    for (int64_t off = 0; off < bytes; off += (int64_t)sizeof(c.data)) {
        const int64_t nb = bytes - off < (int64_t)sizeof(c.data) ? bytes - off : (int64_t)sizeof(c.data);
        c.bytes = (int32_t)nb;
        memcpy(c.data, src + off, (size_t)nb);
        k_upload<<<1, 256, 0, s>>>(reinterpret_cast<uint8_t*>(d_vols) + off, c);
    }
    k_zero<<<1, 256, 0, s>>>(reinterpret_cast<uint32_t*>(d_sync), (int)(sizeof(BatchSync) / 4));
    // the scans' tables: rows for the longest line of each phase
    int longest[3] = {0, 0, 0};
    for (int k = 0; k < count; ++k) {
        longest[1] = max(longest[1], h_vols[k].By);
        longest[2] = max(longest[2], h_vols[k].Bz);
    }
    if (single) {
        // every work-group resident at once: the occupancy of this kernel on
        // every compute unit
        const size_t lds = (size_t)scan_table_bytes(max(longest[1], longest[2]));
        int dev = 0, cus = 0, per_cu = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_single, kWave, lds);
        if (e != hipSuccess) return e;
        const int64_t grid = (int64_t)per_cu * cus;
        if (grid < 1 || grid > INT32_MAX) return hipErrorInvalidConfiguration;
        int64_t t0 = totals[0], t1 = totals[1], t2 = totals[2];
        int lm = lines_mult;
        uint64_t limit = 100ull * 1000 * 1000 * 10;  // 10 s of the 100 MHz counter
        const BatchVol* dv = d_vols;
        BatchSync* ds = d_sync;
        int cnt = count;
        void* args[] = {&dv, &cnt, &t0, &t1, &t2, &lm, &ds, &limit};
        e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_batch_single), dim3((unsigned)grid),
                                       dim3(kWave), args, lds, s);
        if (e != hipSuccess) return e;
        return hipGetLastError();
    }
    for (int ph = 0; ph < 3; ++ph) {
        if (totals[ph] <= 0) continue;
        const int64_t grid = (totals[ph] + kXcdSpan - 1) / kXcdSpan * kXcdSpan;
        if (grid > INT32_MAX) return hipErrorInvalidValue;
        if (ph == 0)
            k_batch_rows<<<(unsigned)grid, kWave, 0, s>>>(d_vols, count, totals[0]);
        else
            k_batch_scan<<<(unsigned)grid, kWave, (size_t)scan_table_bytes(longest[ph]), s>>>(
                d_vols, count, ph, totals[ph], lines_mult);
    }
    return hipGetLastError();
}

}  // namespace pdm
