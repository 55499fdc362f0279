// pdm_api.cpp -- host layer of libpdm: argument validation, the active set
// (step 1 of the TF update, Sec. 3.1), kernel-argument packing and launches.
// Every check runs before any HIP call, so invalid arguments are reported
// without touching a device.
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "pdm.h"
#include "pdm_launch.h"

namespace {

using pdm::MapList;
using pdm::AlphaBits;
using pdm::Bounds;

inline bool aligned(const void* p, uintptr_t a) { return ((uintptr_t)p & (a - 1)) == 0; }

pdm_status check_volume(const pdm_volume* v, pdm_grid* g) {
    if (v == nullptr) return PDM_E_INVAL;
    if (v->nx < 1 || v->ny < 1 || v->nz < 1) return PDM_E_INVAL;
    if (v->dtype != PDM_U8 && v->dtype != PDM_U16) return PDM_E_INVAL;
    const int32_t max_levels = v->dtype == PDM_U8 ? 256 : 65536;
    if (v->levels < 1 || v->levels > max_levels) return PDM_E_INVAL;
    if (v->brick < 1) return PDM_E_INVAL;
    if (v->brick != PDM_BRICK) return PDM_E_UNSUPPORTED;
    const int64_t bx = ((int64_t)v->nx + v->brick - 1) / v->brick;
    const int64_t by = ((int64_t)v->ny + v->brick - 1) / v->brick;
    const int64_t bz = ((int64_t)v->nz + v->brick - 1) / v->brick;
    if (bx > PDM_MAX_GRID_X || by > PDM_MAX_GRID_AXIS || bz > PDM_MAX_GRID_AXIS)
        return PDM_E_UNSUPPORTED;
    g->bx = (int32_t)bx;
    g->by = (int32_t)by;
    g->bz = (int32_t)bz;
    g->count = bx * by * bz;
    return PDM_OK;
}

pdm_status check_bounds(const int32_t* b, int32_t n, int32_t levels) {
    if (b == nullptr) return PDM_E_INVAL;
    if (n < 1 || n > PDM_MAX_PARTITIONS) return PDM_E_INVAL;
    if (b[0] != 0 || b[n] != levels) return PDM_E_INVAL;
    for (int32_t p = 0; p < n; ++p)
        if (b[p + 1] <= b[p]) return PDM_E_INVAL;
    return PDM_OK;
}

// Opacities are tested on their bit patterns: non-zero when any bit besides
// the sign is set (NaN and subnormals count, -0 does not), independent of the
// host's floating-point mode.
typedef uint32_t __attribute__((may_alias)) opacity_bits;
constexpr uint32_t kMagnitude = 0x7fffffffu;

// Step 1 (Sec. 3.1): partitions holding an intensity with non-zero opacity.
// The OR over a partition has no early exit so that it vectorises (a
// 4096-entry table in a fraction of a microsecond).
void active_mask(const int32_t* b, int32_t n, const float* alpha, uint64_t mask[4]) {
    const opacity_bits* u = reinterpret_cast<const opacity_bits*>(alpha);
    mask[0] = mask[1] = mask[2] = mask[3] = 0;
    for (int32_t p = 0; p < n; ++p) {
        uint32_t acc = 0;
        for (int32_t i = b[p]; i < b[p + 1]; ++i) acc |= u[i];
        if (acc & kMagnitude) mask[p >> 6] |= 1ull << (p & 63);
    }
}

pdm_status from_hip(hipError_t e) { return e == hipSuccess ? PDM_OK : PDM_E_DEVICE; }

// Validation and kernel arguments shared by both readings of the plain
// method: the non-zero opacity levels and the volume geometry.  Up to
// PDM_MAX_PLAIN_BITMAP_LEVELS levels they go as a bitmap with per-word prefix
// counts; above, when `allow_runs`, as the maximal runs of non-zero levels
// (at most PDM_MAX_PLAIN_RUNS of them).
pdm_status plain_args(const pdm_volume* v, const void* d_volume, const float* h_alpha,
                      uint8_t* d_dist, pdm::PlainArgs* a, AlphaBits* bits, bool allow_runs) {
    pdm_grid g;
    const pdm_status st = check_volume(v, &g);
    if (st != PDM_OK) return st;
    if (d_volume == nullptr || h_alpha == nullptr || d_dist == nullptr) return PDM_E_INVAL;
    static_assert(PDM_MAX_PLAIN_BITMAP_LEVELS == 32 * PDM_ALPHA_WORDS, "bitmap size");
    static_assert(PDM_MAX_PLAIN_RUNS <= PDM_ALPHA_WORDS, "run list size");
    const bool runs = v->levels > PDM_MAX_PLAIN_BITMAP_LEVELS;
    if (v->levels > PDM_MAX_PLAIN_LEVELS || (runs && !allow_runs)) return PDM_E_UNSUPPORTED;
    memset(bits, 0, sizeof(*bits));
    const opacity_bits* u = reinterpret_cast<const opacity_bits*>(h_alpha);
    int32_t count = 0;
    if (runs) {
        // levels < 65536, so a run's first and last level take 16 bits each
        for (int32_t i = 0; i < v->levels;) {
            if (!(u[i] & kMagnitude)) {
                ++i;
                continue;
            }
            int32_t j = i;
            while (j + 1 < v->levels && (u[j + 1] & kMagnitude)) ++j;
            if (count == PDM_MAX_PLAIN_RUNS) return PDM_E_UNSUPPORTED;
            bits->w[count++] = (uint32_t)i | ((uint32_t)j << 16);
            i = j + 1;
        }
    } else {
        for (int32_t i = 0; i < v->levels; ++i)
            if (u[i] & kMagnitude) bits->w[i >> 5] |= 1u << (i & 31);
        // prefix counts of set bits per word: any set bit in [lo, hi] is O(1)
        count = (v->levels + 31) / 32;
        uint32_t acc = 0;
        for (int32_t i = 0; i < count; ++i) {
            bits->pre[i] = (uint16_t)acc;
            acc += (uint32_t)__builtin_popcount(bits->w[i]);
        }
        bits->pre[count] = (uint16_t)acc;
    }
    a->vol = d_volume;
    a->dist = d_dist;
    a->nx = v->nx;
    a->ny = v->ny;
    a->nz = v->nz;
    a->Bx = g.bx;
    a->By = g.by;
    a->Bz = g.bz;
    a->bytes = v->dtype;
    a->nwords = count;
    a->levels = v->levels;
    a->store_vec = g.bx % 4 == 0 && aligned(d_dist, 4);
    a->runs = runs ? 1 : 0;
    return PDM_OK;
}


}  // namespace

extern "C" {

pdm_status pdm_grid_of(const pdm_volume* v, pdm_grid* out) {
    if (out == nullptr) return PDM_E_INVAL;
    pdm_grid g;
    const pdm_status st = check_volume(v, &g);
    if (st == PDM_OK) *out = g;
    return st;
}

pdm_status pdm_active_set(const int32_t* h_bounds, int32_t n, const float* h_alpha, int32_t levels,
                          uint64_t* h_active) {
    if (h_alpha == nullptr || h_active == nullptr) return PDM_E_INVAL;
    const pdm_status st = check_bounds(h_bounds, n, levels);
    if (st != PDM_OK) return st;
    active_mask(h_bounds, n, h_alpha, h_active);
    return PDM_OK;
}

pdm_status pdm_build_bricks(const pdm_volume* v, const void* d_volume, void* d_bmin, void* d_bmax,
                            int32_t* d_range_err, hipStream_t stream) {
    pdm_grid g;
    pdm_status st = check_volume(v, &g);
    if (st != PDM_OK) return st;
    if (d_volume == nullptr || d_bmin == nullptr || d_bmax == nullptr) return PDM_E_INVAL;
    pdm::BrickArgs a;
    a.vol = d_volume;
    a.bmin = d_bmin;
    a.bmax = d_bmax;
    a.range_err = d_range_err;
    a.nx = v->nx;
    a.ny = v->ny;
    a.nz = v->nz;
    a.Bx = g.bx;
    a.By = g.by;
    a.Bz = g.bz;
    a.bytes = v->dtype;
    a.levels = v->levels;
    // the range flag is only needed when the dtype can hold values >= levels
    if (v->levels == (v->dtype == PDM_U8 ? 256 : 65536)) a.range_err = nullptr;
    return from_hip(pdm::launch_bricks(a, stream));
}

pdm_status pdm_pom_distance_x(const pdm_volume* v, const void* d_bmin, const void* d_bmax,
                              const int32_t* h_bounds, int32_t n, uint8_t* d_pdms,
                              hipStream_t stream) {
    pdm_grid g;
    pdm_status st = check_volume(v, &g);
    if (st != PDM_OK) return st;
    if (d_bmin == nullptr || d_bmax == nullptr || d_pdms == nullptr) return PDM_E_INVAL;
    st = check_bounds(h_bounds, n, v->levels);
    if (st != PDM_OK) return st;
    Bounds b;
    memset(&b, 0, sizeof(b));
    for (int32_t p = 0; p <= n; ++p) b.b[p] = h_bounds[p];
    pdm::PomArgs a;
    a.bmin = d_bmin;
    a.bmax = d_bmax;
    a.pdms = d_pdms;
    a.G = g.count;
    a.Bx = g.bx;
    a.By = g.by;
    a.Bz = g.bz;
    a.bytes = v->dtype;
    a.n = n;
    a.store_vec = g.bx % 4 == 0 && aligned(d_pdms, 4);
    return from_hip(pdm::launch_pom_x(a, b, stream));
}

pdm_status pdm_distance_yz(const pdm_volume* v, uint8_t* d_maps, int32_t count, hipStream_t stream) {
    pdm_grid g;
    const pdm_status st = check_volume(v, &g);
    if (st != PDM_OK) return st;
    if (d_maps == nullptr || count < 1 || count > PDM_MAX_PARTITIONS) return PDM_E_INVAL;
    return from_hip(pdm::launch_distance_yz(d_maps, count, g.bx, g.by, g.bz, stream));
}

pdm_status pdm_build_partitions(const pdm_volume* v, const void* d_bmin, const void* d_bmax,
                                const int32_t* h_bounds, int32_t n, uint8_t* d_pdms,
                                hipStream_t stream) {
    pdm_status st = pdm_pom_distance_x(v, d_bmin, d_bmax, h_bounds, n, d_pdms, stream);
    if (st != PDM_OK) return st;
    return pdm_distance_yz(v, d_pdms, n, stream);
}

pdm_status pdm_tf_update(const pdm_volume* v, const uint8_t* d_pdms, const int32_t* h_bounds,
                         int32_t n, const float* h_alpha, uint8_t* d_dist, uint64_t* h_active,
                         hipStream_t stream) {
    pdm_grid g;
    pdm_status st = check_volume(v, &g);
    if (st != PDM_OK) return st;
    if (d_pdms == nullptr || d_dist == nullptr || h_alpha == nullptr) return PDM_E_INVAL;
    st = check_bounds(h_bounds, n, v->levels);
    if (st != PDM_OK) return st;
    uint64_t mask[4];
    active_mask(h_bounds, n, h_alpha, mask);
    if (h_active != nullptr)
        for (int k = 0; k < 4; ++k) h_active[k] = mask[k];
    MapList maps;
    memset(&maps, 0, sizeof(maps));
    for (int32_t p = 0; p < n; ++p)
        if ((mask[p >> 6] >> (p & 63)) & 1ull) maps.src[maps.count++] = d_pdms + (int64_t)p * g.count;
    return from_hip(pdm::launch_combine(maps, g.count, d_dist, stream));
}

// ------------------------------------------------------------ range tables
namespace {

int32_t range_levels(int32_t n, int32_t max_level) {
    int32_t K = 0;
    while (K < max_level && (2 << K) <= n) ++K;  // 2^(K+1) <= n
    return K;
}

// First map of level k (1-based level) within the table.
int64_t level_first(int32_t n, int32_t k) {
    int64_t off = 0;
    for (int32_t j = 1; j < k; ++j) off += n - (1 << j) + 1;
    return off;
}

// Map indices (i < n: PDM i; i >= n: table map i - n) whose min is the min
// over the partitions of `mask`: each maximal run [a, b] of length L takes
// one PDM (L = 1), the one or two maps of level floor(log2 L) that cover it,
// or, past the top level K, level-K maps every 2^K partitions plus one
// ending at b.  Maps may overlap; min is idempotent.
int32_t cover(int32_t n, int32_t K, const uint64_t* mask, int32_t* out) {
    int32_t cnt = 0;
    auto on = [&](int32_t p) { return ((mask[p >> 6] >> (p & 63)) & 1ull) != 0; };
    auto tmap = [&](int32_t k, int32_t p) { return (int32_t)(n + level_first(n, k) + p); };
    for (int32_t a = 0; a < n;) {
        if (!on(a)) {
            ++a;
            continue;
        }
        int32_t b = a;
        while (b + 1 < n && on(b + 1)) ++b;
        const int32_t L = b - a + 1;
        int32_t k = 0;
        while ((2 << k) <= L) ++k;  // floor(log2 L)
        if (k == 0 || K == 0) {
            for (int32_t p = a; p <= b; ++p) out[cnt++] = p;
        } else if (k <= K) {
            out[cnt++] = tmap(k, a);
            if (L != (1 << k)) out[cnt++] = tmap(k, b - (1 << k) + 1);
        } else {
            const int32_t w = 1 << K;
            int32_t p = a;
            for (; p + w - 1 < b; p += w) out[cnt++] = tmap(K, p);
            out[cnt++] = tmap(K, b - w + 1);
        }
        a = b + 1;
    }
    return cnt;
}

}  // namespace

int64_t pdm_range_table_maps(int32_t n, int32_t max_level) {
    if (n < 1 || n > PDM_MAX_PARTITIONS || max_level < 0) return -1;
    const int32_t K = range_levels(n, max_level);
    return level_first(n, K + 1);
}

pdm_status pdm_range_cover(int32_t n, int32_t max_level, const uint64_t* h_active, int32_t* h_maps,
                           int32_t* h_count) {
    if (n < 1 || n > PDM_MAX_PARTITIONS || max_level < 0 || h_active == nullptr ||
        h_maps == nullptr || h_count == nullptr)
        return PDM_E_INVAL;
    *h_count = cover(n, range_levels(n, max_level), h_active, h_maps);
    return PDM_OK;
}

pdm_status pdm_build_range_table(const pdm_volume* v, const uint8_t* d_pdms, int32_t n,
                                 int32_t max_level, uint8_t* d_table, hipStream_t stream) {
    pdm_grid g;
    const pdm_status st = check_volume(v, &g);
    if (st != PDM_OK) return st;
    if (d_pdms == nullptr || n < 1 || n > PDM_MAX_PARTITIONS || max_level < 0) return PDM_E_INVAL;
    const int32_t K = range_levels(n, max_level);
    if (K == 0) return PDM_OK;
    if (d_table == nullptr) return PDM_E_INVAL;
    const int64_t G = g.count;
    for (int32_t k = 1; k <= K; ++k) {
        const uint8_t* src = k == 1 ? d_pdms : d_table + level_first(n, k - 1) * G;
        uint8_t* dst = d_table + level_first(n, k) * G;
        const int64_t count = n - (1 << k) + 1;
        const hipError_t e = pdm::launch_range_level(src, 1 << (k - 1), dst, count, G, stream);
        if (e != hipSuccess) return PDM_E_DEVICE;
    }
    return PDM_OK;
}

pdm_status pdm_tf_update_ranges(const pdm_volume* v, const uint8_t* d_pdms, const uint8_t* d_table,
                                const int32_t* h_bounds, int32_t n, int32_t max_level,
                                const float* h_alpha, uint8_t* d_dist, uint64_t* h_active,
                                hipStream_t stream) {
    pdm_grid g;
    pdm_status st = check_volume(v, &g);
    if (st != PDM_OK) return st;
    if (d_pdms == nullptr || d_dist == nullptr || h_alpha == nullptr || max_level < 0)
        return PDM_E_INVAL;
    st = check_bounds(h_bounds, n, v->levels);
    if (st != PDM_OK) return st;
    const int32_t K = range_levels(n, max_level);
    if (K > 0 && d_table == nullptr) return PDM_E_INVAL;
    uint64_t mask[4];
    active_mask(h_bounds, n, h_alpha, mask);
    if (h_active != nullptr)
        for (int k = 0; k < 4; ++k) h_active[k] = mask[k];
    int32_t idx[PDM_MAX_PARTITIONS];
    const int32_t cnt = cover(n, K, mask, idx);
    MapList maps;
    memset(&maps, 0, sizeof(maps));
    maps.count = cnt;
    for (int32_t j = 0; j < cnt; ++j)
        maps.src[j] = idx[j] < n ? d_pdms + (int64_t)idx[j] * g.count
                                 : d_table + (int64_t)(idx[j] - n) * g.count;
    return from_hip(pdm::launch_combine(maps, g.count, d_dist, stream));
}

pdm_status pdm_batch_tf_update(const pdm_batch_update* h_items, int32_t count,
                               uint64_t* h_active, hipStream_t stream) {
    if (h_items == nullptr || count < 1 || count > PDM_BATCH_MAX) return PDM_E_INVAL;
    static_assert(PDM_BATCH_MAX <= PDM_BATCH_MAX_ITEMS, "batch descriptors exceed kernel arguments");
    pdm::BatchArgs a;
    memset(&a, 0, sizeof(a));
    a.count = count;
    for (int32_t k = 0; k < count; ++k) {
        const pdm_batch_update& it = h_items[k];
        pdm_grid g;
        pdm_status st = check_volume(it.v, &g);
        if (st != PDM_OK) return st;
        if (it.d_pdms == nullptr || it.d_dist == nullptr || it.h_alpha == nullptr) return PDM_E_INVAL;
        st = check_bounds(it.h_bounds, it.n, it.v->levels);
        if (st != PDM_OK) return st;
        pdm::BatchItem& b = a.it[k];
        active_mask(it.h_bounds, it.n, it.h_alpha, b.mask);
        if (h_active != nullptr)
            for (int w = 0; w < 4; ++w) h_active[4 * k + w] = b.mask[w];
        b.pdms = it.d_pdms;
        b.out = it.d_dist;
        b.G = g.count;
    }
    return from_hip(pdm::launch_batch_combine(a, stream));
}

pdm_status pdm_batch_tf_update_ranges(const pdm_batch_range_update* h_items, int32_t count,
                                      uint64_t* h_active, hipStream_t stream) {
    if (h_items == nullptr || count < 1 || count > PDM_BATCH_MAX) return PDM_E_INVAL;
    static_assert(PDM_BATCH_MAX <= PDM_BATCH_MAX_ITEMS, "batch descriptors exceed kernel arguments");
    static_assert(PDM_MAX_PARTITIONS <= PDM_BATCH_MAX_MAPS, "one cover must fit one launch");
    // every request validated and its cover found before anything is launched
    uint16_t maps[PDM_BATCH_MAX][PDM_MAX_PARTITIONS];
    int32_t cnt[PDM_BATCH_MAX];
    int64_t G[PDM_BATCH_MAX];
    for (int32_t k = 0; k < count; ++k) {
        const pdm_batch_range_update& it = h_items[k];
        pdm_grid g;
        pdm_status st = check_volume(it.v, &g);
        if (st != PDM_OK) return st;
        if (it.d_pdms == nullptr || it.d_dist == nullptr || it.h_alpha == nullptr || it.max_level < 0)
            return PDM_E_INVAL;
        st = check_bounds(it.h_bounds, it.n, it.v->levels);
        if (st != PDM_OK) return st;
        const int32_t K = range_levels(it.n, it.max_level);
        if (K > 0 && it.d_table == nullptr) return PDM_E_INVAL;
        uint64_t mask[4];
        active_mask(it.h_bounds, it.n, it.h_alpha, mask);
        if (h_active != nullptr)
            for (int w = 0; w < 4; ++w) h_active[4 * k + w] = mask[w];
        int32_t idx[PDM_MAX_PARTITIONS];
        cnt[k] = cover(it.n, K, mask, idx);
        for (int32_t j = 0; j < cnt[k]; ++j) maps[k][j] = (uint16_t)idx[j];
        G[k] = g.count;
    }
    // as few launches as the kernel-argument room for map indices allows
    pdm::BatchMapsArgs a;
    memset(&a, 0, sizeof(a));
    for (int32_t k = 0; k < count; ++k) {
        if (a.nidx + cnt[k] > PDM_BATCH_MAX_MAPS) {
            const hipError_t e = pdm::launch_batch_maps(a, stream);
            if (e != hipSuccess) return PDM_E_DEVICE;
            memset(&a, 0, sizeof(a));
        }
        const pdm_batch_range_update& it = h_items[k];
        pdm::MapsItem& m = a.it[a.count++];
        m.pdms = it.d_pdms;
        m.table = it.d_table;
        m.out = it.d_dist;
        m.G = G[k];
        m.map_first = a.nidx;
        m.map_count = cnt[k];
        m.n = it.n;
        for (int32_t j = 0; j < cnt[k]; ++j) a.idx[a.nidx++] = maps[k][j];
    }
    return from_hip(pdm::launch_batch_maps(a, stream));
}

size_t pdm_batch_workspace_bytes(int32_t count) {
    if (count < 1 || count > PDM_BATCH_MAX) return 0;
    return sizeof(pdm::BatchSync) + (size_t)count * sizeof(pdm::BatchVol);
}

}  // extern "C"

namespace {

// Validation and descriptor packing shared by both batched-build entry
// points (host only, no HIP call): vols[0..count) in launch order, the item
// totals per phase and the configuration with defaults filled in.
pdm_status batch_prepare(const pdm_batch_volume* h_vols, int32_t count, const pdm_batch_config* cfg,
                         pdm::BatchVol* vols, int64_t totals[3], pdm_batch_config* out_cfg) {
    pdm_batch_config c = {0, 0, 0, 0};
    if (cfg != nullptr) c = *cfg;
    if (c.rows_per_item < 0 || c.rows_per_item > 256 || c.lines_mult < 0 || c.lines_mult > 16 ||
        c.single_launch < 0 || c.single_launch > 1)
        return PDM_E_INVAL;
    if (c.lines_mult == 0) c.lines_mult = 1;
    if (c.rows_per_item == 0) c.rows_per_item = 2;
    pdm::BatchVol tmp[PDM_BATCH_MAX];
    int64_t work[PDM_BATCH_MAX];
    for (int32_t k = 0; k < count; ++k) {
        const pdm_batch_volume& it = h_vols[k];
        pdm_grid g;
        pdm_status st = check_volume(it.v, &g);
        if (st != PDM_OK) return st;
        if (it.d_volume == nullptr || it.d_bmin == nullptr || it.d_bmax == nullptr ||
            it.d_pdms == nullptr)
            return PDM_E_INVAL;
        st = check_bounds(it.h_bounds, it.n, it.v->levels);
        if (st != PDM_OK) return st;
        if (g.bx > 256 || g.by > 256 || g.bz > 256) return PDM_E_UNSUPPORTED;
        pdm::BatchVol& d = tmp[k];
        memset(&d, 0, sizeof(d));
        d.vol = it.d_volume;
        d.bmin = it.d_bmin;
        d.bmax = it.d_bmax;
        d.pdms = it.d_pdms;
        d.G = g.count;
        d.nx = it.v->nx;
        d.ny = it.v->ny;
        d.nz = it.v->nz;
        d.Bx = g.bx;
        d.By = g.by;
        d.Bz = g.bz;
        d.bytes = it.v->dtype;
        d.n = it.n;
        d.levels = it.v->levels;
        d.store_vec = g.bx % 4 == 0 && aligned(it.d_pdms, 4);
        for (int32_t p = 0; p <= it.n; ++p) d.bounds[p] = it.h_bounds[p];
        const int64_t lines = (int64_t)it.n * g.bx;
        d.chunks = (int32_t)((lines + 64 * c.lines_mult - 1) / (64 * c.lines_mult));
        // first phase: a row takes the power-of-two lane count >= Bx/4, so
        // narrow rows share a wave; an item is rows_per_item wave passes
        int32_t lanes = 1;
        while (4 * lanes < g.bx) lanes *= 2;
        d.row_lanes = lanes;
        d.rows = c.rows_per_item * (64 / lanes);
        d.row_groups = (g.by + d.rows - 1) / d.rows;
        d.items[0] = g.bz * d.row_groups;
        d.items[1] = g.by > 1 ? g.bz * d.chunks : 0;  // a pass over lines of 1 brick is the identity
        d.items[2] = g.bz > 1 ? g.by * d.chunks : 0;
        work[k] = (int64_t)it.n * g.count;
    }
    // order of the volumes' items (the same in every phase)
    int32_t order[PDM_BATCH_MAX];
    for (int32_t k = 0; k < count; ++k) order[k] = k;
    if (c.largest_first)
        for (int32_t a = 1; a < count; ++a)
            for (int32_t b = a; b > 0 && work[order[b]] > work[order[b - 1]]; --b) {
                const int32_t t = order[b];
                order[b] = order[b - 1];
                order[b - 1] = t;
            }
    for (int32_t k = 0; k < count; ++k) vols[k] = tmp[order[k]];
    totals[0] = totals[1] = totals[2] = 0;
    for (int ph = 0; ph < 3; ++ph)
        for (int32_t k = 0; k < count; ++k) {
            vols[k].first[ph] = totals[ph];
            totals[ph] += vols[k].items[ph];
        }
    for (int ph = 0; ph < 3; ++ph)
        if (totals[ph] > INT32_MAX - 64) return PDM_E_UNSUPPORTED;
    *out_cfg = c;
    return PDM_OK;
}

}  // namespace

extern "C" {

pdm_status pdm_batch_build(const pdm_batch_volume* h_vols, int32_t count, void* d_workspace,
                           size_t workspace_bytes, const pdm_batch_config* cfg,
                           hipStream_t stream) {
    if (h_vols == nullptr || count < 1 || count > PDM_BATCH_MAX) return PDM_E_INVAL;
    if (d_workspace == nullptr || !aligned(d_workspace, 16) ||
        workspace_bytes < pdm_batch_workspace_bytes(count))
        return PDM_E_INVAL;
    pdm::BatchVol vols[PDM_BATCH_MAX];
    int64_t totals[3];
    pdm_batch_config c;
    const pdm_status st = batch_prepare(h_vols, count, cfg, vols, totals, &c);
    if (st != PDM_OK) return st;
    uint8_t* ws = static_cast<uint8_t*>(d_workspace);
    pdm::BatchSync* sync = reinterpret_cast<pdm::BatchSync*>(ws);
    pdm::BatchVol* dv = reinterpret_cast<pdm::BatchVol*>(ws + sizeof(pdm::BatchSync));
    return from_hip(pdm::launch_batch_build(vols, count, dv, sync, totals, c.lines_mult,
                                            c.single_launch, stream));
}

pdm_status pdm_batch_build_noalloc(const pdm_batch_volume* h_vols, int32_t count,
                                   const pdm_batch_config* cfg, uint32_t* d_error,
                                   hipStream_t stream) {
    if (h_vols == nullptr || count < 1 || count > PDM_BATCH_MAX) return PDM_E_INVAL;
    pdm::BatchVol vols[PDM_BATCH_MAX];
    int64_t totals[3];
    pdm_batch_config c;
    const pdm_status st = batch_prepare(h_vols, count, cfg, vols, totals, &c);
    if (st != PDM_OK) return st;
    // the scratch array of the current device; the stream must belong to it
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PDM_E_DEVICE;
    if (stream != nullptr) {
        int sdev = -1;
        if (hipStreamGetDevice(stream, &sdev) != hipSuccess) return PDM_E_DEVICE;
        if (sdev != dev) return PDM_E_INVAL;
    }
    uint8_t* ws = nullptr;
    size_t cap = 0;
    if (pdm::batch_scratch(dev, &ws, &cap) != hipSuccess) return PDM_E_DEVICE;
    if (cap < pdm_batch_workspace_bytes(count)) return PDM_E_UNSUPPORTED;
    pdm::BatchSync* sync = reinterpret_cast<pdm::BatchSync*>(ws);
    pdm::BatchVol* dv = reinterpret_cast<pdm::BatchVol*>(ws + sizeof(pdm::BatchSync));
    hipError_t e = pdm::launch_batch_build(vols, count, dv, sync, totals, c.lines_mult,
                                           c.single_launch, stream);
    if (e == hipSuccess && d_error != nullptr) e = pdm::launch_copy_word(&sync->error, d_error, stream);
    return from_hip(e);
}

pdm_status pdm_plain_distance_x(const pdm_volume* v, const void* d_volume, const float* h_alpha,
                                uint8_t* d_dist, hipStream_t stream) {
    pdm::PlainArgs a;
    AlphaBits bits;
    const pdm_status st = plain_args(v, d_volume, h_alpha, d_dist, &a, &bits, true);
    if (st != PDM_OK) return st;
    return from_hip(pdm::launch_plain_x(a, bits, stream));
}

pdm_status pdm_full_recompute(const pdm_volume* v, const void* d_volume, const float* h_alpha,
                              uint8_t* d_dist, hipStream_t stream) {
    pdm_status st = pdm_plain_distance_x(v, d_volume, h_alpha, d_dist, stream);
    if (st != PDM_OK) return st;
    return pdm_distance_yz(v, d_dist, 1, stream);
}

pdm_status pdm_plain_cached_distance_x(const pdm_volume* v, const void* d_bmin, const void* d_bmax,
                                       const float* h_alpha, uint8_t* d_dist, hipStream_t stream) {
    if (d_bmin == nullptr || d_bmax == nullptr) return PDM_E_INVAL;
    pdm::PlainArgs pa;
    AlphaBits bits;
    // the bitmap and the geometry as for the plain method (d_bmin stands in
    // for the volume pointer in the shared checks)
    const pdm_status st = plain_args(v, d_bmin, h_alpha, d_dist, &pa, &bits, true);
    if (st != PDM_OK) return st;
    pdm::CachedArgs a;
    a.bmin = d_bmin;
    a.bmax = d_bmax;
    a.dist = d_dist;
    a.Bx = pa.Bx;
    a.By = pa.By;
    a.Bz = pa.Bz;
    a.bytes = pa.bytes;
    a.nwords = pa.nwords;
    a.levels = pa.levels;
    a.store_vec = pa.store_vec;
    a.runs = pa.runs;
    a.load_vec = pa.Bx % 4 == 0 && aligned(d_bmin, 4 * (uintptr_t)v->dtype) &&
                 aligned(d_bmax, 4 * (uintptr_t)v->dtype);
    return from_hip(pdm::launch_plain_cached_x(a, bits, stream));
}

pdm_status pdm_full_recompute_cached(const pdm_volume* v, const void* d_bmin, const void* d_bmax,
                                     const float* h_alpha, uint8_t* d_dist, hipStream_t stream) {
    pdm_status st = pdm_plain_cached_distance_x(v, d_bmin, d_bmax, h_alpha, d_dist, stream);
    if (st != PDM_OK) return st;
    return pdm_distance_yz(v, d_dist, 1, stream);
}

pdm_status pdm_pom_exact_distance_x(const pdm_volume* v, const void* d_volume,
                                    const int32_t* h_bounds, int32_t n, uint8_t* d_pdms,
                                    hipStream_t stream) {
    pdm_grid g;
    pdm_status st = check_volume(v, &g);
    if (st != PDM_OK) return st;
    if (d_volume == nullptr || d_pdms == nullptr) return PDM_E_INVAL;
    st = check_bounds(h_bounds, n, v->levels);
    if (st != PDM_OK) return st;
    if (v->levels > PDM_MAX_EXACT_LEVELS || g.bx > PDM_MAX_EXACT_GRID_X) return PDM_E_UNSUPPORTED;
    Bounds b;
    memset(&b, 0, sizeof(b));
    for (int32_t p = 0; p <= n; ++p) b.b[p] = h_bounds[p];
    pdm::PomExactArgs a;
    a.vol = d_volume;
    a.pdms = d_pdms;
    a.G = g.count;
    a.nx = v->nx;
    a.ny = v->ny;
    a.nz = v->nz;
    a.Bx = g.bx;
    a.By = g.by;
    a.Bz = g.bz;
    a.bytes = v->dtype;
    a.n = n;
    a.levels = v->levels;
    a.store_vec = g.bx % 4 == 0 && aligned(d_pdms, 4);
    return from_hip(pdm::launch_pom_exact_x(a, b, stream));
}

pdm_status pdm_build_partitions_exact(const pdm_volume* v, const void* d_volume,
                                      const int32_t* h_bounds, int32_t n, uint8_t* d_pdms,
                                      hipStream_t stream) {
    pdm_status st = pdm_pom_exact_distance_x(v, d_volume, h_bounds, n, d_pdms, stream);
    if (st != PDM_OK) return st;
    return pdm_distance_yz(v, d_pdms, n, stream);
}

pdm_status pdm_plain_exact_distance_x(const pdm_volume* v, const void* d_volume,
                                      const float* h_alpha, uint8_t* d_dist, hipStream_t stream) {
    pdm::PlainArgs a;
    AlphaBits bits;
    // the EXACT test looks every voxel up in the bitmap: at most
    // PDM_MAX_EXACT_LEVELS (= PDM_MAX_PLAIN_BITMAP_LEVELS) levels, no runs
    static_assert(PDM_MAX_EXACT_LEVELS == PDM_MAX_PLAIN_BITMAP_LEVELS, "EXACT plain bitmap");
    const pdm_status st = plain_args(v, d_volume, h_alpha, d_dist, &a, &bits, false);
    if (st != PDM_OK) return st;
    return from_hip(pdm::launch_plain_exact_x(a, bits, stream));
}

pdm_status pdm_full_recompute_exact(const pdm_volume* v, const void* d_volume,
                                    const float* h_alpha, uint8_t* d_dist, hipStream_t stream) {
    pdm_status st = pdm_plain_exact_distance_x(v, d_volume, h_alpha, d_dist, stream);
    if (st != PDM_OK) return st;
    return pdm_distance_yz(v, d_dist, 1, stream);
}

const char* pdm_status_string(pdm_status s) {
    switch (s) {
        case PDM_OK: return "ok";
        case PDM_E_INVAL: return "invalid argument";
        case PDM_E_RANGE: return "value out of range";
        case PDM_E_UNSUPPORTED: return "unsupported argument";
        case PDM_E_DEVICE: return "device error";
    }
    return "unknown status";
}

const char* pdm_version(void) { return "pdm 0.1.0 gfx950"; }

}  // extern "C"
