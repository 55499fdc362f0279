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

using pdm::ActiveList;
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

// Step 1 (Sec. 3.1): partitions holding an intensity with non-zero opacity.
void active_mask(const int32_t* b, int32_t n, const float* alpha, uint64_t mask[4]) {
    mask[0] = mask[1] = mask[2] = mask[3] = 0;
    for (int32_t p = 0; p < n; ++p)
        for (int32_t i = b[p]; i < b[p + 1]; ++i)
            if (alpha[i] != 0.0f) {  // NaN != 0: conservative
                mask[p >> 6] |= 1ull << (p & 63);
                break;
            }
}

pdm_status from_hip(hipError_t e) { return e == hipSuccess ? PDM_OK : PDM_E_DEVICE; }

// Validation and kernel arguments shared by both readings of the plain
// method: the non-zero opacity bitmap and the volume geometry.
pdm_status plain_args(const pdm_volume* v, const void* d_volume, const float* h_alpha,
                      uint8_t* d_dist, pdm::PlainArgs* a, AlphaBits* bits) {
    pdm_grid g;
    const pdm_status st = check_volume(v, &g);
    if (st != PDM_OK) return st;
    if (d_volume == nullptr || h_alpha == nullptr || d_dist == nullptr) return PDM_E_INVAL;
    if (v->levels > PDM_MAX_PLAIN_LEVELS) return PDM_E_UNSUPPORTED;
    memset(bits, 0, sizeof(*bits));
    for (int32_t i = 0; i < v->levels; ++i)
        if (h_alpha[i] != 0.0f) bits->w[i >> 5] |= 1u << (i & 31);
    a->vol = d_volume;
    a->dist = d_dist;
    a->nx = v->nx;
    a->ny = v->ny;
    a->nz = v->nz;
    a->Bx = g.bx;
    a->By = g.by;
    a->Bz = g.bz;
    a->bytes = v->dtype;
    a->nwords = (v->levels + 31) / 32;
    a->levels = v->levels;
    a->vec_ok = ((int64_t)v->nx * v->dtype) % 16 == 0 && aligned(d_volume, 16);
    a->store_vec = g.bx % 4 == 0 && aligned(d_dist, 4);
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
    a.vec_ok = ((int64_t)v->nx * v->dtype) % 16 == 0 && aligned(d_volume, 16);
    a.store_vec = g.bx % 4 == 0 && aligned(d_bmin, 4 * v->dtype) && aligned(d_bmax, 4 * v->dtype);
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
    ActiveList act;
    memset(&act, 0, sizeof(act));
    for (int32_t p = 0; p < n; ++p)
        if ((mask[p >> 6] >> (p & 63)) & 1ull) act.p[act.count++] = (uint8_t)p;
    int vec = 1;
    if (g.count % 16 == 0 && aligned(d_pdms, 16) && aligned(d_dist, 16))
        vec = 16;
    else if (g.count % 4 == 0 && aligned(d_pdms, 4) && aligned(d_dist, 4))
        vec = 4;
    return from_hip(pdm::launch_combine(d_pdms, g.count, act, d_dist, vec, stream));
}

pdm_status pdm_plain_distance_x(const pdm_volume* v, const void* d_volume, const float* h_alpha,
                                uint8_t* d_dist, hipStream_t stream) {
    pdm::PlainArgs a;
    AlphaBits bits;
    const pdm_status st = plain_args(v, d_volume, h_alpha, d_dist, &a, &bits);
    if (st != PDM_OK) return st;
    return from_hip(pdm::launch_plain_x(a, bits, stream));
}

pdm_status pdm_full_recompute(const pdm_volume* v, const void* d_volume, const float* h_alpha,
                              uint8_t* d_dist, hipStream_t stream) {
    pdm_status st = pdm_plain_distance_x(v, d_volume, h_alpha, d_dist, stream);
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
    a.vec_ok = ((int64_t)v->nx * v->dtype) % 16 == 0 && aligned(d_volume, 16);
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
    const pdm_status st = plain_args(v, d_volume, h_alpha, d_dist, &a, &bits);
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
