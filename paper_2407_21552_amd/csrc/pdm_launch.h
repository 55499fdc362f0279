// pdm_launch.h -- internal interface between the host API layer and the
// kernel launchers.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

#define PDM_PLAIN_MAX_SEGS 64    // x segments of 256 bricks: Bx <= 16384
#define PDM_ALPHA_WORDS 512      // non-zero opacity bitmap: levels <= 16384
#define PDM_EXACT_MAX_LEVELS 16384  // intensity -> partition table of the EXACT build
#define PDM_BATCH_MAX_ITEMS 48     // volumes per batched TF update (kernel-argument space)
#define PDM_BATCH_MAX_MAPS 640     // map indices per batched range-table launch (kernel-argument space)


namespace pdm {

// Partition borders, passed by value as kernel arguments.
struct Bounds {
    int32_t b[257];
};

// Indices of the active partitions (S), passed by value.
// The maps one TF-update launch combines: pointers to G-byte maps (PDMs or
// range-table maps), at most one per partition.
struct MapList {
    int32_t count;
    int32_t pad;
    const uint8_t* src[256];
};

// The non-zero opacity levels, passed by value.  Up to 16384 levels: bit i
// of w set when alpha[i] != 0, with per-word prefix counts.  Above that: the
// maximal runs of non-zero levels, w[j] = first | last << 16, increasing.
struct AlphaBits {
    uint32_t w[PDM_ALPHA_WORDS];
    uint16_t pre[PDM_ALPHA_WORDS + 2];  // pre[i] = set bits in w[0..i-1] (i <= nwords)
};

// One volume of a batched TF update (72 bytes), passed by value.
struct BatchItem {
    const uint8_t* pdms;
    uint8_t* out;
    int64_t G;
    int64_t first_block;  // first work-group of this volume (set by the launcher)
    int64_t pad;
    uint64_t mask[4];     // active partitions
};

struct BatchArgs {
    int32_t count;
    int32_t pad;
    BatchItem it[PDM_BATCH_MAX_ITEMS];
};

// One request of a batched update through range tables (56 bytes): the maps
// of its cover are idx[map_first .. map_first + map_count), index i < n
// naming PDM i and i >= n table map i - n.
struct MapsItem {
    const uint8_t* pdms;
    const uint8_t* table;
    uint8_t* out;
    int64_t G;
    int64_t first_block;  // first work-group of this request (set by the launcher)
    int32_t map_first;
    int32_t map_count;
    int32_t n;
    int32_t pad;
};

struct BatchMapsArgs {
    int32_t count;
    int32_t nidx;
    MapsItem it[PDM_BATCH_MAX_ITEMS];
    uint16_t idx[PDM_BATCH_MAX_MAPS];
};
static_assert(sizeof(BatchMapsArgs) <= 4000, "kernel arguments of the batched range-table update");
static_assert(offsetof(BatchMapsArgs, idx) % 4 == 0, "map indices are read as 32-bit words");

// Persistent batched build: one descriptor per volume in device memory.
struct BatchVol {
    const void* vol;
    void* bmin;
    void* bmax;
    uint8_t* pdms;
    int64_t G;
    int64_t first[3];  // first item of this volume in each phase (rows, y, z)
    int32_t items[3];  // items per phase
    int32_t chunks;    // items per slice (y) or row (z): ceil(n*Bx / (64*lines_mult))
    int32_t nx, ny, nz, Bx, By, Bz, bytes, n, levels, store_vec;
    int32_t rows;        // brick rows per first-phase item
    int32_t row_groups;  // first-phase items per z slice: ceil(By / rows)
    int32_t row_lanes;   // lanes per brick row in the first phase (power of two)
    int32_t pad1[6];
    int32_t bounds[257];
};

// Grid-barrier state of the single-launch batched build, one word per
// 128-byte line, zeroed before each launch.
struct BatchSync {
    uint32_t error;  // non-zero: a barrier wait gave up
    uint32_t pad0[31];
    uint32_t arrive;  // arrivals so far, over all barriers
    uint32_t pad1[31];
    uint32_t generation;  // barriers completed
    uint32_t pad2[31];
    uint32_t ticket[3][32];  // next item of each phase (one line each)
};

struct BrickArgs {
    const void* vol;
    void* bmin;
    void* bmax;
    int32_t* range_err;
    int nx, ny, nz, Bx, By, Bz, bytes, levels;
};

struct PomArgs {
    const void* bmin;
    const void* bmax;
    uint8_t* pdms;
    int64_t G;
    int Bx, By, Bz, bytes, n;
    int store_vec;
};

struct PlainArgs {
    const void* vol;
    uint8_t* dist;
    int nx, ny, nz, Bx, By, Bz, bytes, nwords, levels;
    int store_vec;
    int runs;  // AlphaBits holds runs (nwords of them), not the bitmap
};

struct CachedArgs {
    const void* bmin;
    const void* bmax;
    uint8_t* dist;
    int Bx, By, Bz, bytes, nwords, levels;
    int store_vec;  // packed stores of 4 distances allowed
    int load_vec;   // vector loads of 4 bricks' [min,max] allowed
    int runs;       // AlphaBits holds runs (nwords of them), not the bitmap
};

struct PomExactArgs {
    const void* vol;
    uint8_t* pdms;
    int64_t G;
    int nx, ny, nz, Bx, By, Bz, bytes, n, levels;
    int store_vec;
};

hipError_t launch_bricks(const BrickArgs& a, hipStream_t s);
hipError_t launch_pom_x(const PomArgs& a, const Bounds& b, hipStream_t s);
hipError_t launch_plain_x(const PlainArgs& a, const AlphaBits& bits, hipStream_t s);
hipError_t launch_plain_cached_x(const CachedArgs& a, const AlphaBits& bits, hipStream_t s);
hipError_t launch_pom_exact_x(const PomExactArgs& a, const Bounds& b, hipStream_t s);
hipError_t launch_plain_exact_x(const PlainArgs& a, const AlphaBits& bits, hipStream_t s);
hipError_t launch_batch_combine(BatchArgs& a, hipStream_t s);
// One launch for the a.count requests of `a` (sets first_block).
hipError_t launch_batch_maps(BatchMapsArgs& a, hipStream_t s);
// Uploads `count` descriptors into d_vols and zeroes d_sync, then runs the
// build over totals[ph] items per phase: three grouped launches, or with
// `single` one cooperative launch with grid barriers between the phases; a
// y/z item covers 64*lines_mult lines.
hipError_t launch_batch_build(const BatchVol* h_vols, int count, BatchVol* d_vols,
                              BatchSync* d_sync, const int64_t totals[3], int lines_mult,
                              int single, hipStream_t s);
// Device address and size of the calling device's scratch array of the
// allocation-free batched build (dev must be the current device); looked up
// on the first call per device.
hipError_t batch_scratch(int dev, uint8_t** ptr, size_t* bytes);
// *dst = *src (one word, device memory), on the stream.
hipError_t launch_copy_word(const uint32_t* src, uint32_t* dst, hipStream_t s);
hipError_t launch_distance_yz(uint8_t* maps, int count, int Bx, int By, int Bz, hipStream_t s);
// out = element-wise min of the listed maps of G bytes (255 for none); any
// size and pointer alignment.
hipError_t launch_combine(const MapList& maps, int64_t G, uint8_t* out, hipStream_t s);
// dst[p] = min(src[p], src[p + h]) for maps p = 0..count-1 (maps of G bytes,
// contiguous): one level of the range table from the level below.
hipError_t launch_range_level(const uint8_t* src, int64_t h, uint8_t* dst, int64_t count, int64_t G,
                              hipStream_t s);

}  // namespace pdm
