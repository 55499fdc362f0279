// pdm_launch.h -- internal interface between the host API layer and the
// kernel launchers.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime_api.h>
#include <stdint.h>

#define PDM_PLAIN_MAX_SEGS 64    // x segments of 256 bricks: Bx <= 16384
#define PDM_ALPHA_WORDS 512      // non-zero opacity bitmap: levels <= 16384
#define PDM_EXACT_MAX_LEVELS 16384  // intensity -> partition table of the EXACT build


namespace pdm {

// Partition borders, passed by value as kernel arguments.
struct Bounds {
    int32_t b[257];
};

// Indices of the active partitions (S), passed by value.
struct ActiveList {
    int32_t count;
    uint8_t p[256];
};

// Bit i set when alpha[i] != 0, passed by value.
struct AlphaBits {
    uint32_t w[PDM_ALPHA_WORDS];
};

struct BrickArgs {
    const void* vol;
    void* bmin;
    void* bmax;
    int32_t* range_err;
    int nx, ny, nz, Bx, By, Bz, bytes, levels;
    int vec_ok;     // 16-byte voxel-row loads allowed
    int store_vec;  // packed stores of 4 bricks allowed
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
    int vec_ok, store_vec;
};

struct PomExactArgs {
    const void* vol;
    uint8_t* pdms;
    int64_t G;
    int nx, ny, nz, Bx, By, Bz, bytes, n, levels;
    int vec_ok, store_vec;
};

hipError_t launch_bricks(const BrickArgs& a, hipStream_t s);
hipError_t launch_pom_x(const PomArgs& a, const Bounds& b, hipStream_t s);
hipError_t launch_plain_x(const PlainArgs& a, const AlphaBits& bits, hipStream_t s);
hipError_t launch_pom_exact_x(const PomExactArgs& a, const Bounds& b, hipStream_t s);
hipError_t launch_plain_exact_x(const PlainArgs& a, const AlphaBits& bits, hipStream_t s);
hipError_t launch_distance_yz(uint8_t* maps, int count, int Bx, int By, int Bz, hipStream_t s);
hipError_t launch_combine(const uint8_t* pdms, int64_t G, const ActiveList& act, uint8_t* out,
                          int vec, hipStream_t s);

}  // namespace pdm
