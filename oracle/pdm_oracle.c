/*
 * pdm_oracle.c -- CPU oracle for partitioned distance maps (PDMs).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * statement of what the GPU library computes.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code, header or table with the HIP library and includes nothing from it.
 *
 * Paper: "Accelerating Transfer Function Update for Distance Map based Volume
 * Rendering" (arXiv 2407.21552).  Every function cites the passage it follows.
 * All arithmetic is integer; there is no floating point except the test
 * alpha != 0 on the transfer function, which is exact.
 *
 * Layouts: a volume is [nz][ny][nx], x fastest, voxels of 1 byte (u8) or
 * 2 bytes (u16, little endian as in host memory).  A brick grid is
 * [Bz][By][Bx], x fastest.  A stack of n grids is [p][Bz][By][Bx].
 * Bricks, partitions, maps: see the readings listed per function.
 *
 * Parallelism: OpenMP over independent bricks, lines or partitions only; no
 * step is reordered, blocked or fused beyond its definition, so the result is
 * identical for any thread count.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define CAP 255 /* distances are stored as uint8 and clamped (Sec. 3.2) */

int oracle_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

static inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

/* Sec. 3.1: the volume is cut into non-overlapping blocks of b^3 voxels.  A
 * block on a far face of the volume holds only the voxels inside the volume. */
void oracle_grid(int nx, int ny, int nz, int b, int* bx, int* by, int* bz) {
    *bx = ceil_div(nx, b);
    *by = ceil_div(ny, b);
    *bz = ceil_div(nz, b);
}

static inline int voxel(const void* vol, int bytes, int64_t idx) {
    if (bytes == 1) return ((const uint8_t*)vol)[idx];
    return ((const uint16_t*)vol)[idx];
}

/* Per-brick intensity minimum and maximum over the voxels of the brick that
 * lie inside the volume (Sec. 3.1 block reduction; partial blocks clipped). */
void oracle_bricks(const void* vol, int bytes, int nx, int ny, int nz, int b,
                   uint16_t* bmin, uint16_t* bmax) {
    int Bx, By, Bz;
    oracle_grid(nx, ny, nz, b, &Bx, &By, &Bz);
    int64_t G = (int64_t)Bx * By * Bz;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < G; ++c) {
        int i = (int)(c % Bx), j = (int)((c / Bx) % By), k = (int)(c / ((int64_t)Bx * By));
        int lo = 1 << 30, hi = -1;
        for (int z = k * b; z < k * b + b && z < nz; ++z)
            for (int y = j * b; y < j * b + b && y < ny; ++y)
                for (int x = i * b; x < i * b + b && x < nx; ++x) {
                    int v = voxel(vol, bytes, ((int64_t)z * ny + y) * nx + x);
                    if (v < lo) lo = v;
                    if (v > hi) hi = v;
                }
        bmin[c] = (uint16_t)lo;
        bmax[c] = (uint16_t)hi;
    }
}

/* Partition table (Sec. 3.1): partition p covers the integer intensities
 * [bounds[p], bounds[p+1]-1]; bounds[0] = 0, bounds[n] = L, strictly
 * increasing.  Returns 0 when valid, -1 otherwise. */
int oracle_check_bounds(const int32_t* bounds, int n, int levels) {
    if (n < 1 || n > 256 || levels < 1) return -1;
    if (bounds[0] != 0 || bounds[n] != levels) return -1;
    for (int p = 0; p < n; ++p)
        if (bounds[p + 1] <= bounds[p]) return -1;
    return 0;
}

/* POM of one partition, RANGE reading: a brick is occupied for [lo,hi] when
 * its intensity interval [bmin,bmax] meets [lo,hi] (Sec. 3.1, POM definition,
 * taken on the brick's [min,max] summary). */
void oracle_pom_range(const uint16_t* bmin, const uint16_t* bmax, int64_t G,
                      int lo, int hi, uint8_t* occ) {
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < G; ++c)
        occ[c] = (bmin[c] <= hi && bmax[c] >= lo) ? 1 : 0;
}

/* POM of one partition, EXACT reading: a brick is occupied when at least one
 * of its voxels has an intensity in [lo,hi] (Sec. 3.1, literal wording). */
void oracle_pom_exact(const void* vol, int bytes, int nx, int ny, int nz, int b,
                      int lo, int hi, uint8_t* occ) {
    int Bx, By, Bz;
    oracle_grid(nx, ny, nz, b, &Bx, &By, &Bz);
    int64_t G = (int64_t)Bx * By * Bz;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < G; ++c) {
        int i = (int)(c % Bx), j = (int)((c / Bx) % By), k = (int)(c / ((int64_t)Bx * By));
        int found = 0;
        for (int z = k * b; z < k * b + b && z < nz && !found; ++z)
            for (int y = j * b; y < j * b + b && y < ny && !found; ++y)
                for (int x = i * b; x < i * b + b && x < nx && !found; ++x) {
                    int v = voxel(vol, bytes, ((int64_t)z * ny + y) * nx + x);
                    if (v >= lo && v <= hi) found = 1;
                }
        occ[c] = (uint8_t)found;
    }
}

/* One 1-D max-min pass along a line of m samples f[0], f[s], f[2s], ...:
 *   g(i) = min over j of max(|i - j|, f(j)).
 * Candidates with |i - j| >= the best value found so far cannot lower it, so
 * the search widens from i until that bound.  Inputs are <= CAP, hence so is
 * the result. */
static void maxmin_line(const uint8_t* f, int m, int64_t s, uint8_t* g) {
    for (int i = 0; i < m; ++i) {
        int best = f[(int64_t)i * s];
        for (int d = 1; d < best; ++d) {
            int cand = CAP + 1;
            if (i - d >= 0) {
                int v = f[(int64_t)(i - d) * s];
                int c = v > d ? v : d;
                if (c < cand) cand = c;
            }
            if (i + d < m) {
                int v = f[(int64_t)(i + d) * s];
                int c = v > d ? v : d;
                if (c < cand) cand = c;
            }
            if (cand < best) best = cand;
        }
        g[(int64_t)i * s] = (uint8_t)best;
    }
}

/* Chessboard (L-infinity) distance transform of an occupancy grid, in brick
 * units, clamped at 255 (Sec. 3.1 PDM definition; uint8 clamp of Sec. 3.2).
 *   dist(c) = min(255, min over occupied c' of max(|dx|,|dy|,|dz|)),
 * and 255 everywhere when nothing is occupied.  Computed as three separable
 * max-min passes (x, then y, then z): max distributes over min and is
 * associative, so the passes compose to the 3-D minimum; clamping each pass at
 * 255 gives the same result as clamping once at the end.  The first pass
 * starts from f = 0 on occupied bricks and 255 elsewhere. */
void oracle_dt(const uint8_t* occ, int Bx, int By, int Bz, uint8_t* dist) {
    int64_t G = (int64_t)Bx * By * Bz;
    uint8_t* f = (uint8_t*)malloc((size_t)G);
    uint8_t* g = (uint8_t*)malloc((size_t)G);
    for (int64_t c = 0; c < G; ++c) f[c] = occ[c] ? 0 : CAP;
    /* x pass: lines are rows, stride 1 */
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < (int64_t)By * Bz; ++r)
        maxmin_line(f + r * Bx, Bx, 1, g + r * Bx);
    /* y pass: lines run along y, stride Bx */
#pragma omp parallel for schedule(static)
    for (int64_t l = 0; l < (int64_t)Bx * Bz; ++l) {
        int64_t k = l / Bx, i = l % Bx;
        int64_t base = k * (int64_t)Bx * By + i;
        maxmin_line(g + base, By, Bx, f + base);
    }
    /* z pass: lines run along z, stride Bx*By */
#pragma omp parallel for schedule(static)
    for (int64_t l = 0; l < (int64_t)Bx * By; ++l)
        maxmin_line(f + l, Bz, (int64_t)Bx * By, dist + l);
    free(f);
    free(g);
}

/* PDMs (Sec. 3.1): for every partition p independently, the POM of p and its
 * clamped chessboard distance transform; stored [p][Bz][By][Bx].  mode 0 is
 * the RANGE reading from the brick [min,max] summary, mode 1 the EXACT
 * reading from the voxels (vol may be NULL in mode 0). */
int oracle_pdms(const void* vol, int bytes, int nx, int ny, int nz, int b,
                const uint16_t* bmin, const uint16_t* bmax,
                const int32_t* bounds, int n, int levels, int mode, uint8_t* pdms) {
    if (oracle_check_bounds(bounds, n, levels)) return -1;
    int Bx, By, Bz;
    oracle_grid(nx, ny, nz, b, &Bx, &By, &Bz);
    int64_t G = (int64_t)Bx * By * Bz;
    uint8_t* occ = (uint8_t*)malloc((size_t)G);
    for (int p = 0; p < n; ++p) {
        int lo = bounds[p], hi = bounds[p + 1] - 1;
        if (mode == 0)
            oracle_pom_range(bmin, bmax, G, lo, hi, occ);
        else
            oracle_pom_exact(vol, bytes, nx, ny, nz, b, lo, hi, occ);
        oracle_dt(occ, Bx, By, Bz, pdms + (int64_t)p * G);
    }
    free(occ);
    return 0;
}

/* Step 1 of the update (Sec. 3.1): S = partitions holding at least one
 * intensity whose opacity is non-zero.  Every intensity of the partition is
 * tested, present in the volume or not.  NaN compares unequal to zero and so
 * counts as non-zero.  S is returned as a 256-bit mask, bit p of word p/64. */
int oracle_active(const int32_t* bounds, int n, const float* alpha, int levels,
                  uint64_t mask[4]) {
    if (oracle_check_bounds(bounds, n, levels)) return -1;
    mask[0] = mask[1] = mask[2] = mask[3] = 0;
    for (int p = 0; p < n; ++p)
        for (int v = bounds[p]; v < bounds[p + 1]; ++v)
            if (alpha[v] != 0.0f) {
                mask[p >> 6] |= (uint64_t)1 << (p & 63);
                break;
            }
    return 0;
}

/* Step 2 of the update (Sec. 3.1, Eq. 1): D'(c) = min over p in S of PDM_p(c);
 * with S empty nothing is occupied and D' is 255 everywhere. */
void oracle_combine(const uint8_t* pdms, int n, int64_t G, const uint64_t mask[4],
                    uint8_t* out) {
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < G; ++c) {
        int m = CAP;
        for (int p = 0; p < n; ++p)
            if ((mask[p >> 6] >> (p & 63)) & 1) {
                int v = pdms[(int64_t)p * G + c];
                if (v < m) m = v;
            }
        out[c] = (uint8_t)m;
    }
}

/* Plain method (Sec. 2, Deakin and Knackstedt; compared in Sec. 4.2): the
 * occupancy of each brick under the transfer function, RANGE reading: the
 * brick is occupied when some intensity i in [bmin,bmax] has alpha[i] != 0.
 * Uses the count of non-zero entries below each intensity,
 *   cnt[i] = #{ j < i : alpha[j] != 0 },
 * so the test is cnt[bmax+1] - cnt[bmin] > 0.  Returns -1 if a brick maximum
 * is not below the number of levels. */
int oracle_plain_occ_range(const uint16_t* bmin, const uint16_t* bmax, int64_t G,
                           const float* alpha, int levels, uint8_t* occ) {
    int32_t* cnt = (int32_t*)malloc(sizeof(int32_t) * ((size_t)levels + 1));
    cnt[0] = 0;
    for (int i = 0; i < levels; ++i) cnt[i + 1] = cnt[i] + (alpha[i] != 0.0f ? 1 : 0);
    int bad = 0;
    for (int64_t c = 0; c < G; ++c)
        if (bmax[c] >= levels) bad = 1;
    if (!bad) {
#pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < G; ++c)
            occ[c] = (cnt[bmax[c] + 1] - cnt[bmin[c]]) > 0 ? 1 : 0;
    }
    free(cnt);
    return bad ? -1 : 0;
}

/* Plain method occupancy, EXACT reading: the brick is occupied when one of
 * its voxels maps to a non-zero opacity. */
int oracle_plain_occ_exact(const void* vol, int bytes, int nx, int ny, int nz, int b,
                           const float* alpha, int levels, uint8_t* occ) {
    int Bx, By, Bz;
    oracle_grid(nx, ny, nz, b, &Bx, &By, &Bz);
    int64_t G = (int64_t)Bx * By * Bz;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t c = 0; c < G; ++c) {
        int i = (int)(c % Bx), j = (int)((c / Bx) % By), k = (int)(c / ((int64_t)Bx * By));
        int found = 0;
        for (int z = k * b; z < k * b + b && z < nz; ++z)
            for (int y = j * b; y < j * b + b && y < ny; ++y)
                for (int x = i * b; x < i * b + b && x < nx; ++x) {
                    int v = voxel(vol, bytes, ((int64_t)z * ny + y) * nx + x);
                    if (v >= levels) bad = 1;
                    else if (alpha[v] != 0.0f) found = 1;
                }
        occ[c] = (uint8_t)found;
    }
    return bad ? -1 : 0;
}

/* Plain method end to end (Sec. 4.2, the comparison): from the raw volume,
 * recompute the brick occupancy under the transfer function and its clamped
 * chessboard distance map D.  mode 0 RANGE, mode 1 EXACT. */
int oracle_full_recompute(const void* vol, int bytes, int nx, int ny, int nz, int b,
                          const float* alpha, int levels, int mode, uint8_t* dist) {
    int Bx, By, Bz;
    oracle_grid(nx, ny, nz, b, &Bx, &By, &Bz);
    int64_t G = (int64_t)Bx * By * Bz;
    uint8_t* occ = (uint8_t*)malloc((size_t)G);
    int rc;
    if (mode == 0) {
        uint16_t* bmin = (uint16_t*)malloc(sizeof(uint16_t) * (size_t)G);
        uint16_t* bmax = (uint16_t*)malloc(sizeof(uint16_t) * (size_t)G);
        oracle_bricks(vol, bytes, nx, ny, nz, b, bmin, bmax);
        rc = oracle_plain_occ_range(bmin, bmax, G, alpha, levels, occ);
        free(bmin);
        free(bmax);
    } else {
        rc = oracle_plain_occ_exact(vol, bytes, nx, ny, nz, b, alpha, levels, occ);
    }
    if (rc == 0) oracle_dt(occ, Bx, By, Bz, dist);
    free(occ);
    return rc;
}
