/*
 * pdm.h -- C ABI of libpdm: partitioned distance maps on MI355X (gfx950).
 *
 * Method: "Accelerating Transfer Function Update for Distance Map based Volume
 * Rendering" (arXiv 2407.21552).  A volume of integer intensities is cut into
 * 4x4x4 bricks (Sec. 3.1).  The intensity range [0, L) is cut into n
 * partitions given by integer borders (Sec. 3.1).  For every partition p a
 * partitioned occupancy map (POM) marks the bricks holding intensities of p,
 * and its partitioned distance map (PDM) stores, per brick, the chessboard
 * distance in bricks to the nearest occupied brick, as uint8 clamped at 255
 * (Sec. 3.1, Sec. 3.2).  On a transfer-function (TF) change the active set S
 * (partitions holding an intensity of non-zero opacity) is found and the new
 * distance map is D' = min over p in S of PDM_p (Sec. 3.1, Eq. 1).  The plain
 * method recomputes occupancy and distance map from the volume on every TF
 * change (Sec. 2, Sec. 4.2).
 *
 * Occupancy reading: a brick is occupied for an intensity interval when its
 * intensity range [min, max] meets the interval (RANGE).  POMs and the plain
 * method use the same reading, so D' <= D holds element-wise, with equality
 * whenever no active partition mixes zero and non-zero opacity (Sec. 3.1).
 *
 * Layouts (all C order, x fastest):
 *   volume  [nz][ny][nx] of uint8 or uint16 (dtype), voxel < levels.
 *   bricks  [Bz][By][Bx] with Bx = ceil(nx/4) etc.; G = Bx*By*Bz.
 *   bmin/bmax [Bz][By][Bx] of the volume's dtype.
 *   pdms    [n][Bz][By][Bx] uint8 (n*G bytes, Sec. 5 memory n*V/b^3).
 *   dist    [Bz][By][Bx] uint8 (D' or D).
 *
 * Conventions for every call:
 *   - Pointers named d_* are device pointers; h_* are host pointers.  The
 *     caller owns and allocates every buffer; the library allocates nothing
 *     and keeps no pointer after returning.  Host arrays are read during the
 *     call only and may be freed as soon as it returns.
 *   - Device work is enqueued on `stream` (0 = the null stream) and the call
 *     returns without synchronising.  There is no global state (one
 *     exception: pdm_batch_build_noalloc keeps its scratch in a static device
 *     array): calls are reentrant; calls that write the same buffers must be
 *     ordered by the caller (same stream or events).
 *   - Arguments are validated on the host before any device work; a failed
 *     check returns PDM_E_INVAL or PDM_E_UNSUPPORTED and enqueues nothing.
 *     PDM_E_DEVICE reports a failed kernel launch.
 *   - On PDM_OK every output element is written, including the empty active
 *     set (D' = 255 everywhere).
 */
#ifndef PDM_H
#define PDM_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PDM_MAX_PARTITIONS 256  /* Table 1 goes up to 256 partitions */
#define PDM_DIST_CAP 255        /* uint8 distances, clamped (Sec. 3.2) */
#define PDM_BRICK 4             /* block size b = 4 (Sec. 3.1) */
#define PDM_MAX_GRID_AXIS 65535 /* bricks per axis */
#define PDM_MAX_GRID_X 16384    /* bricks along x */
#define PDM_MAX_PLAIN_LEVELS 65536 /* levels accepted by the plain method (any u16 range) */
#define PDM_MAX_PLAIN_BITMAP_LEVELS 16384 /* above this, the non-zero opacity levels go as runs */
#define PDM_MAX_PLAIN_RUNS 512     /* runs of non-zero opacity accepted above 16384 levels */
#define PDM_MAX_EXACT_LEVELS 16384 /* levels accepted by the EXACT calls */
#define PDM_MAX_EXACT_GRID_X 256   /* bricks along x accepted by the EXACT build */

typedef enum {
    PDM_OK = 0,
    PDM_E_INVAL = -1,       /* bad pointer, size, dtype, levels or bounds */
    PDM_E_RANGE = -2,       /* reserved: data-dependent range errors go to d_range_err */
    PDM_E_UNSUPPORTED = -3, /* valid but not handled by these kernels (brick != 4, sizes) */
    PDM_E_DEVICE = -4       /* a kernel launch failed */
} pdm_status;

typedef enum { PDM_U8 = 1, PDM_U16 = 2 } pdm_dtype;

typedef struct {
    int32_t nx, ny, nz; /* voxels per axis, each >= 1; index ((z*ny)+y)*nx+x */
    int32_t dtype;      /* pdm_dtype: bytes per voxel */
    int32_t levels;     /* L: every voxel < L; u8: 1..256, u16: 1..65536 */
    int32_t brick;      /* b; only 4 is supported (PDM_E_UNSUPPORTED otherwise) */
} pdm_volume;

typedef struct {
    int32_t bx, by, bz; /* bricks per axis */
    int64_t count;      /* G = bx*by*bz */
} pdm_grid;

/* Brick grid of a volume: Bx = ceil(nx/b), ... (Sec. 3.1).  Host only. */
pdm_status pdm_grid_of(const pdm_volume* v, pdm_grid* out);

/* Step 1 of the TF update (Sec. 3.1): S = { p : some intensity i in
 * [h_bounds[p], h_bounds[p+1]-1] has h_alpha[i] != 0 }.  Every intensity of a
 * partition is tested, present in the volume or not.  The test is on the bit
 * pattern, independent of the host's floating-point mode: NaN and subnormal
 * opacities count as non-zero, -0 as zero.
 * h_bounds: n+1 int32, h_bounds[0] = 0 < ... < h_bounds[n] = levels,
 * n in [1, 256].  h_alpha: `levels` floats.  h_active: 4 words out, bit p of
 * word p/64 set when p is in S.  Host only. */
pdm_status pdm_active_set(const int32_t* h_bounds, int32_t n, const float* h_alpha,
                          int32_t levels, uint64_t* h_active);

/* Per-brick intensity minimum and maximum over the brick's voxels inside the
 * volume; partial bricks on the far faces are clipped, never padded (Sec. 3.1
 * block reduction).  d_volume: nx*ny*nz voxels of v->dtype.  d_bmin, d_bmax:
 * G elements of v->dtype each.  d_range_err: nullable int32; if non-null it is
 * set to 1 by the device when some voxel is >= levels (it is never cleared:
 * zero it before the call). */
pdm_status pdm_build_bricks(const pdm_volume* v, const void* d_volume, void* d_bmin,
                            void* d_bmax, int32_t* d_range_err, hipStream_t stream);

/* One-time initialisation (Sec. 3.1): for every partition p the POM
 * (brick occupied when [bmin, bmax] meets [h_bounds[p], h_bounds[p+1]-1]) and
 * its PDM, the exact chessboard distance in bricks to the nearest occupied
 * brick of p, clamped at 255, and 255 everywhere when p occupies no brick.
 * d_bmin/d_bmax: output of pdm_build_bricks.  d_pdms: n*G bytes, [p][brick].
 * Equivalent to pdm_pom_distance_x followed by pdm_distance_yz(count = n). */
pdm_status pdm_build_partitions(const pdm_volume* v, const void* d_bmin, const void* d_bmax,
                                const int32_t* h_bounds, int32_t n, uint8_t* d_pdms,
                                hipStream_t stream);

/* TF update (Sec. 3.1, both steps; Eq. 1): S from h_alpha as in
 * pdm_active_set, then d_dist[c] = min over p in S of d_pdms[p*G + c]; 255
 * when S is empty.  Only the PDMs of S are read.  Any G and any pointer
 * alignment (d_dist must not overlap d_pdms).  h_active: nullable, 4 words
 * out (the S mask). */
pdm_status pdm_tf_update(const pdm_volume* v, const uint8_t* d_pdms, const int32_t* h_bounds,
                         int32_t n, const float* h_alpha, uint8_t* d_dist, uint64_t* h_active,
                         hipStream_t stream);

/* Range tables: a way to run step 2 of the TF update (Eq. 1) that reads
 * fewer maps.  The distance map of a union of partitions is the element-wise
 * min of their maps (the distance to a union is the min of the distances;
 * Sec. 3.1), so the maps of runs of 2^k consecutive partitions can be built
 * once and reused.  Level k (1 <= k <= K, K = min(max_level, floor(log2 n)))
 * holds the n - 2^k + 1 maps T_k[p] = min(PDM_p, ..., PDM_{p+2^k-1}),
 * p = 0 .. n-2^k, each G bytes like the PDMs, level after level in one
 * buffer.  A TF whose S is R runs of consecutive partitions is then combined
 * from at most 2R maps (runs longer than 2^(K+1) take more) instead of |S|;
 * D' is identical.  Memory: pdm_range_table_maps(n, max_level) * G bytes
 * (n = 64, max_level 6: 264 maps).
 *
 * pdm_range_table_maps: maps in the table; 0 when K = 0; -1 for n outside
 * [1, 256] or max_level < 0.  Host only. */
int64_t pdm_range_table_maps(int32_t n, int32_t max_level);

/* Builds levels 1..K of the table from d_pdms (n*G bytes) into d_table
 * (pdm_range_table_maps(n, max_level) * G bytes, caller-owned; may be null
 * when K = 0).  One launch per level; level k reads two maps of level k-1
 * per map written. */
pdm_status pdm_build_range_table(const pdm_volume* v, const uint8_t* d_pdms, int32_t n,
                                 int32_t max_level, uint8_t* d_table, hipStream_t stream);

/* The maps combined for the active set h_active (4 words, as from
 * pdm_active_set): *h_count indices into h_maps (room for 256), index i < n
 * is PDM i and i >= n is table map i - n.  Every maximal run [a, b] of S
 * takes PDM a when a = b, else the one or two level-floor(log2(b-a+1)) maps
 * covering it (past level K: level-K maps every 2^K partitions and one
 * ending at b).  The union of the covered partitions is exactly S.  Host
 * only. */
pdm_status pdm_range_cover(int32_t n, int32_t max_level, const uint64_t* h_active,
                           int32_t* h_maps, int32_t* h_count);

/* pdm_tf_update reading the cover's maps instead of every PDM of S: the same
 * D' and S mask.  d_table: built by pdm_build_range_table with the same n and
 * max_level (null allowed when K = 0). */
pdm_status pdm_tf_update_ranges(const pdm_volume* v, const uint8_t* d_pdms, const uint8_t* d_table,
                                const int32_t* h_bounds, int32_t n, int32_t max_level,
                                const float* h_alpha, uint8_t* d_dist, uint64_t* h_active,
                                hipStream_t stream);


/* Plain method (Sec. 2 and Sec. 4.2): from the raw volume, the occupancy of
 * every brick under the TF (occupied when some intensity i in the brick's
 * [min, max] has h_alpha[i] != 0, tested as in pdm_active_set) and its
 * clamped chessboard distance map D.
 * h_alpha: v->levels floats, levels <= PDM_MAX_PLAIN_LEVELS.  Up to
 * PDM_MAX_PLAIN_BITMAP_LEVELS levels any table is accepted; above, the
 * levels with h_alpha != 0 must form at most PDM_MAX_PLAIN_RUNS maximal runs
 * (a TF of a few ramps forms a few), else PDM_E_UNSUPPORTED.  d_dist: G bytes.
 * Equivalent to pdm_plain_distance_x followed by pdm_distance_yz(count = 1).
 * Voxels >= levels are a precondition violation (see pdm_build_bricks). */
pdm_status pdm_full_recompute(const pdm_volume* v, const void* d_volume, const float* h_alpha,
                              uint8_t* d_dist, hipStream_t stream);

/* Plain method from the cached brick [min, max] instead of the volume: the
 * same occupancy test as pdm_full_recompute (some intensity i in
 * [bmin, bmax] has h_alpha[i] != 0) and the same D, but reading 2*G*s bytes
 * of brick ranges instead of the whole volume.  This is the comparator that
 * an implementation of the plain method (Sec. 2, Sec. 4.2) keeping the
 * brick ranges of the one-time initialisation would run per TF change.
 * d_bmin/d_bmax: output of pdm_build_bricks (G elements of v->dtype each).
 * levels and h_alpha as for pdm_full_recompute.  d_dist: G bytes.  Equivalent
 * to pdm_plain_cached_distance_x followed by pdm_distance_yz(count = 1). */
pdm_status pdm_full_recompute_cached(const pdm_volume* v, const void* d_bmin, const void* d_bmax,
                                     const float* h_alpha, uint8_t* d_dist, hipStream_t stream);

/* Batched TF update: the update of pdm_tf_update for up to PDM_BATCH_MAX
 * volumes, each with its own PDMs, partitions, opacity table and output, in
 * one kernel launch (the step a server runs per tick).  h_items: `count`
 * descriptors (host, read during the call); every volume is validated as in
 * pdm_tf_update before anything is launched.  Outputs must not overlap.
 * h_active: nullable, 4 words per item (the S masks, item-major). */
#define PDM_BATCH_MAX 48
typedef struct {
    const pdm_volume* v;     /* geometry and levels of the volume */
    const uint8_t* d_pdms;   /* n*G bytes */
    const int32_t* h_bounds; /* n+1 partition borders */
    int32_t n;               /* partitions */
    const float* h_alpha;    /* v->levels entries */
    uint8_t* d_dist;         /* G bytes: D' */
} pdm_batch_update;

pdm_status pdm_batch_tf_update(const pdm_batch_update* h_items, int32_t count,
                               uint64_t* h_active, hipStream_t stream);

/* Batched update through range tables: pdm_tf_update_ranges for up to
 * PDM_BATCH_MAX requests (volume, TF, output), each reading the maps of its
 * own cover, in one kernel launch; the same D' and S masks as the single
 * calls.  The covers' map indices travel in the kernel arguments (room for
 * 640); a batch whose covers hold more is split into several launches on
 * `stream`, in order.  h_items: `count` descriptors (host, read during the
 * call); every request is validated as in pdm_tf_update_ranges before
 * anything is launched.  Outputs must not overlap.  h_active: nullable, 4
 * words per item (the S masks, item-major). */
typedef struct {
    const pdm_volume* v;     /* geometry and levels of the volume */
    const uint8_t* d_pdms;   /* n*G bytes */
    const uint8_t* d_table;  /* the volume's range table (n, max_level); null when K = 0 */
    const int32_t* h_bounds; /* n+1 partition borders */
    int32_t n;               /* partitions */
    int32_t max_level;       /* as given to pdm_build_range_table */
    const float* h_alpha;    /* v->levels entries */
    uint8_t* d_dist;         /* G bytes: D' */
} pdm_batch_range_update;

pdm_status pdm_batch_tf_update_ranges(const pdm_batch_range_update* h_items, int32_t count,
                                      uint64_t* h_active, hipStream_t stream);

/* Batched one-time initialisation: pdm_build_bricks + pdm_build_partitions
 * (Sec. 3.1: brick [min,max], then every partition's POM and its distance
 * transform) for up to PDM_BATCH_MAX volumes of different sizes, dtypes and
 * partition counts.  Three phases, each covering every volume: bricks + POM
 * x distances per group of brick rows, then all y passes, then all z passes;
 * either as three grouped launches or (cfg->single_launch) as ONE cooperative
 * launch of resident work-groups with a grid barrier between the phases.
 * Results are identical to the single-volume calls.  Every grid axis must be
 * <= 256 bricks (else PDM_E_UNSUPPORTED).  Voxel values are not range-checked
 * here (pdm_build_bricks reports them).
 *
 * d_workspace: device memory of pdm_batch_workspace_bytes(count) bytes,
 * 16-byte aligned, owned by the caller; it receives the barrier state and the
 * volume descriptors and must not be used by another call until the stream
 * has passed this batched build.  Its first 4 bytes are an error word, zeroed by the
 * call: non-zero once the stream has passed the build means a single-launch
 * barrier wait gave up after its time limit (never expected; the outputs
 * are then incomplete).  The grouped launches leave it zero.
 * cfg: nullable tuning knobs (see pdm_batch_config); results do not depend on
 * them. */
typedef struct {
    const pdm_volume* v;     /* geometry and levels */
    const void* d_volume;    /* voxels */
    void* d_bmin;            /* G elements of v->dtype */
    void* d_bmax;            /* G elements of v->dtype */
    const int32_t* h_bounds; /* n+1 partition borders */
    int32_t n;               /* partitions */
    uint8_t* d_pdms;         /* n*G bytes */
} pdm_batch_volume;

typedef struct {
    int32_t rows_per_item;  /* wave passes per first-phase work item, 1..256; 0 = 2 (a
                               pass covers 64/W brick rows, W = lanes per row, the
                               power of two >= Bx/4) */
    int32_t lines_mult;     /* 64-line groups per y/z work item, 1..16; 0 = 1 */
    int32_t largest_first;  /* 1: order the volumes' items by decreasing work */
    int32_t single_launch;  /* 0: three grouped launches; 1: one cooperative launch */
} pdm_batch_config;

size_t pdm_batch_workspace_bytes(int32_t count);

pdm_status pdm_batch_build(const pdm_batch_volume* h_vols, int32_t count, void* d_workspace,
                           size_t workspace_bytes, const pdm_batch_config* cfg,
                           hipStream_t stream);

/* pdm_batch_build without a workspace and without any allocation, for
 * callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  The descriptors and
 * the barrier state live in a static device array of the library (57,600
 * bytes: room for PDM_BATCH_MAX volumes, the limit of count; more is
 * PDM_E_INVAL), one per device, held until the process ends; its address is
 * looked up once per device on the first call.  Same validation, kernels and
 * results as pdm_batch_build; calls nothing that allocates.
 * The array is shared by every call on a device and keeps the last call's
 * contents (each call rewrites the descriptors and zeroes the barrier state
 * before its kernels run): calls on one device that overlap in time (on
 * different streams, or from several threads without ordering) race and
 * must not be made.  `stream` must belong to the current device
 * (PDM_E_INVAL otherwise).  d_error: nullable device uint32; when given, the
 * build's error word (see pdm_batch_build) is copied there on the stream
 * after the build. */
pdm_status pdm_batch_build_noalloc(const pdm_batch_volume* h_vols, int32_t count,
                                   const pdm_batch_config* cfg, uint32_t* d_error,
                                   hipStream_t stream);

/* EXACT occupancy reading (Sec. 3.1, literal wording): a brick is occupied
 * for an intensity interval when one of its voxels lies in it (for the plain
 * method: when one of its voxels has non-zero opacity), instead of the RANGE
 * test on [min, max].  EXACT occupancy is contained in RANGE occupancy, so
 * EXACT distances are element-wise >= RANGE ones; D' <= D and the equality
 * case hold within each reading. */

/* PDMs in the EXACT reading, built from the volume directly (no brick
 * [min, max] needed).  levels <= PDM_MAX_EXACT_LEVELS and
 * ceil(nx/4) <= PDM_MAX_EXACT_GRID_X, else PDM_E_UNSUPPORTED.  d_pdms: n*G
 * bytes.  The TF update (pdm_tf_update) is the same for both readings.
 * Equivalent to pdm_pom_exact_distance_x + pdm_distance_yz(count = n). */
pdm_status pdm_build_partitions_exact(const pdm_volume* v, const void* d_volume,
                                      const int32_t* h_bounds, int32_t n, uint8_t* d_pdms,
                                      hipStream_t stream);

/* Plain method in the EXACT reading: D from the volume, a brick being
 * occupied when one of its voxels has h_alpha[voxel] != 0.
 * levels <= PDM_MAX_EXACT_LEVELS.  Equivalent to pdm_plain_exact_distance_x +
 * pdm_distance_yz(count = 1). */
pdm_status pdm_full_recompute_exact(const pdm_volume* v, const void* d_volume,
                                    const float* h_alpha, uint8_t* d_dist, hipStream_t stream);

/* Phases, exposed so that each kernel can be timed on its own. */

/* First phase of pdm_build_partitions: for every partition, the POM and the
 * distance to the nearest occupied brick along x only (clamped at 255),
 * written to d_pdms[p*G + c]. */
pdm_status pdm_pom_distance_x(const pdm_volume* v, const void* d_bmin, const void* d_bmax,
                              const int32_t* h_bounds, int32_t n, uint8_t* d_pdms,
                              hipStream_t stream);

/* First phase of pdm_full_recompute: brick occupancy under the TF from the
 * volume and the distance to the nearest occupied brick along x only. */
pdm_status pdm_plain_distance_x(const pdm_volume* v, const void* d_volume, const float* h_alpha,
                                uint8_t* d_dist, hipStream_t stream);

/* First phase of pdm_full_recompute_cached: brick occupancy under the TF
 * from the cached [min, max] and the distance along x only. */
pdm_status pdm_plain_cached_distance_x(const pdm_volume* v, const void* d_bmin, const void* d_bmax,
                                       const float* h_alpha, uint8_t* d_dist, hipStream_t stream);

/* First phase of pdm_build_partitions_exact: EXACT POMs and x distances. */
pdm_status pdm_pom_exact_distance_x(const pdm_volume* v, const void* d_volume,
                                    const int32_t* h_bounds, int32_t n, uint8_t* d_pdms,
                                    hipStream_t stream);

/* First phase of pdm_full_recompute_exact: EXACT occupancy and x distances. */
pdm_status pdm_plain_exact_distance_x(const pdm_volume* v, const void* d_volume,
                                      const float* h_alpha, uint8_t* d_dist, hipStream_t stream);

/* Second phase of all of the above: completes `count` stacked grids [count][G]
 * in place from x-only distances to full chessboard distances with 1-D max-min passes
 * along y and then z, g(i) = min over j of max(|i-j|, f(j)), clamped at 255. */
pdm_status pdm_distance_yz(const pdm_volume* v, uint8_t* d_maps, int32_t count,
                           hipStream_t stream);

/* Human-readable name of a status code (static storage). */
const char* pdm_status_string(pdm_status s);

/* Library version string (static storage). */
const char* pdm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PDM_H */
