/*
 * pgm.h -- C ABI of libpgm, pyramidal gradient matching on AMD Instinct MI355X (gfx950).
 *
 * The method is that of Y. Li, "Pyramidal Gradient Matching for Optical Flow Estimation"
 * (arXiv:1704.03217): two images in, the gradient image of every level of their pyramids
 * (Sec. III-A, Eq. 1-2; Sec. III-D), coarse-to-fine limited PatchMatch (Sec. III-B, Eq. 3-5)
 * on a regular seed grid, a forward-backward consistency check with an outlier record at
 * every level (Sec. III-C/D, Eq. 6-8), and the level-0 matches on the grid out (Sec. III-G).
 *
 * Conventions for every entry point
 *  - Image and output pointers passed to pgm_match are DEVICE pointers owned by the caller
 *    (e.g. torch tensors). Pointers named host_* are host pointers owned by the caller.
 *  - Images are interleaved RGB uint8 (HWC), `pitch_bytes` apart between rows (>= 3*w); one
 *    image spans pitch_bytes * (h - 1) + 3 * w bytes, which must stay below 2^31 (PGM_EINVAL).
 *  - A context owns one device workspace allocated once by pgm_create; pgm_match never
 *    allocates device memory and returns PGM_ENOMEM when the workspace is too small.
 *  - pgm_match is asynchronous on the caller's HIP stream (a hipStream_t passed as void*;
 *    NULL is the default stream). Argument errors are reported synchronously; device errors
 *    are reported by the call that observes them. Calls on one context must not overlap:
 *    use one context per stream / host thread.
 *  - All functions return a pgm_status; pgm_last_error() describes the last failure of a
 *    context in text.
 *  - Logging to stderr by the environment variable PGM_LOG (read once): 1 failures, 2 also
 *    contexts, servers and each server request (shape, requests sharing its launch sequence,
 *    latency from submission to completion as seen by polling, pool bytes in use), 3 also
 *    each matching call (pairs, launches); unset or 0: nothing.
 */
#ifndef PGM_H
#define PGM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__) || defined(__clang__)
#define PGM_API __attribute__((visibility("default")))
#else
#define PGM_API
#endif

typedef int32_t pgm_status;
enum {
    PGM_OK = 0,
    PGM_EINVAL = -1,       /* invalid argument (bad sizes, parameters or null pointers)   */
    PGM_ENOMEM = -2,       /* the context's workspace is smaller than pgm_query's figure  */
    PGM_EDEVICE = -3,      /* a HIP runtime error (message in pgm_last_error)             */
    PGM_EBUSY = -4,        /* try again later: a server's request queue is full (poll to  */
                           /* take finished requests, then submit again)                  */
    PGM_EUNSUPPORTED = -5  /* valid but not supported by this build                       */
};

enum { PGM_FEAT_INT16 = 0,     /* full gradient image, int16 (PGM-C / PGM-G, Sec. III-F)      */
       PGM_FEAT_F32_DIR = 1,   /* direction-only unit gradients, float (PGM-CD / PGM-GD)      */
       PGM_FEAT_SIGN = 2 };    /* direction-only, "G./|G|" read element-wise: the sign of     */
                               /* every gradient component in {-1, 0, 1} (integer distance)   */
enum { PGM_RGB = 0, PGM_GRAY = 1 };                    /* 6- or 2-channel gradient image       */
enum { PGM_SPACE_RGB = 0,    /* colour spaces of the gradient pyramids (Sec. III-E, Table II)  */
       PGM_SPACE_YCRCB = 1,  /* integer BT.601: Y = (77R + 150G + 29B + 128) >> 8, Cr and Cb  */
                             /* 128 + round((R - Y) 183 / 256), 128 + round((B - Y) 144 / 256) */
       PGM_SPACE_LAB = 2 };  /* 8-bit CIELab (sRGB curve, D65): L* 255/100, a* + 128, b* + 128 */
enum { PGM_INIT_RANDOM = 0, PGM_INIT_EXHAUSTIVE = 1 }; /* initial field at the coarsest level  */
enum { PGM_RS_FLOOR = 0,      /* limited random search (Sec. III-B, Eq. 5): the i-th offset   */
                             /* floor(R_i W / 2^i), R_i uniform in (-1, 1)                  */
       PGM_RS_SYMMETRIC = 1 };  /* the i-th offset uniform over the integers of [-w_i, w_i],  */
                                /* w_i = floor(W / 2^i)                                       */
enum { PGM_METRIC_SAD = 0,   /* patch distance: sum of absolute feature differences          */
       PGM_METRIC_SSD = 1 }; /* sum of squared differences (Eq. 3 as printed), integer       */
                             /* features only, exact in 64 bits                              */

#define PGM_MAX_LEVELS 8

/* flags of a match */
#define PGM_FLAG_INIT   1u  /* the field is initialised at this seed                         */
#define PGM_FLAG_INLIER 2u  /* the outlier record says "no" after the last update (Eq. 7)    */
#define PGM_FLAG_RECORD 4u  /* the record propagated into this level said "no" (Eq. 8)       */

/* Matching parameters (Sec. IV lists the paper's values: W=2, S=5, L=3, s=1/2, N=2, m=2,
 * 6 iterations at full resolution and 4 elsewhere; patch radius 7 forward / 5 backward). */
typedef struct {
    int32_t levels;                  /* L, pyramid levels, 1..8; the coarsest is m = L-1     */
    int32_t seed_stride;             /* seed grid spacing in pixels, >= 1 (1 = dense field)  */
    int32_t patch_fwd, patch_bwd;    /* patch side of the forward / backward field, 1..16    */
    int32_t iters[PGM_MAX_LEVELS];   /* propagation-search iterations per level (0 = full)   */
    int32_t radius;                  /* W of Eq. 5 below the initial field, >= 1             */
    int32_t max_disp;                /* |d| bound at full resolution for the initial field;  */
                                     /* 0 = the whole image; -k (k in 1..1024) = ceil(w / k) */
                                     /* for a w-wide pair (pairs of many sizes)              */
    int32_t sobel_ksize;             /* S of Eq. 1: 3 or 5                                   */
    int32_t feature;                 /* PGM_FEAT_*                                           */
    int32_t color;                   /* PGM_RGB or PGM_GRAY                                  */
    int32_t fwd_bwd;                 /* 1 = forward-backward consistency check at each level */
    int32_t consistency_px;          /* tau: consistent iff |d_fwd + d_bwd|^2 <= tau^2      */
    int32_t init_mode;               /* PGM_INIT_*                                           */
    int32_t refine_rounds;           /* N of Sec. III-D: round trips between m and m-1       */
    int32_t min_region_px;           /* small-region removal (Sec. III-E): forward inliers   */
                                     /* in regions of fewer pixels (seeds x stride^2) become */
                                     /* outliers; 0 = off (the paper uses 9)                 */
    int32_t region_link_px;          /* 4-neighbouring inliers share a region when their     */
                                     /* displacements differ by less than this (1..65535)   */
    int32_t space_fwd[PGM_MAX_LEVELS]; /* PGM_SPACE_* of the forward / backward gradient    */
    int32_t space_bwd[PGM_MAX_LEVELS]; /* pyramid per level (PGM_RGB only; 0 = RGB)         */
    int32_t metric;                  /* PGM_METRIC_*                                         */
    int32_t rs_mode;                 /* PGM_RS_*: offsets of the limited random search       */
    uint64_t rng_seed;               /* key of the counter-based random generator            */
} pgm_params;

/* One match on the level-0 seed grid: seed (x1, y1) in the first image of the pair and its
 * match (x2, y2) in the second. dist is the patch distance (the integer sum of the metric,
 * clamped to 0x7FFFFFFE, or the bits of a float for PGM_FEAT_F32_DIR); 0x7FFFFFFF and
 * (x2, y2) = (x1, y1) where the field is uninitialised. flags: PGM_FLAG_*. 24 bytes. */
typedef struct { int32_t x1, y1, x2, y2, dist; uint32_t flags; } pgm_match_t;

/* Sizes for an image size and parameter set. */
typedef struct {
    int32_t levels;
    int32_t level_w[PGM_MAX_LEVELS], level_h[PGM_MAX_LEVELS];   /* image size per level     */
    int32_t level_nx[PGM_MAX_LEVELS], level_ny[PGM_MAX_LEVELS]; /* seed grid per level      */
    int32_t nx, ny;                  /* level-0 grid: pgm_match writes nx*ny matches          */
    uint64_t workspace_bytes;        /* device workspace pgm_match needs for one pair         */
    uint64_t workspace_shared_bytes; /* part of it shared by all pairs of a batch (random    */
                                     /* numbers); a batch of n pairs needs                    */
    uint64_t workspace_pair_bytes;   /* shared + n * pair bytes                               */
} pgm_sizes;

/* Presets. */
enum {
    PGM_PRESET_PAPER = 0,    /* Sec. IV parameters on a dense field (stride 1, P 15 / 11)    */
    PGM_PRESET_CONFIG1 = 1,  /* 256x192 pairs: L=3, stride 3, 8x8, 4 iterations, |d|<=20    */
    PGM_PRESET_CONFIG2 = 2,  /* 1024x436 pairs: L=5, stride 3, 8x8, 6 iterations, |d|<=200  */
    PGM_PRESET_CONFIG3 = 3,  /* 1242x375 pairs, direction-only float features, |d|<=250     */
    PGM_PRESET_CONFIG4 = 4,  /* batches of pairs of many sizes: configuration 2's matching  */
                             /* with |d| <= ceil(w / 5) per pair (max_disp = -5)            */
    PGM_PRESET_CONFIG5 = 5   /* served pairs of any size: as configuration 4                */
};

/* Fill *p with a preset. Host only. PGM_EINVAL for an unknown preset or p == NULL. */
PGM_API pgm_status pgm_default_params(pgm_params* p, int32_t preset);

/* Validate parameters for a w x h pair and report the grid and workspace sizes (Sec. III-D:
 * level l is ceil(w / 2^l) x ceil(h / 2^l)). Host only, no device work. */
PGM_API pgm_status pgm_query(const pgm_params* p, int32_t w, int32_t h, pgm_sizes* out);

/* Create a context on HIP device `device` with a device workspace of `workspace_bytes`
 * (0 picks 256 MiB). The context owns the workspace until pgm_destroy. */
PGM_API pgm_status pgm_create(int32_t device, uint64_t workspace_bytes, void** out_ctx);

/* Match one pair (the whole method of Sec. III on the GPU).
 *  img1, img2      device, HWC RGB uint8, w x h, rows pitch_bytes apart (may alias).
 *  out_fwd         device, nx*ny pgm_match_t, forward matches (image 1 -> image 2).
 *  out_bwd         device or NULL, nx*ny backward matches (image 2 -> image 1).
 *  out_n_inliers   device or NULL, one int32: the number of forward inliers.
 *  out_compact     device or NULL, nx*ny pgm_match_t: forward inliers in row-major seed
 *                  order, the first *out_n_inliers entries valid (Sec. III-G hands these to
 *                  the interpolator).
 *  out_n_evals     device or NULL, one uint64: patch-distance evaluations are ADDED to it.
 *  stream          hipStream_t or NULL.
 * The context's workspace keeps every level's state until the next call (pgm_dump_*). */
PGM_API pgm_status pgm_match(void* ctx, const pgm_params* p, const uint8_t* img1, const uint8_t* img2,
                     int32_t w, int32_t h, int32_t pitch_bytes, pgm_match_t* out_fwd,
                     pgm_match_t* out_bwd, int32_t* out_n_inliers, pgm_match_t* out_compact,
                     uint64_t* out_n_evals, void* stream);

/* Match n_pairs pairs of the same size and parameters in one pass: every kernel launch of the
 * method covers all pairs (the pair is one more dimension of each grid), so launch latency is
 * paid once per batch. Pair k's images are img1 + k * image_stride_bytes and
 * img2 + k * image_stride_bytes (stride >= pitch_bytes * h); its outputs are out_* + k * nx * ny
 * matches and out_n_inliers[k]; out_n_evals receives the total. Each pair's results are
 * identical to those of pgm_match on that pair alone (the random numbers depend only on the
 * parameters). The workspace must hold workspace_shared_bytes + n_pairs * workspace_pair_bytes
 * (pgm_query), else PGM_ENOMEM. The dump entry points then show pair 0. */
PGM_API pgm_status pgm_match_batch(void* ctx, const pgm_params* p, int32_t n_pairs, const uint8_t* img1,
                                   const uint8_t* img2, int32_t w, int32_t h, int32_t pitch_bytes,
                                   int64_t image_stride_bytes, pgm_match_t* out_fwd, pgm_match_t* out_bwd,
                                   int32_t* out_n_inliers, pgm_match_t* out_compact, uint64_t* out_n_evals,
                                   void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): pgm_match without a context. The workspace is a
 * fixed device array of PGM_STATIC_SCRATCH_BYTES inside the library, one per GPU (it occupies
 * device memory on every GPU the library's code is loaded on, whether or not this entry point
 * is called), whose address is looked up on the first call on each device (with that device
 * current) and kept until the process ends; the call itself allocates nothing. It runs on the current HIP device, with the arguments,
 * outputs and stream of pgm_match. PGM_ENOMEM, before any device work, when the pair's
 * workspace (pgm_query's workspace_bytes) exceeds the array: 64 MiB holds a 1024x436 or a
 * 1242x375 pair with the configuration presets, not the dense paper preset at that size.
 * Every call on one GPU uses the same array: calls that overlap on a GPU (different streams
 * or host threads without ordering between them) race and give undefined results. The dump
 * entry points do not see these calls; pgm_last_error(NULL) describes the last failure. */
#define PGM_STATIC_SCRATCH_BYTES (64ull << 20)
PGM_API pgm_status pgm_match_static(const pgm_params* p, const uint8_t* img1, const uint8_t* img2, int32_t w,
                                    int32_t h, int32_t pitch_bytes, pgm_match_t* out_fwd, pgm_match_t* out_bwd,
                                    int32_t* out_n_inliers, pgm_match_t* out_compact, uint64_t* out_n_evals,
                                    void* stream);

/* One group of a pgm_match_groups call: n_pairs pairs of one size and one parameter set, laid
 * out as for pgm_match_batch (pair k at img1/img2 + k * image_stride_bytes, outputs at
 * out_* + k * nx * ny and out_n_inliers[k]). All pointers are device pointers except params. */
typedef struct {
    const pgm_params* params;
    int32_t n_pairs, w, h, pitch_bytes;
    int64_t image_stride_bytes;
    const uint8_t* img1;
    const uint8_t* img2;
    pgm_match_t* out_fwd;
    pgm_match_t* out_bwd;        /* or NULL */
    int32_t* out_n_inliers;      /* or NULL */
    pgm_match_t* out_compact;    /* or NULL */
} pgm_group;

/* Match several groups of pairs whose sizes and parameters differ between groups. The groups
 * run concurrently on the context's internal streams (each exactly as pgm_match_batch runs
 * it, so every pair's results equal pgm_match on that pair alone), forked from and joined
 * back into `stream`. Group g uses the workspace after the parts of groups 0..g-1, each part
 * workspace_shared_bytes + n_pairs * workspace_pair_bytes rounded up to 256 bytes; the call
 * returns PGM_ENOMEM, before any device work, when the parts do not fit. out_n_evals (device
 * or NULL) receives the total evaluation count. With use_graph = 1 the call's launches are
 * captured into one HIP graph that later calls with identical arguments (pointers and
 * parameter values) replay with a single launch; any other call re-captures it. use_graph
 * is ignored while profiling is on. The dump entry points then show group n_groups-1, pair 0. */
PGM_API pgm_status pgm_match_groups(void* ctx, int32_t n_groups, const pgm_group* groups,
                                    uint64_t* out_n_evals, int32_t use_graph, void* stream);

/* Request server: pairs of any size and parameters arrive one at a time and are matched
 * concurrently. A server owns a device memory pool of pool_bytes and n_streams HIP streams
 * (1..16); at most max_queued requests wait for memory (0 = 4096), and up to max_batch
 * requests (1..16, 0 = 16) may share one launch sequence.
 * pgm_server_submit queues a request (the pgm_match arguments plus a caller tag) and starts
 * queued requests, oldest first, when no launch sequence is in flight (pgm_server_poll and
 * pgm_server_drain: while fewer than 2 * n_streams are) and the head's workspace
 * (pgm_query's workspace_bytes rounded up to 256) fits in the pool; under load requests
 * gather in the queue meanwhile. The head starts together with the later queued
 * requests of the same width, height, pitch and parameters that ask for the same outputs
 * (at most max_batch, as many as the free memory holds): they run as one batch whose kernels
 * cover every pair (each pair's buffers from a pointer table), so per-pair launch costs are
 * paid once, on the least loaded stream. Every request's results equal pgm_match on that pair
 * alone. A request's launches are ordered after the work the caller had issued on `stream`
 * (hipStream_t or NULL) when it submitted, so inputs and zero-filled outputs produced there
 * are seen. PGM_EBUSY when max_queued requests are already waiting (nothing is queued:
 * poll, then submit again).
 * pgm_server_poll reports finished requests: it writes up to max_tags tags to host_tags and,
 * when host_status is not NULL, each request's status (PGM_OK, or the error that stopped its
 * launches: its outputs are then undefined), returns their number (or a negative
 * pgm_status), frees their memory and starts queued requests. A request whose launches failed
 * keeps its memory until its stream has passed them. The caller keeps a request's images and
 * outputs alive until its tag is reported. pgm_server_drain waits until nothing is queued or
 * running (the finished tags stay for pgm_server_poll). pgm_server_stats reports the launch
 * sequences and the requests started so far and the pool bytes in use. Argument errors are reported by
 * pgm_server_submit synchronously, and PGM_ENOMEM when the request alone exceeds the pool.
 * One host thread per server. */
PGM_API pgm_status pgm_server_create(int32_t device, uint64_t pool_bytes, int32_t n_streams, int32_t max_queued,
                                     int32_t max_batch, void** out_server);
PGM_API pgm_status pgm_server_submit(void* server, const pgm_params* p, const uint8_t* img1,
                                     const uint8_t* img2, int32_t w, int32_t h, int32_t pitch_bytes,
                                     pgm_match_t* out_fwd, pgm_match_t* out_bwd, int32_t* out_n_inliers,
                                     pgm_match_t* out_compact, uint64_t* out_n_evals, uint64_t tag,
                                     void* stream);
PGM_API int32_t pgm_server_poll(void* server, uint64_t* host_tags, int32_t* host_status, int32_t max_tags);
PGM_API pgm_status pgm_server_stats(void* server, int64_t* host_sequences, int64_t* host_started,
                                    uint64_t* host_bytes_in_use);
PGM_API pgm_status pgm_server_pending(void* server, int32_t* host_queued, int32_t* host_running,
                                      int32_t* host_finished);
PGM_API pgm_status pgm_server_drain(void* server);
PGM_API const char* pgm_server_last_error(void* server);
PGM_API void pgm_server_destroy(void* server);

/* Matches as text for an external sparse-to-dense interpolator (Sec. III-G hands the
 * grid matches to EpicFlow, whose match files hold one "x1 y1 x2 y2" line per match). Host
 * only: formats the n matches at host_matches (copied from a pgm_match output), all of them
 * or only those flagged PGM_FLAG_INLIER, as decimal lines "x1 y1 x2 y2\n" into host_buf
 * (capacity cap bytes, not NUL-terminated) and stores the bytes needed in *host_len (always,
 * so a call with host_buf NULL sizes the buffer). PGM_ENOMEM, with *host_len set, when cap
 * is too small; nothing is written then. */
PGM_API pgm_status pgm_format_matches(const pgm_match_t* host_matches, int64_t n, int32_t inliers_only,
                                      char* host_buf, uint64_t cap, uint64_t* host_len);

/* Debug copies of the last pgm_match's intermediate state into host memory; each waits for
 * the last call's stream to finish.
 *  pgm_dump_level:    level_nx*level_ny records of 4 int32 {dx, dy, dist, flags} of field
 *                     `dir` (0 forward, 1 backward) after the level's last update.
 *  pgm_dump_gradient: level_w*level_h*2C values of image `image` at `level`, int16 (integer
 *                     features) or float, channel order [Gx_0..Gx_C-1, Gy_0..Gy_C-1]; images
 *                     0 and 1 in the forward pyramid's colour space, 2 and 3 (images 1 and 2)
 *                     in the backward one's.
 *  pgm_dump_pyramid:  level_w*level_h*3 uint8 of image `image` at `level`. */
PGM_API pgm_status pgm_dump_level(void* ctx, int32_t level, int32_t dir, int32_t* host_out);
PGM_API pgm_status pgm_dump_gradient(void* ctx, int32_t level, int32_t image, void* host_out);
PGM_API pgm_status pgm_dump_pyramid(void* ctx, int32_t level, int32_t image, uint8_t* host_out);

/* Per-kernel timing for measurement. While enabled, pgm_match records HIP events on the
 * caller's stream around every run of consecutive launches of one kernel kind (no event
 * between the kernels of a run; its time includes the gaps between them) and counts the
 * distance evaluations of each kernel kind. pgm_profile(ctx, 1) enables and clears the totals, pgm_profile(ctx, 0)
 * disables. pgm_profile_read waits for the last call's stream and returns, for one kind,
 * the number of launches, their summed duration in milliseconds and their summed distance
 * evaluations since the last clear. Kinds (PGM_K_PREP: the first launch of a call, which
 * draws the random numbers and builds the level-0 gradients and pyramid level 1;
 * PGM_K_PYRAMID: pyramid levels 2 and up; PGM_K_GRADIENT: gradients of levels 1 and up;
 * PGM_K_LEVEL: all sweeps of a level small enough for one work-group's LDS, whose distance
 * evaluations count under PGM_K_SWEEP; PGM_K_OUTPUT: the
 * matches of both directions and the compaction, so nothing is recorded under PGM_K_COMPACT;
 * PGM_K_REGION: small-region removal; PGM_K_SWEEP_MULTI: two to four half-sweeps of a small
 * level in one launch, PGM_K_SWEEP_PAIR: two half-sweeps of a somewhat larger level in one
 * launch, whose evaluations count under each): */
enum { PGM_K_PYRAMID = 0, PGM_K_GRADIENT = 1, PGM_K_PREP = 2, PGM_K_INIT = 3, PGM_K_DOWN = 4,
       PGM_K_UP = 5, PGM_K_SWEEP = 6, PGM_K_CHECK = 7, PGM_K_OUTPUT = 8, PGM_K_COMPACT = 9,
       PGM_K_LEVEL = 10, PGM_K_REGION = 11, PGM_K_SWEEP_MULTI = 12, PGM_K_SWEEP_PAIR = 13,
       PGM_K_KINDS = 14 };
PGM_API pgm_status pgm_profile(void* ctx, int32_t enable);
PGM_API pgm_status pgm_profile_read(void* ctx, int32_t kind, int64_t* host_launches,
                                    double* host_total_ms, uint64_t* host_evals);

/* Launch schedule of later calls on ctx. The library picks, per level, among schedules that
 * give identical results: a small level's half-sweeps in one work-group per pair and direction
 * from LDS or as separate launches, and a level's entry (the coarser level's check, the
 * transition, the first half-sweep) in one launch or in several. flags 0 (the default) lets it
 * choose by size and concurrency; the bits force a choice wherever it applies, for tests of
 * schedule invariance and for measurements. PGM_EINVAL for unknown bits or a contradiction. */
enum { PGM_SCHED_AUTO = 0,
       PGM_SCHED_LEVEL_LDS = 1,      /* small levels in one work-group from LDS wherever they fit */
       PGM_SCHED_LEVEL_LAUNCHES = 2, /* small levels as half-sweep launches                       */
       PGM_SCHED_SEPARATE = 4 };     /* every check, transition and half-sweep its own launch     */
PGM_API pgm_status pgm_schedule(void* ctx, int32_t flags);

/* Autotune the launch schedule for one workload: runs pgm_match_batch on the given pairs and
 * outputs (same layout and rules as pgm_match_batch; the outputs hold the matches afterwards)
 * once untimed and `repeats` times timed (1..1000) under each schedule pgm_schedule can force
 * (AUTO, LEVEL_LDS, LEVEL_LAUNCHES, SEPARATE and the two combinations with SEPARATE), keeps the
 * fastest for later calls on ctx and writes its flags to *host_flags (host, may be NULL).
 * Synchronous: waits for `stream`. Every schedule gives the same results, so tuning changes
 * only speed. PGM_EINVAL while profiling is on. */
PGM_API pgm_status pgm_tune(void* ctx, const pgm_params* p, int32_t n_pairs, const uint8_t* img1,
                            const uint8_t* img2, int32_t w, int32_t h, int32_t pitch_bytes,
                            int64_t image_stride_bytes, pgm_match_t* out_fwd, pgm_match_t* out_bwd,
                            int32_t* out_n_inliers, pgm_match_t* out_compact, int32_t repeats, void* stream,
                            int32_t* host_flags);

/* Text of the last error of ctx (or of the last failed pgm_create when ctx is NULL). */
PGM_API const char* pgm_last_error(void* ctx);

/* Free the workspace and the context. Waits for the context's work to finish. */
PGM_API void pgm_destroy(void* ctx);

#ifdef __cplusplus
}
#endif
#endif /* PGM_H */
