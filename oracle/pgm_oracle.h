/*
 * pgm_oracle.h -- CPU oracle for pyramidal gradient matching
 * (Y. Li, "Pyramidal Gradient Matching for Optical Flow Estimation", arXiv:1704.03217).
 *
 * TEST INFRASTRUCTURE. This is a plain, slow, single-threaded reference used only to check
 * the GPU library: by the test-suite, by the smoke check and by the benchmark's CPU-baseline
 * leg. The GPU library never includes, links or calls it, and it shares no code with it.
 *
 * Everything here is host memory. All images are HWC uint8 (3 channels, RGB) with a row pitch
 * in bytes. Gradient images are int16 (full gradient) or float (direction-only variant), with
 * 2*C channels per pixel in the order [Gx_0..Gx_{C-1}, Gy_0..Gy_{C-1}] (Sec. III-A, Eq. 2).
 *
 * Parity status: the gradient image, pyramid, patch distance, Philox generator, random-search
 * offsets, exhaustive initialisation, propagation/search on small cases, the consistency check,
 * the level transitions and the small-region removal are pinned by independent tests. The scan-order schedule
 * (PGMO_SCAN), for which the paper prints no worked example, is pinned by invariants and by a hand-worked pass
 * (a one-pixel translation whose optimum one seed finds by its random search and every later seed takes
 * from an updated neighbour, with the evaluation count derived from the draws).
 */
#ifndef PGM_ORACLE_H
#define PGM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PGMO_MAX_LEVELS 8

enum { PGMO_FEAT_INT16 = 0, PGMO_FEAT_F32_DIR = 1, PGMO_FEAT_SIGN = 2 };
enum { PGMO_RGB = 0, PGMO_GRAY = 1 };
enum { PGMO_SPACE_RGB = 0, PGMO_SPACE_YCRCB = 1, PGMO_SPACE_LAB = 2 };
enum { PGMO_METRIC_SAD = 0, PGMO_METRIC_SSD = 1 };
enum { PGMO_INIT_RANDOM = 0, PGMO_INIT_EXHAUSTIVE = 1 };
enum { PGMO_SYNC = 0, PGMO_SCAN = 1 };
enum { PGMO_RS_FLOOR = 0, PGMO_RS_SYMMETRIC = 1 };

/* per-seed flags reported by the oracle */
#define PGMO_F_INIT   1u   /* the correspondence field is initialised at this seed      */
#define PGMO_F_INLIER 2u   /* outlier record says "no" after the level's update (Eq. 7) */
#define PGMO_F_RECORD 4u   /* record propagated into the level says "no" (Eq. 8)        */

typedef struct {
    int32_t levels;                    /* L, pyramid levels (Sec. III-D)                     */
    int32_t seed_stride;               /* spacing of the seed grid in pixels (Sec. III-G)    */
    int32_t patch_fwd, patch_bwd;      /* patch side for the forward / backward field        */
    int32_t iters[PGMO_MAX_LEVELS];    /* propagation-search iterations per level, 0 = full  */
    int32_t radius;                    /* W of Eq. 5 below the initial level                 */
    int32_t max_disp;                  /* bound on |d| at full resolution, 0 = image size;   */
                                       /* negative -k: ceil(w / k) for a w-wide image        */
    int32_t sobel_ksize;               /* S of Eq. 1: 3 or 5                                 */
    int32_t feature;                   /* PGMO_FEAT_*                                        */
    int32_t color;                     /* PGMO_RGB (C = 3) or PGMO_GRAY (C = 1)              */
    int32_t fwd_bwd;                   /* forward-backward consistency check on/off          */
    int32_t consistency_px;            /* tau: consistent iff |d_f + d_b|^2 <= tau^2         */
    int32_t init_mode;                 /* PGMO_INIT_*                                        */
    int32_t refine_rounds;             /* N of Sec. III-D (refinement between m and m-1)     */
    int32_t min_region_px;             /* small-region removal (Sec. III-E): 0 = off         */
    int32_t region_link_px;            /* neighbours link when |d_a - d_b| < this            */
    int32_t space_fwd[PGMO_MAX_LEVELS]; /* colour space of the forward / backward gradient   */
    int32_t space_bwd[PGMO_MAX_LEVELS]; /* pyramid per level (Table II), PGMO_SPACE_*        */
    int32_t metric;                    /* PGMO_METRIC_*: Eq. 3 summed absolutely or squared */
    int32_t rs_mode;                   /* PGMO_RS_*: offsets of the limited random search    */
    uint64_t rng_seed;                 /* key of the counter-based generator                 */
} pgmo_params;

typedef struct { int32_t x1, y1, x2, y2, dist; uint32_t flags; } pgmo_match_t;

/* ---- building blocks (exported so that tests can pin each one) ---- */

/* reflect-101 border index */
int pgmo_reflect101(int i, int n);
/* one pyramid step: 5x5 binomial, decimation by 2; dst is ceil(w/2) x ceil(h/2), packed */
void pgmo_pyr_down(const uint8_t* src, int w, int h, int pitch, int ch, uint8_t* dst);
/* colour conversion of npx packed RGB pixels into PGMO_SPACE_* (3 uint8 channels) */
void pgmo_convert(const uint8_t* rgb, int npx, int space, uint8_t* out);
/* integer luma Y = (77 R + 150 G + 29 B + 128) >> 8, packed w x h */
void pgmo_gray(const uint8_t* rgb, int w, int h, int pitch, uint8_t* y);
/* gradient image of Eq. 1-2: G is w*h*2*ch int16 */
void pgmo_gradient_image(const uint8_t* img, int w, int h, int pitch, int ch, int ksize, int16_t* G);
/* direction-only gradient image (Sec. III-F): per channel (Gx,Gy)/|(Gx,Gy)|, 0 -> (0,0) */
void pgmo_direction(const int16_t* G, int npix, int ch, float* U);
/* literal reading of "G./|G|" (Sec. III-F): every element divided by its own absolute
 * value, i.e. its sign in {-1, 0, 1} (0 stays 0); in place on npix*C2 values */
void pgmo_sign(int16_t* G, int n);
/* patch distance (Eq. 3, absolute-difference reading) between the patch of Ga at (xa,ya)
 * and the patch of Gb at (xb,yb); C2 = channels per pixel (2*ch); P = patch side */
int64_t pgmo_dist_i16(const int16_t* Ga, const int16_t* Gb, int w, int h, int C2, int P,
                      int xa, int ya, int xb, int yb);
float pgmo_dist_f32(const float* Ua, const float* Ub, int w, int h, int C2, int P,
                    int xa, int ya, int xb, int yb);
/* Eq. 3 as printed: sum of squared differences of integer features, exact in 64 bits */
int64_t pgmo_ssd_i16(const int16_t* Ga, const int16_t* Gb, int w, int h, int C2, int P,
                     int xa, int ya, int xb, int yb);
/* Philox4x32 with 10 rounds (Salmon et al., SC'11) */
void pgmo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* offset floor(R W / 2^i) of Eq. 5 for R = (2u+1)/2^32 - 1 */
int pgmo_search_offset(uint32_t u, int W, int i);
/* offset of Eq. 5 read as a uniform integer in [-w_i, w_i], w_i = floor(W / 2^i):
 * floor(u (2 w_i + 1) / 2^32) - w_i (PGMO_RS_SYMMETRIC) */
int pgmo_search_offset_sym(uint32_t u, int W, int i);
/* uniform integer in [-R, R] from a 32-bit draw: floor(u (2R+1) / 2^32) - R */
int pgmo_init_offset(uint32_t u, int R);
/* seeds along an axis of n pixels */
int pgmo_grid_count(int n, int stride);
int pgmo_grid_pos(int i, int n, int stride);
int pgmo_grid_nearest(int x, int nseeds, int stride);
/* level geometry: sizes and seed counts of every level; returns 0 or -1 on bad input */
int pgmo_geometry(const pgmo_params* p, int w, int h, int32_t* lw, int32_t* lh, int32_t* lnx, int32_t* lny);
/* search radius of the initial (coarsest) level */
int pgmo_top_radius(const pgmo_params* p, int w, int h);

/* Small-region removal (Sec. III-E) on one grid field: inlier seeds are segmented into
 * regions -- two 4-neighbouring inliers belong together when their displacements differ by
 * less than link_px (Euclidean) -- and the inliers of every region whose area (seeds x
 * stride^2 pixels) is below min_px become outliers. inl (0/1) is updated in place. */
/* Test entry: the lift toward the coarser level (Sec. III-D, Eq. 6 with k = j+1) of a given
 * finer field (fw x fh grid, spacing stride) onto a cw x ch grid; 0, or -1 for bad sizes. */
int pgmo_lift(int fw, int fh, int cw, int ch, int stride, const int32_t* fdx, const int32_t* fdy,
              const uint8_t* finl, int32_t* cdx, int32_t* cdy, uint8_t* cinit);
void pgmo_remove_small_regions(const int32_t* dx, const int32_t* dy, uint8_t* inl, int nx, int ny,
                               int stride, int min_px, int link_px);

/* Step 1 alone (propagation + limited random search, Eq. 4-5) on one field, for tests:
 * iterations t0 .. t0+n_iter-1 with search radius W. Ga / Gb are the features of this and
 * the other image (int16 or float, w*h*2C). State in/out: dx, dy, dist (int32 or float bits),
 * init (0/1), nx*ny seeds each. Returns 0 or -1. */
int pgmo_sweep(const pgmo_params* p, int level, int dir, int stage, int W, const void* Ga,
               const void* Gb, int w, int h, int t0, int n_iter, int schedule, int32_t* dx,
               int32_t* dy, int32_t* dist, uint8_t* init, uint64_t* n_evals);

/* ---- the whole method ----
 * out_fwd / out_bwd: nx*ny matches of level 0 (nullable);
 * out_compact: forward inliers in row-major seed order (nullable), count in *n_inliers;
 * trace (nullable): for dir 0 then 1, for level 0..L-1, n_l seeds x {dx, dy, dist, flags}
 *   int32, the state after that level's last consistency update;
 * n_evals (nullable): number of patch-distance evaluations.
 * A match's dist is the patch distance, the bits of a float for the float features, and for
 * the squared metric the 64-bit sum clamped to 0x7FFFFFFE (the decisions use the exact sum).
 * Returns 0, or -1 on invalid parameters. */
int pgmo_match(const pgmo_params* p, const uint8_t* img1, const uint8_t* img2, int w, int h,
               int pitch, int schedule, pgmo_match_t* out_fwd, pgmo_match_t* out_bwd,
               int32_t* n_inliers, pgmo_match_t* out_compact, int32_t* trace, uint64_t* n_evals);

#ifdef __cplusplus
}
#endif
#endif
