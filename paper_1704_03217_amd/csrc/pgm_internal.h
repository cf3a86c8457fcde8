// Internal declarations shared by the kernels and the C ABI of libpgm (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/pgm.h"

namespace pgm {

// Every gradient image is stored with a replicated border of PAD pixels on each side, so a
// patch read of side <= 16 around any in-image pixel needs no clamping (the patch distance
// takes the nearest edge pixel outside the image).
constexpr int PAD = 8;
// Packed displacement (dx in the low, dy in the high 16 bits); this value marks an
// uninitialised seed (|d| never reaches 32768 since images are at most 16384 wide).
constexpr uint32_t UNINIT = 0x80008000u;
constexpr uint64_t NO_DIST = 0x7FFFFFFFull;
// Integer gradients are stored biased to unsigned 16 bit (g + 32768) for v_sad_u16.
constexpr uint32_t BIAS = 32768u;
// Per-seed state flags in the workspace.
constexpr uint8_t ST_REC = 1;   // record propagated into this visit says "inlier"
constexpr uint8_t ST_INL = 2;   // outlier record after the level's update says "inlier"

constexpr int MAX_STAGES = 1 + 2 * 16 + PGM_MAX_LEVELS;

// Caller buffers of one pair of a batch whose pairs each bring their own images and outputs
// (the request server's shared launches). The table lives in the batch's workspace; a kernel
// that reads or writes caller memory takes pair z's pointers from entry z when the table is
// set, and the uniform pair strides otherwise.
struct PairTab {
    const uint8_t* img[2];
    pgm_match_t* out[2];                 // forward, backward (null when not wanted)
    pgm_match_t* compact;
    int32_t* n_in;
    unsigned long long* n_evals;         // the pair's evaluation count is added here (or null)
    const void* unused;
};
constexpr int TAB_MAX = 16;              // pairs of a table-driven batch

// One correspondence field (one direction at one level) in device memory.
struct Field {
    uint32_t* disp;   // packed (dx, dy) or UNINIT
    void* dist;       // patch distance: uint32 (absolute-difference sum, or float bits, as
                      // non-negative floats order as unsigned integers) or uint64 (squared sum)
    uint8_t* flags;   // ST_*
};

// Arguments for one direction of a matching kernel.
struct DirArgs {
    const void* Ga;        // padded gradient of this field's image, at pixel (0, 0)
    const void* Gb;        // padded gradient of the other image, at pixel (0, 0)
    Field f;
    const short2* rnd;     // random-search offsets of this stage and direction: [t][seed][nI]
    const short2* rnd0;    // initial displacements (initial stage only): [seed]
    int P;                 // patch side
};

// floor(n / d) for every 32-bit n by multiplication: M = ceil(2^64 / d) for d >= 2, whose
// excess e = M d - 2^64 < d adds n e / (d 2^64) < 1 / d to n / d, too little to reach the next
// integer, so floor(n M / 2^64) is the quotient; d == 1 passes n through. Set up on the host.
struct DivM {
    uint32_t d, lo, hi;    // the divisor and the low and high words of M
};
inline DivM div_magic(uint32_t d)
{
    DivM m{d, 0u, 0u};
    if (d >= 2) {
        const uint64_t M = ~0ull / d + 1;   // ceil(2^64 / d)
        m.lo = (uint32_t)M;
        m.hi = (uint32_t)(M >> 32);
    }
    return m;
}
// floor(n / m.d): n M / 2^64 as n hi + the high word of n lo, two multiplications
__host__ __device__ inline uint32_t fdiv(uint32_t n, const DivM& m)
{
    const uint64_t p = (uint64_t)n * m.hi + (uint32_t)(((uint64_t)n * m.lo) >> 32);
    return m.d == 1 ? n : (uint32_t)(p >> 32);
}

struct Geo {
    int w, h;              // level image size
    int pw;                // padded row length in pixels (w + 2 PAD)
    int nx, ny;            // seed grid
    int stride, off;       // grid spacing and first seed position
    DivM dnx, dhx, d2s;    // division by nx, by (nx + 1) / 2 and by 2 stride (geo_divs)
};
inline void geo_divs(Geo& g)
{
    g.dnx = div_magic((uint32_t)g.nx);
    g.dhx = div_magic((uint32_t)(g.nx + 1) / 2);
    g.d2s = div_magic((uint32_t)(2 * g.stride));
}

// Pairs of one batch: every per-pair workspace pointer of the kernel arguments points into
// pair 0's slice; pair z's is `zs` bytes further (the random-number table is shared).
struct Batch {
    int npairs;
    int ndir;              // directions covered by the launch (1 or 2)
    long long zs;          // workspace bytes per pair
    DivM dnb;              // division by the work-groups per direction and pair (set by the launcher)
    int inter;             // both directions read the same two images (set by the launcher)
};

struct SweepArgs {
    DirArgs d[2];
    Geo g;
    Batch b;
    int t, colour, nI;
    uint32_t* cnt;         // per-block evaluation counts of this launch, pair 0 (or null)
};

// Two to four consecutive half-sweeps of one level in one launch, the field read from one
// buffer (d[].f) and written whole to another (out[]): half-sweep m updates the seeds of colour
// c[m] at iteration t[m] (the colours alternate).
struct SweepMultiArgs {
    DirArgs d[2];
    Field out[2];          // disp and dist of the output buffer of each direction, pair 0
    Geo g;
    Batch b;
    int nph, t[4], c[4], nI;
    uint32_t* cnt;         // per-block evaluation counts of this launch, pair 0 (or null)
    // set by the launcher: division by the tiles per seed row, and per half-sweep the
    // rectangle it updates relative to the tile (see k_sweep_multi)
    DivM dtx;
    uint32_t ph[4];
};

struct InitArgs {
    DirArgs d[2];
    Geo g;
    Batch b;
    int exhaustive, R;
    uint32_t* cnt;
};

struct TransArgs {         // level-down (to the finer level) or level-up (to the coarser)
    DirArgs d[2];          // the level being entered
    Field src[2];          // the level the field comes from
    Geo g, gs;             // geometry of the entered level and of the source level
    Batch b;
    int carry_record;
    uint32_t* cnt;
};

// Entering a finer level in one launch: the coarser level's check (Steps 2-3), the
// transition (Steps 4-5) and the first half-sweep of Step 1 at the finer level.
struct EnterArgs {
    DirArgs d[2];          // the finer level being entered (both directions), pair 0
    Field src[2];          // the coarser level (both directions), pair 0
    Geo g, gs;             // geometry of the finer and of the coarser level
    Batch b;
    int carry_record;      // a child's record takes its parent's inlier flag (Eq. 8)
    int fwd_bwd, tau2, rec_valid;   // the coarser level's check
    int nI;                // random-search candidates of the half-sweep
    int nb_col, nb_chk;    // work-groups per direction and pair: per colour, for the check
    uint32_t* cnt;         // per-block evaluation counts, pair 0 (or null)
};

struct CheckArgs {
    Field f[2];
    Geo g;
    Batch b;
    int fwd_bwd, tau2, rec_valid;
};

// LDS layout of a whole-level sweep launch (byte offsets; gstride: bytes per gradient image;
// rnd: the level's random-search offsets of one direction)
struct LevelLayout {
    size_t gstride, disp, dist, rnd, total;
};
struct LevelArgs {
    DirArgs d[2];          // both directions, pair 0 (in HBM)
    Geo g;
    Batch b;
    int iters, nI;
    uint32_t* cnt;         // two sweep-count slots (one per direction) per pair, pair 0 (or null)
    size_t gbytes;         // bytes of one padded gradient image (a multiple of 16)
    size_t gorig;          // byte offset of pixel (0, 0) inside it
    LevelLayout lay;
};

struct OutArgs {
    Field f[2];            // level-0 fields (forward, backward), pair 0
    pgm_match_t* out[2];   // pair z writes out[d] + z * nx * ny (out[1] used when ndir == 2)
    Geo g;
    Batch b;               // b.ndir: 1 = forward only, 2 = both
    // compaction of the forward inliers (both null: none)
    pgm_match_t* compact;  // pair z writes compact + z * nx * ny (or null)
    int32_t* n_out;        // pair z writes n_out[z] (or null)
    const PairTab* tab;    // outputs per pair instead of the strides above (or null)
    int dist8;             // the field's distances are uint64
};

struct RngStage {
    int n, iters, nI, W, level, stage;
    long long base;        // first short2 of the stage in the table
    int bpt, b0;           // work-groups per (direction, iteration) and the stage's first one
};

struct RngArgs {
    RngStage st[MAX_STAGES];
    int nstages;
    short2* table;
    short2* init;          // 2 * n_top initial displacements
    int n_top, R_top, top_level;
    int rs_sym;            // PGM_RS_SYMMETRIC: search offsets uniform in [-(W >> i), W >> i]
    uint32_t key0, key1;
    int init_blocks;       // work-groups of the initial displacements (filled in by the launcher)
};

struct CountArgs {
    static constexpr int KINDS = 6;      // init, down, up, sweep, multi-sweep and paired-sweep launches
    const uint32_t* table[KINDS];        // pair 0
    long long n[KINDS];
    int npairs;
    long long zs;
    int kind[KINDS];                     // PGM_K_* of each table
    unsigned long long* user;            // caller's counter (or null)
    unsigned long long* prof;            // PGM_K_KINDS profiling counters (or null)
    const PairTab* tab;                  // per-pair counters instead of user (or null)
};


// Threads per work-group of the matching kernels (k_sweep, k_init, k_down, k_up and the
// k_enter family): one wave. A launch's waves then spread over as many CUs and L1 caches as
// there are waves, up to the whole chip. Four-wave work-groups left most CUs idle on the
// small levels, whose launches wait on their seeds' dependent memory round trips, and were
// slower at every size measured (plain 1024x436 pass 8% slower).
constexpr int MATCH_TPB = 64;

// Work-groups of a matching kernel: one seed per 8 lanes (patch side <= 8) or per 16 lanes
// (side <= 16).
inline int match_blocks(int groups, int P)
{
    const int gpb = MATCH_TPB / (P <= 8 ? 8 : 16);
    return (groups + gpb - 1) / gpb;
}

// Work-groups of one half-sweep launch per direction and pair.
inline int sweep_blocks(int nx, int ny, int P) { return match_blocks(ny * ((nx + 1) / 2), P); }

// Tiles of seeds of a launch of several half-sweeps (four-wave work-groups of 32 seed groups,
// patch sides <= 8): 4 x 6 seeds, so that the rectangle of the first of up to four half-sweeps
// (7 x 9 seeds) holds at most 32 seeds of its colour.
constexpr int MULTI_TPB = 256;
inline int sweep_multi_blocks(int nx, int ny) { return ((nx + 3) / 4) * ((ny + 5) / 6); }
// two half-sweeps per launch on 6 x 8-seed tiles (half as many work-groups)
inline int sweep_pair_blocks(int nx, int ny) { return ((nx + 5) / 6) * ((ny + 7) / 8); }

// Launch wrappers (pgm_kernels.hip). Each returns hipSuccess or the launch error.
// Per-image pointers are those of pair 0; pair z's source is src_zs bytes further and its
// destination dst_zs bytes further.
// one pyramid level (tx, tiles filled in by the launchers)
struct PyrArgs {
    const uint8_t* src[2];   // pair 0's source images (the finer level)
    long long src_zs;        // bytes between pairs' source images
    int pitch, w, h;         // source pitch (bytes) and size
    uint8_t* dst[2];         // pair 0's destination images (packed rows of (w + 1) / 2 pixels)
    long long dst_zs;        // bytes between pairs' destination images (both levels)
    int two;                 // also the level after it, from the same pass
    uint8_t* dst2[2];        // pair 0's images of that level (two)
    const PairTab* tab;      // source images per pair (or null: src + pair * src_zs)
    int tx, tiles;
};
// gradient images of one or more levels (tx, tiles and base filled in by the launchers)
struct GradLevel {
    const uint8_t* src[2];   // pair 0's source images
    long long src_zs;        // bytes between pairs' source images
    int pitch, w, h;
    void* G[2];              // pair 0's padded gradient images
    const PairTab* tab;      // source images per pair (or null: src + pair * src_zs)
    int space;               // PGM_SPACE_* the pixels are converted into first
    int tx, tiles, base;
};
struct GradArgs {
    GradLevel lv[2 * PGM_MAX_LEVELS];
    int n;
    long long dst_zs;
};
// the first launch of a call: random numbers, level-0 gradients and (with_pyr) pyramid level 1
struct PrepArgs {
    RngArgs rng;
    GradArgs grad;           // level 0 (one entry per colour space)
    PyrArgs pyr;
    int with_pyr;
    int rng_blocks, grad_blocks, grad_tiles, pyr_blocks;   // filled in by the launcher
};
// feat: PGM_FEAT_* (0 integer gradients, 1 direction-only float, 2 literal signs)
hipError_t launch_prep(PrepArgs a, int npairs, int gray, int ksize, int feat, hipStream_t s);
hipError_t launch_pyr(PyrArgs a, int npairs, hipStream_t s);
hipError_t launch_gradient(GradArgs a, int npairs, int gray, int ksize, int feat, hipStream_t s);
hipError_t launch_init(InitArgs a, int C2, int kind, hipStream_t s);
hipError_t launch_sweep(SweepArgs a, int C2, int kind, hipStream_t s);
hipError_t launch_sweep_multi(SweepMultiArgs a, int C2, int kind, hipStream_t s);
hipError_t launch_sweep_pair(SweepMultiArgs a, int C2, int kind, hipStream_t s);   // nph == 2
hipError_t launch_down(TransArgs a, int C2, int kind, hipStream_t s);
hipError_t launch_up(TransArgs a, int C2, int kind, hipStream_t s);
hipError_t launch_check(const CheckArgs& a, hipStream_t s);
// ENTER_LAUNCH_START: the check and the transition (k_enter_start); ENTER_LAUNCH_SWEEP: and the
// first half-sweep (k_enter); ENTER_LAUNCH_INIT: the initial level's random starts and its
// first half-sweep (k_enter_init; no coarser level)
enum { ENTER_LAUNCH_START = 0, ENTER_LAUNCH_SWEEP = 1, ENTER_LAUNCH_INIT = 2 };
hipError_t launch_enter(EnterArgs a, int C2, int kind, int mode, hipStream_t s);
// work-groups of one k_enter launch per direction and pair
inline int enter_blocks(int nx, int ny, int P, int n_coarse)
{
    return 2 * sweep_blocks(nx, ny, P) + (n_coarse + MATCH_TPB - 1) / MATCH_TPB;
}
// small-region removal on the level-0 forward field: four launches (labels, unions, region
// sizes, flags)
struct RegionArgs {
    Field f;               // level-0 forward field, pair 0
    Geo g;
    Batch b;
    int32_t* label;        // nx*ny per pair, pair 0
    int32_t* size;         // nx*ny per pair, pair 0
    int min_px;
    long long link2;       // region_link_px^2
};
hipError_t launch_regions(const RegionArgs& a, hipStream_t s);
// every sweep of a small level, one work-group per pair and direction
hipError_t launch_level(const LevelArgs& a, int C2, int kind, hipStream_t s);
// let every whole-level kernel use up to `bytes` of dynamic LDS (once per context)
hipError_t level_allow_lds(size_t bytes);
hipError_t launch_output(const OutArgs& a, hipStream_t s);
// part: pair 0's array of COUNT_SLICES * CountArgs::KINDS partial sums; pair z's array is at
// the same offset of its own workspace slice (z * zs bytes further)
constexpr int COUNT_SLICES = 16;
hipError_t launch_count(const CountArgs& a, unsigned long long* part, hipStream_t s);
// writes the n <= TAB_MAX entries of host into the device table dst (through the kernel's
// arguments: nothing on the host side has to outlive the call)
hipError_t launch_fill_tab(PairTab* dst, const PairTab* host, int n, hipStream_t s);

}  // namespace pgm
