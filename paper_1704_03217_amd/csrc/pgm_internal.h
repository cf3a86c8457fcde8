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
constexpr uint32_t NO_DIST = 0x7FFFFFFFu;
// Integer gradients are stored biased to unsigned 16 bit (g + 32768) for v_sad_u16.
constexpr uint32_t BIAS = 32768u;
// Per-seed state flags in the workspace.
constexpr uint8_t ST_REC = 1;   // record propagated into this visit says "inlier"
constexpr uint8_t ST_INL = 2;   // outlier record after the level's update says "inlier"

constexpr int MAX_STAGES = 1 + 2 * 16 + PGM_MAX_LEVELS;

// One correspondence field (one direction at one level) in device memory.
struct Field {
    uint32_t* disp;   // packed (dx, dy) or UNINIT
    uint32_t* dist;   // int32 distance, or float bits (non-negative floats order as uints)
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

struct Geo {
    int w, h;              // level image size
    int pw;                // padded row length in pixels (w + 2 PAD)
    int nx, ny;            // seed grid
    int stride, off;       // grid spacing and first seed position
};

struct SweepArgs {
    DirArgs d[2];
    Geo g;
    int t, colour, nI;
    unsigned long long* n_evals;     // caller's counter (or null)
    unsigned long long* n_evals2;    // per-kind profiling counter (or null)
};

struct InitArgs {
    DirArgs d[2];
    Geo g;
    int exhaustive, R;
    unsigned long long* n_evals;
    unsigned long long* n_evals2;
};

struct TransArgs {         // level-down (to the finer level) or level-up (to the coarser)
    DirArgs d[2];          // the level being entered
    Field src[2];          // the level the field comes from
    Geo g, gs;             // geometry of the entered level and of the source level
    int carry_record;
    unsigned long long* n_evals;
    unsigned long long* n_evals2;
};

struct CheckArgs {
    Field f[2];
    Geo g;
    int fwd_bwd, tau2, rec_valid;
};

struct RngStage {
    int n, iters, nI, W, level, stage;
    long long base;        // first short2 of the stage in the table
};

struct RngArgs {
    RngStage st[MAX_STAGES];
    int nstages;
    long long total_items; // sum over stages of 2 * n * iters * ceil(nI / 2)
    short2* table;
    short2* init;          // 2 * n_top initial displacements
    int n_top, R_top, top_level;
    uint32_t key0, key1;
};

// Launch wrappers (pgm_kernels.hip). Each returns hipSuccess or the launch error.
hipError_t launch_pyr_down(const uint8_t* src0, const uint8_t* src1, int pitch, int w, int h,
                           uint8_t* dst0, uint8_t* dst1, hipStream_t s);
hipError_t launch_gradient(const uint8_t* img0, const uint8_t* img1, int pitch, int w, int h,
                           void* G0, void* G1, int gray, int ksize, int f32, hipStream_t s);
hipError_t launch_rng(const RngArgs& a, hipStream_t s);
hipError_t launch_init(const InitArgs& a, int C2, int f32, int ndir, hipStream_t s);
hipError_t launch_sweep(const SweepArgs& a, int C2, int f32, int ndir, hipStream_t s);
hipError_t launch_down(const TransArgs& a, int C2, int f32, int ndir, hipStream_t s);
hipError_t launch_up(const TransArgs& a, int C2, int f32, int ndir, hipStream_t s);
hipError_t launch_check(const CheckArgs& a, hipStream_t s);
hipError_t launch_output(const Field& f, const Geo& g, pgm_match_t* out, hipStream_t s);
hipError_t launch_compact(const pgm_match_t* dense, int n, pgm_match_t* out, int32_t* n_out,
                          hipStream_t s);

}  // namespace pgm
