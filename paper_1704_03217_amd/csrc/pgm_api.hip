// C ABI of libpgm (declared in include/pgm.h): parameter validation, workspace layout, the
// level schedule of Sec. III-D and the kernel launches of one pair.
#include <stdarg.h>
#include <stddef.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <chrono>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "pgm_internal.h"

using namespace pgm;

namespace {

struct Layout {
    int L = 0, ch = 3, C2 = 6, esize = 2, f32 = 0;
    int kind = 0, dsize = 4;   // matching kernel family; bytes per stored distance
    int lw[PGM_MAX_LEVELS], lh[PGM_MAX_LEVELS], lnx[PGM_MAX_LEVELS], lny[PGM_MAX_LEVELS];
    size_t pyr[2][PGM_MAX_LEVELS];                       // level >= 1 RGB images
    size_t grad[4][PGM_MAX_LEVELS];                      // padded gradient images (4 slots)
    size_t disp[2][PGM_MAX_LEVELS], dist[2][PGM_MAX_LEVELS], flags[2][PGM_MAX_LEVELS];
    size_t disp2[2][PGM_MAX_LEVELS], dist2[2][PGM_MAX_LEVELS];   // second field buffer (k_sweep_multi)
    size_t rnd = 0, rnd_init = 0;
    size_t tab = 0;                                      // PairTab entries of a table-driven batch
    // stages of the schedule
    int nst = 0;
    int st_level[MAX_STAGES], st_enter[MAX_STAGES], st_W[MAX_STAGES], st_nI[MAX_STAGES];
    long long st_base[MAX_STAGES];                       // short2 offset of the stage's offsets
    int R_top = 0;
    // per-block evaluation counts of the matching launches, one table per kernel kind
    // (init, down, up, sweep, multi-sweep launches, paired-sweep launches)
    size_t cnt[6] = {0, 0, 0, 0, 0, 0};
    long long cnt_cap[6] = {0, 0, 0, 0, 0, 0};
    size_t cntpart = 0;
    size_t cclabel = 0, ccsize = 0;
    // the random-number table is shared by all pairs of a batch; everything else is per pair
    // (offsets above are relative to the pair's slice, except rnd / rnd_init)
    size_t shared_bytes = 0, pair_bytes = 0;
    size_t total = 0;   // shared + one pair
};

enum { CNT_INIT = 0, CNT_DOWN = 1, CNT_UP = 2, CNT_SWEEP = 3, CNT_MULTI = 4, CNT_PAIR = 5 };

// both directions share a launch when their patch sides select the same kernel variant
int variant(int P) { return P == 8 ? 0 : P < 8 ? 1 : P == 16 ? 2 : 3; }

// work-groups launched for `groups` seeds in both directions
long long dir_blocks(const pgm_params* p, int groups)
{
    if (variant(p->patch_fwd) == variant(p->patch_bwd)) return 2LL * match_blocks(groups, p->patch_fwd);
    return (long long)match_blocks(groups, p->patch_fwd) + match_blocks(groups, p->patch_bwd);
}

enum { ENTER_INIT = 0, ENTER_DOWN_F = 1, ENTER_DOWN_FO = 2, ENTER_UP_FO = 3 };
// largest level (seeds x pairs) entered by one fused launch
constexpr long long FUSE_MAX_SEEDS = 8192;
// largest level (seeds x pairs) whose half-sweeps run up to four per launch (4 x 6-seed
// tiles), and up to two (6 x 8-seed tiles: half as many work-groups, one round of the chip
// where 4 x 6 tiles would take two)
constexpr long long MULTI_MAX_SEEDS = 8192, PAIR_MAX_SEEDS = 16384;

size_t take(size_t& cur, size_t bytes)
{
    size_t at = (cur + 255) & ~(size_t)255;
    cur = at + bytes;
    return at;
}

int grid_count(int n, int stride)
{
    int off = stride / 2;
    return n - 1 < off ? 1 : (n - 1 - off) / stride + 1;
}

int n_offsets(int W)   // floor(log2 W) + 1 candidates of Eq. 5
{
    int n = 1;
    while ((2 << (n - 1)) <= W) n++;
    return n;
}

const char* validate(const pgm_params* p, int w, int h)
{
    if (!p) return "null parameters";
    if (w < 1 || h < 1 || w > 16384 || h > 16384) return "image size must be within 1..16384";
    if (p->levels < 1 || p->levels > PGM_MAX_LEVELS) return "levels must be within 1..8";
    if (p->seed_stride < 1 || p->seed_stride > 64) return "seed_stride must be within 1..64";
    if (p->patch_fwd < 1 || p->patch_fwd > 16 || p->patch_bwd < 1 || p->patch_bwd > 16)
        return "patch sides must be within 1..16";
    for (int l = 0; l < p->levels; l++)
        if (p->iters[l] < 0 || p->iters[l] > 255) return "iterations must be within 0..255";
    if (p->radius < 1 || p->radius > 16384) return "radius must be within 1..16384";
    if (p->max_disp < -1024 || p->max_disp > 65535) return "max_disp must be within -1024..65535";
    if (p->rs_mode != PGM_RS_FLOOR && p->rs_mode != PGM_RS_SYMMETRIC) return "unknown rs_mode";
    if (p->sobel_ksize != 3 && p->sobel_ksize != 5) return "sobel_ksize must be 3 or 5";
    if (p->feature != PGM_FEAT_INT16 && p->feature != PGM_FEAT_F32_DIR && p->feature != PGM_FEAT_SIGN)
        return "unknown feature";
    if (p->color != PGM_RGB && p->color != PGM_GRAY) return "unknown color";
    if (p->fwd_bwd != 0 && p->fwd_bwd != 1) return "fwd_bwd must be 0 or 1";
    if (p->consistency_px < 0 || p->consistency_px > 46340) return "consistency_px must be within 0..46340";
    if (p->init_mode != PGM_INIT_RANDOM && p->init_mode != PGM_INIT_EXHAUSTIVE) return "unknown init_mode";
    if (p->refine_rounds < 0 || p->refine_rounds > 16) return "refine_rounds must be within 0..16";
    if (p->refine_rounds > 0 && p->levels < 2) return "refinement needs at least two levels";
    for (int l = 0; l < p->levels; l++) {
        if (p->space_fwd[l] < PGM_SPACE_RGB || p->space_fwd[l] > PGM_SPACE_LAB || p->space_bwd[l] < PGM_SPACE_RGB ||
            p->space_bwd[l] > PGM_SPACE_LAB)
            return "unknown colour space";
        if (p->color == PGM_GRAY && (p->space_fwd[l] != PGM_SPACE_RGB || p->space_bwd[l] != PGM_SPACE_RGB))
            return "colour spaces need color = PGM_RGB";
    }
    if (p->metric != PGM_METRIC_SAD && p->metric != PGM_METRIC_SSD) return "unknown metric";
    if (p->metric == PGM_METRIC_SSD && p->feature == PGM_FEAT_F32_DIR)
        return "the squared metric needs integer features";
    if (p->min_region_px < 0) return "min_region_px must not be negative";
    if (p->min_region_px > 0 && (p->region_link_px < 1 || p->region_link_px > 65535))
        return "region_link_px must be within 1..65535";
    return nullptr;
}

void plan(const pgm_params* p, int w, int h, Layout& Y)
{
    Y = Layout();
    Y.L = p->levels;
    Y.ch = p->color == PGM_GRAY ? 1 : 3;
    Y.C2 = 2 * Y.ch;
    Y.f32 = p->feature == PGM_FEAT_F32_DIR;
    Y.kind = Y.f32 ? 1 : (p->metric == PGM_METRIC_SSD ? 2 : 0);
    Y.dsize = Y.kind == 2 ? 8 : 4;
    Y.esize = Y.f32 ? 4 : 2;
    int cw = w, chh = h;
    for (int l = 0; l < Y.L; l++) {
        Y.lw[l] = cw; Y.lh[l] = chh;
        Y.lnx[l] = grid_count(cw, p->seed_stride);
        Y.lny[l] = grid_count(chh, p->seed_stride);
        cw = (cw + 1) / 2; chh = (chh + 1) / 2;
    }
    const int m = Y.L - 1;
    if (p->max_disp == 0) Y.R_top = Y.lw[m] > Y.lh[m] ? Y.lw[m] : Y.lh[m];
    else {   // a negative bound -k scales with the pair: ceil(w / k) pixels at full resolution
        const int bound = p->max_disp > 0 ? p->max_disp : (w + (-p->max_disp) - 1) / (-p->max_disp);
        Y.R_top = (bound + (1 << m) - 1) >> m;
    }

    // Sec. III-D: initial field at m, N refinement round trips between m and m-1 carrying
    // field and record, the field alone from m to m-1, then field and record to level 0.
    auto add = [&](int level, int enter) { Y.st_level[Y.nst] = level; Y.st_enter[Y.nst] = enter; Y.nst++; };
    add(m, ENTER_INIT);
    for (int k = 0; k < p->refine_rounds; k++) { add(m - 1, ENTER_DOWN_FO); add(m, ENTER_UP_FO); }
    for (int l = m - 1; l >= 0; l--) add(l, l == m - 1 ? ENTER_DOWN_F : ENTER_DOWN_FO);

    // shared slice: random numbers
    long long base = 0;
    for (int k = 0; k < Y.nst; k++) {
        const int l = Y.st_level[k];
        const bool rand_init = Y.st_enter[k] == ENTER_INIT && p->init_mode == PGM_INIT_RANDOM;
        Y.st_W[k] = rand_init ? (Y.R_top > 0 ? Y.R_top : 1) : p->radius;
        Y.st_nI[k] = n_offsets(Y.st_W[k]);
        Y.st_base[k] = base;
        const long long n = (long long)Y.lnx[l] * Y.lny[l];
        base += 2LL * p->iters[l] * n * Y.st_nI[k];
    }
    size_t cur = 0;
    Y.rnd = take(cur, (size_t)base * sizeof(short2) + 4);
    Y.rnd_init = take(cur, (size_t)2 * Y.lnx[m] * Y.lny[m] * sizeof(short2));
    Y.tab = take(cur, (size_t)TAB_MAX * sizeof(PairTab));
    Y.shared_bytes = (cur + 255) & ~(size_t)255;

    // per-pair slice
    cur = 0;
    // gradient images: slots 0, 1 = images 1, 2 in the forward pyramid's colour space, slots
    // 2, 3 = images 1, 2 in the backward one's (the same memory when the spaces agree)
    for (int im = 0; im < 2; im++)
        for (int l = 0; l < Y.L; l++) {
            Y.pyr[im][l] = l ? take(cur, (size_t)Y.lw[l] * Y.lh[l] * 3) : 0;
            Y.grad[im][l] = take(cur, (size_t)(Y.lw[l] + 2 * PAD) * (Y.lh[l] + 2 * PAD) * Y.C2 * Y.esize);
        }
    for (int l = 0; l < Y.L; l++)
        for (int im = 0; im < 2; im++)
            Y.grad[2 + im][l] = p->space_fwd[l] == p->space_bwd[l]
                                    ? Y.grad[im][l]
                                    : take(cur, (size_t)(Y.lw[l] + 2 * PAD) * (Y.lh[l] + 2 * PAD) * Y.C2 * Y.esize);
    for (int d = 0; d < 2; d++)
        for (int l = 0; l < Y.L; l++) {
            size_t n = (size_t)Y.lnx[l] * Y.lny[l];
            Y.disp[d][l] = take(cur, n * 4);
            Y.dist[d][l] = take(cur, n * Y.dsize);
            Y.flags[d][l] = take(cur, n);
            Y.disp2[d][l] = take(cur, n * 4);
            Y.dist2[d][l] = take(cur, n * Y.dsize);
        }
    for (int k = 0; k < Y.nst; k++) {
        const int l = Y.st_level[k];
        const int kind = Y.st_enter[k] == ENTER_INIT ? CNT_INIT : Y.st_enter[k] == ENTER_UP_FO ? CNT_UP : CNT_DOWN;
        Y.cnt_cap[kind] += dir_blocks(p, Y.lnx[l] * Y.lny[l]);
        if (kind == CNT_DOWN && l + 1 < Y.L)   // room for a launch that enters the level whole
            Y.cnt_cap[kind] += 2LL * enter_blocks(Y.lnx[l], Y.lny[l], p->patch_fwd, Y.lnx[l + 1] * Y.lny[l + 1]);
        if (kind == CNT_INIT) Y.cnt_cap[kind] += 2LL * enter_blocks(Y.lnx[l], Y.lny[l], p->patch_fwd, 0);
        auto sb = [&](int P) { return (long long)sweep_blocks(Y.lnx[l], Y.lny[l], P); };
        const long long per_sweep = variant(p->patch_fwd) == variant(p->patch_bwd) ? 2 * sb(p->patch_fwd)
                                                                                   : sb(p->patch_fwd) + sb(p->patch_bwd);
        Y.cnt_cap[CNT_SWEEP] += 2LL * p->iters[l] * per_sweep;
        // one launch per half-sweep at most
        Y.cnt_cap[CNT_MULTI] += 2LL * p->iters[l] * 2 * sweep_multi_blocks(Y.lnx[l], Y.lny[l]);
        Y.cnt_cap[CNT_PAIR] += 2LL * p->iters[l] * 2 * sweep_pair_blocks(Y.lnx[l], Y.lny[l]);
    }
    for (int k = 0; k < 6; k++) Y.cnt[k] = take(cur, (size_t)Y.cnt_cap[k] * 4 + 4);
    // partial evaluation sums of the count reduction: COUNT_SLICES x KINDS per pair
    Y.cntpart = take(cur, (size_t)COUNT_SLICES * CountArgs::KINDS * sizeof(unsigned long long));
    // region labels and sizes on the level-0 grid (small-region removal)
    Y.cclabel = take(cur, (size_t)Y.lnx[0] * Y.lny[0] * 4);
    Y.ccsize = take(cur, (size_t)Y.lnx[0] * Y.lny[0] * 4);
    Y.pair_bytes = (cur + 255) & ~(size_t)255;
    Y.total = Y.shared_bytes + Y.pair_bytes;
}

void fill_sizes(const Layout& Y, pgm_sizes* s)
{
    memset(s, 0, sizeof *s);
    s->levels = Y.L;
    for (int l = 0; l < Y.L; l++) {
        s->level_w[l] = Y.lw[l]; s->level_h[l] = Y.lh[l];
        s->level_nx[l] = Y.lnx[l]; s->level_ny[l] = Y.lny[l];
    }
    s->nx = Y.lnx[0]; s->ny = Y.lny[0];
    s->workspace_bytes = Y.total;
    s->workspace_shared_bytes = Y.shared_bytes;
    s->workspace_pair_bytes = Y.pair_bytes;
}

// LDS layout of a whole-level sweep launch at level l, if it fits in lds_max bytes
bool level_layout(const Layout& Y, int l, int iters, int nI, size_t lds_max, LevelLayout& o)
{
    const size_t n = (size_t)Y.lnx[l] * Y.lny[l];
    const size_t graw = (size_t)(Y.lw[l] + 2 * PAD) * (Y.lh[l] + 2 * PAD) * Y.C2 * Y.esize;
    o.gstride = (graw + 15) & ~(size_t)15;
    o.disp = 2 * o.gstride;
    o.dist = (o.disp + n * 4 + 15) & ~(size_t)15;   // 8-byte distances need 8-byte alignment
    o.rnd = (o.dist + n * Y.dsize + 15) & ~(size_t)15;
    o.total = (o.rnd + (size_t)iters * n * nI * sizeof(short2) + 15) & ~(size_t)15;
    return o.total + 64 <= lds_max;   // room for the kernel's static LDS
}

}  // namespace

struct pgm_ctx_s {
    int device = 0;
    // the pairs of a call share the GPU with other work (concurrent groups, the server's
    // requests): small levels then run in one work-group per pair and direction
    bool concurrent = false;
    int sched = PGM_SCHED_AUTO;   // pgm_schedule
    size_t lds_max = 0;            // LDS bytes a work-group may use on this device
    uint8_t* ws = nullptr;
    size_t ws_bytes = 0;
    std::string err;
    // the last pgm_match, for the dump entry points
    bool have_last = false;
    uint8_t* last_ws = nullptr;                   // workspace region of the last batch
    Layout last;
    pgm_params last_p;
    hipStream_t last_stream = nullptr;
    const uint8_t* last_img[2] = {nullptr, nullptr};
    int last_pitch = 0;
    int rec_valid[PGM_MAX_LEVELS];
    // profiling (pgm_profile): events around launches and per-kind evaluation counters
    bool prof = false;
    unsigned long long* prof_evals = nullptr;     // PGM_K_KINDS device counters
    std::vector<hipEvent_t> events;               // pool, reused after each clear
    size_t next_event = 0;
    struct Rec { int kind; int n; hipEvent_t a, b; };   // n consecutive launches of one kind
    std::vector<Rec> recs;
    bool run_open = false;   // recs.back() still waits for its end event
    // pgm_match_groups: internal streams (default priority), fork/join events, and the graph
    // of the last captured call with the bytes of its arguments
    static constexpr int NSTREAMS = 4;
    hipStream_t gs[NSTREAMS] = {};
    hipStream_t cap = nullptr;
    hipEvent_t fork = nullptr, join[NSTREAMS] = {};
    hipGraphExec_t gexec = nullptr;
    std::string gkey;
    long long nlaunch = 0;                        // kernel launches issued (capture check)
};

static std::string g_create_error;

// Logging to stderr, by the level in the environment variable PGM_LOG (read once): 0 or unset
// nothing, 1 failures, 2 also contexts, servers and every server request (its shape, the
// requests sharing its launch sequence, its latency from submission to completion as seen by
// polling, and the pool bytes in use), 3 also every matching call (pairs, launches).
static int log_level()
{
    static const int level = [] {
        const char* e = getenv("PGM_LOG");
        return e ? atoi(e) : 0;
    }();
    return level;
}

__attribute__((format(printf, 2, 3))) static void pgm_log(int level, const char* fmt, ...)
{
    if (log_level() < level) return;
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    fprintf(stderr, "[pgm] %s\n", buf);
}

static pgm_status fail(pgm_ctx_s* c, pgm_status st, const std::string& msg)
{
    if (c) c->err = msg;
    else g_create_error = msg;
    pgm_log(1, "error %d: %s", (int)st, msg.c_str());
    return st;
}

#define PGM_HIP(ctx, expr)                                                                      \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return fail((ctx), PGM_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e_));    \
    } while (0)

extern "C" {

pgm_status pgm_default_params(pgm_params* p, int32_t preset)
{
    if (!p) return PGM_EINVAL;
    memset(p, 0, sizeof *p);
    p->levels = 3;
    p->seed_stride = 3;
    p->patch_fwd = p->patch_bwd = 8;
    for (int l = 0; l < PGM_MAX_LEVELS; l++) p->iters[l] = 4;
    p->radius = 2;
    p->max_disp = 20;
    p->sobel_ksize = 5;
    p->feature = PGM_FEAT_INT16;
    p->color = PGM_RGB;
    p->fwd_bwd = 1;
    p->consistency_px = 1;
    p->init_mode = PGM_INIT_RANDOM;
    p->refine_rounds = 0;
    p->min_region_px = 0;
    p->region_link_px = 12;
    switch (preset) {
    case PGM_PRESET_PAPER:   // Sec. IV: W=2, S=5, L=3, N=2, 6 / 4 iterations; r = 7 / 5
        // Table II: forward pyramid RGB, CIELab, YCrCb; backward CIELab, YCrCb, RGB
        p->space_fwd[0] = PGM_SPACE_RGB;
        p->space_fwd[1] = PGM_SPACE_LAB;
        p->space_fwd[2] = PGM_SPACE_YCRCB;
        p->space_bwd[0] = PGM_SPACE_LAB;
        p->space_bwd[1] = PGM_SPACE_YCRCB;
        p->space_bwd[2] = PGM_SPACE_RGB;
        p->seed_stride = 1;
        p->patch_fwd = 15;
        p->patch_bwd = 11;
        p->iters[0] = 6;
        p->max_disp = 0;
        p->refine_rounds = 2;
        p->min_region_px = 9;    // Sec. III-E: regions below 9 pixels are removed
        p->rng_seed = 0;
        return PGM_OK;
    case PGM_PRESET_CONFIG1:
        p->rng_seed = 1000;
        return PGM_OK;
    case PGM_PRESET_CONFIG2:
    case PGM_PRESET_CONFIG3:
    case PGM_PRESET_CONFIG4:
    case PGM_PRESET_CONFIG5:
        p->levels = 5;
        for (int l = 0; l < PGM_MAX_LEVELS; l++) p->iters[l] = 6;
        p->max_disp = preset == PGM_PRESET_CONFIG2 ? 200 : preset == PGM_PRESET_CONFIG3 ? 250 : -5;
        p->feature = preset == PGM_PRESET_CONFIG3 ? PGM_FEAT_F32_DIR : PGM_FEAT_INT16;
        p->rng_seed = 1000ull * (uint64_t)preset;
        return PGM_OK;
    default:
        return PGM_EINVAL;
    }
}

pgm_status pgm_query(const pgm_params* p, int32_t w, int32_t h, pgm_sizes* out)
{
    if (!out) return PGM_EINVAL;
    if (validate(p, w, h)) return PGM_EINVAL;
    Layout Y;
    plan(p, w, h, Y);
    fill_sizes(Y, out);
    return PGM_OK;
}

pgm_status pgm_create(int32_t device, uint64_t workspace_bytes, void** out_ctx)
{
    if (!out_ctx) return fail(nullptr, PGM_EINVAL, "out_ctx is null");
    *out_ctx = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0) return fail(nullptr, PGM_EDEVICE, "no HIP device available");
    if (device < 0 || device >= n) return fail(nullptr, PGM_EINVAL, "device index out of range");
    pgm_ctx_s* c = new pgm_ctx_s();
    c->device = device;
    c->ws_bytes = workspace_bytes ? workspace_bytes : (256ull << 20);
    e = hipSetDevice(device);
    if (e == hipSuccess) e = hipMalloc((void**)&c->ws, c->ws_bytes);
    if (e == hipSuccess) e = hipMalloc((void**)&c->prof_evals, PGM_K_KINDS * sizeof(unsigned long long));
    if (e == hipSuccess) {
        int v = 0;
        e = hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
        c->lds_max = v > 0 ? (size_t)v : 0;
        // (HIP may not need the attribute for dynamic LDS up to the device limit; a refusal
        // is left to the launch to report)
        if (e == hipSuccess && c->lds_max > 65536 && level_allow_lds(c->lds_max - 64) != hipSuccess)
            (void)hipGetLastError();
    }
    if (e != hipSuccess) {
        if (c->ws) (void)hipFree(c->ws);
        if (c->prof_evals) (void)hipFree(c->prof_evals);
        std::string msg = std::string("workspace allocation failed: ") + hipGetErrorString(e);
        delete c;
        return fail(nullptr, e == hipErrorOutOfMemory ? PGM_ENOMEM : PGM_EDEVICE, msg);
    }
    *out_ctx = c;
    pgm_log(2, "context on device %d: workspace %zu bytes", device, c->ws_bytes);
    return PGM_OK;
}

void pgm_destroy(void* ctx)
{
    pgm_ctx_s* c = (pgm_ctx_s*)ctx;
    if (!c) return;
    pgm_log(2, "context on device %d destroyed", c->device);
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    if (c->ws) (void)hipFree(c->ws);
    if (c->prof_evals) (void)hipFree(c->prof_evals);
    for (hipEvent_t ev : c->events) (void)hipEventDestroy(ev);
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    for (int i = 0; i < pgm_ctx_s::NSTREAMS; i++) {
        if (c->gs[i]) (void)hipStreamDestroy(c->gs[i]);
        if (c->join[i]) (void)hipEventDestroy(c->join[i]);
    }
    if (c->cap) (void)hipStreamDestroy(c->cap);
    if (c->fork) (void)hipEventDestroy(c->fork);
    delete c;
}

const char* pgm_last_error(void* ctx)
{
    pgm_ctx_s* c = (pgm_ctx_s*)ctx;
    return c ? c->err.c_str() : g_create_error.c_str();
}

// Checks of one batch's arguments; fills the layout.
static pgm_status check_batch(pgm_ctx_s* c, const pgm_params* p, int32_t npairs, const uint8_t* img1,
                              const uint8_t* img2, int32_t w, int32_t h, int32_t pitch_bytes,
                              int64_t image_stride_bytes, const pgm_match_t* out_fwd, Layout& Y)
{
    if (const char* why = validate(p, w, h)) return fail(c, PGM_EINVAL, why);
    if (npairs < 1) return fail(c, PGM_EINVAL, "n_pairs must be at least 1");
    if (!img1 || !img2 || !out_fwd) return fail(c, PGM_EINVAL, "img1, img2 and out_fwd must not be null");
    if (pitch_bytes < 3 * w) return fail(c, PGM_EINVAL, "pitch_bytes must be at least 3 * w");
    // the image kernels address an image's bytes with 32-bit offsets
    if ((int64_t)pitch_bytes * (h - 1) + 3LL * w + 4 > INT32_MAX)
        return fail(c, PGM_EINVAL, "an image must span less than 2^31 bytes: pitch_bytes * (h - 1) + 3 * w");
    if (npairs > 1 && image_stride_bytes < (int64_t)pitch_bytes * h)
        return fail(c, PGM_EINVAL, "image_stride_bytes must be at least pitch_bytes * h");
    plan(p, w, h, Y);
    return PGM_OK;
}

// The whole method for a batch of pairs, with the workspace region [wsb, wsb + wsn).
// With host_tab (npairs <= TAB_MAX entries), every pair brings its own images and outputs:
// img1, img2 and the out_* arguments are then those of entry 0 (for the checks) and are not
// used otherwise; out_n_evals must be null (each entry has its own counter).
static pgm_status match_impl(pgm_ctx_s* c, const pgm_params* p, int32_t npairs, const uint8_t* img1,
                             const uint8_t* img2, int32_t w, int32_t h, int32_t pitch_bytes,
                             int64_t image_stride_bytes, pgm_match_t* out_fwd, pgm_match_t* out_bwd,
                             int32_t* out_n_inliers, pgm_match_t* out_compact, uint64_t* out_n_evals,
                             hipStream_t s, uint8_t* wsb, size_t wsn, const PairTab* host_tab = nullptr)
{
    Layout Y;
    if (host_tab) image_stride_bytes = (int64_t)pitch_bytes * h;   // unused: the table has the images
    if (pgm_status st = check_batch(c, p, npairs, img1, img2, w, h, pitch_bytes, image_stride_bytes, out_fwd, Y))
        return st;
    if (host_tab && (npairs > TAB_MAX || out_n_evals))
        return fail(c, PGM_EINVAL, "a table-driven batch holds at most 16 pairs and counts per pair");
    const size_t need = Y.shared_bytes + (size_t)npairs * Y.pair_bytes;
    if (need > wsn)
        return fail(c, PGM_ENOMEM, "workspace of " + std::to_string(wsn) + " bytes is smaller than the " +
                                       std::to_string(need) + " bytes this batch needs");
    PGM_HIP(c, hipSetDevice(c->device));
    const long long nlaunch0 = c->nlaunch;
    uint8_t* ws = wsb;                            // shared slice
    uint8_t* pw0 = wsb + Y.shared_bytes;          // pair 0's slice
    const long long zs = (long long)Y.pair_bytes;
    unsigned long long* nev = (unsigned long long*)out_n_evals;
    // with profiling on, every launch is bracketed by two events on the caller's stream
    auto event = [&](hipEvent_t* ev) -> hipError_t {
        if (c->next_event == c->events.size()) {
            hipEvent_t e;
            hipError_t err = hipEventCreate(&e);
            if (err != hipSuccess) return err;
            c->events.push_back(e);
        }
        *ev = c->events[c->next_event++];
        return hipSuccess;
    };
    // Profiling times runs of consecutive launches of one kind between two events, so that no
    // event packet sits between the kernels of a run (a run's time includes the gaps between
    // its kernels). A run left open by a failed call is dropped.
    if (c->run_open) {
        c->recs.pop_back();
        c->run_open = false;
    }
    auto close_run = [&]() -> hipError_t {
        if (!c->run_open) return hipSuccess;
        c->run_open = false;
        return hipEventRecord(c->recs.back().b, s);
    };
    auto timed = [&](int kind, auto&& launch) -> hipError_t {
        c->nlaunch++;
        if (!c->prof) return launch();
        if (c->run_open && c->recs.back().kind == kind) {
            hipError_t e = launch();
            if (e == hipSuccess) c->recs.back().n++;
            return e;
        }
        hipError_t e = close_run();
        pgm_ctx_s::Rec r;
        r.kind = kind;
        r.n = 1;
        if (e == hipSuccess) e = event(&r.a);
        if (e == hipSuccess) e = event(&r.b);
        if (e == hipSuccess) e = hipEventRecord(r.a, s);
        if (e == hipSuccess) e = launch();
        if (e == hipSuccess) {
            c->recs.push_back(r);
            c->run_open = true;
        }
        return e;
    };
    // the per-pair buffers of a table-driven batch, written into the workspace first
    const PairTab* dtab = nullptr;
    bool tab_counts = false;
    if (host_tab) {
        dtab = (const PairTab*)(ws + Y.tab);
        for (int k = 0; k < npairs; k++) tab_counts = tab_counts || host_tab[k].n_evals;
        c->nlaunch++;
        PGM_HIP(c, launch_fill_tab((PairTab*)dtab, host_tab, npairs, s));
    }
    // evaluation counts: each matching launch stores one count per work-group into its kind's
    // table (per pair); k_count adds them up at the end
    const bool counting = nev || c->prof || tab_counts;
    long long cnt_off[6] = {0, 0, 0, 0, 0, 0};
    auto ctable = [&](int kind, long long blocks) -> uint32_t* {
        if (!counting) return nullptr;
        uint32_t* t = (uint32_t*)(pw0 + Y.cnt[kind]) + cnt_off[kind];
        cnt_off[kind] += blocks;
        return t;
    };

    // The image stage. One launch draws every random number (shared by the pairs: they depend
    // only on the parameters), builds the level-0 gradient images and the first pyramid level;
    // then the further pyramid levels, then the gradient images of levels 1.. in one launch
    // (Sec. III-D, III-A).
    PrepArgs pa;
    memset(&pa, 0, sizeof pa);
    RngArgs& ra = pa.rng;
    ra.nstages = Y.nst;
    for (int k = 0; k < Y.nst; k++) {
        const int l = Y.st_level[k];
        ra.st[k].n = Y.lnx[l] * Y.lny[l];
        ra.st[k].iters = p->iters[l];
        ra.st[k].nI = Y.st_nI[k];
        ra.st[k].W = Y.st_W[k];
        ra.st[k].level = l;
        ra.st[k].stage = k;
        ra.st[k].base = Y.st_base[k];
    }
    ra.table = (short2*)(ws + Y.rnd);
    ra.init = (short2*)(ws + Y.rnd_init);
    const int m = Y.L - 1;
    ra.n_top = p->init_mode == PGM_INIT_RANDOM ? Y.lnx[m] * Y.lny[m] : 0;
    ra.R_top = Y.R_top;
    ra.rs_sym = p->rs_mode == PGM_RS_SYMMETRIC;
    ra.top_level = m;
    ra.key0 = (uint32_t)p->rng_seed;
    ra.key1 = (uint32_t)(p->rng_seed >> 32);

    // one entry per colour space the level needs (two when the pyramids differ there)
    auto grad_level = [&](GradArgs& ga, int l, const uint8_t* s0, const uint8_t* s1, long long szs, int pitch) {
        for (int half = 0; half < 2; half++) {
            if (half == 1 && p->space_fwd[l] == p->space_bwd[l]) break;
            GradLevel& L = ga.lv[ga.n++];
            L.src[0] = s0;
            L.src[1] = s1;
            L.src_zs = szs;
            L.pitch = pitch;
            L.w = Y.lw[l];
            L.h = Y.lh[l];
            L.G[0] = pw0 + Y.grad[2 * half][l];
            L.G[1] = pw0 + Y.grad[2 * half + 1][l];
            L.tab = l == 0 ? dtab : nullptr;   // level 0 reads the caller's images
            L.space = half ? p->space_bwd[l] : p->space_fwd[l];
        }
    };
    auto pyr_level = [&](PyrArgs& pr, int l, const uint8_t* s0, const uint8_t* s1, long long szs, int pitch) {
        pr.src[0] = s0;
        pr.src[1] = s1;
        pr.src_zs = szs;
        pr.pitch = pitch;
        pr.w = Y.lw[l - 1];
        pr.h = Y.lh[l - 1];
        pr.dst[0] = pw0 + Y.pyr[0][l];
        pr.dst[1] = pw0 + Y.pyr[1][l];
        pr.dst_zs = zs;
    };
    const bool gray = p->color == PGM_GRAY;
    pa.grad.dst_zs = zs;
    grad_level(pa.grad, 0, img1, img2, image_stride_bytes, pitch_bytes);
    // pyramid levels two at a time where two remain (one pass computes both)
    auto second_level = [&](PyrArgs& pr, int l) {
        if (l + 1 >= Y.L) return;
        pr.two = 1;
        pr.dst2[0] = pw0 + Y.pyr[0][l + 1];
        pr.dst2[1] = pw0 + Y.pyr[1][l + 1];
    };
    pa.with_pyr = Y.L > 1;
    if (pa.with_pyr) {
        pyr_level(pa.pyr, 1, img1, img2, image_stride_bytes, pitch_bytes);
        pa.pyr.tab = dtab;
        second_level(pa.pyr, 1);
    }
    PGM_HIP(c, timed(PGM_K_PREP, [&] { return launch_prep(pa, npairs, gray, p->sobel_ksize, p->feature, s); }));
    for (int l = pa.pyr.two ? 3 : 2; l < Y.L;) {
        PyrArgs pr;
        memset(&pr, 0, sizeof pr);
        pyr_level(pr, l, pw0 + Y.pyr[0][l - 1], pw0 + Y.pyr[1][l - 1], zs, Y.lw[l - 1] * 3);
        second_level(pr, l);
        PGM_HIP(c, timed(PGM_K_PYRAMID, [&] { return launch_pyr(pr, npairs, s); }));
        l += pr.two ? 2 : 1;
    }
    GradArgs gl;
    memset(&gl, 0, sizeof gl);
    gl.dst_zs = zs;
    for (int l = 1; l < Y.L; l++) grad_level(gl, l, pw0 + Y.pyr[0][l], pw0 + Y.pyr[1][l], zs, Y.lw[l] * 3);
    if (gl.n) PGM_HIP(c, timed(PGM_K_GRADIENT, [&] { return launch_gradient(gl, npairs, gray, p->sobel_ksize, p->feature, s); }));

    auto geo = [&](int l) {
        Geo g;
        g.w = Y.lw[l]; g.h = Y.lh[l]; g.pw = Y.lw[l] + 2 * PAD;
        g.nx = Y.lnx[l]; g.ny = Y.lny[l];
        g.stride = p->seed_stride; g.off = p->seed_stride / 2;
        geo_divs(g);
        return g;
    };
    auto field = [&](int d, int l) {
        Field f;
        f.disp = (uint32_t*)(pw0 + Y.disp[d][l]);
        f.dist = pw0 + Y.dist[d][l];
        f.flags = pw0 + Y.flags[d][l];
        return f;
    };
    // the second buffer of a level's field (displacements and distances; the flags are shared)
    auto field2 = [&](int d, int l) {
        Field f = field(d, l);
        f.disp = (uint32_t*)(pw0 + Y.disp2[d][l]);
        f.dist = pw0 + Y.dist2[d][l];
        return f;
    };
    auto gorigin = [&](int slot, int l) {
        return (const void*)(pw0 + Y.grad[slot][l] + ((size_t)PAD * (Y.lw[l] + 2 * PAD) + PAD) * Y.C2 * Y.esize);
    };
    auto dirargs = [&](int d, int l, int k) {
        DirArgs a;
        // forward: image 1 against image 2 in the forward space; backward: image 2 against
        // image 1 in the backward space
        a.Ga = d == 0 ? gorigin(0, l) : gorigin(3, l);
        a.Gb = d == 0 ? gorigin(1, l) : gorigin(2, l);
        a.f = field(d, l);
        a.rnd = (const short2*)(ws + Y.rnd) + Y.st_base[k] + (long long)d * p->iters[l] * Y.lnx[l] * Y.lny[l] * Y.st_nI[k];
        a.rnd0 = (const short2*)(ws + Y.rnd_init) + (size_t)d * Y.lnx[m] * Y.lny[m];
        a.P = d == 0 ? p->patch_fwd : p->patch_bwd;
        return a;
    };
    const bool shared = variant(p->patch_fwd) == variant(p->patch_bwd);
    auto batch = [&](int nd) {
        Batch b;
        b.npairs = npairs;
        b.ndir = nd;
        b.zs = zs;
        return b;
    };

    // A small level runs in one work-group per pair and direction (k_level) where other work
    // shares the GPU (concurrent groups, the server) or the batch has 16 pairs or more;
    // otherwise it runs faster as half-sweep launches across the chip (measured: one pair
    // 65 -> 55 us at 64x28, 8 pairs slightly faster, 32 pairs slightly slower).
    auto lds_level = [&](int k, LevelLayout& lay) {
        const int l = Y.st_level[k];
        const bool want = (c->sched & PGM_SCHED_LEVEL_LDS) ||
                          (!(c->sched & PGM_SCHED_LEVEL_LAUNCHES) && (npairs >= 16 || c->concurrent));
        return shared && p->iters[l] > 0 && want && level_layout(Y, l, p->iters[l], Y.st_nI[k], c->lds_max, lay);
    };
    // Stages whose level is entered from the coarser one in one launch together with the
    // coarser level's check: the transition alone (2; batches under 16 pairs), or also the
    // first half-sweep (1) for small levels, where the separate launches cost mostly their
    // latency (the half-sweep needs more registers per lane, which costs more than it saves
    // once a level fills the chip). Both directions share the kernels, and patch sides are
    // at most 8 (six-channel float features excepted: their three candidate patches do not
    // fit the registers).
    const bool can_fuse = shared && std::max(p->patch_fwd, p->patch_bwd) <= 8 && !(Y.kind == 1 && Y.C2 == 6) &&
                          !(c->sched & PGM_SCHED_SEPARATE);
    // The initial level of a random start is entered the same way (3): its starts and its
    // first half-sweep in one launch.
    auto fused = [&](int k) -> int {
        if (k < 0 || k >= Y.nst || !can_fuse) return 0;
        const int e = Y.st_enter[k];
        const int l = Y.st_level[k];
        LevelLayout lay;
        const bool small =
            p->iters[l] > 0 && (long long)Y.lnx[l] * Y.lny[l] * npairs <= FUSE_MAX_SEEDS && !lds_level(k, lay);
        if (e == ENTER_INIT) return p->init_mode == PGM_INIT_RANDOM && small ? 3 : 0;
        if (k == 0 || (e != ENTER_DOWN_F && e != ENTER_DOWN_FO)) return 0;
        if (small) return 1;
        return npairs < 16 ? 2 : 0;   // large batches: the separate check is cheaper per pair
    };
    int rec_valid[PGM_MAX_LEVELS] = {0};
    int check_rec_valid = 0;   // rec_valid of the check deferred into the next stage's launch
    for (int k = 0; k < Y.nst; k++) {
        const int l = Y.st_level[k];
        const Geo g = geo(l);
        const int enter = Y.st_enter[k];
        const int fuse = fused(k);
        LevelArgs la;
        memset(&la, 0, sizeof la);
        const bool in_lds = lds_level(k, la.lay);
        // Step 1's half-sweeps (iteration, colour), red then black. A small level's run
        // several per launch, each launch reading the field from one buffer and writing it
        // whole to the other: chunks of 4 with the rest as 2 or 3 (k_sweep_multi), or on a
        // larger level chunks of 2 (k_sweep_pair) and a last odd one alone, in place on the
        // buffer that holds the field. With an odd number of two-buffer launches the level's
        // entry writes the second buffer, so that the last of them writes the level's own.
        int hs_t[2 * 256], hs_c[2 * 256], nhs = 0;   // iterations are at most 255
        for (int t = 0; t < (in_lds ? 0 : p->iters[l]); t++)
            for (int colour = ((fuse == 1 || fuse == 3) && t == 0) ? 1 : 0; colour < 2; colour++) {
                hs_t[nhs] = t;
                hs_c[nhs++] = colour;
            }
        // (six-channel float features excepted: that kernel variant needs 295 registers per
        // lane, one wave per SIMD)
        const long long lseeds = (long long)g.nx * g.ny * npairs;
        const bool multi = shared && nhs >= 2 && std::max(p->patch_fwd, p->patch_bwd) <= 8 &&
                           !(Y.kind == 1 && Y.C2 == 6) && !(c->sched & PGM_SCHED_SEPARATE) &&
                           lseeds <= PAIR_MAX_SEEDS;
        const bool pairs_only = lseeds > MULTI_MAX_SEEDS;
        int chunk[2 * 256], nch = 0, nflip = 0;
        if (multi && !pairs_only) {
            for (int h = 0; h + 4 <= nhs; h += 4) chunk[nch++] = 4;
            const int rest = nhs % 4;
            if (rest == 1) {   // 4 + 1 as 3 + 2
                chunk[nch - 1] = 3;
                chunk[nch++] = 2;
            } else if (rest) {
                chunk[nch++] = rest;
            }
        } else if (multi) {
            for (int h = 0; h + 2 <= nhs; h += 2) chunk[nch++] = 2;
            if (nhs & 1) chunk[nch++] = 1;
        }
        for (int q = 0; q < nch; q++) nflip += chunk[q] > 1;
        const bool entry_second = multi && (nflip & 1);
        auto entry_dir = [&](int d) {
            DirArgs a = dirargs(d, l, k);
            if (entry_second) a.f = field2(d, l);
            return a;
        };
        if (fuse) {
            const bool init = fuse == 3;
            EnterArgs ea;
            memset(&ea, 0, sizeof ea);
            for (int q = 0; q < 2; q++) {
                ea.d[q] = entry_dir(q);
                if (!init) ea.src[q] = field(q, l + 1);
            }
            ea.g = g;
            ea.gs = init ? g : geo(l + 1);
            ea.b = batch(2);
            ea.carry_record = enter != ENTER_DOWN_F && !init;
            ea.fwd_bwd = p->fwd_bwd;
            ea.tau2 = p->consistency_px * p->consistency_px;
            ea.rec_valid = check_rec_valid;
            ea.nI = Y.st_nI[k];
            const int mode = init ? ENTER_LAUNCH_INIT : fuse == 1 ? ENTER_LAUNCH_SWEEP : ENTER_LAUNCH_START;
            ea.cnt = ctable(init ? CNT_INIT : CNT_DOWN,
                            2LL * enter_blocks(g.nx, g.ny, ea.d[0].P, init ? 0 : ea.gs.nx * ea.gs.ny));
            PGM_HIP(c, timed(init ? PGM_K_INIT : PGM_K_DOWN, [&] { return launch_enter(ea, Y.C2, Y.kind, mode, s); }));
        }
        for (int pass = 0; pass < (fuse ? 0 : shared ? 1 : 2); pass++) {
            const int nd = shared ? 2 : 1;
            const int d0 = shared ? 0 : pass;
            if (enter == ENTER_INIT) {
                InitArgs a;
                memset(&a, 0, sizeof a);
                for (int q = 0; q < nd; q++) a.d[q] = entry_dir(d0 + q);
                a.g = g;
                a.b = batch(nd);
                a.exhaustive = p->init_mode == PGM_INIT_EXHAUSTIVE;
                a.R = Y.R_top;
                a.cnt = ctable(CNT_INIT, (long long)nd * match_blocks(g.nx * g.ny, a.d[0].P));
                PGM_HIP(c, timed(PGM_K_INIT, [&] { return launch_init(a, Y.C2, Y.kind, s); }));
            } else {
                TransArgs a;
                memset(&a, 0, sizeof a);
                const int src = enter == ENTER_UP_FO ? l - 1 : l + 1;
                for (int q = 0; q < nd; q++) {
                    a.d[q] = entry_dir(d0 + q);
                    a.src[q] = field(d0 + q, src);
                }
                a.g = g;
                a.gs = geo(src);
                a.b = batch(nd);
                a.carry_record = enter != ENTER_DOWN_F;
                const long long nb = (long long)nd * match_blocks(g.nx * g.ny, a.d[0].P);
                if (enter == ENTER_UP_FO) {
                    a.cnt = ctable(CNT_UP, nb);
                    PGM_HIP(c, timed(PGM_K_UP, [&] { return launch_up(a, Y.C2, Y.kind, s); }));
                } else {
                    a.cnt = ctable(CNT_DOWN, nb);
                    PGM_HIP(c, timed(PGM_K_DOWN, [&] { return launch_down(a, Y.C2, Y.kind, s); }));
                }
            }
        }
        // Step 1 of a small level in one work-group per pair and direction, from LDS
        if (in_lds) {
            for (int q = 0; q < 2; q++) la.d[q] = dirargs(q, l, k);
            la.g = g;
            la.b = batch(2);
            la.iters = p->iters[l];
            la.nI = Y.st_nI[k];
            la.cnt = ctable(CNT_SWEEP, 2);
            la.gbytes = la.lay.gstride;
            la.gorig = ((size_t)PAD * (Y.lw[l] + 2 * PAD) + PAD) * Y.C2 * Y.esize;
            PGM_HIP(c, timed(PGM_K_LEVEL, [&] { return launch_level(la, Y.C2, Y.kind, s); }));
        }
        bool second = entry_second;   // which buffer holds the field
        for (int q = 0, h = 0; q < nch; q++) {
            if (chunk[q] == 1) {   // alone, in place
                SweepArgs a;
                memset(&a, 0, sizeof a);
                for (int d = 0; d < 2; d++) {
                    a.d[d] = dirargs(d, l, k);
                    a.d[d].f = second ? field2(d, l) : field(d, l);
                }
                a.g = g;
                a.b = batch(2);
                a.t = hs_t[h];
                a.colour = hs_c[h];
                a.nI = Y.st_nI[k];
                a.cnt = ctable(CNT_SWEEP, 2LL * sweep_blocks(g.nx, g.ny, a.d[0].P));
                PGM_HIP(c, timed(PGM_K_SWEEP, [&] { return launch_sweep(a, Y.C2, Y.kind, s); }));
                h++;
                continue;
            }
            SweepMultiArgs a;
            memset(&a, 0, sizeof a);
            for (int d = 0; d < 2; d++) {
                a.d[d] = dirargs(d, l, k);
                a.d[d].f = second ? field2(d, l) : field(d, l);
                a.out[d] = second ? field(d, l) : field2(d, l);
            }
            a.g = g;
            a.b = batch(2);
            a.nph = chunk[q];
            for (int m = 0; m < a.nph; m++) {
                a.t[m] = hs_t[h + m];
                a.c[m] = hs_c[h + m];
            }
            a.nI = Y.st_nI[k];
            if (pairs_only) {
                a.cnt = ctable(CNT_PAIR, 2LL * sweep_pair_blocks(g.nx, g.ny));
                PGM_HIP(c, timed(PGM_K_SWEEP_PAIR, [&] { return launch_sweep_pair(a, Y.C2, Y.kind, s); }));
            } else {
                a.cnt = ctable(CNT_MULTI, 2LL * sweep_multi_blocks(g.nx, g.ny));
                PGM_HIP(c, timed(PGM_K_SWEEP_MULTI, [&] { return launch_sweep_multi(a, Y.C2, Y.kind, s); }));
            }
            h += chunk[q];
            second = !second;
        }
        for (int t = 0; t < (in_lds || multi ? 0 : p->iters[l]); t++)
            for (int colour = ((fuse == 1 || fuse == 3) && t == 0) ? 1 : 0; colour < 2; colour++)
                for (int pass = 0; pass < (shared ? 1 : 2); pass++) {
                    const int nd = shared ? 2 : 1;
                    const int d0 = shared ? 0 : pass;
                    SweepArgs a;
                    memset(&a, 0, sizeof a);
                    for (int q = 0; q < nd; q++) a.d[q] = dirargs(d0 + q, l, k);
                    a.g = g;
                    a.b = batch(nd);
                    a.t = t;
                    a.colour = colour;
                    a.nI = Y.st_nI[k];
                    a.cnt = ctable(CNT_SWEEP, (long long)nd * sweep_blocks(g.nx, g.ny, a.d[0].P));
                    PGM_HIP(c, timed(PGM_K_SWEEP, [&] { return launch_sweep(a, Y.C2, Y.kind, s); }));
                }
        // Step 2-3
        CheckArgs ca;
        ca.f[0] = field(0, l);
        ca.f[1] = field(1, l);
        ca.g = g;
        ca.b = batch(2);
        ca.fwd_bwd = p->fwd_bwd;
        ca.tau2 = p->consistency_px * p->consistency_px;
        ca.rec_valid = enter == ENTER_DOWN_FO || enter == ENTER_UP_FO;
        rec_valid[l] = ca.rec_valid;
        check_rec_valid = ca.rec_valid;
        if (!fused(k + 1)) PGM_HIP(c, timed(PGM_K_CHECK, [&] { return launch_check(ca, s); }));
    }

    // small-region removal on the forward field at full resolution (Sec. III-E)
    if (p->min_region_px > 0) {
        RegionArgs ra2;
        ra2.f = field(0, 0);
        ra2.g = geo(0);
        ra2.b = batch(1);
        ra2.label = (int32_t*)(pw0 + Y.cclabel);
        ra2.size = (int32_t*)(pw0 + Y.ccsize);
        ra2.min_px = p->min_region_px;
        ra2.link2 = (long long)p->region_link_px * p->region_link_px;
        c->nlaunch += 3;   // four launches, one counted by timed()
        PGM_HIP(c, timed(PGM_K_REGION, [&] { return launch_regions(ra2, s); }));
    }

    // level-0 matches on the grid and the compacted forward inliers (Sec. III-G)
    OutArgs oa;
    memset(&oa, 0, sizeof oa);
    oa.g = geo(0);
    oa.b = batch(out_bwd ? 2 : 1);
    oa.f[0] = field(0, 0);
    oa.f[1] = field(1, 0);
    oa.out[0] = out_fwd;
    oa.out[1] = out_bwd;
    oa.compact = out_compact;
    oa.n_out = out_n_inliers;
    oa.tab = dtab;
    oa.dist8 = Y.dsize == 8;
    PGM_HIP(c, timed(PGM_K_OUTPUT, [&] { return launch_output(oa, s); }));
    PGM_HIP(c, close_run());
    if (counting) {
        CountArgs ca;
        const int kinds[6] = {PGM_K_INIT, PGM_K_DOWN, PGM_K_UP, PGM_K_SWEEP, PGM_K_SWEEP_MULTI, PGM_K_SWEEP_PAIR};
        for (int k = 0; k < 6; k++) {
            ca.table[k] = (const uint32_t*)(pw0 + Y.cnt[k]);
            ca.n[k] = cnt_off[k];
            ca.kind[k] = kinds[k];
        }
        ca.npairs = npairs;
        ca.zs = zs;
        ca.user = nev;
        ca.prof = c->prof ? c->prof_evals : nullptr;
        ca.tab = dtab;
        c->nlaunch += 2;
        PGM_HIP(c, launch_count(ca, (unsigned long long*)(pw0 + Y.cntpart), s));
    }

    pgm_log(3, "match: %d pair(s) of %dx%d, %lld launches", (int)npairs, (int)w, (int)h, c->nlaunch - nlaunch0);
    c->have_last = true;
    c->last_ws = wsb;
    c->last = Y;
    c->last_p = *p;
    c->last_stream = s;
    c->last_img[0] = img1;
    c->last_img[1] = img2;
    c->last_pitch = pitch_bytes;
    memcpy(c->rec_valid, rec_valid, sizeof rec_valid);
    return PGM_OK;
}

pgm_status pgm_match(void* ctx, const pgm_params* p, const uint8_t* img1, const uint8_t* img2,
                     int32_t w, int32_t h, int32_t pitch_bytes, pgm_match_t* out_fwd,
                     pgm_match_t* out_bwd, int32_t* out_n_inliers, pgm_match_t* out_compact,
                     uint64_t* out_n_evals, void* stream)
{
    pgm_ctx_s* c = (pgm_ctx_s*)ctx;
    if (!c) return PGM_EINVAL;
    return match_impl(c, p, 1, img1, img2, w, h, pitch_bytes, 0, out_fwd, out_bwd, out_n_inliers, out_compact,
                      out_n_evals, (hipStream_t)stream, c->ws, c->ws_bytes);
}

pgm_status pgm_match_batch(void* ctx, const pgm_params* p, int32_t n_pairs, const uint8_t* img1,
                           const uint8_t* img2, int32_t w, int32_t h, int32_t pitch_bytes,
                           int64_t image_stride_bytes, pgm_match_t* out_fwd, pgm_match_t* out_bwd,
                           int32_t* out_n_inliers, pgm_match_t* out_compact, uint64_t* out_n_evals,
                           void* stream)
{
    pgm_ctx_s* c = (pgm_ctx_s*)ctx;
    if (!c) return PGM_EINVAL;
    return match_impl(c, p, n_pairs, img1, img2, w, h, pitch_bytes, image_stride_bytes, out_fwd, out_bwd,
                      out_n_inliers, out_compact, out_n_evals, (hipStream_t)stream, c->ws, c->ws_bytes);
}

}  // extern "C"

// ---------------------------------------------------------------------------------------
// pgm_match_static: pgm_match for callers that cannot allocate device memory. Its workspace
// is this fixed device array (one copy per GPU, held until the process ends); host code uses
// only the address hipGetSymbolAddress reports for the current device, never the array's
// name. Every call on one GPU shares the array.
// ---------------------------------------------------------------------------------------

static __device__ __align__(256) uint8_t scratch[PGM_STATIC_SCRATCH_BYTES];

namespace {
constexpr int STATIC_MAX_DEVICES = 64;
std::mutex g_static_mu;
pgm_ctx_s g_static_ctx[STATIC_MAX_DEVICES];     // host state per device (no workspace of its own)
uint8_t* g_scratch_ptr[STATIC_MAX_DEVICES];     // device address of `scratch` on each device
bool g_static_ready[STATIC_MAX_DEVICES];
}  // namespace

extern "C" {

pgm_status pgm_match_static(const pgm_params* p, const uint8_t* img1, const uint8_t* img2, int32_t w, int32_t h,
                            int32_t pitch_bytes, pgm_match_t* out_fwd, pgm_match_t* out_bwd,
                            int32_t* out_n_inliers, pgm_match_t* out_compact, uint64_t* out_n_evals,
                            void* stream)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0)
        return fail(nullptr, PGM_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev >= STATIC_MAX_DEVICES) return fail(nullptr, PGM_EUNSUPPORTED, "device index beyond 63");
    pgm_ctx_s* c = &g_static_ctx[dev];
    {
        // set-up once per device, with that device current: the array's device address and
        // the LDS limit of the whole-level kernels
        std::lock_guard<std::mutex> lock(g_static_mu);
        if (!g_static_ready[dev]) {
            void* ptr = nullptr;
            e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !ptr)
                return fail(nullptr, PGM_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            int v = 0;
            e = hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
            if (e != hipSuccess)
                return fail(nullptr, PGM_EDEVICE, std::string("hipDeviceGetAttribute: ") + hipGetErrorString(e));
            c->device = dev;
            c->lds_max = v > 0 ? (size_t)v : 0;
            if (c->lds_max > 65536 && level_allow_lds(c->lds_max - 64) != hipSuccess) (void)hipGetLastError();
            g_scratch_ptr[dev] = (uint8_t*)ptr;
            g_static_ready[dev] = true;
        }
    }
    Layout Y;
    if (pgm_status st = check_batch(c, p, 1, img1, img2, w, h, pitch_bytes, 0, out_fwd, Y))
        return fail(nullptr, st, c->err);
    if (Y.total > (size_t)PGM_STATIC_SCRATCH_BYTES)
        return fail(nullptr, PGM_ENOMEM, "this pair needs " + std::to_string(Y.total) +
                                             " bytes of workspace, more than the " +
                                             std::to_string((unsigned long long)PGM_STATIC_SCRATCH_BYTES) +
                                             " bytes of pgm_match_static's fixed array");
    pgm_status st = match_impl(c, p, 1, img1, img2, w, h, pitch_bytes, 0, out_fwd, out_bwd, out_n_inliers,
                               out_compact, out_n_evals, (hipStream_t)stream, g_scratch_ptr[dev],
                               (size_t)PGM_STATIC_SCRATCH_BYTES);
    if (st != PGM_OK) return fail(nullptr, st, c->err);
    return PGM_OK;
}

pgm_status pgm_tune(void* ctx, const pgm_params* p, int32_t n_pairs, const uint8_t* img1, const uint8_t* img2,
                    int32_t w, int32_t h, int32_t pitch_bytes, int64_t image_stride_bytes, pgm_match_t* out_fwd,
                    pgm_match_t* out_bwd, int32_t* out_n_inliers, pgm_match_t* out_compact, int32_t repeats,
                    void* stream, int32_t* host_flags)
{
    pgm_ctx_s* c = (pgm_ctx_s*)ctx;
    if (!c) return PGM_EINVAL;
    if (repeats < 1 || repeats > 1000) return fail(c, PGM_EINVAL, "repeats must be within 1..1000");
    if (c->prof) return fail(c, PGM_EINVAL, "tuning times the calls itself: turn profiling off first");
    const hipStream_t s = (hipStream_t)stream;
    PGM_HIP(c, hipSetDevice(c->device));
    static const int cand[] = {PGM_SCHED_AUTO,
                               PGM_SCHED_LEVEL_LDS,
                               PGM_SCHED_LEVEL_LAUNCHES,
                               PGM_SCHED_SEPARATE,
                               PGM_SCHED_LEVEL_LDS | PGM_SCHED_SEPARATE,
                               PGM_SCHED_LEVEL_LAUNCHES | PGM_SCHED_SEPARATE};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    PGM_HIP(c, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(c, PGM_EDEVICE, "hipEventCreate failed");
    }
    const int saved = c->sched;
    int best = PGM_SCHED_AUTO;
    float best_ms = 0.0f;
    pgm_status st = PGM_OK;
    for (int f : cand) {
        c->sched = f;
        // one untimed call, then the timed ones
        for (int k = 0; k <= repeats && st == PGM_OK; k++) {
            if (k == 1 && hipEventRecord(e0, s) != hipSuccess) st = fail(c, PGM_EDEVICE, "hipEventRecord failed");
            if (st == PGM_OK)
                st = match_impl(c, p, n_pairs, img1, img2, w, h, pitch_bytes, image_stride_bytes, out_fwd, out_bwd,
                                out_n_inliers, out_compact, nullptr, s, c->ws, c->ws_bytes);
        }
        float ms = 0.0f;
        if (st == PGM_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                             hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            st = fail(c, PGM_EDEVICE, "timing the candidate schedule failed");
        if (st != PGM_OK) break;
        if (f == cand[0] || ms < best_ms) {
            best = f;
            best_ms = ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->sched = st == PGM_OK ? best : saved;
    c->gkey.clear();
    if (st == PGM_OK && host_flags) *host_flags = best;
    return st;
}

static pgm_status groups_eager(pgm_ctx_s* c, int32_t n_groups, const pgm_group* gr, const size_t* off,
                               uint64_t* out_n_evals, hipStream_t s)
{
    const int ns = n_groups < pgm_ctx_s::NSTREAMS ? n_groups : pgm_ctx_s::NSTREAMS;
    PGM_HIP(c, hipEventRecord(c->fork, s));
    for (int i = 0; i < ns; i++) PGM_HIP(c, hipStreamWaitEvent(c->gs[i], c->fork, 0));
    for (int g = 0; g < n_groups; g++) {
        const pgm_group& G = gr[g];
        const size_t end = g + 1 < n_groups ? off[g + 1] : c->ws_bytes;
        c->concurrent = n_groups > 1;
        const pgm_status st = match_impl(c, G.params, G.n_pairs, G.img1, G.img2, G.w, G.h, G.pitch_bytes,
                                         G.image_stride_bytes, G.out_fwd, G.out_bwd, G.out_n_inliers, G.out_compact,
                                         out_n_evals, c->gs[g % ns], c->ws + off[g], end - off[g]);
        c->concurrent = false;
        if (st) return st;
    }
    for (int i = 0; i < ns; i++) {
        PGM_HIP(c, hipEventRecord(c->join[i], c->gs[i]));
        PGM_HIP(c, hipStreamWaitEvent(s, c->join[i], 0));
    }
    return PGM_OK;
}

pgm_status pgm_match_groups(void* ctx, int32_t n_groups, const pgm_group* groups, uint64_t* out_n_evals,
                            int32_t use_graph, void* stream)
{
    pgm_ctx_s* c = (pgm_ctx_s*)ctx;
    if (!c) return PGM_EINVAL;
    if (n_groups < 1 || !groups) return fail(c, PGM_EINVAL, "n_groups must be at least 1 and groups not null");
    if (use_graph != 0 && use_graph != 1) return fail(c, PGM_EINVAL, "use_graph must be 0 or 1");
    // every group's checks first, then the workspace split (no device work before both pass)
    std::vector<size_t> off(n_groups);
    size_t cur = 0;
    for (int g = 0; g < n_groups; g++) {
        const pgm_group& G = groups[g];
        if (!G.params) return fail(c, PGM_EINVAL, "group " + std::to_string(g) + ": params is null");
        Layout Y;
        if (pgm_status st = check_batch(c, G.params, G.n_pairs, G.img1, G.img2, G.w, G.h, G.pitch_bytes,
                                        G.image_stride_bytes, G.out_fwd, Y))
            return fail(c, st, "group " + std::to_string(g) + ": " + c->err);
        off[g] = cur;
        cur += (Y.shared_bytes + (size_t)G.n_pairs * Y.pair_bytes + 255) & ~(size_t)255;
    }
    if (cur > c->ws_bytes)
        return fail(c, PGM_ENOMEM, "workspace of " + std::to_string(c->ws_bytes) + " bytes is smaller than the " +
                                       std::to_string(cur) + " bytes these groups need");
    PGM_HIP(c, hipSetDevice(c->device));
    if (!c->fork) {
        for (int i = 0; i < pgm_ctx_s::NSTREAMS; i++) {
            PGM_HIP(c, hipStreamCreateWithFlags(&c->gs[i], hipStreamNonBlocking));
            PGM_HIP(c, hipEventCreateWithFlags(&c->join[i], hipEventDisableTiming));
        }
        PGM_HIP(c, hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
        PGM_HIP(c, hipEventCreateWithFlags(&c->fork, hipEventDisableTiming));
    }
    hipStream_t s = (hipStream_t)stream;
    if (!use_graph || c->prof) return groups_eager(c, n_groups, groups, off.data(), out_n_evals, s);

    // the graph is reused while every argument (parameter values included) is the same
    std::string key((const char*)&out_n_evals, sizeof out_n_evals);
    for (int g = 0; g < n_groups; g++) {
        key.append((const char*)&groups[g], sizeof(pgm_group));
        key.append((const char*)groups[g].params, sizeof(pgm_params));
    }
    if (!c->gexec || key != c->gkey) {
        if (c->gexec) {
            (void)hipGraphExecDestroy(c->gexec);
            c->gexec = nullptr;
            c->gkey.clear();
        }
        PGM_HIP(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
        const long long launches0 = c->nlaunch;
        pgm_status st = groups_eager(c, n_groups, groups, off.data(), out_n_evals, c->cap);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(c->cap, &graph);
        if (st != PGM_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (e != hipSuccess) return fail(c, PGM_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        // every launch must have become a kernel node of the graph
        size_t nn = 0;
        e = hipGraphGetNodes(graph, nullptr, &nn);
        std::vector<hipGraphNode_t> nodes(nn);
        if (e == hipSuccess && nn) e = hipGraphGetNodes(graph, nodes.data(), &nn);
        long long kernels = 0;
        for (size_t i = 0; e == hipSuccess && i < nn; i++) {
            hipGraphNodeType t;
            e = hipGraphNodeGetType(nodes[i], &t);
            if (e == hipSuccess && t == hipGraphNodeTypeKernel) kernels++;
        }
        if (e != hipSuccess || kernels != c->nlaunch - launches0) {
            (void)hipGraphDestroy(graph);
            return fail(c, PGM_EDEVICE, "graph capture recorded " + std::to_string(kernels) + " kernel nodes of " +
                                            std::to_string(nn) + " for " + std::to_string(c->nlaunch - launches0) +
                                            " launches" + (e != hipSuccess ? std::string(": ") + hipGetErrorString(e) : ""));
        }
        e = hipGraphInstantiate(&c->gexec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            c->gexec = nullptr;
            return fail(c, PGM_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        }
        c->gkey = key;
    }
    PGM_HIP(c, hipGraphLaunch(c->gexec, s));
    c->last_stream = s;
    return PGM_OK;
}

// ---------------------------------------------------------------------------------------
// Request server: continuous admission of single pairs of any size (see pgm.h)
// ---------------------------------------------------------------------------------------

struct pgm_server_s {
    pgm_ctx_s* c = nullptr;                       // its workspace is the memory pool
    std::map<size_t, size_t> free_;               // free pool blocks: offset -> bytes
    std::vector<hipStream_t> streams;
    std::vector<int> load;                        // launch sequences in flight per stream
    std::vector<hipEvent_t> spare;                // events not in use (completion and submission)
    int max_queued = 0;                           // submissions beyond this return PGM_EBUSY
    int max_batch = 1;                            // requests that may share one launch sequence
    int max_running = 2;                          // launch sequences in flight (2 per stream)
    long long n_batches = 0, n_started = 0;       // launch sequences and requests started
    size_t in_use = 0;                            // pool bytes held by launch sequences
    struct Req {
        pgm_params p;
        const uint8_t* img1;
        const uint8_t* img2;
        int32_t w, h, pitch;
        pgm_match_t* out_fwd;
        pgm_match_t* out_bwd;
        int32_t* out_n_inliers;
        pgm_match_t* out_compact;
        uint64_t* out_n_evals;
        uint64_t tag;
        size_t need;        // workspace of the request alone
        hipEvent_t ready;   // recorded on the caller's stream at submission
        std::chrono::steady_clock::time_point t_submit;
    };
    struct Run {            // one launch sequence: one request, or several of the same shape
        std::vector<Req> reqs;
        size_t need, off;
        int stream;
        hipEvent_t done;    // recorded on the server stream after the sequence's launches
        pgm_status status;  // PGM_OK, or the error that stopped the launches
    };
    std::deque<Req> queued;
    std::vector<Run> running;
    std::deque<std::pair<uint64_t, pgm_status>> finished;

    hipError_t take_event(hipEvent_t* ev)
    {
        if (spare.empty()) {
            hipEvent_t e;
            hipError_t err = hipEventCreateWithFlags(&e, hipEventDisableTiming);
            if (err != hipSuccess) return err;
            spare.push_back(e);
        }
        *ev = spare.back();
        spare.pop_back();
        return hipSuccess;
    }
    bool alloc(size_t need, size_t& off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < need) continue;
            off = it->first;
            const size_t rest = it->second - need;
            free_.erase(it);
            if (rest) free_[off + need] = rest;
            in_use += need;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        in_use -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

// Requests share a launch sequence when they have the same size, pitch and parameters (so the
// same random numbers) and ask for the same outputs; each pair's buffers then come from the
// batch's pointer table, and its results equal those of pgm_match on that pair alone.
static bool same_shape(const pgm_server_s::Req& a, const pgm_server_s::Req& b)
{
    return a.w == b.w && a.h == b.h && a.pitch == b.pitch && memcmp(&a.p, &b.p, sizeof a.p) == 0 &&
           !a.out_bwd == !b.out_bwd && !a.out_n_inliers == !b.out_n_inliers && !a.out_compact == !b.out_compact &&
           !a.out_n_evals == !b.out_n_evals;
}

// Start queued requests, oldest first, while fewer than max_running launch sequences are in
// flight and the head fits in the pool: the head together with up to max_batch - 1 later
// requests of its shape, as many as the free memory holds (at least the head). Submission
// starts a request only when no sequence is in flight, polling up to two per stream: a burst
// of submissions or arrivals while the GPU is busy gather in the queue, and then start in
// batches whose launch costs they share (issuing a sequence's ~40 launches costs the host
// about as much as the GPU spends on a pair, so eager one-by-one starts at submission would
// keep the queue from ever forming). A started sequence waits for the submission events of its requests (the
// callers' streams at submit time). A sequence whose launches fail part-way is still tracked
// until its stream passes its completion event, so that its memory is not handed out while
// launches may still use it; its requests are then reported with the error status.
static pgm_status server_admit(pgm_server_s* S, int max_running)
{
    pgm_ctx_s* c = S->c;
    while (!S->queued.empty() && (int)S->running.size() < max_running) {
        const pgm_server_s::Req& head = S->queued.front();
        std::vector<size_t> pick(1, 0);
        for (size_t k = 1; k < S->queued.size() && (int)pick.size() < S->max_batch; k++)
            if (same_shape(head, S->queued[k])) pick.push_back(k);
        Layout Y;
        plan(&head.p, head.w, head.h, Y);
        size_t n = pick.size(), off = 0, need = 0;
        for (; n > 0; n--) {
            need = n == 1 ? head.need : ((Y.shared_bytes + n * Y.pair_bytes + 255) & ~(size_t)255);
            if (S->alloc(need, off)) break;
        }
        if (n == 0) break;
        pgm_server_s::Run r;
        r.need = need;
        r.off = off;
        r.status = PGM_OK;
        for (size_t k = 0; k < n; k++) r.reqs.push_back(S->queued[pick[k]]);
        for (size_t k = n; k-- > 0;) S->queued.erase(S->queued.begin() + (long)pick[k]);
        int q = 0;
        for (int i = 1; i < (int)S->streams.size(); i++)
            if (S->load[i] < S->load[q]) q = i;
        r.stream = q;
        hipError_t e = S->take_event(&r.done);
        if (e != hipSuccess) {
            // nothing launched: back to the head of the queue, in order
            for (size_t k = n; k-- > 0;) S->queued.push_front(r.reqs[k]);
            S->release(off, need);
            return fail(c, PGM_EDEVICE, std::string("hipEventCreate: ") + hipGetErrorString(e));
        }
        const hipStream_t st = S->streams[q];
        for (const auto& rq : r.reqs) {
            e = hipStreamWaitEvent(st, rq.ready, 0);
            if (e != hipSuccess && r.status == PGM_OK)
                r.status = fail(c, PGM_EDEVICE, std::string("hipStreamWaitEvent: ") + hipGetErrorString(e));
        }
        const pgm_server_s::Req& h0 = r.reqs[0];
        if (r.status == PGM_OK) {
            if (n == 1) {
                r.status = match_impl(c, &h0.p, 1, h0.img1, h0.img2, h0.w, h0.h, h0.pitch, 0, h0.out_fwd, h0.out_bwd,
                                      h0.out_n_inliers, h0.out_compact, h0.out_n_evals, st, c->ws + off, need);
            } else {
                PairTab tab[TAB_MAX];
                for (size_t k = 0; k < n; k++) {
                    const pgm_server_s::Req& q2 = r.reqs[k];
                    tab[k].img[0] = q2.img1;
                    tab[k].img[1] = q2.img2;
                    tab[k].out[0] = q2.out_fwd;
                    tab[k].out[1] = q2.out_bwd;
                    tab[k].compact = q2.out_compact;
                    tab[k].n_in = q2.out_n_inliers;
                    tab[k].n_evals = (unsigned long long*)q2.out_n_evals;
                    tab[k].unused = nullptr;
                }
                r.status = match_impl(c, &h0.p, (int32_t)n, h0.img1, h0.img2, h0.w, h0.h, h0.pitch, 0, h0.out_fwd,
                                      h0.out_bwd, h0.out_n_inliers, h0.out_compact, nullptr, st, c->ws + off, need,
                                      tab);
            }
        }
        S->n_batches++;
        S->n_started += (long long)n;
        pgm_log(2, "server: started %zu request(s) of %dx%d on stream %d (tag %llu first); pool in use %zu of %zu bytes",
                n, h0.w, h0.h, q, (unsigned long long)h0.tag, S->in_use, c->ws_bytes & ~(size_t)255);
        e = hipEventRecord(r.done, st);
        if (e != hipSuccess) {
            // without a completion event, wait for the stream before the memory is reused
            (void)hipStreamSynchronize(st);
            S->release(off, need);
            S->spare.push_back(r.done);
            for (const auto& rq : r.reqs) {
                S->spare.push_back(rq.ready);
                S->finished.emplace_back(rq.tag, r.status != PGM_OK ? r.status : PGM_EDEVICE);
            }
            return fail(c, PGM_EDEVICE, std::string("hipEventRecord: ") + hipGetErrorString(e));
        }
        S->load[q]++;
        S->running.push_back(std::move(r));
    }
    return PGM_OK;
}

// move finished requests to the finished list (wait for them all when `wait`)
static pgm_status server_reap(pgm_server_s* S, bool wait)
{
    pgm_ctx_s* c = S->c;
    for (size_t i = 0; i < S->running.size();) {
        pgm_server_s::Run& r = S->running[i];
        hipError_t e = wait ? hipEventSynchronize(r.done) : hipEventQuery(r.done);
        if (e == hipErrorNotReady) {
            i++;
            continue;
        }
        if (e != hipSuccess) return fail(c, PGM_EDEVICE, std::string("request: ") + hipGetErrorString(e));
        S->release(r.off, r.need);
        S->spare.push_back(r.done);
        const auto now = std::chrono::steady_clock::now();
        for (const auto& rq : r.reqs) {
            S->spare.push_back(rq.ready);
            S->finished.emplace_back(rq.tag, r.status);
            pgm_log(2, "server: request tag %llu (%dx%d) finished, status %d, %.3f ms after submission",
                    (unsigned long long)rq.tag, rq.w, rq.h, (int)r.status,
                    std::chrono::duration<double, std::milli>(now - rq.t_submit).count());
        }
        S->load[r.stream]--;
        S->running.erase(S->running.begin() + (long)i);
    }
    return PGM_OK;
}

pgm_status pgm_server_create(int32_t device, uint64_t pool_bytes, int32_t n_streams, int32_t max_queued,
                             int32_t max_batch, void** out_server)
{
    if (!out_server) return fail(nullptr, PGM_EINVAL, "out_server is null");
    *out_server = nullptr;
    if (n_streams < 1 || n_streams > 16) return fail(nullptr, PGM_EINVAL, "n_streams must be in 1..16");
    if (max_queued < 0) return fail(nullptr, PGM_EINVAL, "max_queued must not be negative");
    if (max_batch < 0 || max_batch > TAB_MAX) return fail(nullptr, PGM_EINVAL, "max_batch must be in 0..16");
    void* ctx = nullptr;
    pgm_status st = pgm_create(device, pool_bytes, &ctx);
    if (st != PGM_OK) return st;
    pgm_server_s* S = new pgm_server_s();
    S->c = (pgm_ctx_s*)ctx;
    S->c->concurrent = true;
    S->max_queued = max_queued ? max_queued : 4096;
    S->max_batch = max_batch ? max_batch : TAB_MAX;
    S->max_running = 2 * n_streams;
    pgm_log(2, "server on device %d: pool %zu bytes, %d streams, queue %d, batches of up to %d", device,
            S->c->ws_bytes, n_streams, S->max_queued, S->max_batch);
    S->free_[0] = S->c->ws_bytes & ~(size_t)255;
    for (int i = 0; i < n_streams; i++) {
        hipStream_t q;
        hipError_t e = hipStreamCreateWithFlags(&q, hipStreamNonBlocking);
        if (e != hipSuccess) {
            for (hipStream_t x : S->streams) (void)hipStreamDestroy(x);
            pgm_destroy(ctx);
            delete S;
            return fail(nullptr, PGM_EDEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
        }
        S->streams.push_back(q);
        S->load.push_back(0);
    }
    *out_server = S;
    return PGM_OK;
}

pgm_status pgm_server_submit(void* server, const pgm_params* p, const uint8_t* img1, const uint8_t* img2,
                             int32_t w, int32_t h, int32_t pitch_bytes, pgm_match_t* out_fwd,
                             pgm_match_t* out_bwd, int32_t* out_n_inliers, pgm_match_t* out_compact,
                             uint64_t* out_n_evals, uint64_t tag, void* stream)
{
    pgm_server_s* S = (pgm_server_s*)server;
    if (!S) return PGM_EINVAL;
    pgm_ctx_s* c = S->c;
    Layout Y;
    if (pgm_status st = check_batch(c, p, 1, img1, img2, w, h, pitch_bytes, 0, out_fwd, Y)) return st;
    pgm_server_s::Req r;
    r.p = *p;
    {   // the padding before rng_seed is zeroed so that equal parameters compare equal bytewise
        const size_t a = offsetof(pgm_params, rs_mode) + sizeof(int32_t);
        memset((unsigned char*)&r.p + a, 0, offsetof(pgm_params, rng_seed) - a);
    }
    r.img1 = img1; r.img2 = img2;
    r.w = w; r.h = h; r.pitch = pitch_bytes;
    r.out_fwd = out_fwd; r.out_bwd = out_bwd; r.out_n_inliers = out_n_inliers; r.out_compact = out_compact;
    r.out_n_evals = out_n_evals;
    r.tag = tag;
    r.need = (Y.shared_bytes + Y.pair_bytes + 255) & ~(size_t)255;
    r.ready = nullptr;
    r.t_submit = std::chrono::steady_clock::now();
    if (r.need > (c->ws_bytes & ~(size_t)255))
        return fail(c, PGM_ENOMEM, "request needs " + std::to_string(r.need) + " bytes, more than the pool");
    PGM_HIP(c, hipSetDevice(c->device));
    if (pgm_status st = server_reap(S, false)) return st;
    if (pgm_status st = server_admit(S, 1)) return st;   // may make room
    if ((int)S->queued.size() >= S->max_queued)
        return fail(c, PGM_EBUSY, "the request queue is full (" + std::to_string(S->max_queued) + " requests)");
    // the request's launches are ordered after the caller's work on `stream` so far
    PGM_HIP(c, S->take_event(&r.ready));
    hipError_t e = hipEventRecord(r.ready, (hipStream_t)stream);
    if (e != hipSuccess) {
        S->spare.push_back(r.ready);
        return fail(c, PGM_EDEVICE, std::string("hipEventRecord: ") + hipGetErrorString(e));
    }
    S->queued.push_back(r);
    return server_admit(S, 1);
}

int32_t pgm_server_poll(void* server, uint64_t* host_tags, int32_t* host_status, int32_t max_tags)
{
    pgm_server_s* S = (pgm_server_s*)server;
    if (!S || max_tags < 0 || (max_tags > 0 && !host_tags)) return PGM_EINVAL;
    if (hipSetDevice(S->c->device) != hipSuccess) return fail(S->c, PGM_EDEVICE, "hipSetDevice failed");
    if (pgm_status st = server_reap(S, false)) return st;
    if (pgm_status st = server_admit(S, S->max_running)) return st;
    int32_t n = 0;
    while (n < max_tags && !S->finished.empty()) {
        host_tags[n] = S->finished.front().first;
        if (host_status) host_status[n] = S->finished.front().second;
        n++;
        S->finished.pop_front();
    }
    return n;
}

pgm_status pgm_server_stats(void* server, int64_t* host_sequences, int64_t* host_started,
                            uint64_t* host_bytes_in_use)
{
    pgm_server_s* S = (pgm_server_s*)server;
    if (!S) return PGM_EINVAL;
    if (host_sequences) *host_sequences = S->n_batches;
    if (host_started) *host_started = S->n_started;
    if (host_bytes_in_use) *host_bytes_in_use = S->in_use;
    return PGM_OK;
}

pgm_status pgm_server_pending(void* server, int32_t* queued, int32_t* running, int32_t* finished)
{
    pgm_server_s* S = (pgm_server_s*)server;
    if (!S) return PGM_EINVAL;
    if (queued) *queued = (int32_t)S->queued.size();
    if (running) *running = (int32_t)S->running.size();
    if (finished) *finished = (int32_t)S->finished.size();
    return PGM_OK;
}

pgm_status pgm_server_drain(void* server)
{
    pgm_server_s* S = (pgm_server_s*)server;
    if (!S) return PGM_EINVAL;
    PGM_HIP(S->c, hipSetDevice(S->c->device));
    while (!S->queued.empty() || !S->running.empty()) {
        if (pgm_status st = server_reap(S, true)) return st;
        if (pgm_status st = server_admit(S, S->max_running)) return st;
    }
    return PGM_OK;
}

const char* pgm_server_last_error(void* server)
{
    pgm_server_s* S = (pgm_server_s*)server;
    return S ? S->c->err.c_str() : g_create_error.c_str();
}

void pgm_server_destroy(void* server)
{
    pgm_server_s* S = (pgm_server_s*)server;
    if (!S) return;
    (void)hipSetDevice(S->c->device);
    for (hipStream_t q : S->streams) (void)hipStreamSynchronize(q);
    for (auto& r : S->running) {
        (void)hipEventDestroy(r.done);
        for (auto& rq : r.reqs) (void)hipEventDestroy(rq.ready);
    }
    for (auto& r : S->queued) (void)hipEventDestroy(r.ready);
    for (hipEvent_t ev : S->spare) (void)hipEventDestroy(ev);
    for (hipStream_t q : S->streams) (void)hipStreamDestroy(q);
    pgm_destroy(S->c);
    delete S;
}

pgm_status pgm_format_matches(const pgm_match_t* host_matches, int64_t n, int32_t inliers_only, char* host_buf,
                              uint64_t cap, uint64_t* host_len)
{
    if (!host_len || n < 0 || (n > 0 && !host_matches) || (inliers_only != 0 && inliers_only != 1))
        return PGM_EINVAL;
    std::string out;
    char line[64];
    for (int64_t k = 0; k < n; k++) {
        const pgm_match_t& m = host_matches[k];
        if (inliers_only && !(m.flags & PGM_FLAG_INLIER)) continue;
        const int len = snprintf(line, sizeof line, "%d %d %d %d\n", m.x1, m.y1, m.x2, m.y2);
        out.append(line, (size_t)len);
    }
    *host_len = out.size();
    if (!host_buf) return PGM_OK;
    if (out.size() > cap) return PGM_ENOMEM;
    memcpy(host_buf, out.data(), out.size());
    return PGM_OK;
}

static pgm_status dump_prep(pgm_ctx_s* c, int level)
{
    if (!c) return PGM_EINVAL;
    if (!c->have_last) return fail(c, PGM_EINVAL, "no pgm_match has run on this context");
    if (level < 0 || level >= c->last.L) return fail(c, PGM_EINVAL, "level out of range");
    PGM_HIP(c, hipSetDevice(c->device));
    PGM_HIP(c, hipStreamSynchronize(c->last_stream));
    return PGM_OK;
}

pgm_status pgm_dump_level(void* ctx, int32_t level, int32_t dir, int32_t* host_out)
{
    pgm_ctx_s* c = (pgm_ctx_s*)ctx;
    pgm_status st = dump_prep(c, level);
    if (st != PGM_OK) return st;
    if ((dir != 0 && dir != 1) || !host_out) return fail(c, PGM_EINVAL, "bad dir or null output");
    const Layout& Y = c->last;
    const size_t n = (size_t)Y.lnx[level] * Y.lny[level];
    std::vector<uint64_t> dist(n);
    std::string buf(n * 5, '\0');
    uint32_t* disp = (uint32_t*)&buf[0];
    uint8_t* flags = (uint8_t*)(disp + n);
    PGM_HIP(c, hipMemcpy(disp, c->last_ws + Y.shared_bytes + Y.disp[dir][level], n * 4, hipMemcpyDeviceToHost));
    if (Y.dsize == 8) {
        PGM_HIP(c, hipMemcpy(dist.data(), c->last_ws + Y.shared_bytes + Y.dist[dir][level], n * 8,
                             hipMemcpyDeviceToHost));
    } else {
        std::vector<uint32_t> d32(n);
        PGM_HIP(c, hipMemcpy(d32.data(), c->last_ws + Y.shared_bytes + Y.dist[dir][level], n * 4,
                             hipMemcpyDeviceToHost));
        for (size_t s = 0; s < n; s++) dist[s] = d32[s];
    }
    PGM_HIP(c, hipMemcpy(flags, c->last_ws + Y.shared_bytes + Y.flags[dir][level], n, hipMemcpyDeviceToHost));
    for (size_t s = 0; s < n; s++) {
        const bool init = disp[s] != UNINIT;
        host_out[4 * s + 0] = init ? (int32_t)(int16_t)(disp[s] & 0xFFFF) : 0;
        host_out[4 * s + 1] = init ? (int32_t)(int16_t)(disp[s] >> 16) : 0;
        // squared distances above the int32 range report its largest value below NO_DIST
        host_out[4 * s + 2] = init ? (int32_t)(dist[s] < 0x7FFFFFFEull ? dist[s] : 0x7FFFFFFEull) : (int32_t)NO_DIST;
        host_out[4 * s + 3] = (int32_t)((init ? PGM_FLAG_INIT : 0u) | ((flags[s] & ST_INL) ? PGM_FLAG_INLIER : 0u) |
                                        ((flags[s] & ST_REC) ? PGM_FLAG_RECORD : 0u));
    }
    return PGM_OK;
}

pgm_status pgm_dump_gradient(void* ctx, int32_t level, int32_t image, void* host_out)
{
    pgm_ctx_s* c = (pgm_ctx_s*)ctx;
    pgm_status st = dump_prep(c, level);
    if (st != PGM_OK) return st;
    if (image < 0 || image > 3 || !host_out) return fail(c, PGM_EINVAL, "bad image or null output");
    const Layout& Y = c->last;
    const int w = Y.lw[level], h = Y.lh[level], pw = w + 2 * PAD;
    const size_t row = (size_t)w * Y.C2 * Y.esize;
    for (int y = 0; y < h; y++) {
        const uint8_t* src = c->last_ws + Y.shared_bytes + Y.grad[image][level] + (((size_t)(y + PAD) * pw + PAD) * Y.C2) * Y.esize;
        PGM_HIP(c, hipMemcpy((uint8_t*)host_out + y * row, src, row, hipMemcpyDeviceToHost));
    }
    if (!Y.f32) {
        uint16_t* v = (uint16_t*)host_out;
        for (size_t k = 0; k < (size_t)w * h * Y.C2; k++) v[k] = (uint16_t)((int)v[k] - (int)BIAS);
    }
    return PGM_OK;
}

pgm_status pgm_dump_pyramid(void* ctx, int32_t level, int32_t image, uint8_t* host_out)
{
    pgm_ctx_s* c = (pgm_ctx_s*)ctx;
    pgm_status st = dump_prep(c, level);
    if (st != PGM_OK) return st;
    if ((image != 0 && image != 1) || !host_out) return fail(c, PGM_EINVAL, "bad image or null output");
    const Layout& Y = c->last;
    const int w = Y.lw[level], h = Y.lh[level];
    if (level == 0) {
        PGM_HIP(c, hipMemcpy2D(host_out, (size_t)w * 3, c->last_img[image], c->last_pitch, (size_t)w * 3, h,
                               hipMemcpyDeviceToHost));
    } else {
        PGM_HIP(c, hipMemcpy(host_out, c->last_ws + Y.shared_bytes + Y.pyr[image][level], (size_t)w * h * 3, hipMemcpyDeviceToHost));
    }
    return PGM_OK;
}

pgm_status pgm_schedule(void* ctx, int32_t flags)
{
    pgm_ctx_s* c = (pgm_ctx_s*)ctx;
    if (!c) return PGM_EINVAL;
    const int known = PGM_SCHED_LEVEL_LDS | PGM_SCHED_LEVEL_LAUNCHES | PGM_SCHED_SEPARATE;
    if (flags & ~known) return fail(c, PGM_EINVAL, "unknown schedule bits");
    if ((flags & PGM_SCHED_LEVEL_LDS) && (flags & PGM_SCHED_LEVEL_LAUNCHES))
        return fail(c, PGM_EINVAL, "small levels cannot be both in LDS and launches");
    c->sched = flags;
    c->gkey.clear();   // a captured graph holds the old schedule
    return PGM_OK;
}

pgm_status pgm_profile(void* ctx, int32_t enable)
{
    pgm_ctx_s* c = (pgm_ctx_s*)ctx;
    if (!c || (enable != 0 && enable != 1)) return PGM_EINVAL;
    PGM_HIP(c, hipSetDevice(c->device));
    if (enable) {
        PGM_HIP(c, hipDeviceSynchronize());
        PGM_HIP(c, hipMemset(c->prof_evals, 0, PGM_K_KINDS * sizeof(unsigned long long)));
        c->recs.clear();
        c->run_open = false;
        c->next_event = 0;
    }
    c->prof = enable != 0;
    return PGM_OK;
}

pgm_status pgm_profile_read(void* ctx, int32_t kind, int64_t* host_launches, double* host_total_ms,
                            uint64_t* host_evals)
{
    pgm_ctx_s* c = (pgm_ctx_s*)ctx;
    if (!c || kind < 0 || kind >= PGM_K_KINDS) return PGM_EINVAL;
    PGM_HIP(c, hipSetDevice(c->device));
    PGM_HIP(c, hipDeviceSynchronize());
    int64_t n = 0;
    double ms = 0.0;
    for (const pgm_ctx_s::Rec& r : c->recs) {
        if (r.kind != kind) continue;
        float t = 0.0f;
        PGM_HIP(c, hipEventElapsedTime(&t, r.a, r.b));
        ms += t;
        n += r.n;
    }
    unsigned long long ev[PGM_K_KINDS];
    PGM_HIP(c, hipMemcpy(ev, c->prof_evals, sizeof ev, hipMemcpyDeviceToHost));
    if (host_launches) *host_launches = n;
    if (host_total_ms) *host_total_ms = ms;
    if (host_evals) *host_evals = ev[kind];
    return PGM_OK;
}

}  // extern "C"
