/*
 * pgm_oracle.c -- CPU oracle for pyramidal gradient matching
 * (Y. Li, "Pyramidal Gradient Matching for Optical Flow Estimation", arXiv:1704.03217).
 *
 * TEST INFRASTRUCTURE ONLY: a plain, slow, single-threaded C implementation that the tests,
 * the smoke check and the benchmark's CPU-baseline leg compare the GPU library against. It
 * shares no code with the GPU library. It follows the paper's steps in the paper's order;
 * each function names the passage it implements. Points the paper leaves open are marked
 * READING and take one fixed interpretation (listed with the design notes of the project).
 *
 * Parity status per part: pinned by independent tests (brute force, closed forms, library
 * routines, invariants). The sequential scan schedule, for which the paper prints no worked
 * example, is pinned by invariants and by a hand-worked one-pass case.
 */
#include "pgm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------------------- */
/* Small helpers                                                                          */
/* ------------------------------------------------------------------------------------- */

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* READING (filters at the border): reflect-101, i.e. -1 -> 1 and n -> n-2. */
int pgmo_reflect101(int i, int n)
{
    if (n == 1) return 0;
    while (i < 0 || i >= n) {
        if (i < 0) i = -i;
        if (i >= n) i = 2 * (n - 1) - i;
    }
    return i;
}

/* ------------------------------------------------------------------------------------- */
/* Image pyramid (Sec. III-D): L levels with factor s = 1/2.                              */
/* READING: the paper does not name the low-pass filter; a 5x5 binomial [1 4 6 4 1]^2/256 */
/* with round-half-up, sampled at even pixels, level size ceil(w/2) x ceil(h/2).          */
/* ------------------------------------------------------------------------------------- */

static const int BINOM5[5] = {1, 4, 6, 4, 1};

void pgmo_pyr_down(const uint8_t* src, int w, int h, int pitch, int ch, uint8_t* dst)
{
    int w2 = (w + 1) / 2, h2 = (h + 1) / 2;
    for (int y = 0; y < h2; y++)
        for (int x = 0; x < w2; x++)
            for (int c = 0; c < ch; c++) {
                int sum = 0;
                for (int i = 0; i < 5; i++)
                    for (int j = 0; j < 5; j++) {
                        int sy = pgmo_reflect101(2 * y + i - 2, h);
                        int sx = pgmo_reflect101(2 * x + j - 2, w);
                        sum += BINOM5[i] * BINOM5[j] * src[(size_t)sy * pitch + (size_t)sx * ch + c];
                    }
                dst[((size_t)y * w2 + x) * ch + c] = (uint8_t)((sum + 128) >> 8);
            }
}

/* READING (PGM-G, Sec. III-F, gray image): integer BT.601 luma. */
void pgmo_gray(const uint8_t* rgb, int w, int h, int pitch, uint8_t* y)
{
    for (int r = 0; r < h; r++)
        for (int x = 0; x < w; x++) {
            const uint8_t* p = rgb + (size_t)r * pitch + (size_t)x * 3;
            y[(size_t)r * w + x] = (uint8_t)((77 * p[0] + 150 * p[1] + 29 * p[2] + 128) >> 8);
        }
}

/* ------------------------------------------------------------------------------------- */
/* Gradient image (Sec. III-A, Eq. 1-2).                                                  */
/* Gx = Kx(S) * I and Gy = Ky(S) * I per channel; G(p) = [Gx(p), Gy(p)].                   */
/* READING: Sobel kernels of size S are the outer product of the binomial smoothing taps  */
/* and the binomial derivative taps (S=3: [1 2 1] x [-1 0 1]; S=5: [1 4 6 4 1] x          */
/* [-1 -2 0 2 1]), applied as a correlation so that Gx > 0 where intensity rises with x.  */
/* The patch distance is invariant to the global sign. Borders use reflect-101.           */
/* ------------------------------------------------------------------------------------- */

static void sobel_taps(int ksize, const int** sm, const int** dv)
{
    static const int SM3[3] = {1, 2, 1}, DV3[3] = {-1, 0, 1};
    static const int SM5[5] = {1, 4, 6, 4, 1}, DV5[5] = {-1, -2, 0, 2, 1};
    if (ksize == 3) { *sm = SM3; *dv = DV3; }
    else { *sm = SM5; *dv = DV5; }
}

void pgmo_gradient_image(const uint8_t* img, int w, int h, int pitch, int ch, int ksize, int16_t* G)
{
    const int *sm, *dv;
    sobel_taps(ksize, &sm, &dv);
    int k = ksize / 2;
    for (int y = 0; y < h; y++)
        for (int x = 0; x < w; x++)
            for (int c = 0; c < ch; c++) {
                int gx = 0, gy = 0;
                for (int i = 0; i < ksize; i++)
                    for (int j = 0; j < ksize; j++) {
                        int sy = pgmo_reflect101(y + i - k, h);
                        int sx = pgmo_reflect101(x + j - k, w);
                        int v = img[(size_t)sy * pitch + (size_t)sx * ch + c];
                        gx += sm[i] * dv[j] * v;   /* rows smoothed, columns differentiated */
                        gy += dv[i] * sm[j] * v;   /* rows differentiated, columns smoothed */
                    }
                G[((size_t)y * w + x) * 2 * ch + c] = (int16_t)gx;
                G[((size_t)y * w + x) * 2 * ch + ch + c] = (int16_t)gy;
            }
}

/* Direction-only gradient image (Sec. III-F, PGM-CD / PGM-GD).
 * READING: each channel's gradient vector (Gx_c, Gy_c) divided by its Euclidean length,
 * a zero vector staying zero; computed in double and rounded once to float. */
void pgmo_direction(const int16_t* G, int npix, int ch, float* U)
{
    for (int p = 0; p < npix; p++)
        for (int c = 0; c < ch; c++) {
            int gx = G[(size_t)p * 2 * ch + c], gy = G[(size_t)p * 2 * ch + ch + c];
            float ux = 0.0f, uy = 0.0f;
            if (gx != 0 || gy != 0) {
                double n = sqrt((double)gx * gx + (double)gy * gy);
                ux = (float)(gx / n);
                uy = (float)(gy / n);
            }
            U[(size_t)p * 2 * ch + c] = ux;
            U[(size_t)p * 2 * ch + ch + c] = uy;
        }
}

/* ------------------------------------------------------------------------------------- */
/* Patch distance (Sec. III-B, Eq. 3).                                                    */
/* READING: absolute differences summed over the patch and channels by default (the paper */
/* squares them: PGMO_METRIC_SSD); patch offsets [-floor(P/2), ceil(P/2)-1] so that even */
/* sides work; pixels outside the image take the nearest edge pixel.                      */
/* ------------------------------------------------------------------------------------- */

int64_t pgmo_dist_i16(const int16_t* Ga, const int16_t* Gb, int w, int h, int C2, int P,
                      int xa, int ya, int xb, int yb)
{
    int lo = -(P / 2), hi = (P + 1) / 2 - 1;
    int64_t s = 0;
    for (int oy = lo; oy <= hi; oy++)
        for (int ox = lo; ox <= hi; ox++) {
            size_t ia = ((size_t)clampi(ya + oy, 0, h - 1) * w + clampi(xa + ox, 0, w - 1)) * C2;
            size_t ib = ((size_t)clampi(yb + oy, 0, h - 1) * w + clampi(xb + ox, 0, w - 1)) * C2;
            for (int c = 0; c < C2; c++) s += labs((long)Ga[ia + c] - (long)Gb[ib + c]);
        }
    return s;
}

/* Colour spaces of the two gradient pyramids (Sec. III-E, Table II). READING, YCrCb: integer
 * BT.601 full range, Y = (77 R + 150 G + 29 B + 128) >> 8, Cr = 128 + floor((R - Y) 183 / 256
 * + 1/2), Cb = 128 + floor((B - Y) 144 / 256 + 1/2), clamped to [0, 255], stored (Y, Cr, Cb).
 * READING, CIELab: sRGB (IEC 61966-2-1 transfer curve) to linear, the sRGB / D65 matrix to
 * XYZ, Lab with the D65 white (0.95047, 1, 1.08883), stored as 8-bit (L* 255/100, a* + 128,
 * b* + 128) rounded half up and clamped. The powers are computed with plain IEEE double
 * operations only: u^2.4 = u^2 (u^2)^(1/5) by 40 Newton steps from 1 and t^(1/3) by 20, so
 * the result is a fixed function of the input bits. */
static double root_n(double a, int n, int steps)
{
    double y = 1.0;
    for (int k = 0; k < steps; k++) {
        double p = y;
        for (int m = 2; m < n; m++) p = p * y;        /* y^(n-1) */
        y = y - (p * y - a) / ((double)n * p);
    }
    return y;
}

static double srgb_linear(int c)
{
    double v = (double)c / 255.0;
    if (v <= 0.04045) return v / 12.92;
    double u = (v + 0.055) / 1.055;
    double u2 = u * u;
    return u2 * root_n(u2, 5, 40);
}

static double lab_f(double t)
{
    const double e = (6.0 / 29.0) * (6.0 / 29.0) * (6.0 / 29.0);
    if (t > e) return root_n(t, 3, 20);
    return t / (3.0 * (6.0 / 29.0) * (6.0 / 29.0)) + 4.0 / 29.0;
}

static uint8_t to_u8(double x)
{
    double r = floor(x + 0.5);
    return (uint8_t)(r < 0.0 ? 0.0 : (r > 255.0 ? 255.0 : r));
}

void pgmo_convert(const uint8_t* rgb, int npx, int space, uint8_t* out)
{
    double lin[256];
    if (space == PGMO_SPACE_LAB)
        for (int c = 0; c < 256; c++) lin[c] = srgb_linear(c);
    for (int k = 0; k < npx; k++) {
        const int R = rgb[3 * k], G = rgb[3 * k + 1], B = rgb[3 * k + 2];
        uint8_t* o = out + 3 * k;
        if (space == PGMO_SPACE_YCRCB) {
            const int Y = (77 * R + 150 * G + 29 * B + 128) >> 8;
            const int cr = ((R - Y) * 183 + 32768 + 128), cb = ((B - Y) * 144 + 32768 + 128);
            o[0] = (uint8_t)Y;
            o[1] = (uint8_t)(cr < 0 ? 0 : (cr >> 8 > 255 ? 255 : cr >> 8));
            o[2] = (uint8_t)(cb < 0 ? 0 : (cb >> 8 > 255 ? 255 : cb >> 8));
        } else if (space == PGMO_SPACE_LAB) {
            const double r = lin[R], g = lin[G], b = lin[B];
            const double X = 0.4124564 * r + 0.3575761 * g + 0.1804375 * b;
            const double Yv = 0.2126729 * r + 0.7151522 * g + 0.0721750 * b;
            const double Z = 0.0193339 * r + 0.1191920 * g + 0.9503041 * b;
            const double fx = lab_f(X / 0.95047), fy = lab_f(Yv), fz = lab_f(Z / 1.08883);
            o[0] = to_u8((116.0 * fy - 16.0) * 2.55);
            o[1] = to_u8(500.0 * (fx - fy) + 128.0);
            o[2] = to_u8(200.0 * (fy - fz) + 128.0);
        } else {
            o[0] = (uint8_t)R; o[1] = (uint8_t)G; o[2] = (uint8_t)B;
        }
    }
}

/* Sec. III-F, "G./|G|" read literally: the element-wise division of G by |G| leaves the
 * sign of every gradient component; a zero component stays zero (0/0 taken as 0). */
void pgmo_sign(int16_t* G, int n)
{
    for (int k = 0; k < n; k++) G[k] = (int16_t)(G[k] > 0 ? 1 : (G[k] < 0 ? -1 : 0));
}

/* Eq. 3 read literally (the squared metric, PGMO_METRIC_SSD): the squared differences of
 * integer features summed exactly in 64 bits (at most 16*16*6 terms of 48960^2 < 2^42). */
int64_t pgmo_ssd_i16(const int16_t* Ga, const int16_t* Gb, int w, int h, int C2, int P,
                     int xa, int ya, int xb, int yb)
{
    int lo = -(P / 2), hi = (P + 1) / 2 - 1;
    int64_t s = 0;
    for (int oy = lo; oy <= hi; oy++)
        for (int ox = lo; ox <= hi; ox++) {
            size_t ia = ((size_t)clampi(ya + oy, 0, h - 1) * w + clampi(xa + ox, 0, w - 1)) * C2;
            size_t ib = ((size_t)clampi(yb + oy, 0, h - 1) * w + clampi(xb + ox, 0, w - 1)) * C2;
            for (int c = 0; c < C2; c++) {
                int64_t d = (int64_t)Ga[ia + c] - (int64_t)Gb[ib + c];
                s += d * d;
            }
        }
    return s;
}

/* The float features are unit-vector components: zero or of magnitude >= 2^-14 (the
 * gradient is at most 12240 for S <= 5), hence multiples of 2^-37 in [-1, 1]. Their
 * differences and the sum of up to 16*16*6 of them are therefore exact in double, so this
 * is the exact sum of absolute differences, rounded once to float. */
float pgmo_dist_f32(const float* Ua, const float* Ub, int w, int h, int C2, int P,
                    int xa, int ya, int xb, int yb)
{
    int lo = -(P / 2), hi = (P + 1) / 2 - 1;
    double s = 0.0;
    for (int oy = lo; oy <= hi; oy++)
        for (int ox = lo; ox <= hi; ox++) {
            size_t ia = ((size_t)clampi(ya + oy, 0, h - 1) * w + clampi(xa + ox, 0, w - 1)) * C2;
            size_t ib = ((size_t)clampi(yb + oy, 0, h - 1) * w + clampi(xb + ox, 0, w - 1)) * C2;
            for (int c = 0; c < C2; c++) s += fabs((double)Ua[ia + c] - (double)Ub[ib + c]);
        }
    return (float)s;
}

/* ------------------------------------------------------------------------------------- */
/* Random numbers. READING: the paper only asks for uniform random offsets; we use the    */
/* counter-based Philox4x32-10 generator (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds  */
/* of two 32x32->64 multiplications with the round constants 0xD2511F53 and 0xCD9E8D57,   */
/* the word permutation, and a Weyl key schedule 0x9E3779B9, 0xBB67AE85.                  */
/* ------------------------------------------------------------------------------------- */

void pgmo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        uint64_t p0 = (uint64_t)0xD2511F53u * x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Eq. 5: the i-th candidate offset floor(R_i W / 2^i), R_i uniform in [-1, 1].
 * READING: a 32-bit draw u gives R = (2u+1)/2^32 - 1, the midpoint of the u-th of 2^32
 * equal cells of (-1, 1). Every operation below is exact in double for W < 2^20. */
int pgmo_search_offset(uint32_t u, int W, int i)
{
    double R = (2.0 * (double)u + 1.0) / 4294967296.0 - 1.0;
    return (int)floor(R * (double)W / ldexp(1.0, i));
}

/* Eq. 5 read symmetrically (an option): the i-th offset uniform over the integers of
 * [-w_i, w_i] with w_i = floor(W / 2^i), the radius Eq. 5 halves per step. The same exact
 * floor as the initial displacements below, with R = w_i. */
int pgmo_search_offset_sym(uint32_t u, int W, int i)
{
    int wi = W >> i;
    return (int)floor((double)u / 4294967296.0 * (double)(2 * wi + 1)) - wi;
}

/* Random initial displacement component, uniform over the integers of [-R, R]. */
int pgmo_init_offset(uint32_t u, int R)
{
    return (int)floor((double)u / 4294967296.0 * (double)(2 * R + 1)) - R;
}

/* ------------------------------------------------------------------------------------- */
/* Seed grid. READING: the field is kept on a regular grid of spacing `stride` (the       */
/* paper's output grid, Sec. III-G; stride 1 is the paper's dense field), first seed at   */
/* floor(stride/2), the last seed clamped to the image.                                   */
/* ------------------------------------------------------------------------------------- */

int pgmo_grid_count(int n, int stride)
{
    int off = stride / 2;
    if (n - 1 < off) return 1;
    return (n - 1 - off) / stride + 1;
}

int pgmo_grid_pos(int i, int n, int stride)
{
    int p = stride / 2 + i * stride;
    return p < n - 1 ? p : n - 1;
}

/* nearest seed to pixel coordinate x (ties toward the larger index) */
int pgmo_grid_nearest(int x, int nseeds, int stride)
{
    int off = stride / 2;
    int num = 2 * (x - off) + stride;
    int i = num >= 0 ? num / (2 * stride) : -((-num + 2 * stride - 1) / (2 * stride));
    return clampi(i, 0, nseeds - 1);
}

int pgmo_geometry(const pgmo_params* p, int w, int h, int32_t* lw, int32_t* lh, int32_t* lnx, int32_t* lny)
{
    if (p->levels < 1 || p->levels > PGMO_MAX_LEVELS || p->seed_stride < 1 || w < 1 || h < 1) return -1;
    int cw = w, chh = h;
    for (int l = 0; l < p->levels; l++) {
        lw[l] = cw; lh[l] = chh;
        lnx[l] = pgmo_grid_count(cw, p->seed_stride);
        lny[l] = pgmo_grid_count(chh, p->seed_stride);
        cw = (cw + 1) / 2; chh = (chh + 1) / 2;
    }
    return 0;
}

int pgmo_top_radius(const pgmo_params* p, int w, int h)
{
    int tw = w, th = h;
    for (int l = 1; l < p->levels; l++) { tw = (tw + 1) / 2; th = (th + 1) / 2; }
    if (p->max_disp == 0) return tw > th ? tw : th;
    /* READING (batched and served pairs of many sizes): a negative bound -k scales with the
     * image, ceil(w / k) pixels at full resolution */
    int bound = p->max_disp > 0 ? p->max_disp : (w + (-p->max_disp) - 1) / (-p->max_disp);
    int scale = 1 << (p->levels - 1);
    return (bound + scale - 1) / scale;
}

/* ------------------------------------------------------------------------------------- */
/* Correspondence fields                                                                  */
/* ------------------------------------------------------------------------------------- */

typedef struct {
    int w, h, nx, ny, n, stride;
    int C2, P, feature, metric;
    const int16_t *Gi_self, *Gi_other;   /* integer features of this field's two images */
    const float *Gf_self, *Gf_other;     /* float features (direction-only variant)     */
    int32_t *dx, *dy;                    /* displacement F(p) - p                       */
    double* dist;                        /* patch distance of the current match         */
    uint8_t *init, *rec, *inl;           /* initialised, propagated record, O^l (inlier) */
    int rec_valid;                       /* a record was propagated into this visit     */
} field_t;

typedef struct {
    uint32_t key[2];
    uint64_t evals;
    int rs_sym;                          /* offsets of Eq. 5 read symmetrically         */
} run_t;

static double cost(run_t* r, const field_t* f, int xa, int ya, int xb, int yb)
{
    r->evals++;
    if (f->feature != PGMO_FEAT_F32_DIR && f->metric == PGMO_METRIC_SSD)   /* exact: < 2^53 */
        return (double)pgmo_ssd_i16(f->Gi_self, f->Gi_other, f->w, f->h, f->C2, f->P, xa, ya, xb, yb);
    if (f->feature != PGMO_FEAT_F32_DIR)
        return (double)pgmo_dist_i16(f->Gi_self, f->Gi_other, f->w, f->h, f->C2, f->P, xa, ya, xb, yb);
    return (double)pgmo_dist_f32(f->Gf_self, f->Gf_other, f->w, f->h, f->C2, f->P, xa, ya, xb, yb);
}

static void draws(const run_t* r, uint32_t idx, uint32_t word1, uint32_t block, uint32_t stage, uint32_t out[4])
{
    uint32_t ctr[4] = {idx, word1, block, stage};
    pgmo_philox4x32_10(ctr, r->key, out);
}

/* READING (candidate outside the second image): the target is clamped into the image and
 * the clamped displacement is what is stored. */
static void clamp_target(const field_t* f, int px, int py, int* dx, int* dy)
{
    *dx = clampi(px + *dx, 0, f->w - 1) - px;
    *dy = clampi(py + *dy, 0, f->h - 1) - py;
}

/* Offer candidate displacement (cx, cy) to seed s: evaluated unless it equals the current
 * match, adopted if the seed is uninitialised or the distance is strictly smaller (READING:
 * ties keep the earlier member of the candidate set). */
static void offer(run_t* r, field_t* f, int s, int px, int py, int cx, int cy)
{
    if (f->init[s] && cx == f->dx[s] && cy == f->dy[s]) return;
    double e = cost(r, f, px, py, px + cx, py + cy);
    if (!f->init[s] || e < f->dist[s]) {
        f->dx[s] = cx; f->dy[s] = cy; f->dist[s] = e; f->init[s] = 1;
    }
}

/* The FlowFields order of (Delta_x, Delta_y) that the paper adopts (Sec. III-B):
 * ((1,0),(0,1)) -> ((-1,0),(0,-1)) -> ((-1,0),(0,1)) -> ((1,0),(0,-1)), cycling per
 * iteration. Offsets are in seed-grid units. */
static const int DELTA[4][2][2] = {
    {{1, 0}, {0, 1}}, {{-1, 0}, {0, -1}}, {{-1, 0}, {0, 1}}, {{1, 0}, {0, -1}}};

/* One propagation (Eq. 4) followed by one limited random search (Eq. 5) at seed (i, j). */
static void improve_seed(run_t* r, field_t* f, int i, int j, int t, int level, int dir, int stage, int W)
{
    int s = j * f->nx + i;
    int px = pgmo_grid_pos(i, f->w, f->stride), py = pgmo_grid_pos(j, f->h, f->stride);
    int k = t & 3;

    /* Eq. 4: Omega = {F(p), F(p - Delta_x) + Delta_x, F(p - Delta_y) + Delta_y}; a member
     * whose neighbour is uninitialised (or off the grid) is ignored. On the seed grid,
     * F(p - Delta) + Delta is the neighbour's displacement applied at p. */
    for (int m = 0; m < 2; m++) {
        int ni = i - DELTA[k][m][0], nj = j - DELTA[k][m][1];
        if (ni < 0 || nj < 0 || ni >= f->nx || nj >= f->ny) continue;
        int ns = nj * f->nx + ni;
        if (!f->init[ns]) continue;
        int cx = f->dx[ns], cy = f->dy[ns];
        clamp_target(f, px, py, &cx, &cy);
        offer(r, f, s, px, py, cx, cy);
    }
    if (!f->init[s]) return;   /* READING: no search around an uninitialised match */

    /* Eq. 5: Psi = {F(p)} + {F(p) + floor(R_i W / 2^i)}, i = 0..floor(log2 W), all around
     * the match left by the propagation. */
    int cx0 = f->dx[s], cy0 = f->dy[s];
    int nI = 0;
    while ((1 << (nI + 1)) <= W) nI++;
    nI += 1;   /* floor(log2 W) + 1 candidates */
    uint32_t word1 = (uint32_t)t | ((uint32_t)level << 8) | ((uint32_t)dir << 16) | (1u << 24);
    uint32_t u[4];
    for (int ii = 0; ii < nI; ii++) {
        if ((ii & 1) == 0) draws(r, (uint32_t)s, word1, (uint32_t)(ii >> 1), (uint32_t)stage, u);
        uint32_t ux = u[2 * (ii & 1)], uy = u[2 * (ii & 1) + 1];
        int ox = r->rs_sym ? pgmo_search_offset_sym(ux, W, ii) : pgmo_search_offset(ux, W, ii);
        int oy = r->rs_sym ? pgmo_search_offset_sym(uy, W, ii) : pgmo_search_offset(uy, W, ii);
        int cx = cx0 + ox, cy = cy0 + oy;
        clamp_target(f, px, py, &cx, &cy);
        offer(r, f, s, px, py, cx, cy);
    }
}

/* One basic-gradient-matching iteration over the whole field. SYNC: all seeds of colour
 * (i+j) even, then all of colour odd; a seed's four neighbours have the other colour, so
 * each half is order independent. SCAN: one in-place raster pass in the direction of the
 * current Delta, as in the paper's sequential PatchMatch. */
static void iterate(run_t* r, field_t* f, int t, int level, int dir, int stage, int W, int schedule)
{
    if (schedule == PGMO_SYNC) {
        for (int colour = 0; colour < 2; colour++)
            for (int j = 0; j < f->ny; j++)
                for (int i = 0; i < f->nx; i++)
                    if (((i + j) & 1) == colour) improve_seed(r, f, i, j, t, level, dir, stage, W);
    } else {
        int k = t & 3;
        int xup = DELTA[k][0][0] > 0, yup = DELTA[k][1][1] > 0;
        for (int jj = 0; jj < f->ny; jj++) {
            int j = yup ? jj : f->ny - 1 - jj;
            for (int ii = 0; ii < f->nx; ii++) {
                int i = xup ? ii : f->nx - 1 - ii;
                improve_seed(r, f, i, j, t, level, dir, stage, W);
            }
        }
    }
}

/* Initial field at the coarsest level. READING: the paper initialises F^m with a kd-tree
 * approximate nearest-neighbour step; here either uniform random displacements in
 * [-R, R]^2 (the original PatchMatch start) or, as a test reference, the exact best
 * displacement in that window (dy outer, dx inner, strictly smaller wins). */
static void init_field(run_t* r, field_t* f, int level, int dir, int stage, int mode, int R)
{
    for (int j = 0; j < f->ny; j++)
        for (int i = 0; i < f->nx; i++) {
            int s = j * f->nx + i;
            int px = pgmo_grid_pos(i, f->w, f->stride), py = pgmo_grid_pos(j, f->h, f->stride);
            if (mode == PGMO_INIT_RANDOM) {
                uint32_t u[4];
                draws(r, (uint32_t)s, ((uint32_t)level << 8) | ((uint32_t)dir << 16), 0, (uint32_t)stage, u);
                int cx = pgmo_init_offset(u[0], R), cy = pgmo_init_offset(u[1], R);
                clamp_target(f, px, py, &cx, &cy);
                f->dx[s] = cx; f->dy[s] = cy;
                f->dist[s] = cost(r, f, px, py, px + cx, py + cy);
                f->init[s] = 1;
            } else {
                f->init[s] = 0;
                for (int dy = -R; dy <= R; dy++)
                    for (int dx = -R; dx <= R; dx++) {
                        if (px + dx < 0 || px + dx >= f->w || py + dy < 0 || py + dy >= f->h) continue;
                        double e = cost(r, f, px, py, px + dx, py + dy);
                        if (!f->init[s] || e < f->dist[s]) {
                            f->dx[s] = dx; f->dy[s] = dy; f->dist[s] = e; f->init[s] = 1;
                        }
                    }
            }
            f->rec[s] = 0;
            f->inl[s] = 0;
        }
    f->rec_valid = 0;
}

/* Step 4 and 5 toward the finer level k = j-1 (Eq. 6 with eta = s, Eq. 8).
 * READING: the child at pixel (x, y) looks at aleph = {(x/2, y/2)}, floored, which on the
 * seed grid is the parent seed nearest to (x/2, y/2); fields are carried as displacements,
 * so F^j / eta becomes twice the parent's displacement (clamped into the image). */
static void propagate_down(run_t* r, const field_t* par, field_t* ch, int carry_record)
{
    for (int j = 0; j < ch->ny; j++)
        for (int i = 0; i < ch->nx; i++) {
            int s = j * ch->nx + i;
            int px = pgmo_grid_pos(i, ch->w, ch->stride), py = pgmo_grid_pos(j, ch->h, ch->stride);
            int pi = pgmo_grid_nearest(px / 2, par->nx, par->stride);
            int pj = pgmo_grid_nearest(py / 2, par->ny, par->stride);
            int ps = pj * par->nx + pi;
            if (par->inl[ps]) {                          /* aleph' is not empty */
                int cx = 2 * par->dx[ps], cy = 2 * par->dy[ps];
                clamp_target(ch, px, py, &cx, &cy);
                ch->dx[s] = cx; ch->dy[s] = cy; ch->init[s] = 1;
                ch->dist[s] = cost(r, ch, px, py, px + cx, py + cy);
            } else {
                ch->init[s] = 0;                         /* uninitialized */
                ch->dx[s] = 0; ch->dy[s] = 0; ch->dist[s] = 0.0;
            }
            ch->rec[s] = par->inl[ps];                   /* Eq. 8 */
            ch->inl[s] = 0;
        }
    ch->rec_valid = carry_record;
}

/* round(num / den) to nearest, ties away from zero, den > 0 */
static int round_div(long num, long den)
{
    long a = num < 0 ? -num : num;
    long q = (2 * a + den) / (2 * den);
    return (int)(num < 0 ? -q : q);
}

/* Step 4 and 5 toward the coarser level k = j+1 (Eq. 6 with eta = 1/s, Eq. 8): the mean
 * of the inlier children's displacements, divided by 1/s = 2. READING: the children of a
 * coarse seed are the fine seeds whose parent (as in propagate_down) it is; the mean is
 * rounded to the nearest integer, ties away from zero. */
static void propagate_up(run_t* r, const field_t* fine, field_t* crs)
{
    long* sx = calloc((size_t)crs->n, sizeof(long));
    long* sy = calloc((size_t)crs->n, sizeof(long));
    int* cnt = calloc((size_t)crs->n, sizeof(int));
    for (int j = 0; j < fine->ny; j++)
        for (int i = 0; i < fine->nx; i++) {
            int s = j * fine->nx + i;
            if (!fine->inl[s]) continue;
            int px = pgmo_grid_pos(i, fine->w, fine->stride), py = pgmo_grid_pos(j, fine->h, fine->stride);
            int pi = pgmo_grid_nearest(px / 2, crs->nx, crs->stride);
            int pj = pgmo_grid_nearest(py / 2, crs->ny, crs->stride);
            int ps = pj * crs->nx + pi;
            sx[ps] += fine->dx[s]; sy[ps] += fine->dy[s]; cnt[ps]++;
        }
    for (int j = 0; j < crs->ny; j++)
        for (int i = 0; i < crs->nx; i++) {
            int s = j * crs->nx + i;
            int px = pgmo_grid_pos(i, crs->w, crs->stride), py = pgmo_grid_pos(j, crs->h, crs->stride);
            if (cnt[s] > 0) {
                int cx = round_div(sx[s], 2L * cnt[s]), cy = round_div(sy[s], 2L * cnt[s]);
                clamp_target(crs, px, py, &cx, &cy);
                crs->dx[s] = cx; crs->dy[s] = cy; crs->init[s] = 1;
                crs->dist[s] = cost(r, crs, px, py, px + cx, py + cy);
                crs->rec[s] = 1;
            } else {
                crs->init[s] = 0; crs->dx[s] = 0; crs->dy[s] = 0; crs->dist[s] = 0.0;
                crs->rec[s] = 0;
            }
            crs->inl[s] = 0;
        }
    crs->rec_valid = 1;
    free(sx); free(sy); free(cnt);
}

/* Step 2 and 3: forward-backward consistency check C^l (Sec. III-C/E) and the outlier
 * record update of Eq. 7 (Sec. III-D), read with the record holding "inlier": new = record
 * AND consistent, i.e. a seed is an outlier as soon as the record or the check marks it as
 * one. READING: the backward match consulted for seed p
 * is the one at the backward seed nearest to p + F(p); consistent iff the two
 * displacements cancel within tau pixels (squared Euclidean norm). */
static void check_and_update(field_t* fw, field_t* bw, int fwd_bwd, int tau)
{
    field_t* F[2] = {fw, bw};
    uint8_t* c[2];
    for (int d = 0; d < 2; d++) {
        field_t* a = F[d];
        const field_t* b = F[1 - d];
        c[d] = malloc((size_t)a->n);
        for (int j = 0; j < a->ny; j++)
            for (int i = 0; i < a->nx; i++) {
                int s = j * a->nx + i;
                int ok = a->init[s];
                if (ok && fwd_bwd) {
                    int qx = pgmo_grid_pos(i, a->w, a->stride) + a->dx[s];
                    int qy = pgmo_grid_pos(j, a->h, a->stride) + a->dy[s];
                    int oi = pgmo_grid_nearest(qx, b->nx, b->stride);
                    int oj = pgmo_grid_nearest(qy, b->ny, b->stride);
                    int os = oj * b->nx + oi;
                    if (!b->init[os]) ok = 0;
                    else {
                        long ex = (long)a->dx[s] + b->dx[os], ey = (long)a->dy[s] + b->dy[os];
                        ok = ex * ex + ey * ey <= (long)tau * tau;
                    }
                }
                c[d][s] = (uint8_t)ok;
            }
    }
    for (int d = 0; d < 2; d++) {
        field_t* a = F[d];
        for (int s = 0; s < a->n; s++)
            a->inl[s] = (uint8_t)(a->rec_valid ? (a->rec[s] && c[d][s]) : c[d][s]);
        free(c[d]);
    }
}

/* Small-region removal (Sec. III-E, after FlowFields): segment the field, then drop the
 * regions whose area is too small. READING: only inliers take part; the segments are the
 * connected components of the 4-neighbour graph on the seed grid whose edges join inliers
 * with displacements closer than link_px (Euclidean, integer comparison of squares); a
 * region's area counts stride^2 pixels per seed; it is applied once, to the forward field at
 * full resolution after its consistency check, before the output. Breadth-first search. */
void pgmo_remove_small_regions(const int32_t* dx, const int32_t* dy, uint8_t* inl, int nx, int ny,
                               int stride, int min_px, int link_px)
{
    const int n = nx * ny;
    int* comp = malloc((size_t)n * sizeof(int));
    int* queue = malloc((size_t)n * sizeof(int));
    int* size = malloc((size_t)n * sizeof(int));
    for (int s = 0; s < n; s++) comp[s] = -1;
    const long T2 = (long)link_px * link_px;
    int ncomp = 0;
    for (int s0 = 0; s0 < n; s0++) {
        if (!inl[s0] || comp[s0] >= 0) continue;
        int head = 0, tail = 0;
        queue[tail++] = s0;
        comp[s0] = ncomp;
        while (head < tail) {
            int s = queue[head++];
            int i = s % nx, j = s / nx;
            const int ni[4] = {i - 1, i + 1, i, i};
            const int nj[4] = {j, j, j - 1, j + 1};
            for (int k = 0; k < 4; k++) {
                if (ni[k] < 0 || nj[k] < 0 || ni[k] >= nx || nj[k] >= ny) continue;
                int t = nj[k] * nx + ni[k];
                if (!inl[t] || comp[t] >= 0) continue;
                long ex = (long)dx[s] - dx[t], ey = (long)dy[s] - dy[t];
                if (ex * ex + ey * ey >= T2) continue;
                comp[t] = ncomp;
                queue[tail++] = t;
            }
        }
        size[ncomp++] = tail;
    }
    for (int s = 0; s < n; s++)
        if (inl[s] && (long)size[comp[s]] * stride * stride < (long)min_px) inl[s] = 0;
    free(comp);
    free(queue);
    free(size);
}

static int32_t dist_bits(const field_t* f, int s)
{
    if (!f->init[s]) return 0x7FFFFFFF;
    if (f->feature != PGMO_FEAT_F32_DIR) return (int32_t)(f->dist[s] < 2147483646.0 ? f->dist[s] : 2147483646.0);
    float v = (float)f->dist[s];
    int32_t b;
    memcpy(&b, &v, 4);
    return b;
}

static uint32_t flags_of(const field_t* f, int s)
{
    return (f->init[s] ? PGMO_F_INIT : 0u) | (f->inl[s] ? PGMO_F_INLIER : 0u) |
           (f->rec_valid && f->rec[s] ? PGMO_F_RECORD : 0u);
}

/* Step 1 alone on one field, for tests: iterations t0 .. t0+n_iter-1 of propagation and
 * limited random search (Eq. 4-5) with search radius W, on a field of image size w x h whose
 * features are Ga (this image) and Gb (the other image), int16 or float as p->feature says.
 * State in/out: dx, dy, dist (int32, or float bits), init (0/1). Returns 0 or -1. */
int pgmo_sweep(const pgmo_params* p, int level, int dir, int stage, int W, const void* Ga,
               const void* Gb, int w, int h, int t0, int n_iter, int schedule, int32_t* dx,
               int32_t* dy, int32_t* dist, uint8_t* init, uint64_t* n_evals)
{
    if (w < 1 || h < 1 || p->seed_stride < 1 || W < 1 || t0 < 0 || n_iter < 0 || t0 + n_iter > 256) return -1;
    if (p->rs_mode != PGMO_RS_FLOOR && p->rs_mode != PGMO_RS_SYMMETRIC) return -1;
    int ch = p->color == PGMO_GRAY ? 1 : 3;
    int P = dir == 0 ? p->patch_fwd : p->patch_bwd;
    if (P < 1 || P > 16) return -1;
    field_t f;
    memset(&f, 0, sizeof f);
    f.w = w; f.h = h; f.stride = p->seed_stride;
    f.nx = pgmo_grid_count(w, f.stride); f.ny = pgmo_grid_count(h, f.stride); f.n = f.nx * f.ny;
    f.C2 = 2 * ch; f.P = P; f.feature = p->feature; f.metric = p->metric;
    if (p->metric == PGMO_METRIC_SSD) return -1;   /* a 32-bit distance state cannot hold it */
    if (p->feature != PGMO_FEAT_F32_DIR) { f.Gi_self = Ga; f.Gi_other = Gb; }
    else { f.Gf_self = Ga; f.Gf_other = Gb; }
    f.dx = dx; f.dy = dy; f.init = init;
    f.dist = malloc((size_t)f.n * sizeof(double));
    f.rec = calloc((size_t)f.n, 1); f.inl = calloc((size_t)f.n, 1);
    for (int s = 0; s < f.n; s++) {
        if (p->feature != PGMO_FEAT_F32_DIR) f.dist[s] = (double)dist[s];
        else { float v; memcpy(&v, &dist[s], 4); f.dist[s] = (double)v; }
    }
    run_t run;
    run.key[0] = (uint32_t)p->rng_seed; run.key[1] = (uint32_t)(p->rng_seed >> 32); run.evals = 0;
    run.rs_sym = p->rs_mode == PGMO_RS_SYMMETRIC;
    for (int t = t0; t < t0 + n_iter; t++) iterate(&run, &f, t, level, dir, stage, W, schedule);
    for (int s = 0; s < f.n; s++) dist[s] = dist_bits(&f, s);
    if (n_evals) *n_evals = run.evals;
    free(f.dist); free(f.rec); free(f.inl);
    return 0;
}

/* ------------------------------------------------------------------------------------- */
/* The whole method (Sec. III-D): pyramids, gradient pyramids, initial field at the       */
/* coarsest level m = L-1, then stages of Step 1-5: N refinement round trips between m    */
/* and m-1 carrying field and record, one field-only step from m to m-1, and field plus   */
/* record steps from m-1 down to full resolution.                                         */
/* ------------------------------------------------------------------------------------- */

enum { ENTER_INIT = 0, ENTER_DOWN_F = 1, ENTER_DOWN_FO = 2, ENTER_UP_FO = 3 };

int pgmo_match(const pgmo_params* p, const uint8_t* img1, const uint8_t* img2, int w, int h,
               int pitch, int schedule, pgmo_match_t* out_fwd, pgmo_match_t* out_bwd,
               int32_t* n_inliers, pgmo_match_t* out_compact, int32_t* trace, uint64_t* n_evals)
{
    int32_t lw[PGMO_MAX_LEVELS], lh[PGMO_MAX_LEVELS], lnx[PGMO_MAX_LEVELS], lny[PGMO_MAX_LEVELS];
    if (pgmo_geometry(p, w, h, lw, lh, lnx, lny) != 0) return -1;
    if (p->sobel_ksize != 3 && p->sobel_ksize != 5) return -1;
    if (p->patch_fwd < 1 || p->patch_fwd > 16 || p->patch_bwd < 1 || p->patch_bwd > 16) return -1;
    if (p->radius < 1 || p->consistency_px < 0 || p->refine_rounds < 0 || p->refine_rounds > 16) return -1;
    if (p->feature != PGMO_FEAT_INT16 && p->feature != PGMO_FEAT_F32_DIR && p->feature != PGMO_FEAT_SIGN) return -1;
    if (p->init_mode != PGMO_INIT_RANDOM && p->init_mode != PGMO_INIT_EXHAUSTIVE) return -1;
    if (w > 16384 || h > 16384) return -1;
    if (p->refine_rounds > 0 && p->levels < 2) return -1;
    if (p->min_region_px < 0 || (p->min_region_px > 0 && p->region_link_px < 1)) return -1;
    if (p->metric != PGMO_METRIC_SAD && p->metric != PGMO_METRIC_SSD) return -1;
    if (p->metric == PGMO_METRIC_SSD && p->feature == PGMO_FEAT_F32_DIR) return -1;
    if (p->rs_mode != PGMO_RS_FLOOR && p->rs_mode != PGMO_RS_SYMMETRIC) return -1;
    if (p->max_disp < -1024) return -1;
    for (int l = 0; l < p->levels; l++) {
        if (p->space_fwd[l] < 0 || p->space_fwd[l] > 2 || p->space_bwd[l] < 0 || p->space_bwd[l] > 2) return -1;
        if (p->color == PGMO_GRAY && (p->space_fwd[l] || p->space_bwd[l])) return -1;
    }
    if (pitch < 3 * w) return -1;
    for (int l = 0; l < p->levels; l++) if (p->iters[l] < 0 || p->iters[l] > 255) return -1;
    int L = p->levels;
    int ch = p->color == PGMO_GRAY ? 1 : 3;
    int C2 = 2 * ch;
    int R_top = pgmo_top_radius(p, w, h);

    run_t run;
    run.key[0] = (uint32_t)p->rng_seed;
    run.key[1] = (uint32_t)(p->rng_seed >> 32);
    run.evals = 0;
    run.rs_sym = p->rs_mode == PGMO_RS_SYMMETRIC;

    /* image pyramids {I^l} of both images (RGB), then the gradient pyramids {G^l} (Sec.
     * III-D): one per direction, each level in that direction's colour space (Table II) */
    uint8_t* pyr[2][PGMO_MAX_LEVELS];
    int16_t* Gi[2][2][PGMO_MAX_LEVELS];   /* [direction][image][level] */
    float* Gf[2][2][PGMO_MAX_LEVELS];
    for (int im = 0; im < 2; im++) {
        const uint8_t* src = im == 0 ? img1 : img2;
        for (int l = 0; l < L; l++) {
            size_t npx = (size_t)lw[l] * lh[l];
            pyr[im][l] = malloc(npx * 3);
            if (l == 0)
                for (int y = 0; y < h; y++) memcpy(pyr[im][0] + (size_t)y * w * 3, src + (size_t)y * pitch, (size_t)w * 3);
            else
                pgmo_pyr_down(pyr[im][l - 1], lw[l - 1], lh[l - 1], lw[l - 1] * 3, 3, pyr[im][l]);
            for (int d = 0; d < 2; d++) {
                const int space = d == 0 ? p->space_fwd[l] : p->space_bwd[l];
                Gi[d][im][l] = malloc(npx * C2 * sizeof(int16_t));
                if (ch == 3) {
                    uint8_t* cv = malloc(npx * 3);
                    pgmo_convert(pyr[im][l], (int)npx, space, cv);
                    pgmo_gradient_image(cv, lw[l], lh[l], lw[l] * 3, 3, p->sobel_ksize, Gi[d][im][l]);
                    free(cv);
                } else {
                    uint8_t* gy = malloc(npx);
                    pgmo_gray(pyr[im][l], lw[l], lh[l], lw[l] * 3, gy);
                    pgmo_gradient_image(gy, lw[l], lh[l], lw[l], 1, p->sobel_ksize, Gi[d][im][l]);
                    free(gy);
                }
                Gf[d][im][l] = NULL;
                if (p->feature == PGMO_FEAT_SIGN) pgmo_sign(Gi[d][im][l], (int)(npx * C2));
                if (p->feature == PGMO_FEAT_F32_DIR) {
                    Gf[d][im][l] = malloc(npx * C2 * sizeof(float));
                    pgmo_direction(Gi[d][im][l], (int)npx, ch, Gf[d][im][l]);
                }
            }
        }
    }

    /* fields: dir 0 matches image 1 -> 2 with the forward patch, dir 1 image 2 -> 1 */
    field_t F[2][PGMO_MAX_LEVELS];
    for (int d = 0; d < 2; d++)
        for (int l = 0; l < L; l++) {
            field_t* f = &F[d][l];
            f->w = lw[l]; f->h = lh[l]; f->nx = lnx[l]; f->ny = lny[l]; f->n = lnx[l] * lny[l];
            f->stride = p->seed_stride; f->C2 = C2; f->feature = p->feature; f->metric = p->metric;
            f->P = d == 0 ? p->patch_fwd : p->patch_bwd;
            f->Gi_self = Gi[d][d][l]; f->Gi_other = Gi[d][1 - d][l];
            f->Gf_self = Gf[d][d][l]; f->Gf_other = Gf[d][1 - d][l];
            f->dx = calloc((size_t)f->n, sizeof(int32_t));
            f->dy = calloc((size_t)f->n, sizeof(int32_t));
            f->dist = calloc((size_t)f->n, sizeof(double));
            f->init = calloc((size_t)f->n, 1);
            f->rec = calloc((size_t)f->n, 1);
            f->inl = calloc((size_t)f->n, 1);
            f->rec_valid = 0;
        }

    /* the stage list */
    int st_level[2 * PGMO_MAX_LEVELS + 64], st_enter[2 * PGMO_MAX_LEVELS + 64], nst = 0;
    int m = L - 1;
    st_level[nst] = m; st_enter[nst++] = ENTER_INIT;
    for (int k = 0; k < p->refine_rounds; k++) {
        st_level[nst] = m - 1; st_enter[nst++] = ENTER_DOWN_FO;
        st_level[nst] = m;     st_enter[nst++] = ENTER_UP_FO;
    }
    for (int l = m - 1; l >= 0; l--) {
        st_level[nst] = l;
        st_enter[nst++] = l == m - 1 ? ENTER_DOWN_F : ENTER_DOWN_FO;
    }

    for (int sidx = 0; sidx < nst; sidx++) {
        int l = st_level[sidx];
        int W = p->radius;
        for (int d = 0; d < 2; d++) {
            field_t* f = &F[d][l];
            switch (st_enter[sidx]) {
            case ENTER_INIT:
                init_field(&run, f, l, d, sidx, p->init_mode, R_top);
                if (p->init_mode == PGMO_INIT_RANDOM) W = R_top;
                break;
            case ENTER_DOWN_F: propagate_down(&run, &F[d][l + 1], f, 0); break;
            case ENTER_DOWN_FO: propagate_down(&run, &F[d][l + 1], f, 1); break;
            default: propagate_up(&run, &F[d][l - 1], f); break;
            }
        }
        /* Step 1: basic gradient matching */
        for (int t = 0; t < p->iters[l]; t++)
            for (int d = 0; d < 2; d++) iterate(&run, &F[d][l], t, l, d, sidx, W, schedule);
        /* Step 2 and 3 */
        check_and_update(&F[0][l], &F[1][l], p->fwd_bwd, p->consistency_px);
    }
    if (p->min_region_px > 0) {
        field_t* f = &F[0][0];
        pgmo_remove_small_regions(f->dx, f->dy, f->inl, f->nx, f->ny, f->stride, p->min_region_px,
                                  p->region_link_px);
    }

    if (trace) {
        int32_t* t = trace;
        for (int d = 0; d < 2; d++)
            for (int l = 0; l < L; l++) {
                const field_t* f = &F[d][l];
                for (int s = 0; s < f->n; s++) {
                    *t++ = f->dx[s]; *t++ = f->dy[s]; *t++ = dist_bits(f, s); *t++ = (int32_t)flags_of(f, s);
                }
            }
    }

    /* output: level-0 matches on the seed grid (Sec. III-G) */
    int cnt = 0;
    for (int d = 0; d < 2; d++) {
        pgmo_match_t* out = d == 0 ? out_fwd : out_bwd;
        const field_t* f = &F[d][0];
        for (int j = 0; j < f->ny; j++)
            for (int i = 0; i < f->nx; i++) {
                int s = j * f->nx + i;
                pgmo_match_t mt;
                mt.x1 = pgmo_grid_pos(i, f->w, f->stride);
                mt.y1 = pgmo_grid_pos(j, f->h, f->stride);
                mt.x2 = mt.x1 + (f->init[s] ? f->dx[s] : 0);
                mt.y2 = mt.y1 + (f->init[s] ? f->dy[s] : 0);
                mt.dist = dist_bits(f, s);
                mt.flags = flags_of(f, s);
                if (out) out[s] = mt;
                if (d == 0 && f->inl[s]) {
                    if (out_compact) out_compact[cnt] = mt;
                    cnt++;
                }
            }
    }
    if (n_inliers) *n_inliers = cnt;
    if (n_evals) *n_evals = run.evals;

    for (int d = 0; d < 2; d++)
        for (int l = 0; l < L; l++) {
            field_t* f = &F[d][l];
            free(f->dx); free(f->dy); free(f->dist); free(f->init); free(f->rec); free(f->inl);
        }
    for (int im = 0; im < 2; im++)
        for (int l = 0; l < L; l++) {
            free(pyr[im][l]);
            for (int d = 0; d < 2; d++) { free(Gi[d][im][l]); free(Gf[d][im][l]); }
        }
    return 0;
}

/* Test entry for the lift of Sec. III-D toward the coarser level (Eq. 6 with k = j+1, the
 * step of propagate_up) applied to a given finer field: displacements and inlier flags of a
 * fw x fh grid (spacing `stride`) in, the coarse cw x ch grid's displacements and
 * initialised flags out. The coarse distances are taken on zero features; the lifted
 * displacements do not depend on them. */
int pgmo_lift(int fw, int fh, int cw, int ch, int stride, const int32_t* fdx, const int32_t* fdy,
              const uint8_t* finl, int32_t* cdx, int32_t* cdy, uint8_t* cinit)
{
    if (fw < 1 || fh < 1 || cw < 1 || ch < 1 || stride < 1) return -1;
    field_t fine, crs;
    memset(&fine, 0, sizeof fine);
    memset(&crs, 0, sizeof crs);
    fine.w = fw; fine.h = fh; fine.stride = stride;
    fine.nx = pgmo_grid_count(fw, stride); fine.ny = pgmo_grid_count(fh, stride); fine.n = fine.nx * fine.ny;
    fine.dx = (int32_t*)fdx; fine.dy = (int32_t*)fdy; fine.inl = (uint8_t*)finl;
    crs.w = cw; crs.h = ch; crs.stride = stride;
    crs.nx = pgmo_grid_count(cw, stride); crs.ny = pgmo_grid_count(ch, stride); crs.n = crs.nx * crs.ny;
    crs.C2 = 6; crs.P = 1;
    int16_t* zero = calloc((size_t)cw * ch * 6, sizeof(int16_t));
    crs.Gi_self = zero; crs.Gi_other = zero;
    crs.dx = cdx; crs.dy = cdy; crs.init = cinit;
    crs.dist = malloc((size_t)crs.n * sizeof(double));
    crs.rec = malloc((size_t)crs.n); crs.inl = malloc((size_t)crs.n);
    run_t run;
    memset(&run, 0, sizeof run);
    propagate_up(&run, &fine, &crs);
    free(zero); free(crs.dist); free(crs.rec); free(crs.inl);
    return 0;
}
