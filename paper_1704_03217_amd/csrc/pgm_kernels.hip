// HIP kernels of libpgm for gfx950 (CDNA4): pyramidal gradient matching
// (Y. Li, "Pyramidal Gradient Matching for Optical Flow Estimation", arXiv:1704.03217).
//
// Matching kernels assign one group of LPS lanes (8 for patches up to 8 pixels, 16 up to 16)
// to each seed of the grid: lane c holds pixel column c of every row of the seed's patch of
// the first gradient image in registers (full 8x8 integer patches read from HBM: six 16-byte
// pieces of the patch instead), reads the same part of candidate patches of the second image
// (buffer loads from HBM, plain loads from LDS), and the patch distance is the DPP sum over
// the group. Candidates are priced two at a time, but every seed's decisions
// replay the paper's candidate order one at a time, so they are exactly the sequential ones;
// seeds of one colour of the red-black checkerboard are independent and run in parallel.
#include <string.h>

#include "pgm_internal.h"

namespace pgm {

// two 16-bit lanes of one register (packed integer arithmetic)
typedef short s16x2 __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------------------

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

__device__ __forceinline__ uint32_t pack_d(int dx, int dy)
{
    return (uint32_t)(uint16_t)(int16_t)dx | ((uint32_t)(uint16_t)(int16_t)dy << 16);
}
__device__ __forceinline__ int d_x(uint32_t v) { return (int)(int16_t)(uint16_t)(v & 0xFFFFu); }
__device__ __forceinline__ int d_y(uint32_t v) { return (int)(int16_t)(uint16_t)(v >> 16); }

// clamp the target p + d into the image and return the clamped displacement
__device__ __forceinline__ uint32_t target(int px, int py, int dx, int dy, const Geo& g)
{
    return pack_d(clampi(px + dx, 0, g.w - 1) - px, clampi(py + dy, 0, g.h - 1) - py);
}

__device__ __forceinline__ int grid_pos(int i, int n, const Geo& g)
{
    int p = g.off + i * g.stride;
    return p < n - 1 ? p : n - 1;
}

// index of the grid seed nearest to pixel x >= 0 (ties go to the larger index)
__device__ __forceinline__ int grid_near(int x, int nseeds, const Geo& g)
{
    unsigned num = (unsigned)(2 * (x - g.off) + g.stride);   // >= 0 because off <= stride/2
    int i = (int)fdiv(num, g.d2s);                            // num / (2 stride)
    return i < nseeds - 1 ? i : nseeds - 1;
}

// reflect-101 index into [0, n)
__device__ __forceinline__ int mirror(int i, int n)
{
    if (n == 1) return 0;
    int period = 2 * (n - 1);
    int m = i < 0 ? -i : i;
    m %= period;
    return m < n ? m : period - m;
}

// Philox4x32 with ten rounds (Salmon, Moraes, Dror and Shaw, SC'11).
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; r++) {
        const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
        uint32_t lo0 = m0 * c.x, hi0 = __umulhi(m0, c.x);
        uint32_t lo1 = m1 * c.z, hi1 = __umulhi(m1, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// DPP sums over groups of 8 or 16 consecutive lanes; every lane receives the group total.
template <int LPS>
__device__ __forceinline__ uint32_t group_sum(uint32_t v)
{
    v += __builtin_amdgcn_update_dpp(0u, v, 0xB1, 0xF, 0xF, false);    // quad_perm [1,0,3,2]
    v += __builtin_amdgcn_update_dpp(0u, v, 0x4E, 0xF, 0xF, false);    // quad_perm [2,3,0,1]
    v += __builtin_amdgcn_update_dpp(0u, v, 0x141, 0xF, 0xF, false);   // row_half_mirror
    if (LPS == 16) v += __builtin_amdgcn_update_dpp(0u, v, 0x140, 0xF, 0xF, false);  // row_mirror
    return v;
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    unsigned long long b = (unsigned long long)__double_as_longlong(v);
    uint32_t lo = __builtin_amdgcn_update_dpp(0u, (uint32_t)b, CTRL, 0xF, 0xF, false);
    uint32_t hi = __builtin_amdgcn_update_dpp(0u, (uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

template <int LPS>
__device__ __forceinline__ double group_sum(double v)
{
    v += dpp_f64<0xB1>(v);
    v += dpp_f64<0x4E>(v);
    v += dpp_f64<0x141>(v);
    if (LPS == 16) v += dpp_f64<0x140>(v);
    return v;
}

// ---------------------------------------------------------------------------------------
// one lane's patch column: lane c of a seed's group holds pixel column c of every row of the
// seed's first-image patch in registers and streams the same column of candidate patches.
// The group's lanes read each patch row as one contiguous segment (96 bytes for 8 RGB
// gradient pixels), so a wave's load touches few cache lines.
// ---------------------------------------------------------------------------------------

// Integer gradients, biased u16, two per dword; C2 channels per pixel (C2 even).
// v_sad_u16 adds |a.lo16 - b.lo16| + |a.hi16 - b.hi16| (unsigned halves) to its accumulator,
// so one instruction covers two gradient values of a packed dword.
// Rows past the patch side (P < PMAX) read row P - 1 again and add nothing.
template <int C2, int PMAX, bool FIXED>
struct IntRow {
    static constexpr int ROWS = PMAX;
    static constexpr int W3 = C2 / 2;   // dwords per pixel
    using Acc = uint32_t;
    uint32_t a[PMAX][W3];

    // base: this lane's pixel of the patch's first row; pitch: dwords per image row
    __device__ __forceinline__ void load(const uint32_t* base, ptrdiff_t pitch, int P)
    {
#pragma unroll
        for (int y = 0; y < PMAX; y++) {
            const int yy = (FIXED || y < P) ? y : P - 1;
#pragma unroll
            for (int w = 0; w < W3; w++) a[y][w] = base[yy * pitch + w];
        }
    }
    __device__ __forceinline__ uint32_t sad(const IntRow& B, int P) const
    {
        uint32_t acc = 0;
#pragma unroll
        for (int y = 0; y < PMAX; y++)
            if (FIXED || y < P)
#pragma unroll
                for (int w = 0; w < W3; w++) acc = __builtin_amdgcn_sad_u16(a[y][w], B.a[y][w], acc);
        return acc;
    }
    // The same rows of a padded gradient image in HBM through buffer loads: one VGPR holds
    // the lane's byte offset, the row offsets are scalar (SGPR), and a read outside the
    // image's bytes returns zero instead of touching other memory. (x, y): the lane's pixel
    // of the first row, image coordinates >= -PAD.
    static constexpr bool CAN_BUF = W3 == 1 || W3 == 3;
    __device__ __forceinline__ void load_buf(const void* G, const Geo& g, int x, int y, int P)
    {
        constexpr uint32_t PXB = W3 * 4;
        const uint32_t pitch_b = (uint32_t)g.pw * PXB;
        const char* base = (const char*)G - ((size_t)PAD * g.pw + PAD) * PXB;
        const uint32_t bytes = pitch_b * (uint32_t)(g.h + 2 * PAD);
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)bytes, 0x00020000);
        const uint32_t vo = ((uint32_t)(y + PAD) * (uint32_t)g.pw + (uint32_t)(x + PAD)) * PXB;
#pragma unroll
        for (int r = 0; r < PMAX; r++) {
            const uint32_t so = (uint32_t)((FIXED || r < P) ? r : P - 1) * pitch_b;
            if constexpr (W3 == 3) {
                const auto v = __builtin_amdgcn_raw_buffer_load_b96(rs, vo, so, 0);
                a[r][0] = v[0];
                a[r][1] = v[1];
                a[r][2] = v[2];
            } else if constexpr (W3 == 1) {
                a[r][0] = __builtin_amdgcn_raw_buffer_load_b32(rs, vo, so, 0);
            }
        }
    }
    static __device__ __forceinline__ const uint32_t* at(const void* G, const Geo& g, int x, int y)
    {
        return (const uint32_t*)G + ((ptrdiff_t)y * g.pw + x) * W3;
    }
    static __device__ __forceinline__ ptrdiff_t pitch(const Geo& g) { return (ptrdiff_t)g.pw * W3; }
    // the patch whose top-left pixel is (tlx, tly): lane r reads column r (lanes past the
    // patch side read its last column and add nothing)
    template <bool BUF>
    __device__ __forceinline__ void fetch(const void* G, const Geo& g, int tlx, int tly, int P, int r)
    {
        const int x = tlx + (r < P ? r : P - 1);
        if constexpr (BUF && CAN_BUF) load_buf(G, g, x, tly, P);
        else load(at(G, g, x, tly), pitch(g), P);
    }
    template <int LPS>
    static __device__ __forceinline__ uint32_t finish(uint32_t partial) { return group_sum<LPS>(partial); }
    using Dist = uint32_t;
};

// Full 8x8 patches of 6 integer channels from HBM: the 48 16-byte pieces of a patch (8 rows
// of 96 bytes) are dealt to the group's 8 lanes, piece r + 8 m to lane r (m < 6), so a
// candidate costs six dwordx4 loads per lane instead of eight dwordx3. The texture addresser
// spends the same time on a load instruction whatever its width or its number of active
// lanes (measured: ~16 clocks per wave), so the wider pieces read a patch in 25% less of it.
// Both patches of a distance are read with the same map, so the sum is unchanged; patches in
// LDS (BUF false) keep the column map of IntRow.
struct IntRowQ : IntRow<6, 8, true> {
    __device__ __forceinline__ void load_pieces(const void* G, const Geo& g, int tlx, int tly, int r)
    {
        const uint32_t pitch_b = (uint32_t)g.pw * 12u;
        const char* base = (const char*)G - ((size_t)PAD * g.pw + PAD) * 12;
        const uint32_t bytes = pitch_b * (uint32_t)(g.h + 2 * PAD);
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)bytes, 0x00020000);
        const uint32_t vo = ((uint32_t)(tly + PAD) * (uint32_t)g.pw + (uint32_t)(tlx + PAD)) * 12u;
        uint32_t* f = &a[0][0];   // the 24 dwords as one array: piece m in f[4 m .. 4 m + 3]
#pragma unroll
        for (int m = 0; m < 6; m++) {
            const int k = r + 8 * m;
            const uint32_t off = (uint32_t)(k / 6) * pitch_b + (uint32_t)(k % 6) * 16u;
            const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, vo + off, 0, 0);
            f[4 * m + 0] = v[0];
            f[4 * m + 1] = v[1];
            f[4 * m + 2] = v[2];
            f[4 * m + 3] = v[3];
        }
    }
    template <bool BUF>
    __device__ __forceinline__ void fetch(const void* G, const Geo& g, int tlx, int tly, int P, int r)
    {
        if constexpr (BUF) load_pieces(G, g, tlx, tly, r);
        else IntRow<6, 8, true>::template fetch<false>(G, g, tlx, tly, P, r);
    }
};

// Direction-only float features. The components are unit-vector coordinates (zero or of
// magnitude >= 2^-14), so every difference and the sum over a patch are exact in double and
// the rounded float result does not depend on the order of summation.
template <int C2, int PMAX, bool FIXED>
struct F32Row {
    static constexpr int ROWS = PMAX;
    using Acc = double;
    using Dist = uint32_t;
    static constexpr bool CAN_BUF = false;
    float a[PMAX][C2];

    __device__ __forceinline__ void load(const float* base, ptrdiff_t pitch, int P)
    {
#pragma unroll
        for (int y = 0; y < PMAX; y++) {
            const int yy = (FIXED || y < P) ? y : P - 1;
#pragma unroll
            for (int c = 0; c < C2; c++) a[y][c] = base[yy * pitch + c];
        }
    }
    __device__ __forceinline__ double sad(const F32Row& B, int P) const
    {
        double acc = 0.0;
#pragma unroll
        for (int y = 0; y < PMAX; y++)
            if (FIXED || y < P)
#pragma unroll
                for (int c = 0; c < C2; c++) acc += fabs((double)B.a[y][c] - (double)a[y][c]);
        return acc;
    }
    static __device__ __forceinline__ const float* at(const void* G, const Geo& g, int x, int y)
    {
        return (const float*)G + ((ptrdiff_t)y * g.pw + x) * C2;
    }
    static __device__ __forceinline__ ptrdiff_t pitch(const Geo& g) { return (ptrdiff_t)g.pw * C2; }
    template <bool BUF>
    __device__ __forceinline__ void fetch(const void* G, const Geo& g, int tlx, int tly, int P, int r)
    {
        load(at(G, g, tlx + (r < P ? r : P - 1), tly), pitch(g), P);
    }
    template <int LPS>
    static __device__ __forceinline__ uint32_t finish(double partial)
    {
        return __float_as_uint((float)group_sum<LPS>(partial));
    }
};

// Eq. 3 as printed: squared differences of the same packed integer features, summed exactly
// (a lane's part < 2^38, a group's < 2^42: exact in the double used for the DPP sum).
template <int C2, int PMAX, bool FIXED>
struct SsdRow : IntRow<C2, PMAX, FIXED> {
    using Acc = uint64_t;
    using Dist = uint64_t;
    __device__ __forceinline__ uint64_t sad(const SsdRow& B, int P) const
    {
        uint64_t acc = 0;
#pragma unroll
        for (int y = 0; y < PMAX; y++)
            if (FIXED || y < P)
#pragma unroll
                for (int w = 0; w < IntRow<C2, PMAX, FIXED>::W3; w++) {
                    const uint32_t a = this->a[y][w], b = B.a[y][w];
                    const uint32_t d0 = (uint32_t)abs((int)(a & 0xFFFFu) - (int)(b & 0xFFFFu));
                    const uint32_t d1 = (uint32_t)abs((int)(a >> 16) - (int)(b >> 16));
                    acc += (uint64_t)(d0 * d0) + (uint64_t)(d1 * d1);
                }
        return acc;
    }
    template <int LPS>
    static __device__ __forceinline__ uint64_t finish(uint64_t partial)
    {
        return (uint64_t)group_sum<LPS>((double)partial);
    }
};

// KIND: 0 integer features with absolute differences, 1 float direction features, 2 integer
// features with squared differences
template <int C2, int PMAX, bool FIXED, int KIND>
using RowT = typename std::conditional<
    KIND == 1, F32Row<C2, PMAX, FIXED>,
    typename std::conditional<KIND == 2, SsdRow<C2, PMAX, FIXED>,
                              typename std::conditional<C2 == 6 && PMAX == 8 && FIXED, IntRowQ,
                                                        IntRow<C2, PMAX, FIXED>>::type>::type>::type;

// Patch distance of Eq. 3 (absolute or squared differences) between the patch held by the group and
// the patch of the other image at (qx, qy); every lane of the group gets the result. Lanes
// past the patch side read a valid column and add nothing. All rows of the candidate are
// requested before the first one is used (the scheduling barrier keeps the compiler from
// trading the loads in flight for registers), so a candidate costs one memory round trip.
// rows of the patch whose first-row pixel for this lane is (x, y): buffer loads from HBM
// (BUF) or plain loads (LDS images, float features)

template <class Row, int LPS, bool BUF>
__device__ __forceinline__ typename Row::Dist patch_cost(const Row& A, const void* Gb, const Geo& g, int P,
                                               int r, int qx, int qy)
{
    const int half = P >> 1;
    Row B;
    B.template fetch<BUF>(Gb, g, qx - half, qy - half, P, r);
    __builtin_amdgcn_sched_barrier(0);
    typename Row::Acc part = A.sad(B, P);
    if (r >= P) part = typename Row::Acc(0);
    return Row::template finish<LPS>(part);
}

// Two patch distances with the reads of both candidates in flight together.
template <class Row, int LPS, bool BUF>
__device__ __forceinline__ void patch_cost2(const Row& A, const void* Gb, const Geo& g, int P, int r, int q0x,
                                            int q0y, int q1x, int q1y, typename Row::Dist& e0,
                                            typename Row::Dist& e1)
{
    if constexpr (Row::ROWS == 16) {   // 16-row patches: one at a time (registers for occupancy)
        e0 = patch_cost<Row, LPS, BUF>(A, Gb, g, P, r, q0x, q0y);
        e1 = patch_cost<Row, LPS, BUF>(A, Gb, g, P, r, q1x, q1y);
        return;
    }
    const int half = P >> 1;
    Row B0, B1;
    B0.template fetch<BUF>(Gb, g, q0x - half, q0y - half, P, r);
    B1.template fetch<BUF>(Gb, g, q1x - half, q1y - half, P, r);
    __builtin_amdgcn_sched_barrier(0);
    typename Row::Acc p0 = A.sad(B0, P);
    typename Row::Acc p1 = A.sad(B1, P);
    if (r >= P) {
        p0 = typename Row::Acc(0);
        p1 = typename Row::Acc(0);
    }
    e0 = Row::template finish<LPS>(p0);
    e1 = Row::template finish<LPS>(p1);
}

// Three patch distances with the reads of all three candidates in flight together.
template <class Row, int LPS, bool BUF>
__device__ __forceinline__ void patch_cost3(const Row& A, const void* Gb, const Geo& g, int P, int r, const int qx[3],
                                            const int qy[3], typename Row::Dist e[3])
{
    const int half = P >> 1;
    Row B0, B1, B2;
    B0.template fetch<BUF>(Gb, g, qx[0] - half, qy[0] - half, P, r);
    B1.template fetch<BUF>(Gb, g, qx[1] - half, qy[1] - half, P, r);
    B2.template fetch<BUF>(Gb, g, qx[2] - half, qy[2] - half, P, r);
    __builtin_amdgcn_sched_barrier(0);
    typename Row::Acc p0 = A.sad(B0, P);
    typename Row::Acc p1 = A.sad(B1, P);
    typename Row::Acc p2 = A.sad(B2, P);
    if (r >= P) {
        p0 = typename Row::Acc(0);
        p1 = typename Row::Acc(0);
        p2 = typename Row::Acc(0);
    }
    e[0] = Row::template finish<LPS>(p0);
    e[1] = Row::template finish<LPS>(p1);
    e[2] = Row::template finish<LPS>(p2);
}

// The patch distances of qa and, where `both`, of qb (qb's result is qa's otherwise), for the
// seeds of the wave that call it: both patches' reads in flight together when some of these
// seeds need two, one patch otherwise. A load instruction holds the texture addresser as long
// whatever its number of active lanes, so a second patch that no seed of the wave needs is
// not fetched.
template <class Row, int LPS, bool BUF>
__device__ __forceinline__ void patch_cost_some(const Row& A, const void* Gb, const Geo& g, int P, int r, int px,
                                                int py, uint32_t qa, uint32_t qb, bool both,
                                                typename Row::Dist& ea, typename Row::Dist& eb)
{
    if (__builtin_amdgcn_ballot_w64(both) != 0ull) {   // uniform over the active lanes
        patch_cost2<Row, LPS, BUF>(A, Gb, g, P, r, px + d_x(qa), py + d_y(qa), px + d_x(qb), py + d_y(qb), ea, eb);
    } else {
        ea = patch_cost<Row, LPS, BUF>(A, Gb, g, P, r, px + d_x(qa), py + d_y(qa));
        eb = ea;
    }
}

template <bool BUF, class Row>
__device__ __forceinline__ void load_own(Row& A, const void* Ga, const Geo& g, int P, int r, int px, int py)
{
    const int half = P >> 1;
    A.template fetch<BUF>(Ga, g, px - half, py - half, P, r);
}

// Logical block of a 1-D launch over nbx x ndir x npairs work-groups. Consecutive work-group
// ids are dealt round robin to the 8 XCDs; this remap hands every XCD one contiguous range of
// logical ids (a band of seeds of one pair, or whole pairs of a batch), so each XCD's L2
// caches a compact part of the gradient images. When the two directions read the same two
// images (each image one direction's own and the other's candidates: one colour space for
// both), the two directions of a block of seeds are neighbours in that order and share an
// XCD; with four images (a colour space per direction) each direction keeps its own range.
// The launch holds b.dnb.d work-groups per direction and pair, b.ndir (1 or 2) directions.
struct LBlock {
    int x, dir, z;
};
__device__ __forceinline__ LBlock logical_block(const Batch& bt)
{
    const int N = gridDim.x, L = blockIdx.x;
    const int j = L & 7, q = (N + 7) >> 3, r = N & 7;
    const int id = (r == 0 || j < r) ? j * q + (L >> 3) : r * q + (j - r) * (q - 1) + (L >> 3);
    const int two = bt.ndir == 2;
    const int alt = two & (bt.inter != 0);   // the directions alternate
    const int seq = two & !alt;              // all blocks of one direction, then the other's
    const int xz = id >> alt;
    const int rest = (int)fdiv((uint32_t)xz, bt.dnb);
    LBlock b;
    b.x = xz - rest * (int)bt.dnb.d;
    b.dir = alt ? (id & 1) : (rest & seq);
    b.z = rest >> seq;
    return b;
}

template <class T>
__device__ __forceinline__ T* zoff(T* p, size_t off)
{
    return p ? (T*)((const char*)p + off) : p;
}

__device__ __forceinline__ Field pair_field(const Field& f, size_t off)
{
    Field r;
    r.disp = zoff(f.disp, off);
    r.dist = zoff(f.dist, off);
    r.flags = zoff(f.flags, off);
    return r;
}

__device__ __forceinline__ DirArgs pair_dir(const DirArgs& d, size_t off)
{
    DirArgs r = d;
    r.Ga = zoff(d.Ga, off);
    r.Gb = zoff(d.Gb, off);
    r.f = pair_field(d.f, off);
    return r;   // the random-number table is shared by all pairs
}

// Sum the per-group evaluation counts of the work-group and store the total in its slot of
// the launch's count table (no atomics: one kernel adds the slots up at the end). Every
// thread of the block must call it.
__device__ __forceinline__ void count_evals(uint32_t* cnt, int slot, uint32_t nev, bool leader)
{
    if (!cnt) return;   // uniform over the launch
    __shared__ uint32_t wsum[4];   // work-groups of 64 to 256 threads
    uint32_t v = leader ? nev : 0u;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int k = 0; k < (int)(blockDim.x >> 6); k++) t += wsum[k];
        cnt[slot] = t;
    }
}

// ---------------------------------------------------------------------------------------
// Step 1 (Sec. III-B): one colour of one propagation + limited random search iteration
// ---------------------------------------------------------------------------------------

// Step 1 after the propagation members are priced: the decisions of Eq. 4 in order, then the
// limited random search of Eq. 5 around the result (Psi = {F(p)} + {F(p) + floor(R_i W / 2^i)},
// priced two at a time and decided in order). Returns the evaluations counted; lane 0 hands
// the result to put(displacement, distance, changed).
template <class Row, int LPS, bool BUF, class Put>
__device__ __forceinline__ uint32_t decide_and_search(const Row& A, const DirArgs& D, const Geo& g, int px, int py,
                                                      int r, const short2* R, int nI, short2 o0, short2 o1,
                                                      uint32_t cur0, typename Row::Dist cd0, const uint32_t c[2],
                                                      const bool ok[2], const typename Row::Dist e[2], Put put)
{
    using Dist = typename Row::Dist;
    const int P = D.P;
    const bool init0 = cur0 != UNINIT;
    uint32_t nev = 0;
    uint32_t cur = cur0;
    Dist cd = cd0;
    bool init = init0, changed = false;
#pragma unroll
    for (int m = 0; m < 2; m++) {
        if (!ok[m] || (init && c[m] == cur)) continue;
        nev++;
        if (!init || e[m] < cd) { cur = c[m]; cd = e[m]; init = true; changed = true; }
    }

    // Eq. 5: Psi = {F(p)} + {F(p) + floor(R_i W / 2^i)}, all around the propagated match,
    // priced two at a time in the same way and decided in order
    if (init) {
        const int cx = d_x(cur), cy = d_y(cur);
        const uint32_t curp = cur;
        const Dist cdp = cd;
        for (int ii = 0; ii < nI; ii += 2) {
            if (ii > 0) {
                o0 = R[ii];
                if (ii + 1 < nI) o1 = R[ii + 1];
            }
            const bool two = ii + 1 < nI;
            const uint32_t r0 = target(px, py, cx + o0.x, cy + o0.y, g);
            const uint32_t r1 = two ? target(px, py, cx + o1.x, cy + o1.y, g) : curp;
            const bool n0 = r0 != curp;
            const bool n1 = r1 != curp && r1 != r0;
            Dist f0 = cdp, f1 = cdp;
            if (n0 || n1) {
                const uint32_t qa = n0 ? r0 : r1, qb = n1 ? r1 : r0;
                Dist ea, eb;
                patch_cost_some<Row, LPS, BUF>(A, D.Gb, g, P, r, px, py, qa, qb, n0 && n1, ea, eb);
                if (n0) f0 = ea;
                if (n1) f1 = eb;
            }
            if (two && !n1 && r1 != curp) f1 = f0;
            if (r0 != cur) {
                nev++;
                if (f0 < cd) { cur = r0; cd = f0; changed = true; }
            }
            if (two && r1 != cur) {
                nev++;
                if (f1 < cd) { cur = r1; cd = f1; changed = true; }
            }
        }
    }
    if (r == 0) put(cur, cd, changed);
    return nev;
}

// lane 0's write of a seed's result into field f: always, or only when it changed
template <class Dist>
struct PutSeed {
    Field f;
    int s;
    bool always;
    __device__ __forceinline__ void operator()(uint32_t cur, Dist cd, bool changed) const
    {
        if (changed || always) {
            f.disp[s] = cur;
            ((Dist*)f.dist)[s] = cd;
        }
    }
};

// One seed's half-sweep step (Step 1): propagation (Eq. 4) then limited random search
// (Eq. 5) for seed (i, j) of field D at iteration t. seed_start issues the reads that need
// nothing from other seeds (the seed's first-image patch, its own field, its first two random
// offsets); seed_finish takes the propagation members' displacements from nbr(i', j')
// (called for positions outside the grid too, whose value is then ignored), prices and
// decides, and returns the distance evaluations made. The group's lanes all call both for
// the same seed; lane 0 hands the result to put.
template <class Row>
struct SeedStart {
    Row A;
    uint32_t cur0;
    typename Row::Dist cd0;
    const short2* R;
    short2 o0, o1;
    int s, px, py;
};

// FF: the seed's field and random offsets are read before its patch (the small launches of
// k_sweep_multi and k_sweep_pair, whose propagation decisions wait on the field); the large
// launches of k_sweep, bound by the texture addresser, keep the patch first.
template <class Row, int LPS, bool BUF, bool FF = false>
__device__ __forceinline__ void seed_start(SeedStart<Row>& S, const DirArgs& D, const Geo& g, int i, int j, int t,
                                           int nI, int r)
{
    using Dist = typename Row::Dist;
    S.s = j * g.nx + i;
    S.px = grid_pos(i, g.w, g);
    S.py = grid_pos(j, g.h, g);
    if constexpr (!FF) load_own<BUF>(S.A, D.Ga, g, D.P, r, S.px, S.py);
    S.cur0 = D.f.disp[S.s];
    S.cd0 = ((const Dist*)D.f.dist)[S.s];
    // Eq. 5 offsets of the first two random candidates (nI >= 1), fetched with the field
    S.R = D.rnd + ((size_t)t * (size_t)(g.nx * g.ny) + S.s) * nI;
    S.o0 = S.R[0];
    S.o1 = S.R[nI > 1 ? 1 : 0];
    if constexpr (FF) load_own<BUF>(S.A, D.Ga, g, D.P, r, S.px, S.py);
}

template <class Row, int LPS, bool BUF, class Nbr, class Put>
__device__ __forceinline__ uint32_t seed_finish(const SeedStart<Row>& S, const DirArgs& D, const Geo& g, int i, int j,
                                                int t, int nI, int r, Nbr nbr, Put put)
{
    using Dist = typename Row::Dist;
    const int P = D.P;
    const int px = S.px, py = S.py;
    const uint32_t cur0 = S.cur0;
    const Dist cd0 = S.cd0;
    const bool init0 = cur0 != UNINIT;
    // Eq. 4: Omega = {F(p), F(p - Dx) + Dx, F(p - Dy) + Dy} with the FlowFields order
    // (1,0),(0,1) -> (-1,0),(0,-1) -> (-1,0),(0,1) -> (1,0),(0,-1); members whose
    // neighbour is uninitialised are ignored.
    const int k = t & 3;
    const int sx = (k == 0 || k == 3) ? 1 : -1;
    const int sy = (k == 0 || k == 2) ? 1 : -1;
    uint32_t c[2], nv[2];
    bool ok[2];
#pragma unroll
    for (int m = 0; m < 2; m++) {
        const int ni = m == 0 ? i - sx : i;
        const int nj = m == 0 ? j : j - sy;
        ok[m] = ni >= 0 && nj >= 0 && ni < g.nx && nj < g.ny;
        nv[m] = nbr(ni, nj);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int m = 0; m < 2; m++) {
        ok[m] = ok[m] && nv[m] != UNINIT;
        const uint32_t tg = target(px, py, d_x(nv[m]), d_y(nv[m]), g);
        c[m] = ok[m] ? tg : cur0;
    }
    // Both members are priced together. A member equal to F(p) costs the stored distance
    // and one equal to the other member costs what that one costs, so only new patches
    // are read; the decisions below replay the paper's one-at-a-time order exactly.
    const bool need0 = ok[0] && !(init0 && c[0] == cur0);
    const bool need1 = ok[1] && !(init0 && c[1] == cur0) && !(ok[0] && c[1] == c[0]);
    Dist e[2] = {cd0, cd0};
    if (need0 || need1) {
        const uint32_t qa = need0 ? c[0] : c[1], qb = need1 ? c[1] : c[0];
        Dist ea, eb;
        patch_cost_some<Row, LPS, BUF>(S.A, D.Gb, g, P, r, px, py, qa, qb, need0 && need1, ea, eb);
        if (need0) e[0] = ea;
        if (need1) e[1] = eb;
    }
    if (ok[1] && !need1 && !(init0 && c[1] == cur0)) e[1] = e[0];
    return decide_and_search<Row, LPS, BUF>(S.A, D, g, px, py, r, S.R, nI, S.o0, S.o1, cur0, cd0, c, ok, e, put);
}

template <class Row, int LPS, bool BUF, bool FF = false, class Nbr, class Put>
__device__ __forceinline__ uint32_t sweep_seed_with(const DirArgs& D, const Geo& g, int i, int j, int t, int nI, int r,
                                                    Nbr nbr, Put put)
{
    SeedStart<Row> S;
    seed_start<Row, LPS, BUF, FF>(S, D, g, i, j, t, nI, r);
    return seed_finish<Row, LPS, BUF>(S, D, g, i, j, t, nI, r, nbr, put);
}

// The displacements of the two propagation members of seed (i, j) at iteration t, read from
// clamped indices (a member off the grid is ignored by seed_finish) before the seed's other
// reads, as they start its longest chain of dependent reads; handed to seed_finish as its nbr.
struct Members {
    uint32_t n0, n1;   // the members (i - sx, j) and (i, j - sy)
    int i;
    __device__ __forceinline__ uint32_t operator()(int ni, int) const { return ni == i ? n1 : n0; }
};
__device__ __forceinline__ Members read_members(const uint32_t* disp, const Geo& g, int i, int j, int t)
{
    const int k = t & 3;
    const int sx = (k == 0 || k == 3) ? 1 : -1, sy = (k == 0 || k == 2) ? 1 : -1;
    Members m;
    m.n0 = disp[clampi(j, 0, g.ny - 1) * g.nx + clampi(i - sx, 0, g.nx - 1)];
    m.n1 = disp[clampi(j - sy, 0, g.ny - 1) * g.nx + clampi(i, 0, g.nx - 1)];
    m.i = i;
    return m;
}

// the half-sweep step in place: members from the field itself, a changed seed written back
template <class Row, int LPS, bool BUF>
__device__ __forceinline__ uint32_t sweep_seed(const DirArgs& D, const Geo& g, int i, int j, int t, int nI, int r)
{
    const Members nb = read_members(D.f.disp, g, i, j, t);
    return sweep_seed_with<Row, LPS, BUF>(D, g, i, j, t, nI, r, nb, PutSeed<typename Row::Dist>{D.f, j * g.nx + i, false});
}

// one half-sweep (Step 1, one colour of one iteration) of every seed of the launch
template <int C2, int PMAX, bool FIXED, int KIND>
__global__ __launch_bounds__(MATCH_TPB) void k_sweep(SweepArgs a)
{
    using Row = RowT<C2, PMAX, FIXED, KIND>;
    constexpr int LPS = PMAX;
    constexpr int GPB = MATCH_TPB / LPS;
    const Geo& g = a.g;
    const int nbx = (int)a.b.dnb.d;
    const LBlock lb = logical_block(a.b);
    const size_t zo = (size_t)lb.z * (size_t)a.b.zs;
    const DirArgs D = pair_dir(a.d[lb.dir], zo);
    const int r = threadIdx.x % LPS;
    const int gid = lb.x * GPB + threadIdx.x / LPS;
    const int hx = (g.nx + 1) >> 1;
    const int j = (int)fdiv((uint32_t)gid, g.dhx);   // gid / hx
    const int i = 2 * (gid - j * hx) + ((a.colour + j) & 1);
    uint32_t nev = 0;
    if (j < g.ny && i < g.nx) nev = sweep_seed<Row, LPS, true>(D, g, i, j, a.t, a.nI, r);
    count_evals(zoff(a.cnt, zo), lb.dir * nbx + lb.x, nev, r == 0);
}

// ---------------------------------------------------------------------------------------
// consecutive half-sweeps of a small level in one launch (Step 1 of Sec. III-B, 2-4 times)
// ---------------------------------------------------------------------------------------

// Work-group (x0, y0) owns a MULTI_TX x MULTI_TY tile of seeds, one 8-lane group per seed.
// Half-sweep m = 0 .. nph-1 updates the seeds of colour c[m] at iteration t[m] inside a
// rectangle R_m: R_{nph-1} is the tile, and R_m is R_{m+1} grown by one seed on the sides that
// half-sweep m+1's propagation looks back to, so that every member it reads lies in R_m (the
// launcher lays the rectangles out once for all tiles, plan_multi). The
// first half-sweep reads the field from the input buffer (which no work-group of the launch
// writes), the second its own seeds' values from there too; everything else comes from the
// results of the earlier half-sweeps, kept in LDS per colour over R_0. Every seed thus sees
// exactly the field that the half-sweeps in sequence give it. Only the tile's seeds are
// counted, and they are written to the output buffer after the last half-sweep of their
// colour, so the launch writes the whole field once.
constexpr int MULTI_TX = 4, MULTI_TY = 6, MULTI_MAXPH = 4;
constexpr int MULTI_W = MULTI_TX + MULTI_MAXPH - 1, MULTI_H = MULTI_TY + MULTI_MAXPH - 1;
static_assert((MULTI_W * MULTI_H + 1) / 2 <= MULTI_TPB / 8, "every half-sweep of a tile in one pass");

template <int C2, int PMAX, bool FIXED, int KIND>
__global__ __launch_bounds__(MULTI_TPB) void k_sweep_multi(SweepMultiArgs a)
{
    static_assert(PMAX == 8, "eight lanes per seed");
    using Row = RowT<C2, PMAX, FIXED, KIND>;
    using Dist = typename Row::Dist;
    constexpr int LPS = PMAX;
    __shared__ uint32_t ldisp[2][MULTI_W * MULTI_H];   // per colour, over R_0
    __shared__ Dist ldist[2][MULTI_W * MULTI_H];
    const Geo& g = a.g;
    const int nph = a.nph;   // 2..MULTI_MAXPH, checked by the launcher
    const int nbx = (int)a.b.dnb.d;
    const LBlock lb = logical_block(a.b);
    const size_t zo = (size_t)lb.z * (size_t)a.b.zs;
    const DirArgs D = pair_dir(a.d[lb.dir], zo);
    const Field out = pair_field(a.out[lb.dir], zo);
    const int ty = (int)fdiv((uint32_t)lb.x, a.dtx);   // tile row; a.dtx.d tiles per row
    const int x0 = (lb.x - ty * (int)a.dtx.d) * MULTI_TX, y0 = ty * MULTI_TY;   // both even
    const int r = threadIdx.x % LPS, grp = threadIdx.x / LPS;
    // ph[m]: R_m = [x0 + ax, x0 + ax + W) x [y0 + ay, y0 + ay + H) as bits 0-3 ax + 4, 4-7
    // ay + 4, 8-11 W, 12-15 H, 16 the colour parity (c[m] + ax + ay) & 1, 20-29 the multiplier
    // ceil(1024 / V) with V = W (W odd) or W / 2, which divides every q < 65 exactly as q M >> 10
    const int ox = x0 + (int)(a.ph[0] & 15u) - 4, oy = y0 + (int)((a.ph[0] >> 4) & 15u) - 4;   // R_0: LDS origin
    // group grp's seed of half-sweep m: the grp-th cell of colour c[m] of R_m in row order
    auto pick = [&](int m, int& x, int& y) {
        const uint32_t w = a.ph[m];
        const int Xa = x0 + (int)(w & 15u) - 4, Ya = y0 + (int)((w >> 4) & 15u) - 4;
        const int W = (int)((w >> 8) & 15u), H = (int)((w >> 12) & 15u);
        const int par = (int)((w >> 16) & 1u);   // (c[m] + Xa + Ya) & 1, as x0 + y0 is even
        const int M = (int)(w >> 20);
        x = -1;
        y = -1;
        if (W & 1) {   // colours alternate along the whole row-major order
            const int q = 2 * grp + par;
            if (q < W * H) {
                const int yy = (q * M) >> 10;   // q / W
                x = Xa + q - yy * W;
                y = Ya + yy;
            }
        } else if (grp < (W / 2) * H) {
            const int yy = (grp * M) >> 10;   // grp / (W / 2)
            y = Ya + yy;
            x = Xa + 2 * (grp - yy * (W / 2)) + ((par + yy) & 1);
        }
        return x >= 0 && y >= 0 && x < g.nx && y < g.ny;   // cells outside the grid are skipped
    };
    // The reads of a half-sweep that need nothing from the one before it (the seed's patch,
    // its field, its random offsets) are issued before the barrier that ends that one; the
    // barrier waits for LDS only, so they stay in flight across it.
    auto start = [&](SeedStart<Row>& S, int m, int x, int y) {
        seed_start<Row, LPS, true, true>(S, D, g, x, y, a.t[m], a.nI, r);
        if (m >= 2) {   // the result of half-sweep m - 2, visible since the barrier that ended it
            const int cell = (y - oy) * MULTI_W + (x - ox);
            S.cur0 = ldisp[a.c[m]][cell];
            S.cd0 = ldist[a.c[m]][cell];
        }
    };
    int x, y;
    bool have = pick(0, x, y);
    SeedStart<Row> S;
    if (have) start(S, 0, x, y);
    uint32_t nev = 0;
    for (int m = 0; m < nph; m++) {
        const int c = a.c[m], t = a.t[m];
        if (have) {
            const bool own = x >= x0 && x < x0 + MULTI_TX && y >= y0 && y < y0 + MULTI_TY;
            const bool last = m >= nph - 2;
            const int cell = (y - oy) * MULTI_W + (x - ox);
            const uint32_t* disp = D.f.disp;
            const uint32_t n = seed_finish<Row, LPS, true>(
                S, D, g, x, y, t, a.nI, r,
                [&](int ni, int nj) {
                    if (m == 0) return disp[clampi(nj, 0, g.ny - 1) * g.nx + clampi(ni, 0, g.nx - 1)];
                    return ldisp[c ^ 1][(nj - oy) * MULTI_W + (ni - ox)];   // a member in R_{m-1}
                },
                [&](uint32_t cur, Dist cd, bool) {
                    ldisp[c][cell] = cur;
                    ldist[c][cell] = cd;
                    if (own && last) {
                        out.disp[S.s] = cur;
                        ((Dist*)out.dist)[S.s] = cd;
                    }
                });
            if (own) nev += n;
        }
        if (m + 1 < nph) {
            have = pick(m + 1, x, y);
            if (have) start(S, m + 1, x, y);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    }
    count_evals(zoff(a.cnt, zo), lb.dir * nbx + lb.x, nev, r == 0);
}

// Two consecutive half-sweeps per launch on 6 x 8-seed tiles, for levels whose 4 x 6 tiles would
// take the chip twice over: half as many work-groups. Work-group (x0, y0) owns the tile, one
// 8-lane group per seed; the field is read only from the input buffer and the tile is written
// whole to the output buffer. First pass: the tile's seeds of colour c[0] at iteration t[0] and
// the seeds of that colour in the column and the row just outside the tile that the second
// half-sweep's propagation members come from (their results stay in LDS: 24 + 4 + 3 seeds, one
// pass of 32 groups). Second pass: the tile's seeds of the other colour at iteration t[1], their
// members from LDS. Only the tile's own seeds are counted.
constexpr int PAIR_TX = 6, PAIR_TY = 8;

template <int C2, int PMAX, bool FIXED, int KIND>
__global__ __launch_bounds__(MULTI_TPB) void k_sweep_pair(SweepMultiArgs a)
{
    static_assert(PMAX == 8, "eight lanes per seed");
    using Row = RowT<C2, PMAX, FIXED, KIND>;
    using Dist = typename Row::Dist;
    constexpr int LPS = PMAX;
    constexpr int EX = PAIR_TX + 2;                // row length of the tile and its border in LDS
    constexpr int HALF = PAIR_TX * PAIR_TY / 2;     // seeds of one colour in a tile
    static_assert(PAIR_TX % 2 == 0 && PAIR_TY % 2 == 0 && HALF + PAIR_TX / 2 + PAIR_TY / 2 <= MULTI_TPB / LPS,
                  "one pass per colour");
    __shared__ uint32_t first[(PAIR_TY + 2) * EX];   // first-pass displacements
    const Geo& g = a.g;
    const int c1 = a.c[0];
    const int nbx = (int)a.b.dnb.d;
    const LBlock lb = logical_block(a.b);
    const size_t zo = (size_t)lb.z * (size_t)a.b.zs;
    const DirArgs D = pair_dir(a.d[lb.dir], zo);
    const Field out = pair_field(a.out[lb.dir], zo);
    const int ty = (int)fdiv((uint32_t)lb.x, a.dtx);   // tile row; a.dtx.d tiles per row
    const int x0 = (lb.x - ty * (int)a.dtx.d) * PAIR_TX, y0 = ty * PAIR_TY;
    const int r = threadIdx.x % LPS, grp = threadIdx.x / LPS;
    // the second half-sweep's propagation members are (i - sx, j) and (i, j - sy)
    const int k2 = a.t[1] & 3;
    const int sx = (k2 == 0 || k2 == 3) ? 1 : -1, sy = (k2 == 0 || k2 == 2) ? 1 : -1;
    uint32_t nev = 0;
    {
        int i = -1, j = -1;
        bool own = false;
        if (grp < HALF) {
            j = y0 + grp / (PAIR_TX / 2);
            i = x0 + 2 * (grp % (PAIR_TX / 2)) + ((c1 + j + x0) & 1);
            own = true;
        } else if (grp < HALF + PAIR_TY / 2) {   // the look-back column
            i = sx == 1 ? x0 - 1 : x0 + PAIR_TX;
            j = y0 + 2 * (grp - HALF) + ((c1 + i + y0) & 1);
        } else if (grp < HALF + PAIR_TY / 2 + PAIR_TX / 2) {   // the look-back row
            j = sy == 1 ? y0 - 1 : y0 + PAIR_TY;
            i = x0 + 2 * (grp - HALF - PAIR_TY / 2) + ((c1 + j + x0) & 1);
        }
        if (i >= 0 && j >= 0 && i < g.nx && j < g.ny) {
            const uint32_t* disp = D.f.disp;
            const int s = j * g.nx + i;
            const int slot = (j - y0 + 1) * EX + (i - x0 + 1);
            const uint32_t n = sweep_seed_with<Row, LPS, true, true>(
                D, g, i, j, a.t[0], a.nI, r,
                [=](int ni, int nj) { return disp[clampi(nj, 0, g.ny - 1) * g.nx + clampi(ni, 0, g.nx - 1)]; },
                [&](uint32_t cur, Dist cd, bool) {
                    first[slot] = cur;
                    if (own) {
                        out.disp[s] = cur;
                        ((Dist*)out.dist)[s] = cd;
                    }
                });
            if (own) nev += n;
        }
    }
    __syncthreads();
    if (grp < HALF) {
        const int j = y0 + grp / (PAIR_TX / 2);
        const int i = x0 + 2 * (grp % (PAIR_TX / 2)) + ((1 - c1 + j + x0) & 1);
        if (i < g.nx && j < g.ny) {
            // (ni, nj) lies in the tile or its border: seeds of colour c[0] priced above (or
            // outside the grid, where the value is ignored)
            nev += sweep_seed_with<Row, LPS, true, true>(
                D, g, i, j, a.t[1], a.nI, r, [&](int ni, int nj) { return first[(nj - y0 + 1) * EX + (ni - x0 + 1)]; },
                PutSeed<Dist>{out, j * g.nx + i, true});
        }
    }
    count_evals(zoff(a.cnt, zo), lb.dir * nbx + lb.x, nev, r == 0);
}

// ---------------------------------------------------------------------------------------
// initial field at the coarsest level: random displacement in [-R, R]^2 (drawn in k_prep) or
// the exact best displacement in that window (dy outer, dx inner, strictly smaller wins)
// ---------------------------------------------------------------------------------------

template <int C2, int PMAX, bool FIXED, int KIND>
__global__ __launch_bounds__(MATCH_TPB) void k_init(InitArgs a)
{
    using Row = RowT<C2, PMAX, FIXED, KIND>;
    constexpr int LPS = PMAX;
    constexpr int GPB = MATCH_TPB / LPS;
    const Geo& g = a.g;
    const int nbx = (int)a.b.dnb.d;
    const LBlock lb = logical_block(a.b);
    const size_t zo = (size_t)lb.z * (size_t)a.b.zs;
    const DirArgs D = pair_dir(a.d[lb.dir], zo);
    const int r = threadIdx.x % LPS;
    const int s = lb.x * GPB + threadIdx.x / LPS;
    uint32_t nev = 0;
    if (s < g.nx * g.ny) {
        const int j = (int)fdiv((uint32_t)s, g.dnx), i = s - j * g.nx;
        const int px = grid_pos(i, g.w, g), py = grid_pos(j, g.h, g);
        const int P = D.P;
        const short2 o = a.exhaustive ? make_short2(0, 0) : D.rnd0[s];   // read before the patch
        Row A;
        load_own<true>(A, D.Ga, g, P, r, px, py);
        using Dist = typename Row::Dist;
        uint32_t best = UNINIT;
        Dist bd = NO_DIST;
        if (!a.exhaustive) {
            best = target(px, py, o.x, o.y, g);
            bd = patch_cost<Row, LPS, true>(A, D.Gb, g, P, r, px + d_x(best), py + d_y(best));
            nev++;
        } else {
            // the window clipped to the image, in the same (dy outer, dx inner) order
            const int y0 = max(-a.R, -py), y1 = min(a.R, g.h - 1 - py);
            const int x0 = max(-a.R, -px), x1 = min(a.R, g.w - 1 - px);
            for (int dy = y0; dy <= y1; dy++) {
                for (int dx = x0; dx <= x1; dx++) {
                    const Dist e = patch_cost<Row, LPS, true>(A, D.Gb, g, P, r, px + dx, py + dy);
                    nev++;
                    if (best == UNINIT || e < bd) { best = pack_d(dx, dy); bd = e; }
                }
            }
        }
        if (r == 0) {
            D.f.disp[s] = best;
            ((Dist*)D.f.dist)[s] = bd;
            D.f.flags[s] = 0;
        }
    }
    count_evals(zoff(a.cnt, zo), lb.dir * nbx + lb.x, nev, r == 0);
}

// ---------------------------------------------------------------------------------------
// Step 4-5 toward the finer level (Eq. 6 with eta = s, Eq. 8): the child takes twice the
// displacement of the nearest parent seed to (x/2, y/2) if that parent is an inlier
// ---------------------------------------------------------------------------------------

template <int C2, int PMAX, bool FIXED, int KIND>
__global__ __launch_bounds__(MATCH_TPB) void k_down(TransArgs a)
{
    using Row = RowT<C2, PMAX, FIXED, KIND>;
    constexpr int LPS = PMAX;
    constexpr int GPB = MATCH_TPB / LPS;
    const Geo& g = a.g;
    const int nbx = (int)a.b.dnb.d;
    const LBlock lb = logical_block(a.b);
    const size_t zo = (size_t)lb.z * (size_t)a.b.zs;
    const DirArgs D = pair_dir(a.d[lb.dir], zo);
    const Field S = pair_field(a.src[lb.dir], zo);
    const int r = threadIdx.x % LPS;
    const int s = lb.x * GPB + threadIdx.x / LPS;
    uint32_t nev = 0;
    if (s < g.nx * g.ny) {
        const int j = (int)fdiv((uint32_t)s, g.dnx), i = s - j * g.nx;
        const int px = grid_pos(i, g.w, g), py = grid_pos(j, g.h, g);
        const int ps = grid_near(py >> 1, a.gs.ny, a.gs) * a.gs.nx + grid_near(px >> 1, a.gs.nx, a.gs);
        // the parent's state, then this seed's patch (all in flight together)
        const uint8_t pf = S.flags[ps];
        const uint32_t pd = S.disp[ps];
        Row A;
        load_own<true>(A, D.Ga, g, D.P, r, px, py);
        const bool par_inl = (pf & ST_INL) != 0;
        uint32_t disp = UNINIT;
        typename Row::Dist dist = NO_DIST;
        if (par_inl) {
            disp = target(px, py, 2 * d_x(pd), 2 * d_y(pd), g);
            dist = patch_cost<Row, LPS, true>(A, D.Gb, g, D.P, r, px + d_x(disp), py + d_y(disp));
            nev++;
        }
        if (r == 0) {
            D.f.disp[s] = disp;
            ((typename Row::Dist*)D.f.dist)[s] = dist;
            D.f.flags[s] = (a.carry_record && par_inl) ? ST_REC : 0;
        }
    }
    count_evals(zoff(a.cnt, zo), lb.dir * nbx + lb.x, nev, r == 0);
}

// ---------------------------------------------------------------------------------------
// Step 4-5 toward the coarser level (Eq. 6 with eta = 1/s, Eq. 8): the mean displacement of
// the inlier children divided by 2, rounded to nearest with ties away from zero
// ---------------------------------------------------------------------------------------

__device__ __forceinline__ int div_round(int num, int den)   // den > 0
{
    int a = num < 0 ? -num : num;
    int q = (2 * a + den) / (2 * den);
    return num < 0 ? -q : q;
}

template <int C2, int PMAX, bool FIXED, int KIND>
__global__ __launch_bounds__(MATCH_TPB) void k_up(TransArgs a)
{
    using Row = RowT<C2, PMAX, FIXED, KIND>;
    constexpr int LPS = PMAX;
    constexpr int GPB = MATCH_TPB / LPS;
    const Geo& g = a.g;     // coarse level being entered
    const Geo& f = a.gs;    // finer source level
    const int nbx = (int)a.b.dnb.d;
    const LBlock lb = logical_block(a.b);
    const size_t zo = (size_t)lb.z * (size_t)a.b.zs;
    const DirArgs D = pair_dir(a.d[lb.dir], zo);
    const Field S = pair_field(a.src[lb.dir], zo);
    const int r = threadIdx.x % LPS;
    const int s = lb.x * GPB + threadIdx.x / LPS;
    uint32_t nev = 0;
    if (s < g.nx * g.ny) {
        const int cj = (int)fdiv((uint32_t)s, g.dnx), ci = s - cj * g.nx;
        const int px = grid_pos(ci, g.w, g), py = grid_pos(cj, g.h, g);
        int sx = 0, sy = 0, cnt = 0;
        // children: finer seeds whose nearest coarse seed (as in k_down) is this one
        for (int fj = max(0, 2 * cj - 3); fj <= min(f.ny - 1, 2 * cj + 4); fj++) {
            const int fy = grid_pos(fj, f.h, f);
            if (grid_near(fy >> 1, g.ny, g) != cj) continue;
            for (int fi = max(0, 2 * ci - 3); fi <= min(f.nx - 1, 2 * ci + 4); fi++) {
                const int fx = grid_pos(fi, f.w, f);
                if (grid_near(fx >> 1, g.nx, g) != ci) continue;
                const int fs = fj * f.nx + fi;
                if (!(S.flags[fs] & ST_INL)) continue;
                const uint32_t d = S.disp[fs];
                sx += d_x(d); sy += d_y(d); cnt++;
            }
        }
        uint32_t disp = UNINIT;
        typename Row::Dist dist = NO_DIST;
        if (cnt > 0) {
            disp = target(px, py, div_round(sx, 2 * cnt), div_round(sy, 2 * cnt), g);
            Row A;
            load_own<true>(A, D.Ga, g, D.P, r, px, py);
            dist = patch_cost<Row, LPS, true>(A, D.Gb, g, D.P, r, px + d_x(disp), py + d_y(disp));
            nev++;
        }
        if (r == 0) {
            D.f.disp[s] = disp;
            ((typename Row::Dist*)D.f.dist)[s] = dist;
            D.f.flags[s] = cnt > 0 ? ST_REC : 0;
        }
    }
    count_evals(zoff(a.cnt, zo), lb.dir * nbx + lb.x, nev, r == 0);
}

// ---------------------------------------------------------------------------------------
// Step 2-3: forward-backward consistency check and the record update of Eq. 7
// ---------------------------------------------------------------------------------------

// Steps 2-3 (Sec. III-C, Eq. 7) for seed s of field F, whose displacement is d and flags fl,
// against the opposite field O: the backward match consulted is the one at the opposite seed
// nearest to p + d; consistent iff the two displacements cancel within tau. Returns whether
// the seed is an inlier after the record update. (The opposite displacement is read only
// when it is needed.)
__device__ __forceinline__ int check_partner(const Geo& g, int s, uint32_t d)
{
    const int j = (int)fdiv((uint32_t)s, g.dnx), i = s - j * g.nx;
    const int qx = grid_pos(i, g.w, g) + d_x(d), qy = grid_pos(j, g.h, g) + d_y(d);
    return grid_near(qy, g.ny, g) * g.nx + grid_near(qx, g.nx, g);
}
// the same decision from the opposite field's displacement od at check_partner(g, s, d), read
// beforehand (whatever d: the partner index is inside the grid for any d)
__device__ __forceinline__ bool check_decide(uint32_t d, uint32_t od, uint8_t fl, int fwd_bwd, int tau2, int rec_valid)
{
    bool ok = d != UNINIT;
    if (fwd_bwd) {
        const int ex = d_x(d) + d_x(od), ey = d_y(d) + d_y(od);
        ok = ok && od != UNINIT && ex * ex + ey * ey <= tau2;
    }
    return rec_valid ? (ok && (fl & ST_REC)) : ok;
}
__device__ __forceinline__ bool check_inlier(const Field& O, const Geo& g, int s, uint32_t d, uint8_t fl, int fwd_bwd,
                                             int tau2, int rec_valid)
{
    bool ok = d != UNINIT;
    if (ok && fwd_bwd) {
        const uint32_t od = O.disp[check_partner(g, s, d)];
        if (od == UNINIT) ok = false;
        else {
            const int ex = d_x(d) + d_x(od), ey = d_y(d) + d_y(od);
            ok = ex * ex + ey * ey <= tau2;
        }
    }
    return rec_valid ? (ok && (fl & ST_REC)) : ok;
}

// Steps 2-3 for seed s of field F against the opposite field O, written to its flags
__device__ __forceinline__ void check_seed(const Field& F, const Field& O, const Geo& g, int s, int fwd_bwd, int tau2,
                                           int rec_valid)
{
    const uint32_t d = F.disp[s];
    const uint8_t fl = F.flags[s];
    const bool inl = check_inlier(O, g, s, d, fl, fwd_bwd, tau2, rec_valid);
    F.flags[s] = (uint8_t)((fl & ST_REC) | (inl ? ST_INL : 0));
}

__global__ __launch_bounds__(256) void k_check(CheckArgs a)
{
    const Geo& g = a.g;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.nx * g.ny) return;
    const size_t zo = (size_t)blockIdx.z * (size_t)a.b.zs;
    const Field F = pair_field(a.f[blockIdx.y], zo);
    const Field O = pair_field(a.f[1 - blockIdx.y], zo);
    check_seed(F, O, g, s, a.fwd_bwd, a.tau2, a.rec_valid);
}

// ---------------------------------------------------------------------------------------
// Entering a finer level in one launch. The results equal those of the coarser level's check
// (Steps 2-3), the transition of Eq. 6 and 8 (Steps 4-5) and the first half-sweep of Step 1
// launched one after the other. Per direction and pair the work-groups cover: the seeds of
// the first colour, each of which derives its own start and the starts of the two neighbours
// it propagates from (t = 0) from their parents' checks and then takes its step; the seeds of
// the second colour, which take their start; and the coarser seeds, whose check is written
// to their flags. A start depends only on the parent's state, so no seed waits for another.
// ---------------------------------------------------------------------------------------

// INIT: the initial level instead, whose starts are the seeds' random displacements
template <class Row, int LPS, bool SWEEP, bool INIT>
__device__ __forceinline__ uint32_t enter_seed(const EnterArgs& a, const DirArgs& D, const Field& S, const Field& O,
                                               int i, int j, bool first, int r)
{
    constexpr int M = SWEEP ? 3 : 1;   // starts needed: this seed's, and its two neighbours' for the step
    first = SWEEP && first;
    using Dist = typename Row::Dist;
    const Geo& g = a.g;
    const Geo& gs = a.gs;
    const int s = j * g.nx + i;
    const int px = grid_pos(i, g.w, g), py = grid_pos(j, g.h, g);
    const int P = D.P;
    // m = 0: this seed; m = 1, 2: the neighbours (i - 1, j) and (i, j - 1) that the step at
    // t = 0 propagates from (the first of the Delta orders of Eq. 4). Their parents' states are
    // read first (they start the longest chain of reads), then this seed's patch.
    int qx[3], qy[3], ps[3];
    bool on[3] = {false, false, false};
    uint32_t pd[3];
    uint8_t pf[3];
    short2 o_init[3];
#pragma unroll
    for (int m = 0; m < M; m++) {
        const int ni = m == 1 ? i - 1 : i, nj = m == 2 ? j - 1 : j;
        on[m] = m == 0 || (first && ni >= 0 && nj >= 0);
        qx[m] = grid_pos(max(ni, 0), g.w, g);
        qy[m] = grid_pos(max(nj, 0), g.h, g);
        if constexpr (INIT) {
            o_init[m] = D.rnd0[max(nj, 0) * g.nx + max(ni, 0)];
        } else {
            ps[m] = grid_near(qy[m] >> 1, gs.ny, gs) * gs.nx + grid_near(qx[m] >> 1, gs.nx, gs);
            pd[m] = S.disp[ps[m]];
            pf[m] = S.flags[ps[m]];
        }
    }
    Row A;
    load_own<true>(A, D.Ga, g, P, r, px, py);
    const short2* R = D.rnd + (size_t)s * a.nI;   // offsets of the step at t = 0
    const short2 o0 = R[0], o1 = R[a.nI > 1 ? 1 : 0];
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (SWEEP && !INIT) {
        // k_enter (small levels): the parents' checks read the opposite field while the patches
        // at the starts the parents would give are priced, one round trip fewer; a price is
        // used only where its start holds (the decisions are those of the path below)
        uint32_t od[3], spec[3];
#pragma unroll
        for (int m = 0; m < M; m++) {
            od[m] = a.fwd_bwd ? O.disp[check_partner(gs, ps[m], pd[m])] : UNINIT;
            spec[m] = target(qx[m], qy[m], 2 * d_x(pd[m]), 2 * d_y(pd[m]), g);
        }
        if (!first) {   // this seed's start alone
            const Dist ds = patch_cost<Row, LPS, true>(A, D.Gb, g, P, r, px + d_x(spec[0]), py + d_y(spec[0]));
            const bool in0 = check_decide(pd[0], od[0], pf[0], a.fwd_bwd, a.tau2, a.rec_valid);
            if (r == 0) {
                D.f.flags[s] = (a.carry_record && in0) ? ST_REC : 0;
                D.f.disp[s] = in0 ? spec[0] : UNINIT;
                ((Dist*)D.f.dist)[s] = in0 ? ds : (Dist)NO_DIST;
            }
            return in0 ? 1u : 0u;
        }
        const uint32_t cs0 = target(px, py, d_x(spec[1]), d_y(spec[1]), g);
        const uint32_t cs1 = target(px, py, d_x(spec[2]), d_y(spec[2]), g);
        int tx[3] = {px + d_x(spec[0]), px + d_x(cs0), px + d_x(cs1)};
        int ty[3] = {py + d_y(spec[0]), py + d_y(cs0), py + d_y(cs1)};
        Dist pe[3];
        patch_cost3<Row, LPS, true>(A, D.Gb, g, P, r, tx, ty, pe);
        uint32_t st[3];
#pragma unroll
        for (int m = 0; m < 3; m++) {
            const bool in = on[m] && check_decide(pd[m], od[m], pf[m], a.fwd_bwd, a.tau2, a.rec_valid);
            st[m] = in ? spec[m] : UNINIT;
            if (m == 0 && r == 0) D.f.flags[s] = (a.carry_record && in) ? ST_REC : 0;
        }
        const uint32_t cur0 = st[0];
        const bool init0 = cur0 != UNINIT;
        uint32_t c[2];
        bool ok[2];
#pragma unroll
        for (int m = 0; m < 2; m++) {
            ok[m] = st[m + 1] != UNINIT;
            c[m] = ok[m] ? target(px, py, d_x(st[m + 1]), d_y(st[m + 1]), g) : cur0;
        }
        const bool need0 = ok[0] && !(init0 && c[0] == cur0);
        const bool need1 = ok[1] && !(init0 && c[1] == cur0) && !(ok[0] && c[1] == c[0]);
        const Dist cd0 = init0 ? pe[0] : (Dist)NO_DIST;
        Dist e[2] = {need0 ? pe[1] : cd0, need1 ? pe[2] : cd0};
        if (ok[1] && !need1 && !(init0 && c[1] == cur0)) e[1] = e[0];
        return (init0 ? 1u : 0u) + decide_and_search<Row, LPS, true>(A, D, g, px, py, r, R, a.nI, o0, o1, cur0, cd0, c,
                                                                      ok, e, PutSeed<Dist>{D.f, s, true});
    }
    // the parents' checks (Steps 2-3 at the coarser level) and the starts of Eq. 6
    uint32_t st[3] = {UNINIT, UNINIT, UNINIT};
    bool inl[3] = {false, false, false};
#pragma unroll
    for (int m = 0; m < M; m++) {
        if constexpr (INIT) {   // the random start of the initial field, clamped into the image
            inl[m] = false;
            st[m] = on[m] ? target(qx[m], qy[m], o_init[m].x, o_init[m].y, g) : UNINIT;
        } else {
            inl[m] = on[m] && check_inlier(O, gs, ps[m], pd[m], pf[m], a.fwd_bwd, a.tau2, a.rec_valid);
            st[m] = inl[m] ? target(qx[m], qy[m], 2 * d_x(pd[m]), 2 * d_y(pd[m]), g) : UNINIT;
        }
    }
    const uint32_t cur0 = st[0];
    const bool init0 = cur0 != UNINIT;
    if (r == 0) D.f.flags[s] = (a.carry_record && inl[0]) ? ST_REC : 0;
    uint32_t nev = init0 ? 1u : 0u;
    if (!SWEEP || !first) {
        Dist d0 = NO_DIST;
        if (init0) d0 = patch_cost<Row, LPS, true>(A, D.Gb, g, P, r, px + d_x(cur0), py + d_y(cur0));
        if (r == 0) {
            D.f.disp[s] = cur0;
            ((Dist*)D.f.dist)[s] = d0;
        }
        return nev;
    }
    // the step at t = 0, as in sweep_seed, from the starts just derived: this seed's start and
    // the new propagation members are priced in one round trip
    uint32_t c[2];
    bool ok[2];
#pragma unroll
    for (int m = 0; m < 2; m++) {
        ok[m] = st[m + 1] != UNINIT;
        c[m] = ok[m] ? target(px, py, d_x(st[m + 1]), d_y(st[m + 1]), g) : cur0;
    }
    const bool need0 = ok[0] && !(init0 && c[0] == cur0);
    const bool need1 = ok[1] && !(init0 && c[1] == cur0) && !(ok[0] && c[1] == c[0]);
    Dist cd0 = NO_DIST;
    Dist e[2];
    if (init0 || need0 || need1) {
        const uint32_t q0 = init0 ? cur0 : (need0 ? c[0] : c[1]);
        const uint32_t qa = need0 ? c[0] : (need1 ? c[1] : q0), qb = need1 ? c[1] : qa;
        int tx[3] = {px + d_x(q0), px + d_x(qa), px + d_x(qb)};
        int ty[3] = {py + d_y(q0), py + d_y(qa), py + d_y(qb)};
        Dist pe[3];
        patch_cost3<Row, LPS, true>(A, D.Gb, g, P, r, tx, ty, pe);
        if (init0) cd0 = pe[0];
        e[0] = need0 ? pe[1] : cd0;
        e[1] = need1 ? pe[2] : cd0;
    } else {
        e[0] = cd0;
        e[1] = cd0;
    }
    if (ok[1] && !need1 && !(init0 && c[1] == cur0)) e[1] = e[0];
    return nev + decide_and_search<Row, LPS, true>(A, D, g, px, py, r, R, a.nI, o0, o1, cur0, cd0, c, ok, e,
                                                   PutSeed<Dist>{D.f, s, true});
}

template <int C2, int PMAX, bool FIXED, int KIND, bool SWEEP, bool INIT>
__device__ __forceinline__ void enter_body(const EnterArgs& a)
{
    using Row = RowT<C2, PMAX, FIXED, KIND>;
    constexpr int LPS = PMAX;
    constexpr int GPB = MATCH_TPB / LPS;
    const int nbx = 2 * a.nb_col + a.nb_chk;   // == a.b.dnb.d
    const LBlock lb = logical_block(a.b);
    const size_t zo = (size_t)lb.z * (size_t)a.b.zs;
    const Field S = pair_field(a.src[lb.dir], zo);       // the coarser field of this direction
    const Field O = pair_field(a.src[1 - lb.dir], zo);   // and of the opposite direction
    uint32_t nev = 0;
    bool leader = false;
    if (lb.x >= 2 * a.nb_col) {
        // the coarser level's check, one seed per thread
        const int ps = (lb.x - 2 * a.nb_col) * MATCH_TPB + threadIdx.x;
        if (ps < a.gs.nx * a.gs.ny) check_seed(S, O, a.gs, ps, a.fwd_bwd, a.tau2, a.rec_valid);
    } else {
        const DirArgs D = pair_dir(a.d[lb.dir], zo);
        const int colour = lb.x >= a.nb_col ? 1 : 0;
        const int r = threadIdx.x % LPS;
        const int gid = (lb.x - colour * a.nb_col) * GPB + threadIdx.x / LPS;
        const int hx = (a.g.nx + 1) >> 1;
        const int j = (int)fdiv((uint32_t)gid, a.g.dhx);   // gid / hx
        const int i = 2 * (gid - j * hx) + ((colour + j) & 1);
        leader = r == 0;
        if (j < a.g.ny && i < a.g.nx) nev = enter_seed<Row, LPS, SWEEP, INIT>(a, D, S, O, i, j, colour == 0, r);
    }
    count_evals(zoff(a.cnt, zo), lb.dir * nbx + lb.x, nev, leader);
}

// the coarser level's check, the transition and the first half-sweep
template <int C2, int PMAX, bool FIXED, int KIND>
__global__ __launch_bounds__(MATCH_TPB) void k_enter(EnterArgs a)
{
    enter_body<C2, PMAX, FIXED, KIND, true, false>(a);
}

// the coarser level's check and the transition (both colours take their start only)
template <int C2, int PMAX, bool FIXED, int KIND>
__global__ __launch_bounds__(MATCH_TPB) void k_enter_start(EnterArgs a)
{
    enter_body<C2, PMAX, FIXED, KIND, false, false>(a);
}

// the initial level's random starts (Sec. III-B, III-D) and its first half-sweep
template <int C2, int PMAX, bool FIXED, int KIND>
__global__ __launch_bounds__(MATCH_TPB) void k_enter_init(EnterArgs a)
{
    enter_body<C2, PMAX, FIXED, KIND, true, true>(a);
}

// ---------------------------------------------------------------------------------------
// Step 1 of a small level in one work-group per pair and direction: both gradient images and
// the field are copied into LDS, every half-sweep runs between work-group barriers and the
// field goes back to HBM (Steps 2-3 follow in k_check). The seeds and their decisions are
// those of k_sweep; only the memory they live in differs.
// ---------------------------------------------------------------------------------------

// dst[q] = src[q] for q < n by the NT threads of the work-group, U loads in flight per thread
// (whole rounds unguarded, so the values stay in registers; the rest one at a time)
template <int NT, int U, class T>
__device__ __forceinline__ void copy_in(T* dst, const T* src, int n)
{
    int q = threadIdx.x;
    for (; q + (U - 1) * NT < n; q += U * NT) {
        T v[U];
#pragma unroll
        for (int u = 0; u < U; u++) v[u] = src[q + u * NT];
#pragma unroll
        for (int u = 0; u < U; u++) dst[q + u * NT] = v[u];
    }
    for (; q < n; q += NT) dst[q] = src[q];
}

template <int PMAX, bool F32>
struct LevelShape {
    // the sweep's registers per lane bound the work-group size
    static constexpr int threads = !F32 ? (PMAX == 8 ? 1024 : 512) : (PMAX == 8 ? 512 : 256);
};

template <int C2, int PMAX, bool FIXED, int KIND>
__global__ __launch_bounds__((LevelShape<PMAX, KIND == 1>::threads)) void k_level(LevelArgs a)
{
    using Row = RowT<C2, PMAX, FIXED, KIND>;
    constexpr int LPS = PMAX;
    constexpr int NT = LevelShape<PMAX, KIND == 1>::threads;
    constexpr int NG = NT / LPS;
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ uint32_t evsum;
    const Geo& g = a.g;
    const int n = g.nx * g.ny;
    const int dir = blockIdx.x & 1;
    const size_t zo = (size_t)(blockIdx.x >> 1) * (size_t)a.b.zs;
    const DirArgs H = pair_dir(a.d[dir], zo);
    const LevelLayout& Y = a.lay;
    uint8_t* GA = lds;
    uint8_t* GB = lds + Y.gstride;
    uint32_t* disp = (uint32_t*)(lds + Y.disp);
    using Dist = typename Row::Dist;
    Dist* dist = (Dist*)(lds + Y.dist);
    Dist* const hdist = (Dist*)H.f.dist;
    short2* rnd = (short2*)(lds + Y.rnd);
    // copy in: both padded gradient images (16-byte pieces), the field and the level's
    // random-search offsets, several loads in flight per thread
    {
        const int nq = (int)(a.gbytes / 16);   // gbytes is rounded up to 16 inside the 256-aligned image
        copy_in<NT, 4>((uint4*)GA, (const uint4*)((const uint8_t*)H.Ga - a.gorig), nq);
        copy_in<NT, 4>((uint4*)GB, (const uint4*)((const uint8_t*)H.Gb - a.gorig), nq);
        copy_in<NT, 2>(disp, (const uint32_t*)H.f.disp, n);
        copy_in<NT, 2>(dist, (const Dist*)hdist, n);
        copy_in<NT, 4>(rnd, H.rnd, a.iters * n * a.nI);
        if (threadIdx.x == 0) evsum = 0;
    }
    __syncthreads();
    DirArgs L = H;
    L.Ga = GA + a.gorig;
    L.Gb = GB + a.gorig;
    L.f.disp = disp;
    L.f.dist = dist;
    L.rnd = rnd;
    L.f.flags = nullptr;   // not used by Step 1
    const int r = threadIdx.x % LPS;
    const int hx = (g.nx + 1) >> 1;
    const int per = hx * g.ny;
    uint32_t nev = 0;
    for (int t = 0; t < a.iters; t++) {
        for (int colour = 0; colour < 2; colour++) {
            for (int q = threadIdx.x / LPS; q < per; q += NG) {
                const int j = (int)fdiv((uint32_t)q, g.dhx);   // q / hx
                const int i = 2 * (q - j * hx) + ((colour + j) & 1);
                if (i < g.nx) nev += sweep_seed<Row, LPS, false>(L, g, i, j, t, a.nI, r);
            }
            __syncthreads();
        }
    }
    if (r == 0 && nev) atomicAdd(&evsum, nev);
    for (int q = threadIdx.x; q < n; q += NT) {
        H.f.disp[q] = disp[q];
        hdist[q] = dist[q];
    }
    __syncthreads();
    if (a.cnt && threadIdx.x == 0) zoff(a.cnt, zo)[dir] = evsum;
}

// ---------------------------------------------------------------------------------------
// small-region removal (Sec. III-E): the inliers of the level-0 forward field are segmented
// into 4-connected regions of close displacements by union-find on a label array (a root is
// its own label, a label never exceeds its index and only decreases, joins are atomicMin on
// roots), then the inliers of regions smaller than min_px pixels lose their inlier flag. The
// resulting flags do not depend on the order of the joins.
// ---------------------------------------------------------------------------------------

// Root of x. Labels strictly decrease along the walk, so it ends within n steps; the bound
// also holds while other threads lower labels. On the way every visited label is lowered to
// its grandparent (an ancestor, so the regions do not change; atomicMin never raises a label
// another thread has just lowered), which keeps the walks short.
__device__ __forceinline__ int cc_find(int32_t* L, int x, int n)
{
    int y = __atomic_load_n(&L[x], __ATOMIC_RELAXED);
    for (int k = 0; k < n && y != x; k++) {
        const int z = __atomic_load_n(&L[y], __ATOMIC_RELAXED);
        if (z == y) return y;
        atomicMin(&L[x], z);
        x = y;
        y = z;
    }
    return x;
}

// Join the regions of a and b: hook the larger root under the smaller. When another thread
// moved the larger root first, retry from its new parent; every retry lowers that root, so
// the loop ends within n rounds (the bound keeps it finite whatever happens).
__device__ __forceinline__ void cc_union(int32_t* L, int a, int b, int n)
{
    for (int k = 0; k <= n; k++) {
        a = cc_find(L, a, n);
        b = cc_find(L, b, n);
        if (a == b) return;
        if (a < b) { const int t = a; a = b; b = t; }
        const int old = atomicMin(&L[a], b);
        if (old == a) return;
        a = old;
    }
}

__device__ __forceinline__ bool cc_linked(const Field& f, int s, int t, long long link2)
{
    const uint32_t a = f.disp[s], b = f.disp[t];
    const long long ex = d_x(a) - d_x(b), ey = d_y(a) - d_y(b);
    return ex * ex + ey * ey < link2;
}

__global__ __launch_bounds__(256) void k_cc_init(RegionArgs a)
{
    const int n = a.g.nx * a.g.ny;
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    const size_t zo = (size_t)blockIdx.z * (size_t)a.b.zs;
    zoff(a.label, zo)[s] = s;
    zoff(a.size, zo)[s] = 0;
}

__global__ __launch_bounds__(256) void k_cc_union(RegionArgs a)
{
    const Geo& g = a.g;
    const int n = g.nx * g.ny;
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    const size_t zo = (size_t)blockIdx.z * (size_t)a.b.zs;
    const Field f = pair_field(a.f, zo);
    int32_t* L = zoff(a.label, zo);
    if (!(f.flags[s] & ST_INL)) return;
    const int j = (int)fdiv((uint32_t)s, g.dnx), i = s - j * g.nx;
    if (i + 1 < g.nx && (f.flags[s + 1] & ST_INL) && cc_linked(f, s, s + 1, a.link2)) cc_union(L, s, s + 1, n);
    if (j + 1 < g.ny && (f.flags[s + g.nx] & ST_INL) && cc_linked(f, s, s + g.nx, a.link2))
        cc_union(L, s, s + g.nx, n);
}

// Region sizes: each inlier finds its root; the lanes of a wave that share a root add their
// count with one atomic (neighbouring seeds mostly share one region).
__global__ __launch_bounds__(256) void k_cc_size(RegionArgs a)
{
    const int n = a.g.nx * a.g.ny;
    const int s = blockIdx.x * 256 + threadIdx.x;
    const size_t zo = (size_t)blockIdx.z * (size_t)a.b.zs;
    const Field f = pair_field(a.f, zo);
    int32_t* L = zoff(a.label, zo);
    int32_t* size = zoff(a.size, zo);
    bool pending = s < n && (f.flags[s] & ST_INL);
    int r = -1;
    if (pending) {
        r = cc_find(L, s, n);
        L[s] = r;   // a root stays a root now that every join is done
    }
    const int lane = threadIdx.x & 63;
    unsigned long long left = __ballot(pending);
    while (left) {   // one round per distinct root among the wave's lanes
        const int leader = __ffsll((long long)left) - 1;
        const int rl = __shfl(r, leader, 64);
        const unsigned long long same = __ballot(pending && r == rl);
        if (lane == leader) atomicAdd(size + rl, (int)__popcll(same));
        if (pending && r == rl) pending = false;
        left &= ~same;
    }
}

__global__ __launch_bounds__(256) void k_cc_apply(RegionArgs a)
{
    const int n = a.g.nx * a.g.ny;
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    const size_t zo = (size_t)blockIdx.z * (size_t)a.b.zs;
    const Field f = pair_field(a.f, zo);
    const uint8_t fl = f.flags[s];
    if (!(fl & ST_INL)) return;
    const int r = zoff(a.label, zo)[s];
    const long long area = (long long)zoff(a.size, zo)[r] * a.g.stride * a.g.stride;
    if (area < a.min_px) f.flags[s] = (uint8_t)(fl & ~ST_INL);
}

// ---------------------------------------------------------------------------------------
// output on the level-0 grid and the compaction of forward inliers (Sec. III-G)
// ---------------------------------------------------------------------------------------

// Block x of direction y writes the matches of seeds [256 x, 256 x + 256). With compaction,
// a forward block also places its inliers, in seed order, after those of the blocks before
// it: it counts them from the flags itself (no pass between blocks) and ranks its own with
// wave ballots; the last block writes the total.
__global__ __launch_bounds__(256) void k_output(OutArgs a)
{
    __shared__ uint32_t part[4], wtot[4];
    const Geo& g = a.g;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = g.nx * g.ny;
    const int dir = blockIdx.y;
    const size_t zo = (size_t)blockIdx.z * (size_t)a.b.zs;
    const Field f = pair_field(a.f[dir], zo);
    const PairTab* tz = a.tab ? a.tab + blockIdx.z : nullptr;
    pgm_match_t* out = tz ? tz->out[dir] : a.out[dir] + (size_t)blockIdx.z * n;
    pgm_match_t* compact = tz ? tz->compact : (a.compact ? a.compact + (size_t)blockIdx.z * n : nullptr);
    int32_t* n_out = tz ? tz->n_in : (a.n_out ? a.n_out + blockIdx.z : nullptr);
    const bool counts = dir == 0 && (compact || n_out);   // uniform over the block
    // inliers before this block (compaction): the flags of its 256 x seeds, 16 per load
    // (256-aligned array), eight loads in flight per thread; the first eight are issued
    // together with the seed's own reads
    const uint4* fl4 = (const uint4*)f.flags;
    const int nq = counts ? (int)blockIdx.x * 16 : 0;
    uint4 w[8];
#pragma unroll
    for (int u = 0; u < 8; u++) w[u] = (int)threadIdx.x + u * 256 < nq ? fl4[threadIdx.x + u * 256] : make_uint4(0u, 0u, 0u, 0u);
    bool inl = false;
    pgm_match_t m;
    if (s < n) {
        const int j = (int)fdiv((uint32_t)s, g.dnx), i = s - j * g.nx;
        const uint32_t d = f.disp[s];
        const uint8_t fl = f.flags[s];
        m.x1 = grid_pos(i, g.w, g);
        m.y1 = grid_pos(j, g.h, g);
        const bool init = d != UNINIT;
        m.x2 = m.x1 + (init ? d_x(d) : 0);
        m.y2 = m.y1 + (init ? d_y(d) : 0);
        // the squared metric's 64-bit sum is reported clamped to 31 bits (decisions used it whole)
        const uint64_t fd = a.dist8 ? ((const uint64_t*)f.dist)[s] : ((const uint32_t*)f.dist)[s];
        m.dist = init ? (int32_t)(fd < 0x7FFFFFFEull ? fd : 0x7FFFFFFEull) : (int32_t)NO_DIST;
        m.flags = (init ? PGM_FLAG_INIT : 0u) | ((fl & ST_INL) ? PGM_FLAG_INLIER : 0u) |
                  ((fl & ST_REC) ? PGM_FLAG_RECORD : 0u);
        out[s] = m;
        inl = (fl & ST_INL) != 0;
    }
    if (!counts) return;
    uint32_t v = 0;
    for (int q0 = threadIdx.x;;) {
#pragma unroll
        for (int u = 0; u < 8; u++)
            v += __popc(w[u].x & 0x02020202u) + __popc(w[u].y & 0x02020202u) + __popc(w[u].z & 0x02020202u) +
                 __popc(w[u].w & 0x02020202u);
        q0 += 8 * 256;
        if (q0 >= nq) break;
#pragma unroll
        for (int u = 0; u < 8; u++) w[u] = q0 + u * 256 < nq ? fl4[q0 + u * 256] : make_uint4(0u, 0u, 0u, 0u);
    }
    // the wave's total: DPP sums over rows of 16 lanes, then the four rows
    const uint32_t rows = group_sum<16>(v);
    const uint32_t wsum = (uint32_t)__builtin_amdgcn_readlane((int)rows, 0) + (uint32_t)__builtin_amdgcn_readlane((int)rows, 16) +
                          (uint32_t)__builtin_amdgcn_readlane((int)rows, 32) + (uint32_t)__builtin_amdgcn_readlane((int)rows, 48);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const unsigned long long mask = __ballot(inl);
    if (lane == 0) { part[wv] = wsum; wtot[wv] = (uint32_t)__popcll(mask); }
    __syncthreads();
    const uint32_t prefix = part[0] + part[1] + part[2] + part[3];
    uint32_t before = 0;
    for (int k = 0; k < wv; k++) before += wtot[k];
    const uint32_t rank = (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
    if (inl && compact) compact[prefix + before + rank] = m;
    if (n_out && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0)
        *n_out = (int32_t)(prefix + wtot[0] + wtot[1] + wtot[2] + wtot[3]);
}

// Add up the count tables: k_count_part sums slice x of pair y's tables per kernel kind into
// pair y's partial array at [x * KINDS + kind] (each pair's array sits at the same offset of
// its own workspace slice); k_count_sum adds the parts per kind (profiling) and in total (the
// caller's counter), or per pair into the pairs' own counters of a table-driven batch.
__global__ __launch_bounds__(256) void k_count_part(CountArgs a, unsigned long long* part)
{
    __shared__ unsigned long long ws[4];
    const uint32_t z = blockIdx.y;
    for (int k = 0; k < CountArgs::KINDS; k++) {
        const uint32_t* t = zoff(a.table[k], (size_t)z * (size_t)a.zs);
        unsigned long long v = 0;
        for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < a.n[k]; i += (long long)gridDim.x * 256)
            v += t[i];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
        if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
        __syncthreads();
        if (threadIdx.x == 0)
            zoff(part, (size_t)z * (size_t)a.zs)[blockIdx.x * CountArgs::KINDS + k] = ws[0] + ws[1] + ws[2] + ws[3];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_count_sum(CountArgs a, const unsigned long long* part, int slices)
{
    __shared__ unsigned long long ws[4];
    unsigned long long total = 0;
    for (int k = 0; k < CountArgs::KINDS; k++) {
        unsigned long long v = 0;
        for (int i = threadIdx.x; i < slices * a.npairs; i += 256)
            v += zoff(part, (size_t)(i / slices) * (size_t)a.zs)[(i % slices) * CountArgs::KINDS + k];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
        if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
        __syncthreads();
        const unsigned long long sum = ws[0] + ws[1] + ws[2] + ws[3];
        __syncthreads();
        if (threadIdx.x == 0 && a.prof) a.prof[a.kind[k]] += sum;
        total += sum;
    }
    if (threadIdx.x == 0 && a.user) atomicAdd(a.user, total);
    // table-driven batches: each pair's own total into its own counter
    if (a.tab && (int)threadIdx.x < a.npairs && a.tab[threadIdx.x].n_evals) {
        const int z = (int)threadIdx.x;
        const unsigned long long* pz = zoff(part, (size_t)z * (size_t)a.zs);
        unsigned long long t = 0;
        for (int i = 0; i < slices * CountArgs::KINDS; i++) t += pz[i];
        atomicAdd(a.tab[z].n_evals, t);
    }
}

struct TabFill {
    PairTab t[TAB_MAX];
    PairTab* dst;
    int n;
};

__global__ __launch_bounds__(64) void k_fill_tab(TabFill a)
{
    if ((int)threadIdx.x < a.n) a.dst[threadIdx.x] = a.t[threadIdx.x];
}

// ---------------------------------------------------------------------------------------
// image pyramid (Sec. III-D): 5x5 binomial, decimation by 2, reflect-101 borders
// ---------------------------------------------------------------------------------------

__device__ __forceinline__ int mirror_fast(int i, int n) { return (unsigned)i < (unsigned)n ? i : mirror(i, n); }

// [lo, hi]: the interval that holds mirror(i, n) for every i in [a, b] (a <= n - 1). Inside
// the image the values are i itself; below 0 they rise from 0 to at most -a; past n - 1 they
// fall from n - 1 to at least 2 (n - 1) - b; a wider reach covers the whole image.
__device__ __forceinline__ void mirror_span(int a, int b, int n, int& lo, int& hi)
{
    lo = max(0, min(a, 2 * (n - 1) - b));
    hi = min(n - 1, max(b, -a));
}

// LDS dwords per image row that stage_rgb needs for a block SU pixels wide (the row's bytes
// with up to three before them, and one more dword that the last pixel's read may touch), and
// that count padded to whole 64-lane loads
template <int SU> constexpr int stage_row_min() { return (3 * SU + 6) / 4 + 1; }
template <int SU> constexpr int stage_row_dwords() { return (stage_row_min<SU>() + 63) / 64 * 64; }

// Stages the SU x SV block of pixels (mirror(x0 + min(u, nu - 1), w), mirror(y0 + min(v, nv - 1),
// h)), u < SU, v < SV, handing each to put(v, u, R | G << 8 | B << 16). The image rows and
// columns those pixels lie in are first copied to T (SV rows of RB dwords)
// by whole-dword loads, each row from the 4-byte boundary at or below its first byte. The
// loads go through a buffer descriptor that spans the image, from the 4-byte boundary at or
// below its first byte to the end of the dword that holds its last one: no load reaches
// outside that, and one whose offset lies past it returns 0 without a memory access, so the
// loads need no per-lane bounds tests. The pixels are then cut out of T at their byte
// offsets. Wave q of the four handles block rows q, q + 4, ..., so that everything that
// depends on the row alone is wave-uniform and lanes run along the row. Ends after a barrier,
// with what put wrote to LDS visible; T is free again from then on. The host keeps every
// image below 2^31 bytes, so the 32-bit offsets do not wrap.
template <int SU, int SV, int RB = stage_row_dwords<SU>(), typename Put>
__device__ __forceinline__ void stage_rgb(const uint8_t* img, int pitch, int w, int h, int x0, int nu, int y0,
                                          int nv, uint32_t* T, Put put)
{
    static_assert(RB >= stage_row_min<SU>(), "a staged row holds the pixels' bytes");
    // Columns past the last whole 64 go in one flat pass over all rows when they fit 256
    // threads, instead of a nearly idle pass per row.
    constexpr int REM = SU % 64, FLAT = REM > 0 && REM * SV <= 256;
    constexpr int RPW = (SV + 3) / 4, DPL = (RB + 63) / 64, UPL = FLAT ? SU / 64 : (SU + 63) / 64;
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6) & 3, lane = (int)threadIdx.x & 63;
    int c_lo, c_hi, r_lo, r_hi;
    mirror_span(x0, x0 + min(nu, SU) - 1, w, c_lo, c_hi);
    mirror_span(y0, y0 + min(nv, SV) - 1, h, r_lo, r_hi);
    c_hi = min(c_hi, c_lo + SU - 1);   // the bounds above never exceed SU x SV; this keeps T's
    r_hi = min(r_hi, r_lo + SV - 1);   // indices in range whatever the arguments
    const uint32_t mis = (uint32_t)((uintptr_t)img & 3u);
    const uint32_t bytes = mis + (uint32_t)(h - 1) * (uint32_t)pitch + 3u * (uint32_t)w;
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void*)((uintptr_t)img - mis), 0, (int)((bytes + 3u) & ~3u), 0x00020000);
    const uint32_t col0 = mis + 3u * (uint32_t)c_lo;   // offset of column c_lo in row 0
    uint32_t raw[RPW][DPL];
#pragma unroll
    for (int r = 0; r < RPW; r++) {
        const uint32_t ro = (col0 + (uint32_t)min(r_lo + wave + 4 * r, h - 1) * (uint32_t)pitch) & ~3u;
#pragma unroll
        for (int q = 0; q < DPL; q++)
            raw[r][q] = __builtin_amdgcn_raw_buffer_load_b32(rs, (int)(ro + 4u * (uint32_t)(lane + 64 * q)), 0, 0);
    }
#pragma unroll
    for (int r = 0; r < RPW; r++) {
        const int v = wave + 4 * r;
        if (v < SV) {
#pragma unroll
            for (int q = 0; q < DPL; q++)
                if (RB % 64 == 0 || lane + 64 * q < RB) T[v * RB + lane + 64 * q] = raw[r][q];
        }
    }
    // byte offset of each of the lane's columns in a T row whose first byte is 4-aligned
    int xo[UPL];
#pragma unroll
    for (int q = 0; q < UPL; q++) xo[q] = 3 * (clampi(mirror_fast(x0 + min(lane + 64 * q, nu - 1), w), c_lo, c_hi) - c_lo);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RPW; r++) {
        const int v = wave + 4 * r;
        if (v >= SV) break;
        const int y = clampi(mirror_fast(y0 + min(v, nv - 1), h), r_lo, r_hi);
        const int sh = (int)((col0 + (uint32_t)y * (uint32_t)pitch) & 3u);   // the row's misalignment
        const uint32_t* row = T + (y - r_lo) * RB;
#pragma unroll
        for (int q = 0; q < UPL; q++) {
            const int u = lane + 64 * q;
            if (u < SU) {
                const int o = sh + xo[q];
                const uint32_t* c = row + (o >> 2);
                put(v, u, __builtin_amdgcn_alignbyte(c[1], c[0], (uint32_t)(o & 3)) & 0xFFFFFFu);
            }
        }
    }
    if (FLAT && (int)threadIdx.x < REM * SV) {
        const int v = (int)threadIdx.x / (REM > 0 ? REM : 1), u = SU - REM + ((int)threadIdx.x - v * REM);
        const int x = clampi(mirror_fast(x0 + min(u, nu - 1), w), c_lo, c_hi);
        const int y = clampi(mirror_fast(y0 + min(v, nv - 1), h), r_lo, r_hi);
        const int o = (int)((col0 + (uint32_t)y * (uint32_t)pitch) & 3u) + 3 * (x - c_lo);
        const uint32_t* c = T + (y - r_lo) * RB + (o >> 2);
        put(v, u, __builtin_amdgcn_alignbyte(c[1], c[0], (uint32_t)(o & 3)) & 0xFFFFFFu);
    }
    __syncthreads();
}

// Binomial sums of packed pixels. A pixel R | G << 8 | B << 16 contributes (R, B) to the two
// halves of one 32-bit sum (p & 0x00FF00FF) and G << 8 to another (p & 0xFF00). A 5-tap pass
// sums to at most 16 * 255 and two passes to at most 256 * 255 < 2^16 per channel, so the halves
// never carry into each other and each channel's sum is the integer of the separate passes.
__device__ __forceinline__ void binom_add(uint32_t& rb, uint32_t& g, uint32_t tap, uint32_t p)
{
    rb += tap * (p & 0x00FF00FFu);
    g += tap * (p & 0xFF00u);
}

// the rounded level value (sum + 128) >> 8 of each channel, packed again
__device__ __forceinline__ uint32_t binom_pixel(uint32_t rb, uint32_t g)
{
    const uint32_t R = ((rb & 0xFFFFu) + 128u) >> 8, B = ((rb >> 16) + 128u) >> 8, G = ((g >> 8) + 128u) >> 8;
    return R | (G << 8) | (B << 16);
}

__device__ __forceinline__ void put_rgb(uint8_t* o, uint32_t p)
{
    o[0] = (uint8_t)p;
    o[1] = (uint8_t)(p >> 8);
    o[2] = (uint8_t)(p >> 16);
}

// Horizontal 5-tap binomial at even position 2k of a staged row whose stride is even: two
// 8-byte and one 4-byte LDS reads.
__device__ __forceinline__ void binom_row(const uint32_t* row, int k, uint32_t& rb, uint32_t& g)
{
    const uint2 a = *(const uint2*)(row + 2 * k), b = *(const uint2*)(row + 2 * k + 2);
    const uint32_t c = row[2 * k + 4];
    rb = 0;
    g = 0;
    binom_add(rb, g, 1, a.x);
    binom_add(rb, g, 4, a.y);
    binom_add(rb, g, 6, b.x);
    binom_add(rb, g, 4, b.y);
    binom_add(rb, g, 1, c);
}

// A work-group computes 64 x 4 output pixels: it stages the (2*64+3) x (2*4+3) source pixels
// (reflect-101 applied at load time), filters every staged row at the even columns, then the
// columns; the integer result is the 5x5 sum of the same products. Wave q handles staged rows
// q, q + 4, ... and output row q; lanes run along the rows.
constexpr int PY_TW = 64, PY_TH = 4, PY_SU = 2 * PY_TW + 3, PY_SV = 2 * PY_TH + 3;
constexpr int PY_SP = PY_SU + 1;   // even row stride of the staged pixels
constexpr int PY_H = PY_SV * PY_TW * 2 > PY_SV * stage_row_dwords<PY_SU>() ? PY_SV * PY_TW * 2 : PY_SV * stage_row_dwords<PY_SU>();
constexpr int PY_LDS = PY_SV * PY_SP + PY_H;   // dwords
static_assert(PY_TW == 64 && PY_TH == 4, "one lane per output column, one wave per output row");

__device__ __forceinline__ void pyr_tile(const PyrArgs& a, int t, int z, uint32_t* lds)
{
    uint32_t* S = lds;                  // [PY_SV][PY_SP] staged pixels
    uint32_t* H = lds + PY_SV * PY_SP;  // [PY_SV][PY_TW][2] row sums (staging rows before them)
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6) & 3, lane = (int)threadIdx.x & 63;
    const int w = a.w, h = a.h, w2 = (w + 1) >> 1, h2 = (h + 1) >> 1;
    const int X0 = (t % a.tx) * PY_TW, Y0 = (t / a.tx) * PY_TH;
    const size_t pair = (size_t)(z >> 1);
    const uint8_t* src = a.tab ? a.tab[pair].img[z & 1] : a.src[z & 1] + pair * (size_t)a.src_zs;
    uint8_t* dst = a.dst[z & 1] + pair * (size_t)a.dst_zs;
    const int xlo = 2 * X0 - 2, ylo = 2 * Y0 - 2;
    stage_rgb<PY_SU, PY_SV>(src, a.pitch, w, h, xlo, PY_SU, ylo, PY_SV, H, [=](int v, int u, uint32_t p) { S[v * PY_SP + u] = p; });
#pragma unroll
    for (int r = 0; r < (PY_SV + 3) / 4; r++) {
        const int v = wave + 4 * r;
        if (v >= PY_SV) break;
        uint32_t rb, g;
        binom_row(S + v * PY_SP, lane, rb, g);
        *(uint2*)(H + 2 * (v * PY_TW + lane)) = make_uint2(rb, g);
    }
    __syncthreads();
    const int x = X0 + lane, y = Y0 + wave;
    if (x >= w2 || y >= h2) return;
    const uint32_t tap[5] = {1, 4, 6, 4, 1};
    uint32_t rb = 0, g = 0;
#pragma unroll
    for (int i = 0; i < 5; i++) {
        const uint2 q = *(const uint2*)(H + 2 * ((2 * wave + i) * PY_TW + lane));
        rb += tap[i] * q.x;
        g += tap[i] * q.y;
    }
    put_rgb(dst + ((size_t)y * w2 + x) * 3, binom_pixel(rb, g));
}

// Two pyramid levels in one pass. A work-group computes TW x TH pixels of level l+2 and the
// 2 TW x 2 TH pixels of level l+1 above them: it stages the level-l pixels under the level-(l+1)
// pixels that its level-(l+2) pixels read (the reflections at the borders fall inside that
// block), computes those level-(l+1) pixels as pyr_tile does, writes the ones it owns, then
// filters them into level l+2. Each value is the integer of two separate passes. Wave q
// handles rows q, q + 4, ... of each stage, lanes the columns. 29 x 3 makes the level-(l+1)
// block 61 columns wide and the staged block 125: one and two 64-lane passes, for wide levels,
// with the LDS of the gradient tile; 32 x 2 (67 and 137 columns, a nearly empty extra pass)
// tiles a 64-pixel-wide level with two work-groups across instead of three.
template <int TW_, int TH_> struct P2 {
    static constexpr int TW = TW_, TH = TH_;
    static constexpr int RB = stage_row_min<2 * (2 * TW_ + 3) + 3>();   // staging row stride
    static constexpr int C1 = 2 * TW + 3, R1 = 2 * TH + 3;   // level-(l+1) block
    static constexpr int SU = 2 * C1 + 3, SV = 2 * R1 + 3;   // level-l block
    static constexpr int SP = SU + 1;                        // even row stride of the staged pixels
    static constexpr int CP = (C1 + 63) / 64;                // column passes over the level-(l+1) block
    // the level-(l+1) block reuses the staged block's space and its row sums the first row
    // sums' space (each is written after a barrier that ends the last read of what it replaces)
    static constexpr int H = SV * C1 * 2 > SV * RB ? SV * C1 * 2 : SV * RB;
    static constexpr int LDS = SV * SP + H;   // dwords
    static_assert(TW <= 64 && R1 * C1 <= SV * SP && 2 * R1 * TW <= H && TH <= 4, "pyramid tile shape and aliasing");
};
using P2Wide = P2<29, 3>;
using P2Narrow = P2<32, 2>;
constexpr int P2_LDS = P2Wide::LDS > P2Narrow::LDS ? P2Wide::LDS : P2Narrow::LDS;

template <typename D>
__device__ __forceinline__ void pyr2_tile(const PyrArgs& a, int t, int z, uint32_t* lds)
{
    constexpr int TW = D::TW;
    constexpr int TH = D::TH, C1 = D::C1, R1 = D::R1, SU = D::SU, SV = D::SV, SP = D::SP;
    uint32_t* S0 = lds;             // [SV][SP] staged level-l pixels
    uint32_t* H0 = lds + SV * SP;   // [SV][C1][2] row sums (staging rows before them)
    uint32_t* V1 = S0;              // [R1][C1] level-(l+1) pixels (S0 is dead)
    uint32_t* H1 = H0;              // [R1][TW][2] row sums of level l+1 (H0 is dead)
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6) & 3, lane = (int)threadIdx.x & 63;
    const int w0 = a.w, h0 = a.h, w1 = (w0 + 1) >> 1, h1 = (h0 + 1) >> 1, w2 = (w1 + 1) >> 1, h2 = (h1 + 1) >> 1;
    const int X0 = (t % a.tx) * TW, Y0 = (t / a.tx) * TH;
    const size_t pair = (size_t)(z >> 1);
    const uint8_t* src = a.tab ? a.tab[pair].img[z & 1] : a.src[z & 1] + pair * (size_t)a.src_zs;
    uint8_t* dst1 = a.dst[z & 1] + pair * (size_t)a.dst_zs;
    uint8_t* dst2 = a.dst2[z & 1] + pair * (size_t)a.dst_zs;
    const int cx0 = max(0, 2 * X0 - 2), cx1 = min(w1 - 1, 2 * X0 + 2 * TW);
    const int cy0 = max(0, 2 * Y0 - 2), cy1 = min(h1 - 1, 2 * Y0 + 2 * TH);
    const int NU = 2 * (cx1 - cx0 + 1) + 3, NV = 2 * (cy1 - cy0 + 1) + 3;
    const int xlo = 2 * cx0 - 2, ylo = 2 * cy0 - 2;
    stage_rgb<SU, SV, D::RB>(src, a.pitch, w0, h0, xlo, NU, ylo, NV, H0, [=](int v, int u, uint32_t p) { S0[v * SP + u] = p; });
#pragma unroll
    for (int r = 0; r < (SV + 3) / 4; r++) {
        const int v = wave + 4 * r;
        if (v >= SV) break;
#pragma unroll
        for (int q = 0; q < D::CP; q++) {
            const int k = lane + 64 * q;   // level-(l+1) block column
            if (k < C1) {
                uint32_t rb, g;
                binom_row(S0 + v * SP, k, rb, g);
                *(uint2*)(H0 + 2 * (v * C1 + k)) = make_uint2(rb, g);
            }
        }
    }
    __syncthreads();
    const uint32_t tap[5] = {1, 4, 6, 4, 1};
#pragma unroll
    for (int r = 0; r < (R1 + 3) / 4; r++) {
        const int rr = wave + 4 * r;
        if (rr >= R1) break;
#pragma unroll
        for (int q = 0; q < D::CP; q++) {
            const int k = lane + 64 * q;
            if (k < C1) {
                uint32_t rb = 0, g = 0;
#pragma unroll
                for (int i = 0; i < 5; i++) {
                    const uint2 e = *(const uint2*)(H0 + 2 * ((2 * rr + i) * C1 + k));
                    rb += tap[i] * e.x;
                    g += tap[i] * e.y;
                }
                const uint32_t px = binom_pixel(rb, g);
                V1[rr * C1 + k] = px;
                const int c = cx0 + k, y = cy0 + rr;
                if (c >= 2 * X0 && c < 2 * X0 + 2 * TW && c <= cx1 && y >= 2 * Y0 && y < 2 * Y0 + 2 * TH && y <= cy1)
                    put_rgb(dst1 + ((size_t)y * w1 + c) * 3, px);
            }
        }
    }
    __syncthreads();
    // level l+2: rows of the level-(l+1) block at this tile's even columns, then its columns
    const int X2 = X0 + lane;
    int col[5];   // the level-(l+1) block columns of the five taps (reflected at the border)
#pragma unroll
    for (int j = 0; j < 5; j++) col[j] = mirror_fast(2 * X2 - 2 + j, w1) - cx0;
#pragma unroll
    for (int r = 0; r < (R1 + 3) / 4; r++) {
        const int rr = wave + 4 * r;
        if (rr >= R1) break;
        if (lane < TW) {
            uint32_t rb = 0, g = 0;
            if (rr <= cy1 - cy0 && X2 < w2) {
#pragma unroll
                for (int j = 0; j < 5; j++) binom_add(rb, g, tap[j], V1[rr * C1 + col[j]]);
            }
            *(uint2*)(H1 + 2 * (rr * TW + lane)) = make_uint2(rb, g);
        }
    }
    __syncthreads();
    const int Y2 = Y0 + wave;
    if (wave >= TH || lane >= TW || X2 >= w2 || Y2 >= h2) return;
    uint32_t rb = 0, g = 0;
#pragma unroll
    for (int i = 0; i < 5; i++) {
        const uint2 e = *(const uint2*)(H1 + 2 * ((mirror_fast(2 * Y2 - 2 + i, h1) - cy0) * TW + lane));
        rb += tap[i] * e.x;
        g += tap[i] * e.y;
    }
    put_rgb(dst2 + ((size_t)Y2 * w2 + X2) * 3, binom_pixel(rb, g));
}

// ---------------------------------------------------------------------------------------
// gradient image (Sec. III-A, Eq. 1-2) written with a replicated PAD border
// ---------------------------------------------------------------------------------------

// Colour spaces of the gradient pyramids (Sec. III-E, Table II): integer BT.601 YCrCb, and
// 8-bit CIELab (sRGB transfer curve, D65) from plain IEEE double operations in a fixed order
// (u^2.4 = u^2 (u^2)^(1/5) by 40 Newton steps, t^(1/3) by 20), so that each value is a fixed
// function of the pixel; contraction into fused multiply-adds is off for that reason.
__device__ __forceinline__ uint32_t to_ycrcb(uint32_t rgb)
{
    const int R = rgb & 0xFF, G = (rgb >> 8) & 0xFF, B = (rgb >> 16) & 0xFF;
    const int Y = (77 * R + 150 * G + 29 * B + 128) >> 8;
    const int cr = (R - Y) * 183 + 32768 + 128, cb = (B - Y) * 144 + 32768 + 128;
    const int Cr = cr < 0 ? 0 : min(cr >> 8, 255), Cb = cb < 0 ? 0 : min(cb >> 8, 255);
    return (uint32_t)Y | ((uint32_t)Cr << 8) | ((uint32_t)Cb << 16);
}

__device__ double root_newton(double a, int n, int steps)
{
#pragma clang fp contract(off)
    double y = 1.0;
    for (int k = 0; k < steps; k++) {
        double p = y;
        for (int m = 2; m < n; m++) p = p * y;
        y = y - (p * y - a) / ((double)n * p);
    }
    return y;
}

__device__ double srgb_linear(int c)
{
#pragma clang fp contract(off)
    const double v = (double)c / 255.0;
    if (v <= 0.04045) return v / 12.92;
    const double u = (v + 0.055) / 1.055;
    const double u2 = u * u;
    return u2 * root_newton(u2, 5, 40);
}

__device__ double lab_f(double t)
{
#pragma clang fp contract(off)
    const double e = (6.0 / 29.0) * (6.0 / 29.0) * (6.0 / 29.0);
    if (t > e) return root_newton(t, 3, 20);
    return t / (3.0 * (6.0 / 29.0) * (6.0 / 29.0)) + 4.0 / 29.0;
}

__device__ __forceinline__ uint32_t lab_u8(double x)
{
    const double r = floor(x + 0.5);
    return (uint32_t)(r < 0.0 ? 0.0 : (r > 255.0 ? 255.0 : r));
}

// lin: the block's table of srgb_linear(0..255)
__device__ uint32_t to_lab(uint32_t rgb, const double* lin)
{
#pragma clang fp contract(off)
    const double r = lin[rgb & 0xFF], g = lin[(rgb >> 8) & 0xFF], b = lin[(rgb >> 16) & 0xFF];
    const double X = 0.4124564 * r + 0.3575761 * g + 0.1804375 * b;
    const double Yv = 0.2126729 * r + 0.7151522 * g + 0.0721750 * b;
    const double Z = 0.0193339 * r + 0.1191920 * g + 0.9503041 * b;
    const double fx = lab_f(X / 0.95047), fy = lab_f(Yv), fz = lab_f(Z / 1.08883);
    return lab_u8((116.0 * fy - 16.0) * 2.55) | (lab_u8(500.0 * (fx - fy) + 128.0) << 8) |
           (lab_u8(200.0 * (fy - fz) + 128.0) << 16);
}

// A work-group computes a 64 x 12 tile of the padded gradient image (64 x 8 was slower on
// 32-pair batches, 64 x 32 everywhere). It stages the pixels that the windows of its pixels
// read -- the padding maps to the nearest image pixel, the filter reflects (101) -- converted to
// the level's colour space, applies the smoothing and derivative taps along the staged rows,
// then across them: the Sobel sums are separable, so the integer results equal the full
// KS x KS sums. Every partial sum fits in 16 bits (row smoothing <= 16 * 255, row derivative
// <= 6 * 255, columns <= 6 * 4080), so the sums run as packed 16-bit multiply-adds on pairs of
// values: a staged colour pixel is kept as (R, G) and (B, B), a grey one as (Y, Y), and the row
// sums as the planes (smooth R, smooth G), (deriv R, deriv G), (smooth B, deriv B), or (smooth
// Y, deriv Y). Wave q of the four handles rows q, q + 4, ... of each pass, lanes the columns.
// LDS: the staged pixels, then the row-sum planes; the staging rows and the sRGB linearisation
// table of the CIELab conversion (256 doubles) use the planes' space before the row pass.
constexpr int GR_TW = 64, GR_TH = 12, GR_SU = GR_TW + 4, GR_SV = GR_TH + 4;   // kernel radius <= 2
constexpr int GR_LDS = GR_SV * GR_SU * 2 + GR_SV * GR_TW * 3;                 // dwords
constexpr int GR_LIN_AT = GR_SV * GR_SU * 2 + GR_SV * stage_row_dwords<GR_SU>();
static_assert(GR_TW == 64 && GR_SV % 4 == 0 && GR_TH % 4 == 0, "one lane per column, whole rows per wave");
static_assert(GR_LIN_AT % 2 == 0 && GR_LIN_AT + 512 <= GR_LDS, "the linearisation table fits after the staging rows");

__device__ __forceinline__ uint32_t lo_hi(uint32_t lo, uint32_t hi, uint32_t sel) { return __builtin_amdgcn_perm(hi, lo, sel); }
__device__ __forceinline__ s16x2 as_s16x2(uint32_t v) { return __builtin_bit_cast(s16x2, v); }
__device__ __forceinline__ uint32_t as_u32(s16x2 v) { return __builtin_bit_cast(uint32_t, v); }

// FEAT: 0 integer gradients, 1 direction-only unit vectors (float), 2 literal signs
template <int KS, bool GRAY, int FEAT>
__device__ __forceinline__ void grad_tile(const GradLevel& L, long long dst_zs, int t, int z, uint32_t* lds)
{
    constexpr int CH = GRAY ? 1 : 3;
    constexpr int C2 = 2 * CH;
    constexpr int K = KS / 2;
    constexpr int NP = GRAY ? 1 : 3;   // row-sum planes
    constexpr int PL = GR_SV * GR_TW;  // dwords per plane
    uint32_t* S = lds;                             // [GR_SV][GR_SU][1 (gray) or 2 dwords]
    uint32_t* H = lds + GR_SV * GR_SU * 2;         // [NP][GR_SV][GR_TW]
    double* lin = (double*)(lds + GR_LIN_AT);
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6), lane = (int)threadIdx.x & 63;
    const int w = L.w, h = L.h;
    const int pw = w + 2 * PAD, ph = h + 2 * PAD;
    const int X0 = (t % L.tx) * GR_TW, Y0 = (t / L.tx) * GR_TH;
    const size_t pair = (size_t)(z >> 1);
    const uint8_t* img = L.tab ? L.tab[pair].img[z & 1] : L.src[z & 1] + pair * (size_t)L.src_zs;
    void* G = zoff(L.G[z & 1], pair * (size_t)dst_zs);
    // the image columns and rows the tile's pixels map to
    const int cx0 = clampi(X0 - PAD, 0, w - 1), cx1 = clampi(min(X0 + GR_TW - 1, pw - 1) - PAD, 0, w - 1);
    const int cy0 = clampi(Y0 - PAD, 0, h - 1), cy1 = clampi(min(Y0 + GR_TH - 1, ph - 1) - PAD, 0, h - 1);
    const int NU = cx1 - cx0 + 1 + 2 * K, NV = cy1 - cy0 + 1 + 2 * K;
    const int space = L.space;
    if (!GRAY && space == PGM_SPACE_LAB) lin[threadIdx.x] = srgb_linear((int)threadIdx.x);   // read after the staging barrier
    // Staging: a fixed GR_SV x GR_SU block (columns and rows past the needed NU x NV repeat the
    // last needed one).
    stage_rgb<GR_SU, GR_SV>(img, L.pitch, w, h, cx0 - K, NU, cy0 - K, NV, H, [=](int v, int u, uint32_t p) {
        if (GRAY) {
            const uint32_t y = (77 * (p & 0xFFu) + 150 * ((p >> 8) & 0xFFu) + 29 * ((p >> 16) & 0xFFu) + 128) >> 8;
            S[v * GR_SU + u] = y | (y << 16);
        } else {
            if (space == PGM_SPACE_YCRCB) p = to_ycrcb(p);
            else if (space == PGM_SPACE_LAB) p = to_lab(p, lin);
            ((uint2*)S)[v * GR_SU + u] = make_uint2(__builtin_amdgcn_perm(0u, p, 0x0c010c00u), __builtin_amdgcn_perm(0u, p, 0x0c020c02u));
        }
    });
    const short sm3[3] = {1, 2, 1}, dv3[3] = {-1, 0, 1};
    const short sm5[5] = {1, 4, 6, 4, 1}, dv5[5] = {-1, -2, 0, 2, 1};
    // Row pass over the fixed block.
#pragma unroll
    for (int r = 0; r < GR_SV / 4; r++) {
        const int v = wave + 4 * r;
        s16x2 acc[NP];
#pragma unroll
        for (int c = 0; c < NP; c++) acc[c] = s16x2{0, 0};
#pragma unroll
        for (int j = 0; j < KS; j++) {
            const short sm = KS == 3 ? sm3[j] : sm5[j], dv = KS == 3 ? dv3[j] : dv5[j];
            if (GRAY) {
                acc[0] += s16x2{sm, dv} * as_s16x2(S[v * GR_SU + lane + j]);
            } else {
                const uint2 q = ((const uint2*)S)[v * GR_SU + lane + j];
                acc[0] += s16x2{sm, sm} * as_s16x2(q.x);
                acc[1] += s16x2{dv, dv} * as_s16x2(q.x);
                acc[2] += s16x2{sm, dv} * as_s16x2(q.y);
            }
        }
#pragma unroll
        for (int c = 0; c < NP; c++) H[c * PL + v * GR_TW + lane] = as_u32(acc[c]);
    }
    __syncthreads();
    // Column pass: (sum of derivative weights x smoothing, sum of smoothing weights x
    // derivative) = (gy, gx) per channel.
    constexpr int PX = C2 * (FEAT == 1 ? 4 : 2);   // bytes per gradient pixel
    const int X = X0 + lane;
    const int u = clampi(X - PAD, 0, w - 1) - cx0;
    char* const tile = (char*)G + ((size_t)Y0 * pw + X0) * PX;   // the tile's first pixel
    const size_t row_bytes = (size_t)pw * PX;
#pragma unroll
    for (int r = 0; r < GR_TH / 4; r++) {
        const int Y = Y0 + wave + 4 * r;
        if (Y >= ph || X >= pw) continue;
        const int v = clampi(Y - PAD, 0, h - 1) - cy0;
        s16x2 g[NP];   // colour: (gy R, gy G), (gx R, gx G), (gy B, gx B); grey: (gy, gx)
#pragma unroll
        for (int c = 0; c < NP; c++) g[c] = s16x2{0, 0};
#pragma unroll
        for (int i = 0; i < KS; i++) {
            const short sm = KS == 3 ? sm3[i] : sm5[i], dv = KS == 3 ? dv3[i] : dv5[i];
            const uint32_t* q = H + (v + i) * GR_TW + u;
            if (GRAY) {
                g[0] += s16x2{dv, sm} * as_s16x2(q[0]);
            } else {
                g[0] += s16x2{dv, dv} * as_s16x2(q[0]);
                g[1] += s16x2{sm, sm} * as_s16x2(q[PL]);
                g[2] += s16x2{dv, sm} * as_s16x2(q[2 * PL]);
            }
        }
        char* const px = tile + (wave + 4 * r) * row_bytes + (uint32_t)(lane * PX);
        if (FEAT == 0) {
            // biased 16-bit values in the order gx of each channel, then gy of each; adding
            // 2^15 modulo 2^16 flips the top bit of each half
            uint32_t* out = (uint32_t*)px;   // C2 even: pixels are dword aligned
            if (GRAY) {
                out[0] = __builtin_amdgcn_alignbit(as_u32(g[0]), as_u32(g[0]), 16) ^ 0x80008000u;
            } else {
                out[0] = as_u32(g[1]) ^ 0x80008000u;
                out[1] = lo_hi(as_u32(g[2]), as_u32(g[0]), 0x05040302u) ^ 0x80008000u;
                out[2] = lo_hi(as_u32(g[0]), as_u32(g[2]), 0x05040302u) ^ 0x80008000u;
            }
        } else {
            int gx[CH], gy[CH];
            if (GRAY) {
                gy[0] = g[0].x;
                gx[0] = g[0].y;
            } else {
                gy[0] = g[0].x, gy[1] = g[0].y, gy[2] = g[2].x;
                gx[0] = g[1].x, gx[1] = g[1].y, gx[2] = g[2].y;
            }
            if (FEAT == 2) {   // Sec. III-F read element-wise: G./|G| is the sign, 0 stays 0
                uint16_t vals[C2];
#pragma unroll
                for (int c = 0; c < CH; c++) {
                    vals[c] = (uint16_t)(((gx[c] > 0) - (gx[c] < 0)) + (int)BIAS);
                    vals[CH + c] = (uint16_t)(((gy[c] > 0) - (gy[c] < 0)) + (int)BIAS);
                }
                uint32_t* out = (uint32_t*)px;
#pragma unroll
                for (int k = 0; k < C2 / 2; k++) out[k] = (uint32_t)vals[2 * k] | ((uint32_t)vals[2 * k + 1] << 16);
            } else {
                float* out = (float*)px;
#pragma unroll
                for (int c = 0; c < CH; c++) {
                    float ux = 0.0f, uy = 0.0f;
                    if (gx[c] != 0 || gy[c] != 0) {
                        const double n = sqrt((double)gx[c] * gx[c] + (double)gy[c] * gy[c]);
                        ux = (float)((double)gx[c] / n);
                        uy = (float)((double)gy[c] / n);
                    }
                    out[c] = ux;
                    out[CH + c] = uy;
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------------------
// random numbers of a whole pair: initial displacements and every random-search offset
// ---------------------------------------------------------------------------------------

// seeds per thread of a random-search work-group (each seed takes a few Philox blocks per
// stage, direction and iteration: these are k_prep's longest work-groups)
constexpr int RNG_SPT = 4;

__device__ __forceinline__ int search_off(uint32_t u, int W, int i, int sym)
{
    if (sym) {   // uniform over the integers of [-w_i, w_i], w_i = floor(W / 2^i)
        const int wi = W >> i;
        return (int)__umulhi(u, 2u * (uint32_t)wi + 1u) - wi;
    }
    // floor(R W / 2^i) with R = (2u + 1) / 2^32 - 1, in exact integer arithmetic
    const long long A = (long long)(2ull * u + 1ull) * W - ((long long)W << 32);
    return (int)(A >> (32 + i));
}

// Work-group b of the random numbers: the initial displacements first, then per stage one
// range per (direction, iteration) in which thread x of chunk c draws every search offset of
// seeds 256 (RNG_SPT c + m) + x, m < RNG_SPT (one Philox block per two offsets).
__device__ __forceinline__ void rng_block(const RngArgs& a, int b)
{
    if (b < a.init_blocks) {
        const int item = b * 256 + (int)threadIdx.x;
        if (item >= 2 * a.n_top) return;
        const int dir = item / a.n_top, s = item - dir * a.n_top;
        const uint4 u = philox4x32_10(
            make_uint4((uint32_t)s, ((uint32_t)a.top_level << 8) | ((uint32_t)dir << 16), 0u, 0u), a.key0, a.key1);
        const uint32_t span = 2u * (uint32_t)a.R_top + 1u;
        a.init[item] = make_short2((short)((int)__umulhi(u.x, span) - a.R_top), (short)((int)__umulhi(u.y, span) - a.R_top));
        return;
    }
    b -= a.init_blocks;
    int k = 0;
    while (k + 1 < a.nstages && b >= a.st[k + 1].b0) k++;
    const RngStage& S = a.st[k];
    const int local = b - S.b0;
    const int q = local / S.bpt, chunk = local - q * S.bpt;
    const int dir = q / S.iters, t = q - dir * S.iters;
    const uint32_t w1 = (uint32_t)t | ((uint32_t)S.level << 8) | ((uint32_t)dir << 16) | (1u << 24);
    for (int m = 0; m < RNG_SPT; m++) {
        const int s = (chunk * RNG_SPT + m) * 256 + (int)threadIdx.x;
        if (s >= S.n) return;
        short2* out = a.table + S.base + (((long long)dir * S.iters + t) * S.n + s) * S.nI;
        for (int i0 = 0; i0 < S.nI; i0 += 2) {
            const uint4 u = philox4x32_10(make_uint4((uint32_t)s, w1, (uint32_t)(i0 >> 1), (uint32_t)S.stage), a.key0, a.key1);
            out[i0] = make_short2((short)search_off(u.x, S.W, i0, a.rs_sym), (short)search_off(u.y, S.W, i0, a.rs_sym));
            if (i0 + 1 < S.nI)
                out[i0 + 1] = make_short2((short)search_off(u.z, S.W, i0 + 1, a.rs_sym),
                                          (short)search_off(u.w, S.W, i0 + 1, a.rs_sym));
        }
    }
}

// ---------------------------------------------------------------------------------------
// kernels of the image stage. k_prep starts a call with three independent jobs in one launch
// (work-group ranges): the random numbers, the first pyramid levels and the level-0 gradient
// images, dispatched in that order (the longest work-groups, the random ones, first); k_pyr
// builds the further pyramid levels and k_gradient their gradient images (all levels in one
// launch: blockIdx.x runs over the tiles of each level in turn).
// ---------------------------------------------------------------------------------------

constexpr int PREP_LDS = GR_LDS > PY_LDS ? (GR_LDS > P2_LDS ? GR_LDS : P2_LDS) : (PY_LDS > P2_LDS ? PY_LDS : P2_LDS);

template <int KS, bool GRAY, int FEAT>
__global__ __launch_bounds__(256) void k_prep(PrepArgs a)
{
    __shared__ __align__(16) uint32_t lds[PREP_LDS];
    int b = blockIdx.x;
    if (b < a.rng_blocks) {
        rng_block(a.rng, b);
        return;
    }
    b -= a.rng_blocks;
    if (b < a.pyr_blocks) {
        if (a.pyr.two) pyr2_tile<P2Wide>(a.pyr, b % a.pyr.tiles, b / a.pyr.tiles, lds);
        else pyr_tile(a.pyr, b % a.pyr.tiles, b / a.pyr.tiles, lds);
        return;
    }
    b -= a.pyr_blocks;
    if (b < a.grad_blocks) {   // level 0 in each colour space it needs
        const int z = b / a.grad_tiles, tt = b - z * a.grad_tiles;
        int e = 0;
        while (e + 1 < a.grad.n && tt >= a.grad.lv[e + 1].base) e++;
        grad_tile<KS, GRAY, FEAT>(a.grad.lv[e], a.grad.dst_zs, tt - a.grad.lv[e].base, z, lds);
    }
}

__global__ __launch_bounds__(256) void k_pyr(PyrArgs a)
{
    __shared__ __align__(16) uint32_t lds[PY_LDS > P2_LDS ? PY_LDS : P2_LDS];
    if (a.two) pyr2_tile<P2Narrow>(a, blockIdx.x, blockIdx.y, lds);
    else pyr_tile(a, blockIdx.x, blockIdx.y, lds);
}

template <int KS, bool GRAY, int FEAT>
__global__ __launch_bounds__(256) void k_gradient(GradArgs a)
{
    __shared__ __align__(16) uint32_t lds[GR_LDS];
    int lv = 0;
    while (lv + 1 < a.n && (int)blockIdx.x >= a.lv[lv + 1].base) lv++;
    grad_tile<KS, GRAY, FEAT>(a.lv[lv], a.dst_zs, (int)blockIdx.x - a.lv[lv].base, blockIdx.y, lds);
}

// ---------------------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------------------

// tw x th: the level-(l+2) tile of the kernel that runs the plan (two levels)
static void plan_pyr(PyrArgs& a, int tw, int th)
{
    const int w1 = (a.w + 1) / 2, h1 = (a.h + 1) / 2;
    if (a.two) {   // tiles over the second level
        a.tx = ((w1 + 1) / 2 + tw - 1) / tw;
        a.tiles = a.tx * (((h1 + 1) / 2 + th - 1) / th);
    } else {
        a.tx = (w1 + PY_TW - 1) / PY_TW;
        a.tiles = a.tx * ((h1 + PY_TH - 1) / PY_TH);
    }
}

static int plan_grad(GradArgs& a)
{
    int total = 0;
    for (int k = 0; k < a.n; k++) {
        GradLevel& L = a.lv[k];
        L.tx = (L.w + 2 * PAD + GR_TW - 1) / GR_TW;
        L.tiles = L.tx * ((L.h + 2 * PAD + GR_TH - 1) / GR_TH);
        L.base = total;
        total += L.tiles;
    }
    return total;
}

hipError_t launch_pyr(PyrArgs a, int npairs, hipStream_t s)
{
    plan_pyr(a, P2Narrow::TW, P2Narrow::TH);
    hipLaunchKernelGGL(k_pyr, dim3(a.tiles, 2 * npairs), dim3(256), 0, s, a);
    return hipGetLastError();
}

#define PGM_IMG_VARIANTS(M)                                                                    \
    M(3, false, 0) M(3, false, 1) M(3, false, 2) M(3, true, 0) M(3, true, 1) M(3, true, 2)       \
    M(5, false, 0) M(5, false, 1) M(5, false, 2) M(5, true, 0) M(5, true, 1) M(5, true, 2)

hipError_t launch_gradient(GradArgs a, int npairs, int gray, int ksize, int feat, hipStream_t s)
{
    const int total = plan_grad(a);
    if (total == 0) return hipSuccess;
    dim3 grid(total, 2 * npairs);
#define PGM_GRAD(KS, GR, F)                                                                       \
    if (ksize == KS && !!gray == GR && feat == F) {                                                \
        hipLaunchKernelGGL((k_gradient<KS, GR, F>), grid, dim3(256), 0, s, a);                     \
        return hipGetLastError();                                                                  \
    }
    PGM_IMG_VARIANTS(PGM_GRAD)
#undef PGM_GRAD
    return hipErrorInvalidValue;
}

hipError_t launch_prep(PrepArgs a, int npairs, int gray, int ksize, int feat, hipStream_t s)
{
    RngArgs& r = a.rng;
    r.init_blocks = (int)((2LL * r.n_top + 255) / 256);
    long long nb = 0;
    for (int k = 0; k < r.nstages; k++) {
        r.st[k].bpt = (r.st[k].n + 256 * RNG_SPT - 1) / (256 * RNG_SPT);
        r.st[k].b0 = (int)nb;
        nb += 2LL * r.st[k].iters * r.st[k].bpt;
        if (nb > 0x40000000LL) return hipErrorInvalidValue;
    }
    a.rng_blocks = r.init_blocks + (int)nb;
    a.grad_tiles = plan_grad(a.grad);
    a.grad_blocks = a.grad_tiles * 2 * npairs;
    a.pyr_blocks = 0;
    if (a.with_pyr) {
        plan_pyr(a.pyr, P2Wide::TW, P2Wide::TH);
        a.pyr_blocks = a.pyr.tiles * 2 * npairs;
    }
    const long long blocks = (long long)a.rng_blocks + a.grad_blocks + a.pyr_blocks;
    if (blocks > 0x7FFFFFFFLL) return hipErrorInvalidValue;
#define PGM_PREP(KS, GR, F)                                                                       \
    if (ksize == KS && !!gray == GR && feat == F) {                                                \
        hipLaunchKernelGGL((k_prep<KS, GR, F>), dim3((unsigned)blocks), dim3(256), 0, s, a);       \
        return hipGetLastError();                                                                  \
    }
    PGM_IMG_VARIANTS(PGM_PREP)
#undef PGM_PREP
    return hipErrorInvalidValue;
}

#undef PGM_IMG_VARIANTS

// whether the two directions of a launch read the same two gradient images (one colour space)
static int same_images(const DirArgs d[2]) { return d[0].Ga == d[1].Gb && d[0].Gb == d[1].Ga; }

// Kernel variants: patch side exactly 8 or 16 (fully unrolled rows), or any side up to 8 /
// up to 16 with masked rows; 6 or 2 gradient channels; integer or float features.
#define PGM_DISPATCH(KERNEL, ARGS, NGROUPS)                                               \
    do {                                                                                         \
        const int P = (ARGS).d[0].P;                                                             \
        const int pmax = P <= 8 ? 8 : 16;                                                        \
        const bool fixed = P == pmax;                                                            \
        dim3 grid((unsigned)((long long)match_blocks((NGROUPS), P) * (ARGS).b.ndir * (ARGS).b.npairs)); \
        if ((NGROUPS) <= 0) return hipSuccess;                                                   \
        (ARGS).b.dnb = div_magic((uint32_t)match_blocks((NGROUPS), P));                          \
        (ARGS).b.inter = same_images((ARGS).d);                                                  \
        PGM_V(KERNEL, 6, 8, true) PGM_V(KERNEL, 6, 8, false) PGM_V(KERNEL, 6, 16, true)           \
        PGM_V(KERNEL, 6, 16, false) PGM_V(KERNEL, 2, 8, true) PGM_V(KERNEL, 2, 8, false)          \
        PGM_V(KERNEL, 2, 16, true) PGM_V(KERNEL, 2, 16, false)                                    \
        return hipErrorInvalidValue;                                                             \
    } while (0)

#define PGM_V(KERNEL, C2_, PM_, FX_)                                                             \
    if (C2 == C2_ && pmax == PM_ && fixed == FX_) {                                              \
        if (kind == 1) hipLaunchKernelGGL((KERNEL<C2_, PM_, FX_, 1>), grid, dim3(MATCH_TPB), 0, s, a); \
        else if (kind == 2) hipLaunchKernelGGL((KERNEL<C2_, PM_, FX_, 2>), grid, dim3(MATCH_TPB), 0, s, a); \
        else hipLaunchKernelGGL((KERNEL<C2_, PM_, FX_, 0>), grid, dim3(MATCH_TPB), 0, s, a);           \
        return hipGetLastError();                                                                \
    }

hipError_t launch_sweep(SweepArgs a, int C2, int kind, hipStream_t s)
{
    PGM_DISPATCH(k_sweep, a, a.g.ny * ((a.g.nx + 1) / 2));
}

// The rectangles R_m of k_sweep_multi relative to the tile, one packed word per half-sweep:
// R_{nph-1} is the tile, R_m is R_{m+1} grown by a seed on the sides half-sweep m+1 looks back to.
static void plan_multi(SweepMultiArgs& a)
{
    int xa = 0, xb = MULTI_TX, ya = 0, yb = MULTI_TY;
    for (int m = a.nph - 1; m >= 0; m--) {
        if (m < a.nph - 1) {
            const int k = a.t[m + 1] & 3;
            const int sx = (k == 0 || k == 3) ? 1 : -1, sy = (k == 0 || k == 2) ? 1 : -1;
            if (sx == 1) xa--; else xb++;
            if (sy == 1) ya--; else yb++;
        }
        const int W = xb - xa, H = yb - ya;
        const int V = (W & 1) ? W : W / 2;
        const uint32_t M = (uint32_t)((1024 + V - 1) / V);
        a.ph[m] = (uint32_t)(xa + 4) | (uint32_t)(ya + 4) << 4 | (uint32_t)W << 8 | (uint32_t)H << 12 |
                  (uint32_t)((a.c[m] + xa + ya) & 1) << 16 | M << 20;
    }
}

hipError_t launch_sweep_multi(SweepMultiArgs a, int C2, int kind, hipStream_t s)
{
    const int P = a.d[0].P;
    if (P > 8 || a.d[1].P > 8 || a.nph < 2 || a.nph > MULTI_MAXPH) return hipErrorInvalidValue;
    for (int m = 0; m < a.nph; m++)
        if (a.c[m] != ((a.c[0] + m) & 1) || a.t[m] < 0) return hipErrorInvalidValue;   // colours alternate
    const bool fixed = P == 8;
    const long long nb = (long long)sweep_multi_blocks(a.g.nx, a.g.ny) * a.b.ndir * a.b.npairs;
    if (nb <= 0) return hipSuccess;
    if (nb > 0x7FFFFFFFLL) return hipErrorInvalidValue;
    const dim3 grid((unsigned)nb);
    a.b.dnb = div_magic((uint32_t)sweep_multi_blocks(a.g.nx, a.g.ny));
    a.b.inter = same_images(a.d);
    a.dtx = div_magic((uint32_t)(a.g.nx + MULTI_TX - 1) / MULTI_TX);
    plan_multi(a);
#define PGM_MULTI(C2_, FX_)                                                                              \
    if (C2 == C2_ && fixed == FX_) {                                                                      \
        if (kind == 1) hipLaunchKernelGGL((k_sweep_multi<C2_, 8, FX_, 1>), grid, dim3(MULTI_TPB), 0, s, a);  \
        else if (kind == 2) hipLaunchKernelGGL((k_sweep_multi<C2_, 8, FX_, 2>), grid, dim3(MULTI_TPB), 0, s, a); \
        else hipLaunchKernelGGL((k_sweep_multi<C2_, 8, FX_, 0>), grid, dim3(MULTI_TPB), 0, s, a);            \
        return hipGetLastError();                                                                         \
    }
    PGM_MULTI(6, true) PGM_MULTI(6, false) PGM_MULTI(2, true) PGM_MULTI(2, false)
#undef PGM_MULTI
    return hipErrorInvalidValue;
}

hipError_t launch_sweep_pair(SweepMultiArgs a, int C2, int kind, hipStream_t s)
{
    const int P = a.d[0].P;
    if (P > 8 || a.d[1].P > 8 || a.nph != 2 || a.c[1] != 1 - a.c[0] || (a.c[0] & ~1) || a.t[0] < 0 || a.t[1] < 0)
        return hipErrorInvalidValue;
    const bool fixed = P == 8;
    const long long nb = (long long)sweep_pair_blocks(a.g.nx, a.g.ny) * a.b.ndir * a.b.npairs;
    if (nb <= 0) return hipSuccess;
    if (nb > 0x7FFFFFFFLL) return hipErrorInvalidValue;
    const dim3 grid((unsigned)nb);
    a.b.dnb = div_magic((uint32_t)sweep_pair_blocks(a.g.nx, a.g.ny));
    a.b.inter = same_images(a.d);
    a.dtx = div_magic((uint32_t)(a.g.nx + PAIR_TX - 1) / PAIR_TX);
#define PGM_PAIR(C2_, FX_)                                                                              \
    if (C2 == C2_ && fixed == FX_) {                                                                     \
        if (kind == 1) hipLaunchKernelGGL((k_sweep_pair<C2_, 8, FX_, 1>), grid, dim3(MULTI_TPB), 0, s, a); \
        else if (kind == 2) hipLaunchKernelGGL((k_sweep_pair<C2_, 8, FX_, 2>), grid, dim3(MULTI_TPB), 0, s, a); \
        else hipLaunchKernelGGL((k_sweep_pair<C2_, 8, FX_, 0>), grid, dim3(MULTI_TPB), 0, s, a);            \
        return hipGetLastError();                                                                        \
    }
    PGM_PAIR(6, true) PGM_PAIR(6, false) PGM_PAIR(2, true) PGM_PAIR(2, false)
#undef PGM_PAIR
    return hipErrorInvalidValue;
}

hipError_t launch_init(InitArgs a, int C2, int kind, hipStream_t s)
{
    PGM_DISPATCH(k_init, a, a.g.nx * a.g.ny);
}

hipError_t launch_down(TransArgs a, int C2, int kind, hipStream_t s)
{
    PGM_DISPATCH(k_down, a, a.g.nx * a.g.ny);
}

hipError_t launch_up(TransArgs a, int C2, int kind, hipStream_t s)
{
    PGM_DISPATCH(k_up, a, a.g.nx * a.g.ny);
}

hipError_t launch_enter(EnterArgs a, int C2, int kind, int mode, hipStream_t s)
{
    const int P = a.d[0].P;
    a.nb_col = sweep_blocks(a.g.nx, a.g.ny, P);
    a.nb_chk = mode == ENTER_LAUNCH_INIT ? 0 : (a.gs.nx * a.gs.ny + MATCH_TPB - 1) / MATCH_TPB;
    const int pmax = P <= 8 ? 8 : 16;
    const bool fixed = P == pmax;
    const long long nb = (long long)(2 * a.nb_col + a.nb_chk) * a.b.ndir * a.b.npairs;
    if (nb > 0x7FFFFFFFLL || a.b.ndir != 2) return hipErrorInvalidValue;
    const dim3 grid((unsigned)nb);
    a.b.dnb = div_magic((uint32_t)(2 * a.nb_col + a.nb_chk));
    a.b.inter = same_images(a.d);
    // patch sides up to 8 only: three candidate patches of 16 rows do not fit the registers
    if (mode == ENTER_LAUNCH_SWEEP) {
        PGM_V(k_enter, 6, 8, true) PGM_V(k_enter, 6, 8, false) PGM_V(k_enter, 2, 8, true) PGM_V(k_enter, 2, 8, false)
    } else if (mode == ENTER_LAUNCH_INIT) {
        PGM_V(k_enter_init, 6, 8, true) PGM_V(k_enter_init, 6, 8, false) PGM_V(k_enter_init, 2, 8, true)
        PGM_V(k_enter_init, 2, 8, false)
    } else {
        PGM_V(k_enter_start, 6, 8, true) PGM_V(k_enter_start, 6, 8, false) PGM_V(k_enter_start, 2, 8, true)
        PGM_V(k_enter_start, 2, 8, false)
    }
    return hipErrorInvalidValue;
}

#undef PGM_V
#undef PGM_DISPATCH

template <int C2, int PM, bool FX, int K>
static hipError_t launch_level_v(const LevelArgs& a, hipStream_t s)
{
    const size_t bytes = a.lay.total;
    hipLaunchKernelGGL((k_level<C2, PM, FX, K>), dim3(2 * a.b.npairs), dim3(LevelShape<PM, K == 1>::threads), bytes,
                       s, a);
    return hipGetLastError();
}

hipError_t level_allow_lds(size_t bytes)
{
    hipError_t first = hipSuccess;
    auto allow = [&](const void* fn) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess && first == hipSuccess) first = e;
    };
#define PGM_LA(C2_, PM_, FX_)                                                                    \
    allow((const void*)k_level<C2_, PM_, FX_, 0>);                                               \
    allow((const void*)k_level<C2_, PM_, FX_, 1>);                                               \
    allow((const void*)k_level<C2_, PM_, FX_, 2>);
    PGM_LA(6, 8, true) PGM_LA(6, 8, false) PGM_LA(6, 16, true) PGM_LA(6, 16, false)
    PGM_LA(2, 8, true) PGM_LA(2, 8, false) PGM_LA(2, 16, true) PGM_LA(2, 16, false)
#undef PGM_LA
    return first;
}

hipError_t launch_level(const LevelArgs& a, int C2, int kind, hipStream_t s)
{
    const int P = a.d[0].P;
    const int pmax = P <= 8 ? 8 : 16;
    const bool fixed = P == pmax;
#define PGM_LV(C2_, PM_, FX_)                                                                    \
    if (C2 == C2_ && pmax == PM_ && fixed == FX_)                                                \
        return kind == 1 ? launch_level_v<C2_, PM_, FX_, 1>(a, s)                                  \
               : kind == 2 ? launch_level_v<C2_, PM_, FX_, 2>(a, s) : launch_level_v<C2_, PM_, FX_, 0>(a, s);
    PGM_LV(6, 8, true) PGM_LV(6, 8, false) PGM_LV(6, 16, true) PGM_LV(6, 16, false)
    PGM_LV(2, 8, true) PGM_LV(2, 8, false) PGM_LV(2, 16, true) PGM_LV(2, 16, false)
#undef PGM_LV
    return hipErrorInvalidValue;
}

hipError_t launch_check(const CheckArgs& a, hipStream_t s)
{
    const int n = a.g.nx * a.g.ny;
    hipLaunchKernelGGL(k_check, dim3((n + 255) / 256, 2, a.b.npairs), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_regions(const RegionArgs& a, hipStream_t s)
{
    const int n = a.g.nx * a.g.ny;
    const dim3 grid((n + 255) / 256, 1, a.b.npairs);
    hipLaunchKernelGGL(k_cc_init, grid, dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_cc_union, grid, dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_cc_size, grid, dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_cc_apply, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_output(const OutArgs& a, hipStream_t s)
{
    const int n = a.g.nx * a.g.ny;
    hipLaunchKernelGGL(k_output, dim3((n + 255) / 256, a.b.ndir, a.b.npairs), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fill_tab(PairTab* dst, const PairTab* host, int n, hipStream_t s)
{
    if (n < 1 || n > TAB_MAX) return hipErrorInvalidValue;
    TabFill f;
    memset(&f, 0, sizeof f);
    for (int k = 0; k < n; k++) f.t[k] = host[k];
    f.dst = dst;
    f.n = n;
    hipLaunchKernelGGL(k_fill_tab, dim3(1), dim3(64), 0, s, f);
    return hipGetLastError();
}

hipError_t launch_count(const CountArgs& a, unsigned long long* part, hipStream_t s)
{
    long long n = 0;
    for (int k = 0; k < CountArgs::KINDS; k++) n = n > a.n[k] ? n : a.n[k];
    const int slices = (int)std::min<long long>(COUNT_SLICES, std::max<long long>(1, (n + 2047) / 2048));
    hipLaunchKernelGGL(k_count_part, dim3(slices, a.npairs), dim3(256), 0, s, a, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_count_sum, dim3(1), dim3(256), 0, s, a, (const unsigned long long*)part, slices);
    return hipGetLastError();
}

}  // namespace pgm
