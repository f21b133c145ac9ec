// scalp_device.h -- device helpers shared by the hard and soft kernels.
#pragma once

#include "scalp_internal.h"

namespace scalp {
namespace dev {

// First coordinate of grid cell `idx` of `n` along an axis of `len` pixels:
// pixel c is in cell floor(c * n / len), i.e. cell idx starts at
// ceil(idx * len / n).  With n <= len < 2^16 every product fits 32 bits and
// the division is a 32-bit one (len and n are uniform, so is the branch).
__device__ __forceinline__ int cell_lo(int idx, int len, int n) {
    if (len < 65536)
        return (int)(((unsigned)idx * (unsigned)len + (unsigned)(n - 1)) / (unsigned)n);
    return (int)(((long long)idx * len + n - 1) / n);
}

// Grid cell of coordinate c along an axis of `len` pixels cut into n cells:
// floor(c * n / len), in 32 bits when len < 2^16.
__device__ __forceinline__ int cell_of(int c, int n, int len) {
    if (len < 65536) return (int)(((unsigned)c * (unsigned)n) / (unsigned)len);
    return (int)(((long long)c * n) / len);
}

__device__ __forceinline__ float colour_dist(float4 f, float l, float a, float b) {
    float dl = f.x - l;
    float da = f.y - a;
    float db = f.z - b;
    return (dl * dl + da * da) + db * db;
}

__device__ __forceinline__ long long to_fixed(float v) {
    return (long long)rintf(v * kFixScaleF);
}

// Accumulates the samples i = 1 .. n-1 of the path from the pixel at linear
// index `idx` toward (dx, dy): on major-axis step i the minor offset is
// floor((2 i |d_minor| + n) / (2 n)).  stepx / stepy are the index strides
// of one pixel in x / y.  Global-memory variant, used when a candidate's
// path rectangle exceeds the LDS tables; samples are accumulated in path
// order, with up to three texel loads in flight.  Paths of up to 46340
// steps count the minor steps as the carries of a 32-bit accumulator (exact
// there, see walk_table); longer ones (cells over ~15000 pixels wide, or
// caller-supplied endpoints far across a wide image) keep the remainder
// exactly.
__device__ __forceinline__ unsigned step_increment(int am, int n);

__device__ __forceinline__ void walk_path(const float4* __restrict__ base, int idx, int stepx,
                                          int stepy, int dx, int dy, float l, float a, float b,
                                          float& sc, float& sw) {
    const int adx = dx < 0 ? -dx : dx;
    const int ady = dy < 0 ? -dy : dy;
    const bool xmaj = adx >= ady;
    const int n = xmaj ? adx : ady;
    if (n < 2) return;
    const int am = xmaj ? ady : adx;
    const int sx = dx < 0 ? -stepx : stepx;
    const int sy = dy < 0 ? -stepy : stepy;
    const int smaj = xmaj ? sx : sy;
    const int sdiag = smaj + (xmaj ? sy : sx);
#define SCALP_GACC(f)                                             \
    do {                                                          \
        const float dl_ = (f).x - l;                              \
        const float da_ = (f).y - a;                              \
        const float db_ = (f).z - b;                              \
        const float dc_ = (dl_ * dl_ + da_ * da_) + db_ * db_;    \
        sc = sc + dc_;                                            \
        sw = sw + (f).w;                                          \
    } while (0)
    if (n <= 46340) {
        const unsigned F = step_increment(am, n);
        unsigned acc = 0x80000000u;
#define SCALP_CSTEP()                                             \
    do {                                                          \
        const bool c_ = __builtin_add_overflow(acc, F, &acc);     \
        idx += c_ ? sdiag : smaj;                                 \
    } while (0)
        SCALP_CSTEP();
        float4 fa = base[idx];
        unsigned trips = (unsigned)(n - 2) >> 1;
        while (!__builtin_sub_overflow(trips, 1u, &trips)) {
            SCALP_CSTEP();
            const float4 fb = base[idx];
            SCALP_CSTEP();
            const float4 fc = base[idx];
            SCALP_GACC(fa);
            SCALP_GACC(fb);
            fa = fc;
            asm volatile("" : "+v"(acc));
        }
        if ((n - 2) & 1) {
            SCALP_CSTEP();
            const float4 fb = base[idx];
            SCALP_GACC(fa);
            fa = fb;
        }
        SCALP_GACC(fa);
#undef SCALP_CSTEP
        return;
    }
    const int two_n = 2 * n;
    const int inc = 2 * am;
    int rem = n;
#define SCALP_GSTEP()                                             \
    do {                                                          \
        rem += inc;                                               \
        const bool st_ = rem >= two_n;                            \
        rem -= st_ ? two_n : 0;                                   \
        idx += st_ ? sdiag : smaj;                                \
    } while (0)
    SCALP_GSTEP();
    float4 fa = base[idx];
    int left = n - 2;
    while (left >= 2) {
        SCALP_GSTEP();
        const float4 fb = base[idx];
        SCALP_GSTEP();
        const float4 fc = base[idx];
        SCALP_GACC(fa);
        SCALP_GACC(fb);
        fa = fc;
        left -= 2;
    }
    if (left == 1) {
        SCALP_GSTEP();
        const float4 fb = base[idx];
        SCALP_GACC(fa);
        fa = fb;
    }
    SCALP_GACC(fa);
#undef SCALP_GSTEP
#undef SCALP_GACC
}

// Increment of the carry-counting line stepper below for minor extent am and
// major extent n (0 <= am <= n).  Any F with 0 <= F - 2^32 am/n < 2^32/(2 n^2)
// steps exactly (see walk_table).  For n < 1023 a reciprocal good to one ulp
// gives 2^32 am/n within 769, and adding 1025 lands in (256, 1794]: inside
// the window for every n up to 1094.  Longer paths take the correctly
// rounded double quotient, rounded up.
__device__ __forceinline__ unsigned step_increment(int am, int n) {
    if (am == n) return 0xffffffffu;
    if (n < 1023) {
        const float sf = (float)am * __builtin_amdgcn_rcpf((float)n);
        return (unsigned)(sf * 4294967296.0f) + 1025u;
    }
    return (unsigned)ceil((double)am * 4294967296.0 / (double)n);
}

// Fills an LDS table with (d_c(q), w_q) for the texels of a rectangle of
// the packed image: entry e = r * tw + c holds texel (min(tx0 + c, W - 1),
// ty0 + r), for e < area (entries past the rectangle's width only pad the
// row pitch and are never read by a path).  Lanes step by WG entries, i.e.
// by (WG / tw rows, WG mod tw columns), with no division per entry, and
// take two entries per trip with both loads issued before either is used.
template <int WG>
__device__ __forceinline__ void fill_table(float2* tab, const float4* __restrict__ img, int W,
                                           int tx0, int ty0, int tw, int area, float l, float a,
                                           float b) {
    const int tid = threadIdx.x;
    const int dr = WG / tw, dc = WG - dr * tw;
    int r = tid / tw, c = tid - r * tw;
    const float4* row = img + (long long)(ty0 + r) * W;
    int e = tid;
    for (; e + WG < area; e += 2 * WG) {
        const float4 f0 = row[min(tx0 + c, W - 1)];
        c += dc;
        bool wrap = c >= tw;
        c -= wrap ? tw : 0;
        row += (long long)(dr + (wrap ? 1 : 0)) * W;
        const float4 f1 = row[min(tx0 + c, W - 1)];
        c += dc;
        wrap = c >= tw;
        c -= wrap ? tw : 0;
        row += (long long)(dr + (wrap ? 1 : 0)) * W;
        tab[e] = make_float2(colour_dist(f0, l, a, b), f0.w);
        tab[e + WG] = make_float2(colour_dist(f1, l, a, b), f1.w);
    }
    if (e < area) {
        const float4 f = row[min(tx0 + c, W - 1)];
        tab[e] = make_float2(colour_dist(f, l, a, b), f.w);
    }
}

// The same table, filled column by column: with R = WG / tw >= 1 rows per
// pass, lane tid < R tw keeps column c = tid mod tw of rows r0 = tid / tw,
// r0 + R, r0 + 2R, ... (entry e = r tw + c, starting at e = tid), so an
// entry costs one texel load, its colour distance and two index adds.
// r0 = floor(tid m / 2^24) with m = ceil(2^24 / tw): exact for tid < 2^10
// and tw < 2^14, since m tw - 2^24 < tw and tid (m tw - 2^24) < 2^24.  rows:
// the rectangle's rows; the caller supplies R and m (computed once per
// table) and takes fill_table when tw > WG.
template <int WG>
__device__ __forceinline__ void fill_table_cols(float2* tab, const float4* __restrict__ img,
                                                int W, int tx0, int ty0, int tw, int rows, int R,
                                                unsigned m, float l, float a, float b) {
    const int tid = threadIdx.x;
    const int r0 = (int)__umulhi((unsigned)tid << 8, m);
    if (r0 >= R) return;                           // lanes past R tw
    const int c = tid - r0 * tw;
    int p = (ty0 + r0) * W + min(tx0 + c, W - 1);  // < W H < 2^31
    const int dp = R * W, de = R * tw;
    int e = tid, r = r0;
    for (; r + R < rows; r += 2 * R) {
        const float4 f0 = img[p];
        const float4 f1 = img[p + dp];
        tab[e] = make_float2(colour_dist(f0, l, a, b), f0.w);
        tab[e + de] = make_float2(colour_dist(f1, l, a, b), f1.w);
        p += 2 * dp;
        e += 2 * de;
    }
    if (r < rows) {
        const float4 f = img[p];
        tab[e] = make_float2(colour_dist(f, l, a, b), f.w);
    }
}

// The walk over a per-candidate LDS table of (colour distance, w) pairs: the
// colour distance of a texel to the candidate does not depend on the pixel
// the path starts from, so it is computed once per texel (same FP32
// operations, same order) and every path sample costs two adds.
//
// Stepping: the minor-axis offset after i major steps, floor(i s + 1/2) with
// s = |d_minor| / n, is the number of carries out of a 32-bit accumulator
// that starts at 2^31 and adds F = ceil(2^32 s) per step (2^32 - 1 when
// s = 1).  The accumulated excess i (F - 2^32 s) < i stays below the gap
// 2^32 / (2n) between i s + 1/2 and the next integer whenever 2 n^2 < 2^32,
// i.e. n < 46340 (tables never exceed 2 x 9728 entries, so every path over a
// table qualifies), and an exact tie is never undershot since F rounds up.
// One add with carry-out, one select and one address add per sample; four
// samples per loop trip with the loads issued ahead of the adds.  The trip
// counter is decremented with a borrow-out that is itself the exit test, and
// the accumulator passes through an empty asm statement once per trip so
// that the compiler keeps the chain of adds instead of re-deriving acc from
// a separate induction variable (one instruction less per trip each).
__device__ __forceinline__ void walk_table(const float2* tab, int idx, int tw, int dx, int dy,
                                           float& sc, float& sw) {
    const int adx = dx < 0 ? -dx : dx;
    const int ady = dy < 0 ? -dy : dy;
    const bool xmaj = adx >= ady;
    const int n = xmaj ? adx : ady;
    if (n < 2) return;
    const int am = xmaj ? ady : adx;
    const unsigned F = step_increment(am, n);
    const int sx = dx < 0 ? -8 : 8;
    const int sy = dy < 0 ? -8 * tw : 8 * tw;
    const int smaj = xmaj ? sx : sy;
    const int sdiag = smaj + (xmaj ? sy : sx);
    unsigned acc = 0x80000000u;
    const char* q = reinterpret_cast<const char*>(tab + idx);
#define SCALP_STEP()                                              \
    do {                                                          \
        const bool c_ = __builtin_add_overflow(acc, F, &acc);     \
        q += c_ ? sdiag : smaj;                                   \
    } while (0)
#define SCALP_LOAD() (*reinterpret_cast<const float2*>(q))
#define SCALP_ACC(v)                                              \
    do {                                                          \
        sc = sc + (v).x;                                          \
        sw = sw + (v).y;                                          \
    } while (0)
    // samples 1 .. n-1 (sample 0 and the endpoint are added by the caller)
    SCALP_STEP();
    float2 fa = SCALP_LOAD();
    unsigned trips = (unsigned)(n - 2) >> 2;
    while (!__builtin_sub_overflow(trips, 1u, &trips)) {
        SCALP_STEP();
        const float2 fb = SCALP_LOAD();
        SCALP_STEP();
        const float2 fc = SCALP_LOAD();
        SCALP_ACC(fa);
        SCALP_STEP();
        const float2 fd = SCALP_LOAD();
        SCALP_ACC(fb);
        SCALP_STEP();
        fa = SCALP_LOAD();
        SCALP_ACC(fc);
        SCALP_ACC(fd);
        asm volatile("" : "+v"(acc));
    }
    const int rem = (n - 2) & 3;
    if (rem > 0) {
        SCALP_STEP();
        const float2 fb = SCALP_LOAD();
        SCALP_ACC(fa);
        fa = fb;
    }
    if (rem > 1) {
        SCALP_STEP();
        const float2 fb = SCALP_LOAD();
        SCALP_ACC(fa);
        fa = fb;
    }
    if (rem > 2) {
        SCALP_STEP();
        const float2 fb = SCALP_LOAD();
        SCALP_ACC(fa);
        fa = fb;
    }
    SCALP_ACC(fa);
#undef SCALP_STEP
#undef SCALP_LOAD
#undef SCALP_ACC
}

// Correctly rounded FP64 reciprocals 1/1 .. 1/1024, built at compile time.
struct RecipTable {
    double v[1025];
    constexpr RecipTable() : v() {
        for (int i = 1; i <= 1024; ++i) v[i] = 1.0 / (double)i;
    }
};
namespace {
__constant__ const RecipTable kRecip = RecipTable();
}

// RN(1 / (n + 1)) for a path of n steps (np = n + 1 samples), clamped to the
// table; callers fetch it before walking the path so that the load's latency
// hides behind the walk.
__device__ __forceinline__ double path_recip(int n) { return kRecip.v[(n < 1023 ? n : 1023) + 1]; }

// a / np and b / np in IEEE FP32 (np = n + 1) for the two averages of
// Eqs. (1)-(2); inv = path_recip(n).  For np <= 1024 and a, b zero or at
// least 2^-100, the FP32 rounding of the FP64 product a * RN(1/np) is the
// IEEE quotient: a float divided by an integer np is never a rounding
// midpoint of FP32 and stays at least 2^-35 (relative) away from one for
// np <= 1024, while the product's error is below 2^-52.  Other operands take
// the IEEE division itself.
__device__ __forceinline__ void div_path_len(float a, float b, int n, double inv, float& qa,
                                             float& qb) {
    const bool fast = n < 1024 && !(a > 0.0f && a < 0x1p-100f) && !(b > 0.0f && b < 0x1p-100f);
    if (fast) {
        qa = (float)((double)a * inv);
        qb = (float)((double)b * inv);
    } else {
        const float np = (float)(n + 1);
        qa = a / np;
        qb = b / np;
    }
}

__device__ __forceinline__ int round_coord(float v, int hi) {
    int e = (int)floorf(v + 0.5f);
    e = e < 0 ? 0 : e;
    return e > hi ? hi : e;
}

// Workgroup index -> work item.  Workgroups are dispatched round-robin over
// the 8 XCDs; give each XCD a contiguous run of items so that neighbouring
// cells, which read overlapping table rectangles, share an L2.
__device__ __forceinline__ int xcd_remap(int b, int G) {
    const int q = G >> 3, rem = G & 7;
    const int x = b & 7, slot = b >> 3;
    return x < rem ? x * (q + 1) + slot : rem * (q + 1) + (x - rem) * q + slot;
}

// Cell at position i of the cell order of the grid assignment: column
// strips ceil(nx / strips) cells wide (the last one narrower), row-major
// within a strip.  A bijection of [0, nx ny); strips = 1 is row-major order.
__device__ __forceinline__ int cell_in_strips(int i, int nx, int ny, int strips) {
    const int tw = (nx + strips - 1) / strips;
    const int s = i / (tw * ny);
    const int x0 = s * tw;
    const int w = min(tw, nx - x0);
    const int l = i - s * tw * ny;
    const int r = l / w;
    return r * nx + x0 + (l - r * w);
}

__device__ __forceinline__ int find_image(const int* start, int n, int v) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= v) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Pixel t of a cell of width cw and height ch, enumerated in 8-wide column
// strips walked serpentine (down, up, ...): 64 consecutive indices form a
// compact 8x8 block, so the lanes of a wave walk paths of similar length.
__device__ __forceinline__ void cell_pixel(int t, int cw, int ch, int& x, int& y) {
    const int nfull = cw >> 3, wr = cw & 7;
    const int fullpx = nfull * 8 * ch;
    int s, row, col;
    if (t < fullpx) {
        const int per = 8 * ch;
        s = t / per;
        const int r = t - s * per;
        row = r >> 3;
        col = 8 * s + (r & 7);
    } else {
        s = nfull;
        const int r = t - fullpx;
        row = r / wr;
        col = 8 * nfull + (r - row * wr);
    }
    y = (s & 1) ? (ch - 1 - row) : row;
    x = col;
}

// Strip (8-column band) of cell pixel t, in the order of cell_pixel.
__device__ __forceinline__ int strip_of(int t, int cw, int ch) {
    const int fullpx = (cw >> 3) * 8 * ch;
    return t < fullpx ? t / (8 * ch) : (cw >> 3);
}

// x of lane i - CTRL's shift, 0 where that lane is outside the row or the
// row is not in ROW_MASK (DPP: gfx9 row_shr / row_bcast controls).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_or_zero(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xf,
                                                      false));
}

// Sum over the 64 lanes of a wave in six DPP steps (no LDS traffic): row
// prefix sums by shifts of 1, 2, 4 and 8 lanes, then the last lane of each
// row is broadcast into the next row (row_bcast:15) and lane 31 into rows 2
// and 3 (row_bcast:31).  Only lane 63 holds the total.  All lanes must be
// active.
__device__ __forceinline__ float wave_sum_last(float v) {
    v += dpp_or_zero<0x111, 0xf>(v);
    v += dpp_or_zero<0x112, 0xf>(v);
    v += dpp_or_zero<0x114, 0xf>(v);
    v += dpp_or_zero<0x118, 0xf>(v);
    v += dpp_or_zero<0x142, 0xa>(v);
    v += dpp_or_zero<0x143, 0xc>(v);
    return v;
}

// Minimum and maximum over the 64 lanes of a wave (all lanes active), the
// same value in every lane.
__device__ __forceinline__ int wave_min_i32(int v) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ int wave_max_i32(int v) {
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ float wave_sum(float v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

}  // namespace dev
}  // namespace scalp
