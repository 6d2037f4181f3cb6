// gfx950 kernels of the three offloaded loop nests (sweep S, residual R,
// copy-back C), their batched forms, and the transfer/measurement helpers.
//
// The nests are the loop bodies of the Jacobi program whose loops the paper's
// method offloads (Sec. 3.2.1): S computes wrk2 = p + omega*ss from the old
// iterate with the 19-point variable-coefficient stencil, R sums
// ((wrk2 - p)/omega)^2 over the interior, C copies wrk2 back into p on the
// interior. All three are HBM-bound (S: 56 bytes per point for FP32
// coefficients, 32 for bfloat16; R and C: 8), so the design is about streaming:
//
//  * one wave owns one j-row and 64*VEC consecutive i-points (VEC per lane,
//    loaded as one 4/8/16-byte vector), so every load and store is coalesced
//    along the contiguous i axis; a batch runs a grid with short, compactly
//    stored rows in packed form, where a wave's points run across row ends;
//  * the wave marches through a chunk of k-planes keeping rows j-1, j, j+1 of
//    planes k-1, k, k+1 in registers: each p value comes from memory once per
//    row-march, the k+-1 neighbours never reload;
//  * the i+-1 neighbours come from the adjacent lane through a cross-lane
//    shuffle; only the two wave-edge lanes load one halo value each;
//  * stores are whole vectors, so rows are written in full 128-byte lines;
//  * no LDS and no barriers: the j+-1 rows are re-read by the waves of the
//    neighbouring rows and served by L1/L2; every XCD takes one contiguous
//    band of row blocks from each k-chunk, so neighbouring blocks share an L2
//    while all XCDs stream the same window of HBM at once (an XCD-contiguous
//    order over the whole grid is a tile option);
//  * no MFMA: there is no dense contraction here.

#include <algorithm>
#include <array>
#include <atomic>
#include <mutex>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "ofl_internal.hpp"

namespace ofl {
namespace {

typedef float f2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned int u2 __attribute__((ext_vector_type(2)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

constexpr int kXcds = 8;

// Work-groups are handed to the 8 XCDs round-robin by id. With the remap on,
// XCD x receives one contiguous range of logical tiles, so neighbouring tiles
// (which share halo rows) share that XCD's L2. Off (the default), all XCDs
// work through the same window of the grid at the same time, which on MI355X
// streams HBM faster for the sweep (measured: 333 us vs 347 us per sweep at
// 257x257x513) than the L2 sharing saves.
__device__ __forceinline__ int xcd_remap(int bid, int n) {
    const int xcd = bid % kXcds;
    const int local = bid / kXcds;
    const int per = n / kXcds;
    const int rem = n % kXcds;
    return xcd * per + min(xcd, rem) + local;
}

// The sweep's default order when a k-chunk holds a multiple of 8 tiles (`row`
// of them, k-chunk slowest): XCD x takes tiles [x*row/8, (x+1)*row/8) of every
// k-chunk, k-chunk after k-chunk. All XCDs still work on the same k-chunks at
// once, and a block's j-neighbours run beside it on the same XCD, so the halo
// rows they share are fetched into one L2 once instead of into two. Measured at
// 257x257x513: fetched bytes per sweep 1.871 -> 1.776 GB (FP32) and
// 1.115 -> 1.006 GB (bfloat16), the sweep 320.2 -> 319.5 us and 196.2 -> 194.6 us.
__device__ __forceinline__ int xcd_band(int bid, int row) {
    const int xcd = bid % kXcds;
    const int slot = bid / kXcds;
    const int per = row / kXcds;
    return (slot / per) * row + xcd * per + slot % per;
}

// Order of a sweep launch's tiles: round-robin by block id, XCD-contiguous
// ranges (OFL_TILE_XCD_REMAP), or XCD bands of each k-chunk.
enum : int { kOrderPlain = 0, kOrderRemap = 1, kOrderBand = 2 };

template <bool NT, typename T>
__device__ __forceinline__ T ld(const T *ptr) {
    if constexpr (NT)
        return __builtin_nontemporal_load(ptr);
    else
        return *ptr;
}

template <bool NT, typename T>
__device__ __forceinline__ void st(T *ptr, T v) {
    if constexpr (NT)
        __builtin_nontemporal_store(v, ptr);
    else
        *ptr = v;
}

template <int VEC, bool NT>
__device__ __forceinline__ void load_f32(const float *ptr, float (&v)[VEC]) {
    if constexpr (VEC == 1) {
        v[0] = ld<NT>(ptr);
    } else if constexpr (VEC == 2) {
        f2 x = ld<NT>(reinterpret_cast<const f2 *>(ptr));
        v[0] = x.x;
        v[1] = x.y;
    } else if constexpr (VEC == 4) {
        f4 x = ld<NT>(reinterpret_cast<const f4 *>(ptr));
        v[0] = x.x;
        v[1] = x.y;
        v[2] = x.z;
        v[3] = x.w;
    } else {
        static_assert(VEC == 8, "vector width");
        f4 x = ld<NT>(reinterpret_cast<const f4 *>(ptr));
        f4 y = ld<NT>(reinterpret_cast<const f4 *>(ptr) + 1);
        v[0] = x.x;
        v[1] = x.y;
        v[2] = x.z;
        v[3] = x.w;
        v[4] = y.x;
        v[5] = y.y;
        v[6] = y.z;
        v[7] = y.w;
    }
}

template <int VEC, bool NT>
__device__ __forceinline__ void store_f32(float *ptr, const float (&v)[VEC]) {
    if constexpr (VEC == 1) {
        st<NT>(ptr, v[0]);
    } else if constexpr (VEC == 2) {
        f2 x = {v[0], v[1]};
        st<NT>(reinterpret_cast<f2 *>(ptr), x);
    } else if constexpr (VEC == 4) {
        f4 x = {v[0], v[1], v[2], v[3]};
        st<NT>(reinterpret_cast<f4 *>(ptr), x);
    } else {
        static_assert(VEC == 8, "vector width");
        f4 x = {v[0], v[1], v[2], v[3]};
        f4 y = {v[4], v[5], v[6], v[7]};
        st<NT>(reinterpret_cast<f4 *>(ptr), x);
        st<NT>(reinterpret_cast<f4 *>(ptr) + 1, y);
    }
}

// bfloat16 -> FP32 is exact: the 16 stored bits are the high half of the FP32
// encoding. The offset format adds its per-array FP32 bias (0 for plain).
__device__ __forceinline__ float bf16_lo(unsigned u) { return __uint_as_float(u << 16); }
__device__ __forceinline__ float bf16_hi(unsigned u) { return __uint_as_float(u & 0xffff0000u); }

template <int VEC, bool NT>
__device__ __forceinline__ void load_bf16(const uint16_t *ptr, float bias, float (&v)[VEC]) {
    if constexpr (VEC == 1) {
        unsigned u = ld<NT>(ptr);
        v[0] = bias + bf16_lo(u);
    } else if constexpr (VEC == 2) {
        unsigned u = ld<NT>(reinterpret_cast<const unsigned *>(ptr));
        v[0] = bias + bf16_lo(u);
        v[1] = bias + bf16_hi(u);
    } else if constexpr (VEC == 4) {
        u2 x = ld<NT>(reinterpret_cast<const u2 *>(ptr));
        v[0] = bias + bf16_lo(x.x);
        v[1] = bias + bf16_hi(x.x);
        v[2] = bias + bf16_lo(x.y);
        v[3] = bias + bf16_hi(x.y);
    } else {
        // 16 bytes per lane: eight bfloat16 values in one load
        static_assert(VEC == 8, "vector width");
        u4 x = ld<NT>(reinterpret_cast<const u4 *>(ptr));
        v[0] = bias + bf16_lo(x.x);
        v[1] = bias + bf16_hi(x.x);
        v[2] = bias + bf16_lo(x.y);
        v[3] = bias + bf16_hi(x.y);
        v[4] = bias + bf16_lo(x.z);
        v[5] = bias + bf16_hi(x.z);
        v[6] = bias + bf16_lo(x.w);
        v[7] = bias + bf16_hi(x.w);
    }
}

// Lanes that share one row segment: the whole wave, or, with 8 points per
// lane, each half of it (a wave then owns two rows of 256 points, so a tile is
// 256 points wide at every vector width from 4 up and each coefficient load is
// 16 bytes per lane in the bfloat16 formats).
template <int VEC>
constexpr int lanes_per_row() {
    return VEC == 8 ? kWave / 2 : kWave;
}

// One row segment of p: this lane's VEC values plus its outer neighbours
// (left of element 0, right of element VEC-1). The loads are issued for all
// rows of a step before any neighbour exchange, so that one wait covers the
// whole step: issue_prow() starts the vector load and the halo load,
// finish_prow() takes the inner neighbours from the adjacent lanes and the
// two segment-edge neighbours from the halo value. `sub` is the lane's index
// within its row segment. The halo load is branch-free: the segment's last
// lane reads the element after the tile (hr), every other lane the element
// before it (hl, one shared cache line). For the first tile of a row that
// element is row padding or the array's front guard; it only feeds i = 0,
// which is never stored.
template <int VEC>
__device__ __forceinline__ void issue_prow(const float *row, int il, int hl, int hr, int sub, float (&v)[VEC],
                                           float &h) {
    load_f32<VEC, false>(row + il, v);
    h = row[sub == lanes_per_row<VEC>() - 1 ? hr : hl];
}

template <int VEC>
__device__ __forceinline__ void finish_prow(const float (&v)[VEC], float h, int sub, float &l, float &r) {
    const float up = __shfl_up(v[VEC - 1], 1, kWave);
    const float dn = __shfl_down(v[0], 1, kWave);
    l = (sub == 0) ? h : up;
    r = (sub == lanes_per_row<VEC>() - 1) ? h : dn;
}

template <int VEC, bool BF16, bool NT>
__device__ __forceinline__ void load_coefs(const GridView &g, long long off, float (&c)[kNCoef][VEC]) {
#pragma unroll
    for (int n = 0; n < kNCoef; ++n) {
        if constexpr (BF16)
            load_bf16<VEC, NT>(static_cast<const uint16_t *>(g.coef[n]) + off, g.bias[n], c[n]);
        else
            load_f32<VEC, NT>(static_cast<const float *>(g.coef[n]) + off, c[n]);
    }
}

// Nest S for one wave: i-points ts + lane*VEC .. +VEC-1 of one line of the
// grid, marching along it. In packed-row form (a batched grid with
// g.nseg > 0, k-march only) the line is a segment of 64*VEC consecutive
// points of a plane that runs across row ends: `fixed` is 0, ts counts points
// from the plane's start, and rows j-1, j+1 of a point lie one pitch before and
// after it. The pitch is a multiple of 4, so a lane's VEC points share one
// row. Points of row 0 that the first segment covers are never stored.
// Without OFL_TILE_MARCH_J the wave owns row j =
// `fixed` and marches through planes k = m0..m1-1 (consecutive steps one plane
// apart); with it the wave owns plane k = `fixed` and marches through rows
// j = m0..m1-1 (consecutive steps one row apart, so every stream the wave reads
// advances through contiguous memory). Either way rows j-1..j+1 of planes
// k-1..k+1 stay in registers and each step loads only the three new rows.
// With 8 points per lane (k-march, unpacked rows only) the wave owns rows
// `fixed` and `fixed`+1, one per half-wave; a half whose row lies past J-2
// loads row J-2 and stores nothing.
template <int VEC, bool BF16, int FLAGS>
__device__ __forceinline__ void sweep_march(const GridView &g, int ts, int fixed, int m0, int m1, float omega,
                                            double *part) {
    constexpr bool kFuseR = (FLAGS & kFlagFuseResidual) != 0;
    constexpr bool kNtLoads = (FLAGS & OFL_TILE_NT_LOADS) != 0;
    constexpr bool kNtStores = (FLAGS & OFL_TILE_NT_STORES) != 0;
    constexpr bool kPrefetch = (FLAGS & OFL_TILE_PREFETCH) != 0;
    constexpr bool kMarchJ = (FLAGS & OFL_TILE_MARCH_J) != 0;
    constexpr int kLpr = lanes_per_row<VEC>();
    static_assert(VEC != 8 || !kMarchJ, "8 points per lane march along k only");
    const int lane = threadIdx.x & (kWave - 1);
    const int sub = lane & (kLpr - 1);
    const int ib = ts + sub * VEC;
    const bool packed = !kMarchJ && VEC != 8 && g.nseg > 0;
    const int flat_end = (g.J - 1) * g.pitch;  // packed: first point after row J-2
    // Lanes whose vector starts past the row's last element (packed: past row
    // J-2) load the last vector before that instead (same cache line, no extra
    // HBM traffic); their results are never stored.
    const int il = packed ? min(ib, flat_end - VEC) : min(ib, ((g.I - 1) / VEC) * VEC);
    const int hl = ts - 1;
    const int hr = packed ? min(ts + kLpr * VEC, flat_end - 1) : ts + kLpr * VEC;
    // i of the lane's first point, and whether its row is an interior one
    const int jr = packed ? ib / g.pitch : 0;
    const int i0 = ib - jr * g.pitch;
    const int jown = VEC == 8 ? fixed + lane / kLpr : fixed;  // this lane's row (k-march)
    const bool row_ok = packed ? (jr >= 1 && jr <= g.J - 2) : (VEC != 8 || jown <= g.J - 2);
    if constexpr (VEC == 8)
        fixed = min(jown, g.J - 2);
    const long long pitch = g.pitch;
    const long long plane = g.plane;
    const float *__restrict__ p = g.p;
    auto row = [&](int j, int k) { return p + j * pitch + k * plane; };
    // The coefficient arrays have rows of their own pitch, which can end
    // before i = I-1. A lane whose vector would run past that end has no
    // interior point, so it reads the row's last vector instead (packed rows
    // share p's layout and stay as they are).
    const long long cpitch = g.cpitch;
    const long long cplane = g.cplane;
    const int ilc = packed ? il : min(il, g.cpitch - VEC);
    // offset of the coefficients of step m
    auto coef_off = [&](int m) {
        return kMarchJ ? m * cpitch + fixed * cplane + ilc : fixed * cpitch + m * cplane + ilc;
    };

    // P[r][q][e]: row j-1+r, plane k-1+q, element e. EL/ER: outer neighbours.
    float P[3][3][VEC];
    float EL[3][3], ER[3][3];
    {
        // the two lines behind the first step
        float h[2][3];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                if constexpr (kMarchJ)
                    issue_prow<VEC>(row(m0 - 1 + a, fixed - 1 + b), il, hl, hr, sub, P[a][b], h[a][b]);
                else
                    issue_prow<VEC>(row(fixed - 1 + b, m0 - 1 + a), il, hl, hr, sub, P[b][a], h[a][b]);
            }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                if constexpr (kMarchJ)
                    finish_prow<VEC>(P[a][b], h[a][b], sub, EL[a][b], ER[a][b]);
                else
                    finish_prow<VEC>(P[b][a], h[a][b], sub, EL[b][a], ER[b][a]);
            }
    }

    float C[kNCoef][VEC];
    if constexpr (kPrefetch)
        load_coefs<VEC, BF16, kNtLoads>(g, coef_off(m0), C);

    const int I = g.I;
    float *__restrict__ wrk2 = g.wrk2;
    double racc = 0.0;  // fused residual: sum of (wrk2 - p)^2 over this wave's points
    for (int m = m0; m < m1; ++m) {
        const int j = kMarchJ ? m : fixed;
        const int k = kMarchJ ? fixed : m;
        float Cn[kNCoef][VEC];
        if constexpr (kPrefetch) {
            if (m + 1 < m1)
                load_coefs<VEC, BF16, kNtLoads>(g, coef_off(m + 1), Cn);
        } else {
            load_coefs<VEC, BF16, kNtLoads>(g, coef_off(m), C);
        }
        // the three new rows: j+1 of planes k-1..k+1 (j-march) or
        // j-1..j+1 of plane k+1 (k-march)
        float h[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            if constexpr (kMarchJ)
                issue_prow<VEC>(row(j + 1, k - 1 + b), il, hl, hr, sub, P[2][b], h[b]);
            else
                issue_prow<VEC>(row(j - 1 + b, k + 1), il, hl, hr, sub, P[b][2], h[b]);
        }
        // Keep every load of the step ahead of the first use, so one wait
        // covers them all instead of the scheduler trading them for registers.
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            if constexpr (kMarchJ)
                finish_prow<VEC>(P[2][b], h[b], sub, EL[2][b], ER[2][b]);
            else
                finish_prow<VEC>(P[b][2], h[b], sub, EL[b][2], ER[b][2]);
        }

        float out[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            // neighbour at i+1 / i-1 of element e in row r, plane q
            auto rt = [&](int r, int q) { return e < VEC - 1 ? P[r][q][e + 1] : ER[r][q]; };
            auto lf = [&](int r, int q) { return e > 0 ? P[r][q][e - 1] : EL[r][q]; };
            // Every product is fused with its sum explicitly, in one fixed
            // order, so each point gets the same roundings in every tile,
            // width, batched and fused form (the compiler's own contraction
            // may pair a different product with each sum per instantiation).
            const float centre = P[1][1][e];
            float s0 = C[0][e] * rt(1, 1);
            s0 = fmaf(C[1][e], P[2][1][e], s0);
            s0 = fmaf(C[2][e], P[1][2][e], s0);
            s0 = fmaf(C[4][e], (rt(2, 1) - rt(0, 1)) - (lf(2, 1) - lf(0, 1)), s0);
            s0 = fmaf(C[5][e], (P[2][2][e] - P[0][2][e]) - (P[2][0][e] - P[0][0][e]), s0);
            s0 = fmaf(C[6][e], (rt(1, 2) - lf(1, 2)) - (rt(1, 0) - lf(1, 0)), s0);
            s0 = fmaf(C[7][e], lf(1, 1), s0);
            s0 = fmaf(C[8][e], P[0][1][e], s0);
            s0 = fmaf(C[9][e], P[1][0][e], s0);
            s0 += C[11][e];
            const float ss = fmaf(C[3][e], s0, -centre) * C[10][e];
            out[e] = fmaf(omega, ss, centre);
            if constexpr (kFuseR) {
                // the residual nest's own term, (wrk2 - p) in FP32 squared in FP64
                if (row_ok && i0 + e >= 1 && i0 + e <= I - 2) {
                    const double d = static_cast<double>(out[e] - centre);
                    racc = fma(d, d, racc);
                }
            }
        }
        // Points of an interior row outside the interior (its two boundary
        // columns and the row padding) receive p's own value, so every lane that
        // loaded its own points stores one whole vector and the rows of wrk2 are
        // written in full 128-byte lines. The interior is what the nest computes.
        if (row_ok && il == ib) {
#pragma unroll
            for (int e = 0; e < VEC; ++e)
                if (i0 + e < 1 || i0 + e > I - 2)
                    out[e] = P[1][1][e];
            store_f32<VEC, kNtStores>(wrk2 + j * pitch + k * plane + ib, out);
        }

        // slide the register window one step along the march axis
#pragma unroll
        for (int b = 0; b < 3; ++b) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                if constexpr (kMarchJ) {
                    P[0][b][e] = P[1][b][e];
                    P[1][b][e] = P[2][b][e];
                } else {
                    P[b][0][e] = P[b][1][e];
                    P[b][1][e] = P[b][2][e];
                }
            }
            if constexpr (kMarchJ) {
                EL[0][b] = EL[1][b];
                EL[1][b] = EL[2][b];
                ER[0][b] = ER[1][b];
                ER[1][b] = ER[2][b];
            } else {
                EL[b][0] = EL[b][1];
                EL[b][1] = EL[b][2];
                ER[b][0] = ER[b][1];
                ER[b][1] = ER[b][2];
            }
        }
        if constexpr (kPrefetch) {
#pragma unroll
            for (int n = 0; n < kNCoef; ++n)
#pragma unroll
                for (int e = 0; e < VEC; ++e)
                    C[n][e] = Cn[n][e];
        }
    }
    if constexpr (kFuseR) {
        // butterfly over the wave, fixed order; lane 0 writes the wave's partial
#pragma unroll
        for (int d = kWave / 2; d >= 1; d >>= 1)
            racc += __shfl_xor(racc, d, kWave);
        if (lane == 0)
            *part = racc;
    }
}

// Fixed-order sum of n FP64 values by one whole work-group of any size (a
// multiple of 64 threads, at most 512): thread t adds x[t], x[t + size], ... in
// order, each wave folds its lanes by a butterfly, and thread 0 adds the waves
// in index order. The total is returned on thread 0. Every thread of the
// work-group must call it (it holds two barriers).
__device__ __forceinline__ double group_sum_fixed(const double *x, long long n) {
    __shared__ double wsum[512 / kWave];
    const long long step = blockDim.x;
    long long t = threadIdx.x;
    double v = 0.0;
    // eight loads in flight, added in index order
    for (; t + 7 * step < n; t += 8 * step) {
        double a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            a[u] = x[t + u * step];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            v += a[u];
    }
    for (; t < n; t += step)
        v += x[t];
#pragma unroll
    for (int m = kWave / 2; m >= 1; m >>= 1)
        v += __shfl_xor(v, m, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0)
        wsum[threadIdx.x / kWave] = v;
    __syncthreads();
    double total = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < static_cast<int>(blockDim.x / kWave); ++w)
            total += wsum[w];
    __syncthreads();  // wsum may be reused by the caller's next call
    return total;
}

// Lines a wave may own and the extent of its march, per march axis.
template <int FLAGS>
__device__ __forceinline__ void march_extent(const GridView &g, int &fixed_last, int &march_end) {
    constexpr bool kMarchJ = (FLAGS & OFL_TILE_MARCH_J) != 0;
    fixed_last = kMarchJ ? g.K - 2 : g.J - 2;
    march_end = kMarchJ ? g.J - 1 : g.K - 1;
}

template <int VEC, bool BF16, int FLAGS>
__global__ __launch_bounds__(512) void sweep_kernel(GridView g, int chunk, int nti, int nfb, float omega,
                                                    int order, double *parts, PrevParts prev) {
    const int bid = static_cast<int>(blockIdx.x);
    if constexpr ((FLAGS & kFlagFuseResidual) != 0) {
        // the previous iteration's residual, before this work-group's march
        // (whole work-group: no wave has returned yet)
        if (prev.parts && bid == 0) {
            const double total = group_sum_fixed(prev.parts, prev.n);
            if (threadIdx.x == 0)
                *g.gosa = total / (static_cast<double>(omega) * static_cast<double>(omega));
        }
    }
    const int L = order == kOrderBand    ? xcd_band(bid, nti * nfb)
                  : order == kOrderRemap ? xcd_remap(bid, gridDim.x)
                                         : bid;
    // fused residual: one partial per wave of the launch, every slot written
    double *part = nullptr;
    if constexpr ((FLAGS & kFlagFuseResidual) != 0)
        part = parts + static_cast<long long>(blockIdx.x) * (blockDim.x / kWave) + threadIdx.x / kWave;
    const int it = L % nti;
    const int rest = L / nti;
    const int fb = rest % nfb;
    const int mc = rest / nfb;
    const int lines = blockDim.x / kWave;
    // a wave owns one line, or two rows with 8 points per lane
    constexpr int kRowsPerWave = kWave / lanes_per_row<VEC>();
    const int fixed = 1 + (fb * lines + static_cast<int>(threadIdx.x / kWave)) * kRowsPerWave;
    int fixed_last, march_end;
    march_extent<FLAGS>(g, fixed_last, march_end);
    if (fixed > fixed_last) {
        if constexpr ((FLAGS & kFlagFuseResidual) != 0)
            if ((threadIdx.x & (kWave - 1)) == 0)
                *part = 0.0;
        return;
    }
    const int m0 = 1 + mc * chunk;
    const int m1 = min(m0 + chunk, march_end);
    sweep_march<VEC, BF16, FLAGS>(g, it * tile_points(VEC), fixed, m0, m1, omega, part);
}

// One batched sweep item for one wave: its line (or packed segment) and march
// chunk. part (fused residual) receives the wave's partial, 0 for an idle wave.
template <int VEC, bool BF16, int FLAGS>
__device__ __forceinline__ void batch_sweep_item(const GridView &g, const SweepItem &item, int chunk, float omega,
                                                 int lines, int wave, double *part) {
    constexpr bool kFuseR = (FLAGS & kFlagFuseResidual) != 0;
    if constexpr ((FLAGS & OFL_TILE_MARCH_J) == 0) {
        if (g.nseg > 0) {
            // packed rows: the work-group's waves own consecutive segments
            const int seg = item.fblock * lines + wave;
            if (seg >= g.nseg) {
                if constexpr (kFuseR)
                    if ((threadIdx.x & (kWave - 1)) == 0)
                        *part = 0.0;
                return;
            }
            const int m0 = 1 + item.mchunk * chunk;
            const int m1 = min(m0 + chunk, g.K - 1);
            sweep_march<VEC, BF16, FLAGS>(g, packed_seg0(g.pitch) + seg * kWave * VEC, 0, m0, m1, omega, part);
            return;
        }
    }
    const int fixed = 1 + item.fblock * lines + wave;
    int fixed_last, march_end;
    march_extent<FLAGS>(g, fixed_last, march_end);
    if (fixed > fixed_last) {
        if constexpr (kFuseR)
            if ((threadIdx.x & (kWave - 1)) == 0)
                *part = 0.0;
        return;
    }
    const int m0 = 1 + item.mchunk * chunk;
    const int m1 = min(m0 + chunk, march_end);
    sweep_march<VEC, BF16, FLAGS>(g, item.itile * kWave * VEC, fixed, m0, m1, omega, part);
}

// parts (fused residual only): slot w*lines + wave receives the partial of
// wave `wave` of item w; every slot of every item is written. VEC == 0: each
// item runs at its grid's own width (g.vec: 1, 2 or 4), so one launch covers
// grids of every width; the branch is uniform over the work-group.
template <int VEC, bool BF16, int FLAGS>
__global__ __launch_bounds__(512) void batch_sweep_kernel(const GridView *__restrict__ views,
                                                          const SweepItem *__restrict__ items, int nitems,
                                                          int chunk, float omega, int remap, double *parts,
                                                          PrevParts prev) {
    constexpr bool kFuseR = (FLAGS & kFlagFuseResidual) != 0;
    if constexpr (kFuseR) {
        // the previous iteration's residual of grid b, by work-group b (and
        // b + gridDim.x, ...), before any of its items
        if (prev.parts)
            for (int b = static_cast<int>(blockIdx.x); b < prev.ngrids; b += gridDim.x) {
                const long long lo = prev.range[2 * b];
                const double total = group_sum_fixed(prev.parts + lo, prev.range[2 * b + 1] - lo);
                if (threadIdx.x == 0)
                    *views[b].gosa = total / (static_cast<double>(omega) * static_cast<double>(omega));
            }
    }
    const int lines = blockDim.x / kWave;
    const int wave = static_cast<int>(threadIdx.x / kWave);
    const int first = remap ? xcd_remap(blockIdx.x, gridDim.x) : static_cast<int>(blockIdx.x);
    for (int w = first; w < nitems; w += gridDim.x) {
        const SweepItem item = items[w];
        const GridView g = views[item.grid];
        double *part = nullptr;
        if constexpr (kFuseR)
            part = parts + static_cast<long long>(w) * lines + wave;
        if constexpr (VEC == 0) {
            if (g.vec == 1)
                batch_sweep_item<1, BF16, FLAGS>(g, item, chunk, omega, lines, wave, part);
            else if (g.vec == 2)
                batch_sweep_item<2, BF16, FLAGS>(g, item, chunk, omega, lines, wave, part);
            else
                batch_sweep_item<4, BF16, FLAGS>(g, item, chunk, omega, lines, wave, part);
        } else {
            batch_sweep_item<VEC, BF16, FLAGS>(g, item, chunk, omega, lines, wave, part);
        }
    }
}

// ---------------------------------------------------------------- residual

struct Acc {
    double d;     // FP64 running sum
    float s, c;   // Neumaier-compensated FP32 running sum
};

template <int SUM>
__device__ __forceinline__ void acc_add(Acc &a, float diff) {
    if constexpr (SUM == OFL_SUM_F64) {
        const double x = static_cast<double>(diff);
        a.d = fma(x, x, a.d);
    } else {
        const float y = diff * diff;
        const float t = a.s + y;
        if (fabsf(a.s) >= fabsf(y))
            a.c += (a.s - t) + y;
        else
            a.c += (y - t) + a.s;
        a.s = t;
    }
}

template <int SUM>
__device__ __forceinline__ double acc_value(const Acc &a) {
    if constexpr (SUM == OFL_SUM_F64)
        return a.d;
    else
        return static_cast<double>(a.s) + static_cast<double>(a.c);
}

// Row tile rt of a grid -> offset of this lane's load, clamped to the row's
// last vector like the sweep's loads (whole_rows: to the padded row's last
// vector). i0 receives the i of the lane's first point and ok whether its row
// is an interior one. Packed rows (g.nseg > 0): tile rt is segment rt % nseg of
// plane 1 + rt / nseg, the same segments the batched sweep uses.
template <int VEC>
__device__ __forceinline__ long long row_tile_offset(const GridView &g, int rt, int nti, int lane, int &i0,
                                                     bool &ok, bool whole_rows = false) {
    if (g.nseg > 0) {
        const int seg = rt % g.nseg;
        const int k = 1 + rt / g.nseg;
        const int f = packed_seg0(g.pitch) + seg * kWave * VEC + lane * VEC;
        const int jr = f / g.pitch;
        i0 = f - jr * g.pitch;
        ok = jr >= 1 && jr <= g.J - 2;
        return k * g.plane + min(f, (g.J - 1) * g.pitch - VEC);
    }
    ok = true;
    int &ib = i0;
    const int it = rt % nti;
    const int row = rt / nti;
    const int jj = g.J - 2;
    const int j = 1 + row % jj;
    const int k = 1 + row / jj;
    ib = it * kWave * VEC + lane * VEC;
    const int il = min(ib, whole_rows ? g.pitch - VEC : ((g.I - 1) / VEC) * VEC);
    return j * static_cast<long long>(g.pitch) + k * g.plane + il;
}

// Sum of squared differences over row tiles [first, first + count) for one
// wave. The unrolled loads are unconditional (past-the-end slots reload the
// last row tile and are not counted), so all of them are in flight at once.
template <int VEC, int SUM, bool NT>
__device__ __forceinline__ void residual_rows(const GridView &g, int first, int count, Acc &acc) {
    const int lane = threadIdx.x & (kWave - 1);
    const int nti = itiles(g.I, VEC);
    const int I = g.I;
    const int last = first + count - 1;
    for (int r0 = first; r0 <= last; r0 += kRowUnroll) {
        float pv[kRowUnroll][VEC], wv[kRowUnroll][VEC];
        int ib[kRowUnroll];
        bool ok[kRowUnroll];
#pragma unroll
        for (int u = 0; u < kRowUnroll; ++u) {
            const long long off = row_tile_offset<VEC>(g, min(r0 + u, last), nti, lane, ib[u], ok[u]);
            load_f32<VEC, NT>(g.p + off, pv[u]);
            load_f32<VEC, NT>(g.wrk2 + off, wv[u]);
        }
#pragma unroll
        for (int u = 0; u < kRowUnroll; ++u)
            if (r0 + u <= last) {
#pragma unroll
                for (int e = 0; e < VEC; ++e)
                    if (ok[u] && ib[u] + e >= 1 && ib[u] + e <= I - 2)
                        acc_add<SUM>(acc, wv[u][e] - pv[u][e]);
            }
    }
}

// Block sum in a fixed order (wave butterflies, then waves in index order).
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double part[kResidualThreads / kWave];
#pragma unroll
    for (int m = kWave / 2; m >= 1; m >>= 1)
        v += __shfl_xor(v, m, kWave);
    const int wave = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0)
        part[wave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kResidualThreads / kWave; ++w)
            t += part[w];
    return t;
}

template <int VEC, int SUM, bool NT>
__global__ __launch_bounds__(kResidualThreads) void residual_kernel(GridView g, int rows_per_wave, int nrt) {
    const int wave = blockIdx.x * (kResidualThreads / kWave) + static_cast<int>(threadIdx.x / kWave);
    const int first = wave * rows_per_wave;
    const int count = max(0, min(rows_per_wave, nrt - first));
    Acc acc = {0.0, 0.f, 0.f};
    residual_rows<VEC, SUM, NT>(g, first, count, acc);
    const double t = block_sum(acc_value<SUM>(acc));
    if (threadIdx.x == 0)
        g.partials[blockIdx.x] = t;
}

template <int VEC, int SUM, bool NT>
__global__ __launch_bounds__(kResidualThreads) void batch_residual_kernel(const GridView *__restrict__ views,
                                                                          const RowItem *__restrict__ items,
                                                                          int nitems) {
    const int wave = static_cast<int>(threadIdx.x / kWave);
    constexpr int kWaves = kResidualThreads / kWave;
    for (int w = xcd_remap(blockIdx.x, gridDim.x); w < nitems; w += gridDim.x) {
        const RowItem item = items[w];
        const GridView g = views[item.grid];
        const int per = (item.count + kWaves - 1) / kWaves;
        const int first = item.first + wave * per;
        const int count = max(0, min(per, item.first + item.count - first));
        Acc acc = {0.0, 0.f, 0.f};
        if constexpr (VEC == 0) {
            // the grid's own width (uniform over the work-group)
            if (g.vec == 1)
                residual_rows<1, SUM, NT>(g, first, count, acc);
            else if (g.vec == 2)
                residual_rows<2, SUM, NT>(g, first, count, acc);
            else
                residual_rows<4, SUM, NT>(g, first, count, acc);
        } else {
            residual_rows<VEC, SUM, NT>(g, first, count, acc);
        }
        const double t = block_sum(acc_value<SUM>(acc));
        if (threadIdx.x == 0)
            views[item.grid].partials[item.partial] = t;
        __syncthreads();  // block_sum's shared slots are reused by the next item
    }
}

// Fixed-order sum of n partials: thread t adds t, t+256, ... in order, then a
// fixed tree. gosa = total / omega^2, in FP64.
__device__ __forceinline__ void finalize_sum(const double *partials, int n, double omega, double *gosa) {
    __shared__ double s[kResidualThreads];
    double v = 0.0;
    for (int t = threadIdx.x; t < n; t += kResidualThreads)
        v += partials[t];
    s[threadIdx.x] = v;
    __syncthreads();
    for (int h = kResidualThreads / 2; h >= 1; h >>= 1) {
        if (static_cast<int>(threadIdx.x) < h)
            s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        *gosa = s[0] / (omega * omega);
}

__global__ __launch_bounds__(kResidualThreads) void finalize_kernel(const double *partials, int n, double omega,
                                                                    double *gosa) {
    finalize_sum(partials, n, omega, gosa);
}

// First stage of a two-stage fixed-order sum: block b adds partials
// [b*chunk, (b+1)*chunk) into out[b] (thread strides, then a fixed tree).
__global__ __launch_bounds__(kResidualThreads) void reduce_stage_kernel(const double *partials, long long n,
                                                                        long long chunk, double *out) {
    __shared__ double sm[kResidualThreads];
    const long long lo = blockIdx.x * chunk;
    const long long hi = min(n, lo + chunk);
    double v = 0.0;
    for (long long t = lo + threadIdx.x; t < hi; t += kResidualThreads)
        v += partials[t];
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int h = kResidualThreads / 2; h >= 1; h >>= 1) {
        if (static_cast<int>(threadIdx.x) < h)
            sm[threadIdx.x] += sm[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        out[blockIdx.x] = sm[0];
}

__global__ __launch_bounds__(kResidualThreads) void batch_finalize_kernel(const GridView *__restrict__ views,
                                                                          const int *__restrict__ range,
                                                                          double omega) {
    const GridView g = views[blockIdx.x];
    // g.partials already points at this grid's first partial; range gives counts.
    finalize_sum(g.partials, range[blockIdx.x + 1] - range[blockIdx.x], omega, g.gosa);
}

// The fused residual's last sum, after the last iteration's sweep: the same
// fixed-order group sum, with the same work-group size, that the next sweep's
// first work-group(s) apply to every earlier iteration, so the gosa a run
// returns is computed by that code too. One grid: one work-group over n
// partials. A batch: work-group b (and b + gridDim.x, ...) sums grid b's
// range parts[range[2b], range[2b+1]).
__global__ __launch_bounds__(512) void fold_finalize_kernel(const double *parts, long long n, double omega,
                                                            double *gosa) {
    const double total = group_sum_fixed(parts, n);
    if (threadIdx.x == 0)
        *gosa = total / (omega * omega);
}

__global__ __launch_bounds__(512) void batch_fold_finalize_kernel(const GridView *__restrict__ views,
                                                                  const double *__restrict__ parts,
                                                                  const long long *__restrict__ range, int ngrids,
                                                                  double omega) {
    for (int b = static_cast<int>(blockIdx.x); b < ngrids; b += gridDim.x) {
        const long long lo = range[2 * b];
        const double total = group_sum_fixed(parts + lo, range[2 * b + 1] - lo);
        if (threadIdx.x == 0)
            *views[b].gosa = total / (omega * omega);
    }
}

// ---------------------------------------------------------------- copy-back

// whole_rows: the device wrk2 equals p outside the interior (boundary columns
// and row padding), so every interior row is copied whole, boundary columns and
// padding included. The result is the same, and every 128-byte line of those
// rows is written in full instead of in part.
// U row tiles per round: every load of a round is in flight before its first
// store.
template <int VEC, bool NTL, bool NTS, int U>
__device__ __forceinline__ void copyback_rows(const GridView &g, int first, int count, bool whole_rows) {
    const int lane = threadIdx.x & (kWave - 1);
    const int nti = itiles(g.I, VEC);
    const int I = g.I;
    const int last = first + count - 1;
    for (int r0 = first; r0 <= last; r0 += U) {
        float wv[U][VEC];
        long long off[U];
        int ib[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            off[u] = row_tile_offset<VEC>(g, min(r0 + u, last), nti, lane, ib[u], ok[u], whole_rows);
            load_f32<VEC, NTL>(g.wrk2 + off[u], wv[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (r0 + u > last)
                continue;
            if (whole_rows) {
                if (ok[u] && ib[u] + VEC <= g.pitch)
                    store_f32<VEC, NTS>(g.p + off[u], wv[u]);
            } else if (ok[u] && ib[u] >= 1 && ib[u] + VEC - 1 <= I - 2) {
                store_f32<VEC, NTS>(g.p + off[u], wv[u]);
            } else {
#pragma unroll
                for (int e = 0; e < VEC; ++e)
                    if (ok[u] && ib[u] + e >= 1 && ib[u] + e <= I - 2)
                        g.p[off[u] + e] = wv[u][e];
            }
        }
    }
}

// fin_n > 0: the residual nest ran just before as its own kernel and left
// fin_n block partials; block 0 first turns them into gosa (the finalize step,
// with the same fixed order), so that step needs no launch of its own.
template <int VEC, bool NTL, bool NTS, int U>
__global__ __launch_bounds__(kResidualThreads) void copyback_kernel(GridView g, int rows_per_wave, int nrt,
                                                                    int whole_rows, int fin_n, double omega) {
    if (fin_n > 0 && blockIdx.x == 0)
        finalize_sum(g.partials, fin_n, omega, g.gosa);
    const int wave = blockIdx.x * (kResidualThreads / kWave) + static_cast<int>(threadIdx.x / kWave);
    const int first = wave * rows_per_wave;
    const int count = max(0, min(rows_per_wave, nrt - first));
    copyback_rows<VEC, NTL, NTS, U>(g, first, count, whole_rows != 0);
}

template <int VEC, bool NTL, bool NTS>
__global__ __launch_bounds__(kResidualThreads) void batch_copyback_kernel(const GridView *__restrict__ views,
                                                                          const RowItem *__restrict__ items,
                                                                          int nitems, int whole_rows) {
    const int wave = static_cast<int>(threadIdx.x / kWave);
    constexpr int kWaves = kResidualThreads / kWave;
    for (int w = xcd_remap(blockIdx.x, gridDim.x); w < nitems; w += gridDim.x) {
        const RowItem item = items[w];
        const GridView g = views[item.grid];
        const int per = (item.count + kWaves - 1) / kWaves;
        const int first = item.first + wave * per;
        const int count = max(0, min(per, item.first + item.count - first));
        if constexpr (VEC == 0) {
            if (g.vec == 1)
                copyback_rows<1, NTL, NTS, kCopyUnroll>(g, first, count, whole_rows != 0);
            else if (g.vec == 2)
                copyback_rows<2, NTL, NTS, kCopyUnroll>(g, first, count, whole_rows != 0);
            else
                copyback_rows<4, NTL, NTS, kCopyUnroll>(g, first, count, whole_rows != 0);
        } else {
            copyback_rows<VEC, NTL, NTS, kCopyUnroll>(g, first, count, whole_rows != 0);
        }
    }
}

// -------------------------------------------------------- transfer helpers

// Contiguous host-order staging buffer <-> pitched device array. Host row
// `row` is row row % J of plane row / J.
__device__ __forceinline__ long long pitched_at(long long t, int I, int J, int pitch, long long plane) {
    const long long row = t / I;
    const int i = static_cast<int>(t - row * I);
    const long long k = row / J;
    const int j = static_cast<int>(row - k * J);
    return k * plane + static_cast<long long>(j) * pitch + i;
}

template <typename T>
__global__ void pack_kernel(const T *__restrict__ src, T *__restrict__ dst, int I, int J, long long n, int keep,
                            int pitch, long long plane) {
    for (long long t = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; t < n;
         t += static_cast<long long>(gridDim.x) * blockDim.x) {
        const long long row = t / I;
        const int i = static_cast<int>(t - row * I);
        if (i < keep) {
            const long long k = row / J;
            const int j = static_cast<int>(row - k * J);
            dst[k * plane + static_cast<long long>(j) * pitch + i] = src[t];
        }
    }
}

template <typename T>
__global__ void unpack_kernel(const T *__restrict__ src, T *__restrict__ dst, int I, int J, long long n, int pitch,
                              long long plane) {
    for (long long t = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; t < n;
         t += static_cast<long long>(gridDim.x) * blockDim.x)
        dst[t] = src[pitched_at(t, I, J, pitch, plane)];
}

__global__ void fill_zero_kernel(unsigned *__restrict__ dst, long long n) {
    for (long long t = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; t < n;
         t += static_cast<long long>(gridDim.x) * blockDim.x)
        dst[t] = 0u;
}

// Streaming copy, 16 bytes per lane, four independent loads in flight.
__global__ __launch_bounds__(256) void copy_kernel(const u4 *__restrict__ src, u4 *__restrict__ dst, long long n) {
    const long long stride = static_cast<long long>(gridDim.x) * blockDim.x;
    long long t = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x;
    for (; t + 3 * stride < n; t += 4 * stride) {
        const u4 a = __builtin_nontemporal_load(src + t);
        const u4 b = __builtin_nontemporal_load(src + t + stride);
        const u4 c = __builtin_nontemporal_load(src + t + 2 * stride);
        const u4 d = __builtin_nontemporal_load(src + t + 3 * stride);
        __builtin_nontemporal_store(a, dst + t);
        __builtin_nontemporal_store(b, dst + t + stride);
        __builtin_nontemporal_store(c, dst + t + 2 * stride);
        __builtin_nontemporal_store(d, dst + t + 3 * stride);
    }
    for (; t < n; t += stride)
        dst[t] = src[t];
}

// The sweep's access pattern without the stencil: every lane reads 4
// consecutive elements of each of N32 FP32 streams and N16 bfloat16 streams
// (non-temporal, linear order) and writes their sum to one FP32 stream. With
// (13, 0) that is the FP32 sweep's 13 reads and 1 write per point, with
// (1, 12) the bfloat16 sweep's; the rate it reaches is the practical HBM
// ceiling of that pattern. One vector per lane and many work-groups, as in the
// sweep.
struct StreamArgs {
    const float *f[16];
    const uint16_t *h[16];
    float *dst;
};

template <int N32, int N16>
__global__ __launch_bounds__(256) void stream_kernel(StreamArgs a, long long nvec) {
    const long long v = blockIdx.x * 256LL + threadIdx.x;
    if (v >= nvec)
        return;
    f4 x[N32];
    u2 h[N16 > 0 ? N16 : 1];
#pragma unroll
    for (int s = 0; s < N32; ++s)
        x[s] = __builtin_nontemporal_load(reinterpret_cast<const f4 *>(a.f[s]) + v);
#pragma unroll
    for (int s = 0; s < N16; ++s)
        h[s] = __builtin_nontemporal_load(reinterpret_cast<const u2 *>(a.h[s]) + v);
    f4 acc = x[0];
#pragma unroll
    for (int s = 1; s < N32; ++s)
        acc += x[s];
#pragma unroll
    for (int s = 0; s < N16; ++s) {
        acc.x += bf16_lo(h[s].x);
        acc.y += bf16_hi(h[s].x);
        acc.z += bf16_lo(h[s].y);
        acc.w += bf16_hi(h[s].y);
    }
    __builtin_nontemporal_store(acc, reinterpret_cast<f4 *>(a.dst) + v);
}

int grid_for(long long n, int threads, int cap) {
    long long b = (n + threads - 1) / threads;
    if (b < 1)
        b = 1;
    if (b > cap)
        b = cap;
    return static_cast<int>(b);
}

void check_launch(const char *what) { hip_check(hipGetLastError(), what); }

}  // namespace

// ------------------------------------------------------------------ launchers

namespace {

// Launcher tables over (vec, format, flags): one instantiation per combination.
using SweepLaunch = void (*)(const GridView &, const TileCfg &, float, int, int, int, double *, const PrevParts &,
                             hipStream_t);
using BatchSweepLaunch = void (*)(const GridView *, const SweepItem *, int, const TileCfg &, float, int, double *,
                                  const PrevParts &, hipStream_t);

// Dynamic LDS per work-group that lets at most `occ` work-groups of this
// sweep instantiation reside on a CU at once (tile.occupancy of a single
// grid; 0: no reservation). The kernel uses none of it: the reservation only
// bounds residency. The smallest size that does so is found through the
// runtime's own occupancy calculator (which knows the allocation granularity
// and the kernel's static LDS and registers), once per rows and occ; every
// device the library runs on is a gfx950 with the same LDS per CU.
template <int VEC, bool BF16, int FLAGS>
size_t sweep_occupancy_lds(int rows, int occ) {
    if (occ <= 0)
        return 0;
    static std::atomic<long long> memo[9][17];  // bytes + 1; 0: not yet known
    const long long known = memo[rows][occ].load(std::memory_order_relaxed);
    if (known > 0)
        return static_cast<size_t>(known - 1);
    int dev = 0, lds_cu = 0, lds_block = 0;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    hip_check(hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev),
              "hipDeviceGetAttribute(LDS per CU)");
    hip_check(hipDeviceGetAttribute(&lds_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev),
              "hipDeviceGetAttribute(LDS per work-group)");
    constexpr size_t kStep = 256;
    size_t bytes = (static_cast<size_t>(lds_cu) / static_cast<size_t>(occ + 1) / kStep + 1) * kStep;
    for (;; bytes += kStep) {
        if (bytes > static_cast<size_t>(lds_block))
            fail(OFL_EINVAL, "tile.occupancy " + std::to_string(occ) +
                                 ": the device cannot hold the LDS reservation that bounds a CU to that many "
                                 "work-groups");
        int resident = 0;
        hip_check(hipOccupancyMaxActiveBlocksPerMultiprocessor(&resident, sweep_kernel<VEC, BF16, FLAGS>, kWave * rows,
                                                               bytes),
                  "hipOccupancyMaxActiveBlocksPerMultiprocessor(sweep)");
        if (resident <= occ)
            break;
    }
    memo[rows][occ].store(static_cast<long long>(bytes) + 1, std::memory_order_relaxed);
    return bytes;
}

template <int VEC, bool BF16, int FLAGS>
void sweep_one(const GridView &g, const TileCfg &t, float omega, int nti, int nfb, int blocks, double *parts,
               const PrevParts &prev, hipStream_t s) {
    // bands need whole k-chunks of a multiple of 8 tiles (blocks = nti*nfb*nmc)
    const int order = (t.flags & OFL_TILE_XCD_REMAP) ? kOrderRemap
                      : ((nti * nfb) % kXcds == 0) ? kOrderBand
                                                   : kOrderPlain;
    const size_t lds = sweep_occupancy_lds<VEC, BF16, FLAGS>(t.rows, t.occupancy);
    sweep_kernel<VEC, BF16, FLAGS><<<blocks, kWave * t.rows, lds, s>>>(g, t.kchunk, nti, nfb, omega, order, parts,
                                                                         prev);
}

template <int VEC, bool BF16, int FLAGS>
void batch_sweep_one(const GridView *views, const SweepItem *items, int nitems, const TileCfg &t, float omega,
                     int blocks, double *parts, const PrevParts &prev, hipStream_t s) {
    batch_sweep_kernel<VEC, BF16, FLAGS><<<blocks, kWave * t.rows, 0, s>>>(
        views, items, nitems, t.kchunk, omega, (t.flags & OFL_TILE_XCD_REMAP) ? 1 : 0, parts, prev);
}

template <int VEC, bool BF16, int... F>
constexpr std::array<SweepLaunch, sizeof...(F)> sweep_row(std::integer_sequence<int, F...>) {
    return {&sweep_one<VEC, BF16, F>...};
}

template <int VEC, bool BF16, int... F>
constexpr std::array<BatchSweepLaunch, sizeof...(F)> batch_sweep_row(std::integer_sequence<int, F...>) {
    return {&batch_sweep_one<VEC, BF16, F>...};
}

constexpr int kSweepCombos = 32;  // the template flag bits plus the fused-residual bit
using SweepFlagSeq = std::make_integer_sequence<int, kSweepCombos>;
static_assert((kTemplateFlagMask | kFlagFuseResidual) < kSweepCombos, "sweep launcher table too small");

int vec_index(int vec) { return vec == 1 ? 0 : (vec == 2 ? 1 : 2); }

// 8 points per lane: k-march only, so the flag combinations without
// OFL_TILE_MARCH_J (the host refuses such tiles before any launch).
template <bool BF16, int F>
constexpr SweepLaunch sweep_one_vec8() {
    if constexpr ((F & OFL_TILE_MARCH_J) != 0)
        return nullptr;
    else
        return &sweep_one<8, BF16, F>;
}

template <bool BF16, int... F>
constexpr std::array<SweepLaunch, sizeof...(F)> sweep_row_vec8(std::integer_sequence<int, F...>) {
    return {sweep_one_vec8<BF16, F>()...};
}

SweepLaunch sweep_launcher(int vec, bool bf16, int flags) {
    static const std::array<SweepLaunch, kSweepCombos> table[2][4] = {
        {sweep_row<1, false>(SweepFlagSeq{}), sweep_row<2, false>(SweepFlagSeq{}),
         sweep_row<4, false>(SweepFlagSeq{}), sweep_row_vec8<false>(SweepFlagSeq{})},
        {sweep_row<1, true>(SweepFlagSeq{}), sweep_row<2, true>(SweepFlagSeq{}), sweep_row<4, true>(SweepFlagSeq{}),
         sweep_row_vec8<true>(SweepFlagSeq{})}};
    const SweepLaunch f = table[bf16 ? 1 : 0][vec == 8 ? 3 : vec_index(vec)][flags & (kSweepCombos - 1)];
    if (!f)
        fail(OFL_ENOTSUP, "8 points per lane march along k only (no OFL_TILE_MARCH_J)");
    return f;
}

// vec 0: each item at its grid's own width
BatchSweepLaunch batch_sweep_launcher(int vec, bool bf16, int flags) {
    if (vec != 0 && vec != 1 && vec != 2 && vec != 4)
        fail(OFL_ENOTSUP, "batched sweeps run 1, 2 or 4 points per lane");
    static const std::array<BatchSweepLaunch, kSweepCombos> table[2][4] = {
        {batch_sweep_row<1, false>(SweepFlagSeq{}), batch_sweep_row<2, false>(SweepFlagSeq{}),
         batch_sweep_row<4, false>(SweepFlagSeq{}), batch_sweep_row<0, false>(SweepFlagSeq{})},
        {batch_sweep_row<1, true>(SweepFlagSeq{}), batch_sweep_row<2, true>(SweepFlagSeq{}),
         batch_sweep_row<4, true>(SweepFlagSeq{}), batch_sweep_row<0, true>(SweepFlagSeq{})}};
    return table[bf16 ? 1 : 0][vec == 0 ? 3 : vec_index(vec)][flags & (kSweepCombos - 1)];
}

}  // namespace

void launch_sweep(const GridView &g, const TileCfg &t, int bf16, float omega, hipStream_t s, double *fused_parts,
                  const PrevParts &prev) {
    int nti, nfb, nmc;
    sweep_shape(g.I, g.J, g.K, t, &nti, &nfb, &nmc);
    const long long blocks = static_cast<long long>(nti) * nfb * nmc;
    if (blocks > 0x7fffffffLL)
        fail(OFL_EINVAL, "sweep launch too large for this tile");
    const int flags = (t.flags & kTemplateFlagMask) | (fused_parts ? kFlagFuseResidual : 0);
    if (prev.parts && !fused_parts)
        fail(OFL_EINVAL, "a folded residual reduction needs the fused sweep");
    sweep_launcher(t.vec, bf16 != 0, flags)(g, t, omega, nti, nfb, static_cast<int>(blocks), fused_parts, prev, s);
    check_launch("sweep kernel launch");
}

void launch_finalize(const double *partials, long long n, float omega, double *gosa, hipStream_t s,
                     double *scratch, int scratch_len) {
    constexpr long long kStageChunk = 4 * kResidualThreads;
    if (n > kStageChunk && scratch && scratch_len > 0) {
        const long long blocks = std::min<long long>(scratch_len, (n + kStageChunk - 1) / kStageChunk);
        const long long chunk = (n + blocks - 1) / blocks;
        reduce_stage_kernel<<<static_cast<int>(blocks), kResidualThreads, 0, s>>>(partials, n, chunk, scratch);
        check_launch("residual reduce-stage launch");
        finalize_kernel<<<1, kResidualThreads, 0, s>>>(scratch, static_cast<int>(blocks), static_cast<double>(omega),
                                                       gosa);
    } else {
        finalize_kernel<<<1, kResidualThreads, 0, s>>>(partials, static_cast<int>(n), static_cast<double>(omega), gosa);
    }
    check_launch("residual finalize launch");
}

void launch_batch_sweep(const GridView *views, const SweepItem *items, int nitems, const TileCfg &t, int bf16,
                        float omega, int grid_blocks, hipStream_t s, double *fused_parts, const PrevParts &prev) {
    const int flags = (t.flags & kTemplateFlagMask) | (fused_parts ? kFlagFuseResidual : 0);
    if (prev.parts && !fused_parts)
        fail(OFL_EINVAL, "a folded residual reduction needs the fused sweep");
    batch_sweep_launcher(t.vec, bf16 != 0, flags)(views, items, nitems, t, omega, grid_blocks, fused_parts, prev,
                                                  s);
    check_launch("batched sweep kernel launch");
}

void launch_fold_finalize(const double *parts, long long n, float omega, double *gosa, int threads, hipStream_t s) {
    if (threads < kWave || threads > 512 || threads % kWave != 0)
        fail(OFL_EINVAL, "fused residual sum: work-group size must be 64..512 threads in whole waves");
    fold_finalize_kernel<<<1, threads, 0, s>>>(parts, n, static_cast<double>(omega), gosa);
    check_launch("fused residual sum launch");
}

void launch_batch_fold_finalize(const GridView *views, const double *parts, const long long *range, int ngrids,
                                float omega, int threads, hipStream_t s) {
    if (threads < kWave || threads > 512 || threads % kWave != 0)
        fail(OFL_EINVAL, "fused residual sum: work-group size must be 64..512 threads in whole waves");
    if (ngrids < 1)
        return;
    batch_fold_finalize_kernel<<<ngrids, threads, 0, s>>>(views, parts, range, ngrids, static_cast<double>(omega));
    check_launch("batched fused residual sum launch");
}

static int rows_per_wave(int nrt, int blocks) {
    const long long waves = static_cast<long long>(blocks) * (kResidualThreads / kWave);
    const long long per = (nrt + waves - 1) / waves;
    return static_cast<int>(per < 1 ? 1 : per);
}

namespace {

// Dispatch helpers for the residual and copy-back kernels: vec, sum mode and
// the non-temporal choices are template parameters.
template <template <int, int, bool> class K, class... A>
void by_vec_sum_nt(int vec, int sum_mode, bool nt, A &&...a) {
    auto go = [&](auto v, auto sm, auto n) { K<decltype(v)::value, decltype(sm)::value, decltype(n)::value>::run(a...); };
    using F64 = std::integral_constant<int, OFL_SUM_F64>;
    using K32 = std::integral_constant<int, OFL_SUM_KAHAN_F32>;
    auto with_nt = [&](auto v, auto sm) {
        if (nt)
            go(v, sm, std::true_type{});
        else
            go(v, sm, std::false_type{});
    };
    auto with_sum = [&](auto v) {
        if (sum_mode == OFL_SUM_F64)
            with_nt(v, F64{});
        else
            with_nt(v, K32{});
    };
    if (vec == 1)
        with_sum(std::integral_constant<int, 1>{});
    else if (vec == 2)
        with_sum(std::integral_constant<int, 2>{});
    else if (vec == 4)
        with_sum(std::integral_constant<int, 4>{});
    else
        with_sum(std::integral_constant<int, 0>{});  // batches: each item at its grid's width
}

template <int VEC, int SUM, bool NT>
struct ResidualLaunch {
    static void run(dim3 grid, dim3 block, hipStream_t s, const GridView &g, int rpw, int nrt) {
        if constexpr (VEC == 0)
            fail(OFL_EINVAL, "a single grid's residual runs 1, 2 or 4 points per lane");
        else
            residual_kernel<VEC, SUM, NT><<<grid, block, 0, s>>>(g, rpw, nrt);
    }
};

template <int VEC, int SUM, bool NT>
struct BatchResidualLaunch {
    static void run(dim3 grid, dim3 block, hipStream_t s, const GridView *views, const RowItem *items, int n) {
        batch_residual_kernel<VEC, SUM, NT><<<grid, block, 0, s>>>(views, items, n);
    }
};

// copy-back: the "sum mode" slot carries the non-temporal store choice
template <int VEC, int NTS, bool NTL>
struct CopybackLaunch {
    static void run(dim3 grid, dim3 block, hipStream_t s, const GridView &g, int rpw, int nrt, int whole_rows,
                    int fin_n, double omega, bool wide) {
        if constexpr (VEC == 0)
            fail(OFL_EINVAL, "a single grid's copy-back runs 1, 2 or 4 points per lane");
        else if (wide)
            copyback_kernel<VEC, NTL, NTS != 0, kCopyUnroll>
                <<<grid, block, 0, s>>>(g, rpw, nrt, whole_rows, fin_n, omega);
        else
            copyback_kernel<VEC, NTL, NTS != 0, kRowUnroll>
                <<<grid, block, 0, s>>>(g, rpw, nrt, whole_rows, fin_n, omega);
    }
};

template <int VEC, int NTS, bool NTL>
struct BatchCopybackLaunch {
    static void run(dim3 grid, dim3 block, hipStream_t s, const GridView *views, const RowItem *items, int n,
                    int whole_rows) {
        batch_copyback_kernel<VEC, NTL, NTS != 0><<<grid, block, 0, s>>>(views, items, n, whole_rows);
    }
};

}  // namespace

void launch_residual(const GridView &g, int vec, int sum_mode, int flags, float omega, hipStream_t s, bool finalize) {
    vec = std::min(vec, 4);  // p and wrk2 are FP32: 16 bytes per lane at 4 points
    const int nrt = itiles(g.I, vec) * (g.J - 2) * (g.K - 2);
    const int rpw = rows_per_wave(nrt, kResidualBlocks);
    // Ordinary loads: p and wrk2 then stay in the caches for the copy-back that
    // follows (measured 43.2 -> 41.3 us for it at 257x257x513, the residual
    // itself unchanged); OFL_TILE_NT_LOADS concerns the sweep's coefficients.
    (void)flags;
    by_vec_sum_nt<ResidualLaunch>(vec, sum_mode, false, dim3(kResidualBlocks), dim3(kResidualThreads), s, g, rpw,
                                  nrt);
    check_launch("residual kernel launch");
    if (!finalize)
        return;
    finalize_kernel<<<1, kResidualThreads, 0, s>>>(g.partials, kResidualBlocks, static_cast<double>(omega), g.gosa);
    check_launch("residual finalize launch");
}

void launch_copyback(const GridView &g, int vec, int flags, hipStream_t s, bool whole_rows, bool finalize_residual,
                     float omega) {
    vec = std::min(vec, 4);  // p and wrk2 are FP32: 16 bytes per lane at 4 points
    const int nrt = itiles(g.I, vec) * (g.J - 2) * (g.K - 2);
    // A launch with enough row tiles gives each wave one round of 16, all
    // loads in flight before the first store. Per launch at 257x257x513:
    // 39.5-39.6 us, against 42.6 with two rounds of 4, 40.6 with two of 8,
    // 43.4 with two of 16, 39.7 with one of 32 (which slows the batches); the
    // 64-grid batches gain 0.3-1.7%. Below 4096 such waves (16 per CU) the
    // rounds would leave CUs idle, so smaller launches (a grid of 129 x 129 x
    // 257, one plane of a region gene) keep two rounds of 4 per wave. The
    // residual keeps 4 per round: 40.7 us, 41.5 with 8.
    constexpr int kWavesPerBlock = kResidualThreads / kWave;
    const bool wide = nrt / kCopyUnroll >= 4096;
    const int per_wave = wide ? kCopyUnroll : 2 * kRowUnroll;
    const int blocks = grid_for(nrt, kWavesPerBlock * per_wave, kResidualBlocks * 4);
    const int rpw = rows_per_wave(nrt, blocks);
    by_vec_sum_nt<CopybackLaunch>(vec, (flags & OFL_TILE_NT_STORES) ? 1 : 0, (flags & OFL_TILE_NT_LOADS) != 0,
                                  dim3(blocks), dim3(kResidualThreads), s, g, rpw, nrt, whole_rows ? 1 : 0,
                                  finalize_residual ? kResidualBlocks : 0, static_cast<double>(omega), wide);
    check_launch("copy-back kernel launch");
}

void launch_batch_residual(const GridView *views, const RowItem *items, int nitems, int vec, int sum_mode, int flags,
                           int grid_blocks, hipStream_t s) {
    // Unlike a single grid, the batch residual keeps the tile's non-temporal
    // loads: with ordinary ones the batch ran 0.6-0.9% slower (64 mixed grids).
    by_vec_sum_nt<BatchResidualLaunch>(vec, sum_mode, (flags & OFL_TILE_NT_LOADS) != 0, dim3(grid_blocks),
                                       dim3(kResidualThreads), s, views, items, nitems);
    check_launch("batched residual kernel launch");
}

void launch_batch_finalize(const GridView *views, const int *partial_range, int ngrids, float omega, hipStream_t s) {
    batch_finalize_kernel<<<ngrids, kResidualThreads, 0, s>>>(views, partial_range, static_cast<double>(omega));
    check_launch("batched finalize launch");
}

void launch_batch_copyback(const GridView *views, const RowItem *items, int nitems, int vec, int flags,
                           int grid_blocks, hipStream_t s, bool whole_rows) {
    by_vec_sum_nt<BatchCopybackLaunch>(vec, (flags & OFL_TILE_NT_STORES) ? 1 : 0, (flags & OFL_TILE_NT_LOADS) != 0,
                                       dim3(grid_blocks), dim3(kResidualThreads), s, views, items, nitems,
                                       whole_rows ? 1 : 0);
    check_launch("batched copy-back kernel launch");
}

void launch_pack(const void *staging, void *arr, int I, int J, int K, int keep, int pitch, long long plane,
                 int elem_bytes, hipStream_t s) {
    const long long n = static_cast<long long>(J) * K * I;
    const int blocks = grid_for(n, 256, 65536);
    if (elem_bytes == 4)
        pack_kernel<float><<<blocks, 256, 0, s>>>(static_cast<const float *>(staging), static_cast<float *>(arr), I, J,
                                                 n, keep, pitch, plane);
    else
        pack_kernel<uint16_t><<<blocks, 256, 0, s>>>(static_cast<const uint16_t *>(staging),
                                                    static_cast<uint16_t *>(arr), I, J, n, keep, pitch, plane);
    check_launch("pack kernel launch");
}

void launch_unpack(const void *arr, void *staging, int I, int J, int K, int pitch, long long plane, int elem_bytes,
                   hipStream_t s) {
    const long long n = static_cast<long long>(J) * K * I;
    const int blocks = grid_for(n, 256, 65536);
    if (elem_bytes == 4)
        unpack_kernel<float><<<blocks, 256, 0, s>>>(static_cast<const float *>(arr), static_cast<float *>(staging), I,
                                                   J, n, pitch, plane);
    else
        unpack_kernel<uint16_t><<<blocks, 256, 0, s>>>(static_cast<const uint16_t *>(arr),
                                                      static_cast<uint16_t *>(staging), I, J, n, pitch, plane);
    check_launch("unpack kernel launch");
}

void launch_fill_zero(void *ptr, size_t bytes, hipStream_t s) {
    const long long n = static_cast<long long>(bytes / 4);
    if (n == 0)
        return;
    fill_zero_kernel<<<grid_for(n, 256, 65536), 256, 0, s>>>(static_cast<unsigned *>(ptr), n);
    check_launch("fill kernel launch");
}

void launch_copy(void *dst, const void *src, size_t bytes, hipStream_t s) {
    const long long n = static_cast<long long>(bytes / 16);
    if (n == 0)
        return;
    copy_kernel<<<grid_for(n, 256, 256 * 256), 256, 0, s>>>(static_cast<const u4 *>(src), static_cast<u4 *>(dst), n);
    check_launch("copy kernel launch");
}

void launch_stream(const float *const *src32, int n32, const uint16_t *const *src16, int n16, float *dst, size_t n,
                   hipStream_t s) {
    StreamArgs a{};
    for (int t = 0; t < n32; ++t)
        a.f[t] = src32[t];
    for (int t = 0; t < n16; ++t)
        a.h[t] = src16[t];
    a.dst = dst;
    const long long nvec = static_cast<long long>(n / 4);
    if (nvec == 0)
        return;
    const long long blocks = (nvec + 255) / 256;
    if (blocks > 0x7fffffffLL)
        fail(OFL_EINVAL, "stream probe too large");
    if (n32 == 13 && n16 == 0)
        stream_kernel<13, 0><<<static_cast<int>(blocks), 256, 0, s>>>(a, nvec);
    else if (n32 == 1 && n16 == 12)
        stream_kernel<1, 12><<<static_cast<int>(blocks), 256, 0, s>>>(a, nvec);
    else
        fail(OFL_ENOTSUP, "stream probe patterns: 13 FP32 sources, or 1 FP32 and 12 bfloat16 sources");
    check_launch("stream kernel launch");
}

// The fused sweep's per-wave residual partials of ofl_jacobi_run_static live
// here instead of in memory the library allocates. Every slot a launch reads is
// written by the same launch's sweep first, so nothing needs clearing between
// calls. In host code the name stands for a host-side shadow, not a device
// address: only the address hipGetSymbolAddress returns for the current device
// may reach a kernel.
static __device__ __align__(256) double scratch[kStaticScratchParts];

double *static_scratch(int device) {
    static std::mutex mu;
    static std::vector<double *> ptrs;
    std::lock_guard<std::mutex> lock(mu);
    if (device < 0)
        fail(OFL_EINVAL, "static scratch: negative device ordinal");
    if (static_cast<size_t>(device) >= ptrs.size())
        ptrs.resize(static_cast<size_t>(device) + 1, nullptr);
    if (!ptrs[device]) {
        void *ptr = nullptr;
        hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(static scratch)");
        if (!ptr)
            fail(OFL_EDEVICE, "hipGetSymbolAddress returned no address for the static scratch");
        ptrs[device] = static_cast<double *>(ptr);
    }
    return ptrs[device];
}

int device_cu_count(int device) {
    hipDeviceProp_t prop;
    hip_check(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties");
    return prop.multiProcessorCount;
}

}  // namespace ofl
