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
//    along the contiguous i axis;
//  * the wave marches through a chunk of k-planes keeping rows j-1, j, j+1 of
//    planes k-1, k, k+1 in registers: each p value comes from memory once per
//    row-march, the k+-1 neighbours never reload;
//  * the i+-1 neighbours come from the adjacent lane through a cross-lane
//    shuffle; only the two wave-edge lanes load one halo value each;
//  * no LDS and no barriers: the j+-1 rows are re-read by the waves of the
//    neighbouring rows and served by L1/L2, and work-groups are remapped so
//    that neighbouring j-blocks run on the same XCD (shared L2);
//  * no MFMA: there is no dense contraction here.

#include "ofl_internal.hpp"

namespace ofl {
namespace {

typedef float f2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned int u2 __attribute__((ext_vector_type(2)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

constexpr int kXcds = 8;

// Work-groups are handed to the 8 XCDs round-robin by id. Renumber them so
// that XCD x receives one contiguous range of logical tiles: neighbouring
// tiles (which share halo rows) then share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int bid, int n) {
    const int xcd = bid % kXcds;
    const int local = bid / kXcds;
    const int per = n / kXcds;
    const int rem = n % kXcds;
    return xcd * per + min(xcd, rem) + local;
}

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
    } else {
        f4 x = ld<NT>(reinterpret_cast<const f4 *>(ptr));
        v[0] = x.x;
        v[1] = x.y;
        v[2] = x.z;
        v[3] = x.w;
    }
}

template <int VEC, bool NT>
__device__ __forceinline__ void store_f32(float *ptr, const float (&v)[VEC]) {
    if constexpr (VEC == 1) {
        st<NT>(ptr, v[0]);
    } else if constexpr (VEC == 2) {
        f2 x = {v[0], v[1]};
        st<NT>(reinterpret_cast<f2 *>(ptr), x);
    } else {
        f4 x = {v[0], v[1], v[2], v[3]};
        st<NT>(reinterpret_cast<f4 *>(ptr), x);
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
    } else {
        u2 x = ld<NT>(reinterpret_cast<const u2 *>(ptr));
        v[0] = bias + bf16_lo(x.x);
        v[1] = bias + bf16_hi(x.x);
        v[2] = bias + bf16_lo(x.y);
        v[3] = bias + bf16_hi(x.y);
    }
}

// One row segment of p: this lane's VEC values plus its outer neighbours
// (left of element 0, right of element VEC-1). Interior lanes take them from
// the adjacent lanes; lanes 0 and 63 load them (the tile's halo). For the
// first tile of a row lane 0 reads the element before the row (row padding or
// the array's front guard): that value only feeds i = 0, which is never stored.
template <int VEC>
__device__ __forceinline__ void load_prow(const float *row, int ib, int ts, int lane, float (&v)[VEC], float &l,
                                          float &r) {
    load_f32<VEC, false>(row + ib, v);
    const float up = __shfl_up(v[VEC - 1], 1, kWave);
    const float dn = __shfl_down(v[0], 1, kWave);
    float h = 0.f;
    if (lane == 0 || lane == kWave - 1)
        h = row[lane == 0 ? ts - 1 : ts + kWave * VEC];
    l = (lane == 0) ? h : up;
    r = (lane == kWave - 1) ? h : dn;
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

// Nest S for one wave: row j, i-points ts + lane*VEC .. +VEC-1, planes k0..k1-1.
template <int VEC, bool BF16, int FLAGS>
__device__ __forceinline__ void sweep_march(const GridView &g, int ts, int j, int k0, int k1, float omega) {
    constexpr bool kNtLoads = (FLAGS & OFL_TILE_NT_LOADS) != 0;
    constexpr bool kNtStores = (FLAGS & OFL_TILE_NT_STORES) != 0;
    constexpr bool kPrefetch = (FLAGS & OFL_TILE_PREFETCH) != 0;
    const int lane = threadIdx.x & (kWave - 1);
    const int ib = ts + lane * VEC;
    const long long pitch = g.pitch;
    const long long plane = g.plane;
    const float *__restrict__ p = g.p;

    // P[r][q][e]: row j-1+r, plane k-1+q, element e. EL/ER: outer neighbours.
    float P[3][3][VEC];
    float EL[3][3], ER[3][3];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int r = 0; r < 3; ++r)
            load_prow<VEC>(p + (j - 1 + r) * pitch + (k0 - 1 + q) * plane, ib, ts, lane, P[r][q], EL[r][q],
                           ER[r][q]);

    float C[kNCoef][VEC];
    if constexpr (kPrefetch)
        load_coefs<VEC, BF16, kNtLoads>(g, j * pitch + k0 * plane + ib, C);

    const int I = g.I;
    float *__restrict__ wrk2 = g.wrk2;
    for (int k = k0; k < k1; ++k) {
        float Cn[kNCoef][VEC];
        if constexpr (kPrefetch) {
            if (k + 1 < k1)
                load_coefs<VEC, BF16, kNtLoads>(g, j * pitch + (k + 1) * plane + ib, Cn);
        } else {
            load_coefs<VEC, BF16, kNtLoads>(g, j * pitch + k * plane + ib, C);
        }
#pragma unroll
        for (int r = 0; r < 3; ++r)
            load_prow<VEC>(p + (j - 1 + r) * pitch + (k + 1) * plane, ib, ts, lane, P[r][2], EL[r][2], ER[r][2]);

        float out[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            // neighbour at i+1 / i-1 of element e in row r, plane q
            auto rt = [&](int r, int q) { return e < VEC - 1 ? P[r][q][e + 1] : ER[r][q]; };
            auto lf = [&](int r, int q) { return e > 0 ? P[r][q][e - 1] : EL[r][q]; };
            const float centre = P[1][1][e];
            float s0 = C[0][e] * rt(1, 1) + C[1][e] * P[2][1][e] + C[2][e] * P[1][2][e];
            s0 += C[4][e] * ((rt(2, 1) - rt(0, 1)) - (lf(2, 1) - lf(0, 1)));
            s0 += C[5][e] * ((P[2][2][e] - P[0][2][e]) - (P[2][0][e] - P[0][0][e]));
            s0 += C[6][e] * ((rt(1, 2) - lf(1, 2)) - (rt(1, 0) - lf(1, 0)));
            s0 += C[7][e] * lf(1, 1) + C[8][e] * P[0][1][e] + C[9][e] * P[1][0][e] + C[11][e];
            const float ss = (C[3][e] * s0 - centre) * C[10][e];
            out[e] = centre + omega * ss;
        }
        float *w = wrk2 + j * pitch + k * plane + ib;
        if (ib >= 1 && ib + VEC - 1 <= I - 2) {
            store_f32<VEC, kNtStores>(w, out);
        } else {
#pragma unroll
            for (int e = 0; e < VEC; ++e)
                if (ib + e >= 1 && ib + e <= I - 2)
                    w[e] = out[e];
        }

#pragma unroll
        for (int r = 0; r < 3; ++r) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                P[r][0][e] = P[r][1][e];
                P[r][1][e] = P[r][2][e];
            }
            EL[r][0] = EL[r][1];
            EL[r][1] = EL[r][2];
            ER[r][0] = ER[r][1];
            ER[r][1] = ER[r][2];
        }
        if constexpr (kPrefetch) {
#pragma unroll
            for (int n = 0; n < kNCoef; ++n)
#pragma unroll
                for (int e = 0; e < VEC; ++e)
                    C[n][e] = Cn[n][e];
        }
    }
}

template <int VEC, bool BF16, int FLAGS>
__global__ __launch_bounds__(512) void sweep_kernel(GridView g, int kchunk, int nti, int njb, float omega) {
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    const int it = L % nti;
    const int rest = L / nti;
    const int jb = rest % njb;
    const int kc = rest / njb;
    const int rows = blockDim.x / kWave;
    const int j = 1 + jb * rows + static_cast<int>(threadIdx.x / kWave);
    if (j > g.J - 2)
        return;
    const int k0 = 1 + kc * kchunk;
    const int k1 = min(k0 + kchunk, g.K - 1);
    sweep_march<VEC, BF16, FLAGS>(g, it * kWave * VEC, j, k0, k1, omega);
}

template <int VEC, bool BF16, int FLAGS>
__global__ __launch_bounds__(512) void batch_sweep_kernel(const GridView *__restrict__ views,
                                                          const SweepItem *__restrict__ items, int nitems,
                                                          int kchunk, float omega) {
    const int rows = blockDim.x / kWave;
    const int wave = static_cast<int>(threadIdx.x / kWave);
    for (int w = xcd_remap(blockIdx.x, gridDim.x); w < nitems; w += gridDim.x) {
        const SweepItem item = items[w];
        const GridView g = views[item.grid];
        const int j = 1 + item.jblock * rows + wave;
        if (j > g.J - 2)
            continue;
        const int k0 = 1 + item.kchunk * kchunk;
        const int k1 = min(k0 + kchunk, g.K - 1);
        sweep_march<VEC, BF16, FLAGS>(g, item.itile * kWave * VEC, j, k0, k1, omega);
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

// Row tile rt of a grid -> offset of this lane's first element; false if the
// tile index is past the end.
template <int VEC>
__device__ __forceinline__ long long row_tile_offset(const GridView &g, int rt, int nti, int lane, int &ib) {
    const int it = rt % nti;
    const int row = rt / nti;
    const int jj = g.J - 2;
    const int j = 1 + row % jj;
    const int k = 1 + row / jj;
    ib = it * kWave * VEC + lane * VEC;
    return j * static_cast<long long>(g.pitch) + k * g.plane + ib;
}

// Sum of squared differences over row tiles [first, first + count) for one wave.
template <int VEC, int SUM>
__device__ __forceinline__ void residual_rows(const GridView &g, int first, int count, Acc &acc) {
    const int lane = threadIdx.x & (kWave - 1);
    const int nti = itiles(g.I, VEC);
    const int I = g.I;
    for (int r0 = first; r0 < first + count; r0 += kRowUnroll) {
        float pv[kRowUnroll][VEC], wv[kRowUnroll][VEC];
        int ib[kRowUnroll];
#pragma unroll
        for (int u = 0; u < kRowUnroll; ++u) {
            ib[u] = 1 << 30;
            if (r0 + u < first + count) {
                const long long off = row_tile_offset<VEC>(g, r0 + u, nti, lane, ib[u]);
                load_f32<VEC, false>(g.p + off, pv[u]);
                load_f32<VEC, false>(g.wrk2 + off, wv[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < kRowUnroll; ++u)
#pragma unroll
            for (int e = 0; e < VEC; ++e)
                if (ib[u] + e >= 1 && ib[u] + e <= I - 2)
                    acc_add<SUM>(acc, wv[u][e] - pv[u][e]);
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

template <int VEC, int SUM>
__global__ __launch_bounds__(kResidualThreads) void residual_kernel(GridView g, int rows_per_wave, int nrt) {
    const int wave = blockIdx.x * (kResidualThreads / kWave) + static_cast<int>(threadIdx.x / kWave);
    const int first = wave * rows_per_wave;
    const int count = max(0, min(rows_per_wave, nrt - first));
    Acc acc = {0.0, 0.f, 0.f};
    residual_rows<VEC, SUM>(g, first, count, acc);
    const double t = block_sum(acc_value<SUM>(acc));
    if (threadIdx.x == 0)
        g.partials[blockIdx.x] = t;
}

template <int VEC, int SUM>
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
        residual_rows<VEC, SUM>(g, first, count, acc);
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

__global__ __launch_bounds__(kResidualThreads) void batch_finalize_kernel(const GridView *__restrict__ views,
                                                                          const int *__restrict__ range,
                                                                          double omega) {
    const GridView g = views[blockIdx.x];
    // g.partials already points at this grid's first partial; range gives counts.
    finalize_sum(g.partials, range[blockIdx.x + 1] - range[blockIdx.x], omega, g.gosa);
}

// ---------------------------------------------------------------- copy-back

template <int VEC>
__device__ __forceinline__ void copyback_rows(const GridView &g, int first, int count) {
    const int lane = threadIdx.x & (kWave - 1);
    const int nti = itiles(g.I, VEC);
    const int I = g.I;
    for (int r0 = first; r0 < first + count; r0 += kRowUnroll) {
        float wv[kRowUnroll][VEC];
        long long off[kRowUnroll];
        int ib[kRowUnroll];
#pragma unroll
        for (int u = 0; u < kRowUnroll; ++u) {
            ib[u] = 1 << 30;
            off[u] = 0;
            if (r0 + u < first + count) {
                off[u] = row_tile_offset<VEC>(g, r0 + u, nti, lane, ib[u]);
                load_f32<VEC, false>(g.wrk2 + off[u], wv[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < kRowUnroll; ++u) {
            if (ib[u] >= 1 && ib[u] + VEC - 1 <= I - 2) {
                store_f32<VEC, false>(g.p + off[u], wv[u]);
            } else {
#pragma unroll
                for (int e = 0; e < VEC; ++e)
                    if (ib[u] + e >= 1 && ib[u] + e <= I - 2)
                        g.p[off[u] + e] = wv[u][e];
            }
        }
    }
}

template <int VEC>
__global__ __launch_bounds__(kResidualThreads) void copyback_kernel(GridView g, int rows_per_wave, int nrt) {
    const int wave = blockIdx.x * (kResidualThreads / kWave) + static_cast<int>(threadIdx.x / kWave);
    const int first = wave * rows_per_wave;
    const int count = max(0, min(rows_per_wave, nrt - first));
    copyback_rows<VEC>(g, first, count);
}

template <int VEC>
__global__ __launch_bounds__(kResidualThreads) void batch_copyback_kernel(const GridView *__restrict__ views,
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
        copyback_rows<VEC>(g, first, count);
    }
}

// -------------------------------------------------------- transfer helpers

// Contiguous host-order staging buffer <-> pitched device array.
template <typename T>
__global__ void pack_kernel(const T *__restrict__ src, T *__restrict__ dst, int I, long long rows, int pitch) {
    const long long n = rows * I;
    for (long long t = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; t < n;
         t += static_cast<long long>(gridDim.x) * blockDim.x) {
        const long long row = t / I;
        const int i = static_cast<int>(t - row * I);
        dst[row * pitch + i] = src[t];
    }
}

template <typename T>
__global__ void unpack_kernel(const T *__restrict__ src, T *__restrict__ dst, int I, long long rows, int pitch) {
    const long long n = rows * I;
    for (long long t = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; t < n;
         t += static_cast<long long>(gridDim.x) * blockDim.x) {
        const long long row = t / I;
        const int i = static_cast<int>(t - row * I);
        dst[t] = src[row * pitch + i];
    }
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

#define OFL_SWEEP_FLAGS(VEC, BF, KERNEL, ...)                                                   \
    switch (t.flags & 7) {                                                                      \
    case 0: KERNEL<VEC, BF, 0><<<__VA_ARGS__>>>(ARGS); break;                                   \
    case 1: KERNEL<VEC, BF, 1><<<__VA_ARGS__>>>(ARGS); break;                                   \
    case 2: KERNEL<VEC, BF, 2><<<__VA_ARGS__>>>(ARGS); break;                                   \
    case 3: KERNEL<VEC, BF, 3><<<__VA_ARGS__>>>(ARGS); break;                                   \
    case 4: KERNEL<VEC, BF, 4><<<__VA_ARGS__>>>(ARGS); break;                                   \
    case 5: KERNEL<VEC, BF, 5><<<__VA_ARGS__>>>(ARGS); break;                                   \
    case 6: KERNEL<VEC, BF, 6><<<__VA_ARGS__>>>(ARGS); break;                                   \
    default: KERNEL<VEC, BF, 7><<<__VA_ARGS__>>>(ARGS); break;                                  \
    }

#define OFL_SWEEP_DISPATCH(KERNEL, ...)                                                         \
    if (bf16) {                                                                                 \
        if (t.vec == 1) { OFL_SWEEP_FLAGS(1, true, KERNEL, __VA_ARGS__) }                       \
        else if (t.vec == 2) { OFL_SWEEP_FLAGS(2, true, KERNEL, __VA_ARGS__) }                  \
        else { OFL_SWEEP_FLAGS(4, true, KERNEL, __VA_ARGS__) }                                  \
    } else {                                                                                    \
        if (t.vec == 1) { OFL_SWEEP_FLAGS(1, false, KERNEL, __VA_ARGS__) }                      \
        else if (t.vec == 2) { OFL_SWEEP_FLAGS(2, false, KERNEL, __VA_ARGS__) }                 \
        else { OFL_SWEEP_FLAGS(4, false, KERNEL, __VA_ARGS__) }                                 \
    }

void launch_sweep(const GridView &g, const TileCfg &t, int bf16, float omega, hipStream_t s) {
    const int nti = itiles(g.I, t.vec);
    const int njb = (g.J - 2 + t.rows - 1) / t.rows;
    const int nkc = (g.K - 2 + t.kchunk - 1) / t.kchunk;
    const long long blocks = static_cast<long long>(nti) * njb * nkc;
    if (blocks > 0x7fffffffLL)
        fail(OFL_EINVAL, "sweep launch too large for this tile");
    const dim3 grid(static_cast<unsigned>(blocks));
    const dim3 block(kWave * t.rows);
#define ARGS g, t.kchunk, nti, njb, omega
    OFL_SWEEP_DISPATCH(sweep_kernel, grid, block, 0, s)
#undef ARGS
    check_launch("sweep kernel launch");
}

void launch_batch_sweep(const GridView *views, const SweepItem *items, int nitems, const TileCfg &t, int bf16,
                        float omega, int grid_blocks, hipStream_t s) {
    const dim3 grid(static_cast<unsigned>(grid_blocks));
    const dim3 block(kWave * t.rows);
#define ARGS views, items, nitems, t.kchunk, omega
    OFL_SWEEP_DISPATCH(batch_sweep_kernel, grid, block, 0, s)
#undef ARGS
    check_launch("batched sweep kernel launch");
}

static int rows_per_wave(int nrt, int blocks) {
    const long long waves = static_cast<long long>(blocks) * (kResidualThreads / kWave);
    const long long per = (nrt + waves - 1) / waves;
    return static_cast<int>(per < 1 ? 1 : per);
}

void launch_residual(const GridView &g, int vec, int sum_mode, float omega, hipStream_t s) {
    const int nrt = itiles(g.I, vec) * (g.J - 2) * (g.K - 2);
    const int rpw = rows_per_wave(nrt, kResidualBlocks);
    const dim3 grid(kResidualBlocks), block(kResidualThreads);
#define RES(V, S) residual_kernel<V, S><<<grid, block, 0, s>>>(g, rpw, nrt)
    if (sum_mode == OFL_SUM_F64) {
        if (vec == 1) RES(1, OFL_SUM_F64); else if (vec == 2) RES(2, OFL_SUM_F64); else RES(4, OFL_SUM_F64);
    } else {
        if (vec == 1) RES(1, OFL_SUM_KAHAN_F32); else if (vec == 2) RES(2, OFL_SUM_KAHAN_F32); else RES(4, OFL_SUM_KAHAN_F32);
    }
#undef RES
    check_launch("residual kernel launch");
    finalize_kernel<<<1, kResidualThreads, 0, s>>>(g.partials, kResidualBlocks, static_cast<double>(omega), g.gosa);
    check_launch("residual finalize launch");
}

void launch_copyback(const GridView &g, int vec, hipStream_t s) {
    const int nrt = itiles(g.I, vec) * (g.J - 2) * (g.K - 2);
    const int blocks = grid_for(nrt, (kResidualThreads / kWave) * kRowUnroll * 2, kResidualBlocks * 4);
    const int rpw = rows_per_wave(nrt, blocks);
    const dim3 grid(blocks), block(kResidualThreads);
    if (vec == 1)
        copyback_kernel<1><<<grid, block, 0, s>>>(g, rpw, nrt);
    else if (vec == 2)
        copyback_kernel<2><<<grid, block, 0, s>>>(g, rpw, nrt);
    else
        copyback_kernel<4><<<grid, block, 0, s>>>(g, rpw, nrt);
    check_launch("copy-back kernel launch");
}

void launch_batch_residual(const GridView *views, const RowItem *items, int nitems, int vec, int sum_mode,
                           int grid_blocks, hipStream_t s) {
    const dim3 grid(grid_blocks), block(kResidualThreads);
#define RES(V, S) batch_residual_kernel<V, S><<<grid, block, 0, s>>>(views, items, nitems)
    if (sum_mode == OFL_SUM_F64) {
        if (vec == 1) RES(1, OFL_SUM_F64); else if (vec == 2) RES(2, OFL_SUM_F64); else RES(4, OFL_SUM_F64);
    } else {
        if (vec == 1) RES(1, OFL_SUM_KAHAN_F32); else if (vec == 2) RES(2, OFL_SUM_KAHAN_F32); else RES(4, OFL_SUM_KAHAN_F32);
    }
#undef RES
    check_launch("batched residual kernel launch");
}

void launch_batch_finalize(const GridView *views, const int *partial_range, int ngrids, float omega, hipStream_t s) {
    batch_finalize_kernel<<<ngrids, kResidualThreads, 0, s>>>(views, partial_range, static_cast<double>(omega));
    check_launch("batched finalize launch");
}

void launch_batch_copyback(const GridView *views, const RowItem *items, int nitems, int vec, int grid_blocks,
                           hipStream_t s) {
    const dim3 grid(grid_blocks), block(kResidualThreads);
    if (vec == 1)
        batch_copyback_kernel<1><<<grid, block, 0, s>>>(views, items, nitems);
    else if (vec == 2)
        batch_copyback_kernel<2><<<grid, block, 0, s>>>(views, items, nitems);
    else
        batch_copyback_kernel<4><<<grid, block, 0, s>>>(views, items, nitems);
    check_launch("batched copy-back kernel launch");
}

void launch_pack(const void *staging, void *arr, int I, int J, int K, int pitch, int elem_bytes, hipStream_t s) {
    const long long rows = static_cast<long long>(J) * K;
    const int blocks = grid_for(rows * I, 256, 65536);
    if (elem_bytes == 4)
        pack_kernel<float><<<blocks, 256, 0, s>>>(static_cast<const float *>(staging), static_cast<float *>(arr), I,
                                                 rows, pitch);
    else
        pack_kernel<uint16_t><<<blocks, 256, 0, s>>>(static_cast<const uint16_t *>(staging),
                                                    static_cast<uint16_t *>(arr), I, rows, pitch);
    check_launch("pack kernel launch");
}

void launch_unpack(const void *arr, void *staging, int I, int J, int K, int pitch, int elem_bytes, hipStream_t s) {
    const long long rows = static_cast<long long>(J) * K;
    const int blocks = grid_for(rows * I, 256, 65536);
    if (elem_bytes == 4)
        unpack_kernel<float><<<blocks, 256, 0, s>>>(static_cast<const float *>(arr), static_cast<float *>(staging),
                                                   I, rows, pitch);
    else
        unpack_kernel<uint16_t><<<blocks, 256, 0, s>>>(static_cast<const uint16_t *>(arr),
                                                      static_cast<uint16_t *>(staging), I, rows, pitch);
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

int device_cu_count(int device) {
    hipDeviceProp_t prop;
    hip_check(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties");
    return prop.multiProcessorCount;
}

}  // namespace ofl
