// FP32 matrix product on the matrix cores: the GPU routine a recognised host
// matrix-product block is replaced with (function-block offload, Sec. 3.2.2,
// Sec. 4.2.1).
//
// C = A B for row-major FP32 matrices. A work-group of four waves owns a
// 128 x 256 tile of C. Each wave owns a 64 x 128 quarter as 2 x 4 accumulator
// tiles of 32 x 32, updated by v_mfma_f32_32x32x2_f32 (FP32 operands, FP32
// accumulation); each operand value read from LDS feeds two or four products.
// Products whose 128-row tiles leave much of their last round of resident
// work-groups idle use 64 x 256 tiles (four waves of 64 x 64 side by side),
// twice as many (see launch_gemm_f32). The K dimension advances in stages of
// 16: the next stage's A and B tiles are fetched from global memory into
// registers while the current stage, held in LDS, feeds the matrix cores. LDS
// is double-buffered, so one barrier per stage suffices.
//
// Tiles are handed to work-groups so that each XCD works through a contiguous
// run of them. Measured at 4096^3 with 128 x 128 tiles, this order ran at up
// to 132 TFLOP/s against 118 for the hardware's round-robin, but from run to
// run it varied down to the round-robin figure; 128 x 256 tiles ran at 137.
//
// Operand layout of the 32x32x2 instruction (wave64): lane l supplies
// A[l % 32][l / 32] and B[l / 32][l % 32]; accumulator register r of lane l
// holds C[8 (r / 4) + 4 (l / 32) + r % 4][l % 32].
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ofl_internal.hpp"

namespace ofl {

namespace {

constexpr int kGemmThreads = 256;
constexpr int kTileN = 256, kTileK = 16;
constexpr int kCus = 256;  // compute units of an MI355X

// Work-group tile of TM x 256: four waves of 64 rows each, TM / 64 of them along
// m and the rest along n; each thread fetches kAPer consecutive k of one A row.
template <int TM>
struct Shape {
    static constexpr int kWavesM = TM / 64;
    static constexpr int kWavesN = 4 / kWavesM;
    static constexpr int kNJ = kTileN / kWavesN / 32;  // 32-wide accumulator tiles per wave along n
    static constexpr int kAPer = TM * kTileK / kGemmThreads;
    static constexpr int kAThreadsPerRow = kTileK / kAPer;
    static_assert(kWavesM * kWavesN == kGemmThreads / 64 && kAPer % 4 == 0, "unsupported tile");
};
constexpr int kBThreadsPerRow = kTileN / 8;                 // threads loading one B row, 8 floats each
constexpr int kBRowsPerPass = kGemmThreads / kBThreadsPerRow;
constexpr int kBPasses = kTileK / kBRowsPerPass;            // passes over the B tile per stage
static_assert(kBPasses * kBRowsPerPass == kTileK, "B tile rows must split into whole passes");
constexpr int kLdsPad = 4;  // floats of padding per LDS row
constexpr int kXcds = 8;    // accelerator complex dies of an MI355X, each with its own L2

typedef float floatx16 __attribute__((ext_vector_type(16)));

struct GemmArgs {
    int M, N, K;
    const float *A;
    int lda;
    const float *B;
    int ldb;
    float *C;
    int ldc;
};

// Fetch this thread's share of the A (TM x 16) and B (16 x 256) tiles at k0
// into registers: A row tid / kAThreadsPerRow, kAPer columns from
// (tid % kAThreadsPerRow) * kAPer; B rows pass * 8 + tid / 32, columns
// (tid % 32) * 8 .. +8, for pass 0 and 1. Out-of-range elements read as zero.
// `vec`: the block's tiles lie inside the matrices and every row start is
// 16-byte aligned, so whole float4 loads are used.
template <int TM>
__device__ __forceinline__ void fetch(const GemmArgs &g, int m0, int n0, int k0, bool vec, float *ra, float *rb) {
    using S = Shape<TM>;
    const int tid = threadIdx.x;
    const int am = m0 + tid / S::kAThreadsPerRow, ak = k0 + (tid % S::kAThreadsPerRow) * S::kAPer;
    const int bn = n0 + (tid % kBThreadsPerRow) * 8;
    if (vec && k0 + kTileK <= g.K) {
        const float4 *pa = reinterpret_cast<const float4 *>(g.A + static_cast<size_t>(am) * g.lda + ak);
#pragma unroll
        for (int q = 0; q < S::kAPer / 4; ++q) {
            const float4 a = pa[q];
            ra[4 * q] = a.x; ra[4 * q + 1] = a.y; ra[4 * q + 2] = a.z; ra[4 * q + 3] = a.w;
        }
#pragma unroll
        for (int pass = 0; pass < kBPasses; ++pass) {
            const int bk = k0 + pass * kBRowsPerPass + tid / kBThreadsPerRow;
            const float4 *pb = reinterpret_cast<const float4 *>(g.B + static_cast<size_t>(bk) * g.ldb + bn);
            const float4 b0 = pb[0], b1 = pb[1];
            float *r = rb + pass * 8;
            r[0] = b0.x; r[1] = b0.y; r[2] = b0.z; r[3] = b0.w;
            r[4] = b1.x; r[5] = b1.y; r[6] = b1.z; r[7] = b1.w;
        }
        return;
    }
#pragma unroll
    for (int e = 0; e < S::kAPer; ++e) {
        const int k = ak + e;
        ra[e] = (am < g.M && k < g.K) ? g.A[static_cast<size_t>(am) * g.lda + k] : 0.f;
    }
#pragma unroll
    for (int pass = 0; pass < kBPasses; ++pass) {
        const int bk = k0 + pass * kBRowsPerPass + tid / kBThreadsPerRow;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int n = bn + e;
            rb[pass * 8 + e] = (bk < g.K && n < g.N) ? g.B[static_cast<size_t>(bk) * g.ldb + n] : 0.f;
        }
    }
}

template <int TM>
__global__ __launch_bounds__(kGemmThreads) void gemm_f32_kernel(GemmArgs g, int vec_ok) {
    using S = Shape<TM>;
    constexpr int kNJ = S::kNJ;
    // A is kept transposed (k-major) so that a wave's operand fetch for one k
    // reads 32 consecutive floats.
    __shared__ float As[2][kTileK][TM + kLdsPad];
    __shared__ float Bs[2][kTileK][kTileN + kLdsPad];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = (wave / S::kWavesN) * 64, wn = (wave % S::kWavesN) * (kTileN / S::kWavesN);
    // Work-groups are dealt round-robin to the eight XCDs. Give each XCD a
    // contiguous run of tiles in row-major tile order instead, so that tiles
    // sharing rows of A (and neighbouring columns of B) meet in one XCD's L2.
    int bx = blockIdx.x, by = blockIdx.y;
    {
        const int nb = gridDim.x * gridDim.y, b = blockIdx.y * gridDim.x + blockIdx.x;
        const int per = nb / kXcds;
        const int t = b < per * kXcds ? (b % kXcds) * per + b / kXcds : b;
        by = t / gridDim.x;
        bx = t % gridDim.x;
    }
    const int m0 = by * TM, n0 = bx * kTileN;
    const bool vec = vec_ok && m0 + TM <= g.M && n0 + kTileN <= g.N;

    floatx16 acc[2][kNJ];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < kNJ; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r)
                acc[i][j][r] = 0.f;

    float ra[S::kAPer], rb[8 * kBPasses];
    auto stash = [&](int buf) {
        const int am = tid / S::kAThreadsPerRow, ak = (tid % S::kAThreadsPerRow) * S::kAPer;
        const int bn = (tid % kBThreadsPerRow) * 8;
#pragma unroll
        for (int e = 0; e < S::kAPer; ++e)
            As[buf][ak + e][am] = ra[e];
#pragma unroll
        for (int pass = 0; pass < kBPasses; ++pass) {
            const int bk = pass * kBRowsPerPass + tid / kBThreadsPerRow;
#pragma unroll
            for (int e = 0; e < 8; ++e)
                Bs[buf][bk][bn + e] = rb[pass * 8 + e];
        }
    };

    fetch<TM>(g, m0, n0, 0, vec, ra, rb);
    stash(0);
    __syncthreads();
    const int lrow = lane >> 5, lcol = lane & 31;
    int buf = 0;
    for (int k0 = 0; k0 < g.K; k0 += kTileK) {
        const bool more = k0 + kTileK < g.K;
        if (more)
            fetch<TM>(g, m0, n0, k0 + kTileK, vec, ra, rb);
        // The operands of step kk + 2 are read from LDS before step kk's products
        // are issued (two register sets), so the LDS latency hides behind eight
        // matrix instructions; the scheduling barrier keeps the compiler from
        // sinking the reads back next to their use. Measured +1.5-1.9%.
        float a[2][2], b[2][kNJ];
#pragma unroll
        for (int i = 0; i < 2; ++i)
            a[0][i] = As[buf][lrow][wm + i * 32 + lcol];
#pragma unroll
        for (int j = 0; j < kNJ; ++j)
            b[0][j] = Bs[buf][lrow][wn + j * 32 + lcol];
#pragma unroll
        for (int kk = 0; kk < kTileK; kk += 2) {
            const int cur = (kk / 2) & 1, nxt = cur ^ 1;
            if (kk + 2 < kTileK) {
#pragma unroll
                for (int i = 0; i < 2; ++i)
                    a[nxt][i] = As[buf][kk + 2 + lrow][wm + i * 32 + lcol];
#pragma unroll
                for (int j = 0; j < kNJ; ++j)
                    b[nxt][j] = Bs[buf][kk + 2 + lrow][wn + j * 32 + lcol];
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < kNJ; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[cur][i], b[cur][j], acc[i][j], 0, 0, 0);
        }
        if (more)
            stash(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }

#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < kNJ; ++j) {
            const int col = n0 + wn + j * 32 + lcol;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = m0 + wm + i * 32 + 8 * (r >> 2) + 4 * lrow + (r & 3);
                if (row < g.M && col < g.N)
                    g.C[static_cast<size_t>(row) * g.ldc + col] = acc[i][j][r];
            }
        }
}

}  // namespace

namespace {

// Work-groups of a tile height resident on one CU at a time (registers and LDS
// decide: two of the 128-row kernel, three of the 64-row one on gfx950), from
// the runtime's occupancy query, taken once.
template <int TM>
int resident_per_cu() {
    static const int n = [] {
        int blocks = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, gemm_f32_kernel<TM>, kGemmThreads, 0) != hipSuccess ||
            blocks < 1)
            blocks = 1;
        return blocks;
    }();
    return n;
}

// Fraction of the work-group slots busy over the whole product when `tiles`
// tiles run in rounds of `slots`: the last round's idle slots are the tail.
double round_fill(long long tiles, long long slots) {
    const long long rounds = (tiles + slots - 1) / slots;
    return static_cast<double>(tiles) / static_cast<double>(rounds * slots);
}

}  // namespace

void launch_gemm_f32(int M, int N, int K, const float *A, int lda, const float *B, int ldb, float *C, int ldc,
                     hipStream_t s) {
    const GemmArgs g{M, N, K, A, lda, B, ldb, C, ldc};
    const bool aligned = (reinterpret_cast<uintptr_t>(A) % 16 == 0) && (reinterpret_cast<uintptr_t>(B) % 16 == 0) &&
                         lda % 4 == 0 && ldb % 4 == 0;
    // Tile height by the tail of the last round of tiles: the 128-row tiles
    // reuse each operand more and run about 5% faster in steady state (8192^3:
    // 141 against 133.5 TFLOP/s), so they are taken unless the 64-row ones fill
    // the rounds of resident work-groups better by more than that. Measured:
    // 2048^3 104 against 61 TFLOP/s and 3072^3 99 against 79 for 64 rows,
    // 4096^3 138 against 109 for 128 rows, and 6144^3 133 for 64 rows against
    // 105 for 128 (1152 tiles of 128 rows are 2.25 rounds of 512).
    const long long tiles128 = static_cast<long long>((N + kTileN - 1) / kTileN) * ((M + 127) / 128);
    const long long tiles64 = static_cast<long long>((N + kTileN - 1) / kTileN) * ((M + 63) / 64);
    const double fill128 = round_fill(tiles128, static_cast<long long>(kCus) * resident_per_cu<128>());
    const double fill64 = round_fill(tiles64, static_cast<long long>(kCus) * resident_per_cu<64>());
    if (fill128 >= 0.95 * fill64) {
        const dim3 grid((N + kTileN - 1) / kTileN, (M + 127) / 128);
        hipLaunchKernelGGL(gemm_f32_kernel<128>, grid, dim3(kGemmThreads), 0, s, g, aligned ? 1 : 0);
    } else {
        const dim3 grid((N + kTileN - 1) / kTileN, (M + 63) / 64);
        hipLaunchKernelGGL(gemm_f32_kernel<64>, grid, dim3(kGemmThreads), 0, s, g, aligned ? 1 : 0);
    }
    hip_check(hipGetLastError(), "gemm kernel launch");
}

}  // namespace ofl
