// Internal declarations of the offloaded-Jacobi library: device layout, the
// views the kernels read, launch entry points and the error type. Not part of
// the public interface (that is include/ofl.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <stdexcept>
#include <string>

#include "ofl.h"

namespace ofl {

constexpr int kNCoef = 12;
constexpr int kWave = 64;
constexpr int kPitchAlign = 32;   // FP32 elements per 128 bytes (row alignment of the pitched layout)
constexpr size_t kGuard = 1024;   // elements of slack before and after every device array
constexpr int kResidualBlocks = 2048;  // fixed -> deterministic residual partials
constexpr int kResidualThreads = 256;
constexpr int kRowUnroll = 4;   // row tiles a residual wave keeps in flight
constexpr int kCopyUnroll = 16;  // row tiles a copy-back wave keeps in flight
// Template flags of the sweep kernels are the low four OFL_TILE_* bits (the
// XCD order is a launch argument, not a template flag) plus this internal bit,
// which sits where the public tile flags keep OFL_TILE_XCD_REMAP: the sweep
// also accumulates the residual nest's terms into one FP64 partial per wave.
constexpr int kTemplateFlagMask = 15;
constexpr int kFlagFuseResidual = 16;

enum Nest { kS = 0, kR = 1, kC = 2 };

struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] void fail(int code, const std::string &msg);
void hip_check(hipError_t e, const char *what);

inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

// Device layout of one grid: every array pitched along i, rows 128-byte
// aligned by default (or to row_align elements, a multiple of 4), with guard
// elements before and after so that whole-wave vector loads that run past the
// last interior point stay inside the allocation.
struct Layout {
    int I = 0, J = 0, K = 0;
    int pitch = 0;          // elements per row of p and wrk2
    size_t plane = 0;       // elements per plane: pitch * J (compact rows: padded to kSegAlign)
    size_t elems = 0;       // plane * K
    // The twelve coefficient arrays: rows of cpitch elements holding i = 0 ..
    // crow-1 (the default layout leaves out i = I-1, a boundary column that no
    // nest reads), planes of cplane, celems in all. Compact rows: as p.
    int cpitch = 0, crow = 0;
    size_t cplane = 0, celems = 0;
    size_t coef_elem = 4;   // bytes per stored coefficient (4 or 2)
    size_t off[OFL_NARRAYS] = {};  // byte offset of element 0 of each array in the block
    size_t staging_off = 0; // contiguous I*J*K*4-byte staging buffer for transfers
    size_t partials_off = 0;
    size_t gosa_off = 0;
    size_t total = 0;       // bytes of the whole device block
};

Layout make_layout(int I, int J, int K, int coef_format, int row_align = 0);

// What a kernel needs to address one grid on the device.
struct GridView {
    float *p;
    float *wrk2;
    const void *coef[kNCoef];  // float* (FP32) or uint16_t* (bfloat16 formats)
    float bias[kNCoef];
    int I, J, K, pitch;
    int cpitch;  // row pitch of the coefficient arrays (elements)
    // Batched grids only: > 0 when the grid runs in packed rows, as this many
    // segments of 64 * VEC consecutive points per plane (rows 1..J-2), each
    // wave's line running across row ends; 0 for the row-per-wave form.
    int nseg;
    // Batched grids only: the grid's points per lane (1, 2 or 4) in a launch
    // whose items mix vector widths; unused elsewhere.
    int vec;
    long long plane;
    long long cplane;  // plane stride of the coefficient arrays (elements)
    double *partials;  // residual partial sums (batched: base of this grid's range)
    double *gosa;      // device scalar
};

// Sweep work item (batched launch): grid, i-tile, block of lines a work-group
// owns (rows j, or planes k when marching along j), chunk of the march.
struct SweepItem {
    int grid, itile, fblock, mchunk;
};
// Residual / copy-back work item (batched launch): grid and a range of row tiles.
struct RowItem {
    int grid, first, count, partial;
};

struct TileCfg {
    int vec = 4, rows = 4, kchunk = 32, flags = 0, occupancy = 0;
};

bool tile_valid(const ofl_tile &t, std::string *why);
TileCfg to_cfg(const ofl_tile &t);
ofl_tile to_tile(const TileCfg &c);

// Points of one row tile: 64 lanes x vec, except at 8 points per lane, where
// a wave covers two rows of 32 lanes each (the sweep only).
__host__ __device__ inline constexpr int tile_points(int vec) { return vec == 8 ? (kWave / 2) * 8 : kWave * vec; }
__host__ __device__ inline int itiles(int I, int vec) { return (I - 2) / tile_points(vec) + 1; }

// Packed rows (batched grids with short rows): a plane's rows 1..J-2 are cut
// into segments of 64 * vec consecutive points, the first starting at the
// last multiple of kSegAlign elements at or before row 1. With compact rows
// planes are padded to kSegAlign elements, so every segment starts on a
// 128-byte line in the FP32 arrays and in the bfloat16 ones.
constexpr int kSegAlign = 64;
__host__ __device__ inline int packed_seg0(int pitch) { return pitch / kSegAlign * kSegAlign; }
__host__ __device__ inline long long packed_nseg(int J, int pitch, int vec) {
    const long long span = static_cast<long long>(J - 1) * pitch - packed_seg0(pitch);
    return (span + kWave * vec - 1) / (kWave * vec);
}

// Sweep decomposition of a grid: i-tiles, blocks of owned lines, march chunks.
void sweep_shape(int I, int J, int K, const TileCfg &t, int *nti, int *nfb, int *nmc);

// The previous iteration's fused-residual partials, reduced inside the next
// fused sweep launch instead of by kernels of their own: the launch's first
// work-group (a single grid: n partials) or work-groups 0..ngrids-1 (a batch:
// grid b owns parts[range[2b], range[2b+1])) sum them in a fixed order into
// gosa before their own march. parts == nullptr: nothing to reduce.
struct PrevParts {
    const double *parts = nullptr;
    long long n = 0;
    const long long *range = nullptr;
    int ngrids = 0;
};

// Single-grid launches (kernels.hip).
// fused_parts != nullptr: fuse the residual, one partial per wave (sweep_waves() of them).
void launch_sweep(const GridView &g, const TileCfg &t, int bf16, float omega, hipStream_t s,
                  double *fused_parts = nullptr, const PrevParts &prev = PrevParts{});
long long sweep_waves(int I, int J, int K, const TileCfg &t);
// gosa = sum(partials[0..n)) / omega^2 in a fixed order; with scratch (at
// least scratch_len doubles) large n is summed in two stages.
void launch_finalize(const double *partials, long long n, float omega, double *gosa, hipStream_t s,
                     double *scratch = nullptr, int scratch_len = 0);
void launch_residual(const GridView &g, int vec, int sum_mode, int flags, float omega, hipStream_t s,
                     bool finalize = true);
// whole_rows: the device wrk2 equals p outside the interior, so interior rows
// are copied whole (same result, full-line writes).
// finalize_residual: the residual kernel just ran without its finalize step
// (launch_residual(..., false)); the copy-back's block 0 does it first.
void launch_copyback(const GridView &g, int vec, int flags, hipStream_t s, bool whole_rows = false,
                     bool finalize_residual = false, float omega = 1.f);
// Host-order staging (rows of I elements) into a pitched device array that
// keeps the first `keep` elements of every row (keep <= I, keep <= pitch).
void launch_pack(const void *staging, void *arr, int I, int J, int K, int keep, int pitch, long long plane,
                 int elem_bytes, hipStream_t s);
void launch_unpack(const void *arr, void *staging, int I, int J, int K, int pitch, long long plane, int elem_bytes,
                   hipStream_t s);
void launch_fill_zero(void *ptr, size_t bytes, hipStream_t s);
void launch_copy(void *dst, const void *src, size_t bytes, hipStream_t s);
// dst[t] = sum of the n32 FP32 and n16 bfloat16 sources at t, t < n (n a
// multiple of 4): the sweep's streaming pattern, (13, 0) or (1, 12).
void launch_stream(const float *const *src32, int n32, const uint16_t *const *src16, int n16, float *dst, size_t n,
                   hipStream_t s);

// Batched launches (kernels.hip).
// fused_parts != nullptr: fuse the residual, rows partials per item (slot item*rows + wave).
void launch_batch_sweep(const GridView *views, const SweepItem *items, int nitems, const TileCfg &t, int bf16,
                        float omega, int grid_blocks, hipStream_t s, double *fused_parts = nullptr,
                        const PrevParts &prev = PrevParts{});
// The fused residual's last sum by the group sum the sweeps fold in, with the
// sweep's work-group size `threads` (64 x tile rows): one grid's n partials
// into gosa, or each batched grid's range of parts into its gosa.
void launch_fold_finalize(const double *parts, long long n, float omega, double *gosa, int threads, hipStream_t s);
void launch_batch_fold_finalize(const GridView *views, const double *parts, const long long *range, int ngrids,
                                float omega, int threads, hipStream_t s);
void launch_batch_residual(const GridView *views, const RowItem *items, int nitems, int vec, int sum_mode, int flags,
                           int grid_blocks, hipStream_t s);
void launch_batch_finalize(const GridView *views, const int *partial_range, int ngrids, float omega,
                           hipStream_t s);
void launch_batch_copyback(const GridView *views, const RowItem *items, int nitems, int vec, int flags,
                           int grid_blocks, hipStream_t s, bool whole_rows);

// Matrix product on the matrix cores (gemm.hip).
void launch_gemm_f32(int M, int N, int K, const float *A, int lda, const float *B, int ldb, float *C, int ldc,
                     hipStream_t s);

int device_cu_count(int device);
std::string device_arch(int device);  // e.g. "gfx950:sramecc+:xnack-"

// Host ranges for marker traces (trace.cpp): a range per offloaded nest,
// planned transfer, graph launch, batched run and tuner measurement.
void trace_push(const char *name);
void trace_pop();
struct TraceRange {
    explicit TraceRange(const char *name) { trace_push(name); }
    ~TraceRange() { trace_pop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

// Library-owned device scratch for the entry point that allocates nothing
// (ofl_jacobi_run_static): kStaticScratchParts FP64 slots per device, held
// until the process ends. static_scratch() resolves this device's address of
// the array (the current device must be `device`); every call on a device
// shares the same slots.
constexpr long long kStaticScratchParts = 1LL << 19;  // 4 MiB
double *static_scratch(int device);

}  // namespace ofl
