// Kernel launchers that do nothing, for the host-code build that runs against
// the stand-in HIP runtime (tests/csrc/hip_stand_in.cpp): the device state
// exists but no kernel runs, so only status codes, transfer bookkeeping and
// resource handling are meaningful in that build, not the numbers.
#include "ofl_internal.hpp"

namespace ofl {

void launch_sweep(const GridView &, const TileCfg &, int, float, hipStream_t, double *, const PrevParts &) {}
void launch_finalize(const double *, long long, float, double *, hipStream_t, double *, int) {}
void launch_residual(const GridView &, int, int, int, float, hipStream_t, bool) {}
void launch_copyback(const GridView &, int, int, hipStream_t, bool, bool, float) {}
void launch_pack(const void *, void *, int, int, int, int, int, long long, int, hipStream_t) {}
void launch_unpack(const void *, void *, int, int, int, int, long long, int, hipStream_t) {}
void launch_fill_zero(void *, size_t, hipStream_t) {}
void launch_copy(void *, const void *, size_t, hipStream_t) {}
void launch_stream(const float *const *, int, const uint16_t *const *, int, float *, size_t, hipStream_t) {}
void launch_batch_sweep(const GridView *, const SweepItem *, int, const TileCfg &, int, float, int, hipStream_t,
                        double *, const PrevParts &) {}
void launch_fold_finalize(const double *, long long, float, double *, int, hipStream_t) {}
void launch_batch_fold_finalize(const GridView *, const double *, const long long *, int, float, int, hipStream_t) {}
void launch_batch_residual(const GridView *, const RowItem *, int, int, int, int, int, hipStream_t) {}
void launch_batch_finalize(const GridView *, const int *, int, float, hipStream_t) {}
void launch_batch_copyback(const GridView *, const RowItem *, int, int, int, int, hipStream_t, bool) {}
void launch_gemm_f32(int, int, int, const float *, int, const float *, int, float *, int, hipStream_t) {}
int device_cu_count(int) { return 256; }
std::string device_arch(int) { return "stand-in"; }
// The no-op sweep never writes the partials, so one slot stands for the array.
double *static_scratch(int) {
    static double slot[1];
    return slot;
}

// no marker ranges in the host-only builds
void trace_push(const char *) {}
void trace_pop() {}

}  // namespace ofl
