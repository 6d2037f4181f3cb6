// Stand-ins for the device launches, for the sanitizer build of the host
// code: every launch reports a device error, exactly what the library does
// when no GPU is present. Only host paths (all-CPU genes, the planner,
// argument checks, the GA) can succeed in such a build.
#include "ofl_internal.hpp"

namespace ofl {

namespace {
[[noreturn]] void no_device() { fail(OFL_EDEVICE, "this build has no device code"); }
}  // namespace

void launch_sweep(const GridView &, const TileCfg &, int, float, hipStream_t, double *, const PrevParts &) { no_device(); }
void launch_finalize(const double *, long long, float, double *, hipStream_t, double *, int) { no_device(); }
void launch_residual(const GridView &, int, int, int, float, hipStream_t, bool) { no_device(); }
void launch_copyback(const GridView &, int, int, hipStream_t, bool, bool, float) { no_device(); }
void launch_pack(const void *, void *, int, int, int, int, int, long long, int, hipStream_t) { no_device(); }
void launch_unpack(const void *, void *, int, int, int, int, long long, int, hipStream_t) { no_device(); }
void launch_fill_zero(void *, size_t, hipStream_t) { no_device(); }
void launch_copy(void *, const void *, size_t, hipStream_t) { no_device(); }
void launch_stream(const float *const *, int, const uint16_t *const *, int, float *, size_t, hipStream_t) {
    no_device();
}
void launch_batch_sweep(const GridView *, const SweepItem *, int, const TileCfg &, int, float, int, hipStream_t,
                        double *, const PrevParts &) {
    no_device();
}
void launch_fold_finalize(const double *, long long, float, double *, int, hipStream_t) { no_device(); }
void launch_batch_fold_finalize(const GridView *, const double *, const long long *, int, float, int, hipStream_t) { no_device(); }
void launch_batch_residual(const GridView *, const RowItem *, int, int, int, int, int, hipStream_t) { no_device(); }
void launch_batch_finalize(const GridView *, const int *, int, float, hipStream_t) { no_device(); }
void launch_batch_copyback(const GridView *, const RowItem *, int, int, int, int, hipStream_t, bool) { no_device(); }
void launch_gemm_f32(int, int, int, const float *, int, const float *, int, float *, int, hipStream_t) {
    no_device();
}
int device_cu_count(int) { no_device(); }
std::string device_arch(int) { no_device(); }
double *static_scratch(int) { no_device(); }

// no marker ranges in the host-only builds
void trace_push(const char *) {}
void trace_pop() {}

}  // namespace ofl
