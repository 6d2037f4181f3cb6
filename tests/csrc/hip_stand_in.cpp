// Test-only stand-in for the HIP runtime calls the library's host code makes,
// so that the host paths that need device state (a grid whose device block and
// stream exist, a batch with its tables and graph) can run on a machine with no
// GPU, under AddressSanitizer, LeakSanitizer and UBSan. Device memory is host
// memory, streams, events and graphs are tokens, copies are memcpy, and every
// call succeeds, except the one the driver names: stand_in_fail_call(n) makes
// the n-th HIP call after it report an error (once), which is how the tests
// reach every device-error path of the library. A release call (free, destroy)
// that reports an error still releases, as a runtime whose context has failed
// drops its resources with it: the caller cannot do anything else with them.
//
// Never linked into the library: the sanitizer test builds it into its own
// executable together with the host sources and no-op kernel launchers.
#include <hip/hip_runtime_api.h>

#include <cstdlib>
#include <cstring>

namespace {

long g_calls = 0;    // HIP calls since the last stand_in_fail_call
long g_fail_at = 0;  // the call that fails (1-based); 0: none
long g_live = 0;     // allocations and tokens not yet released
long g_alloc_calls = 0;  // calls that allocate or release device memory, streams, events or graphs
bool g_capturing = false;

bool next_fails() {
    ++g_calls;
    if (g_fail_at > 0 && g_calls == g_fail_at) {
        g_fail_at = 0;
        return true;
    }
    return false;
}

// An opaque handle the library only passes back to us.
template <class T>
T token() {
    ++g_live;
    ++g_alloc_calls;
    return reinterpret_cast<T>(new char[16]);
}

template <class T>
void release(T t) {
    ++g_alloc_calls;
    if (t) {
        --g_live;
        delete[] reinterpret_cast<char *>(t);
    }
}

}  // namespace

#define STAND_IN_STEP()                 \
    do {                                \
        if (next_fails())               \
            return hipErrorLaunchFailure; \
    } while (0)

extern "C" void stand_in_fail_call(long n) {
    g_calls = 0;
    g_fail_at = n;
}

extern "C" long stand_in_calls(void) { return g_calls; }

extern "C" long stand_in_live(void) { return g_live; }

extern "C" long stand_in_alloc_calls(void) { return g_alloc_calls; }

hipError_t hipGetDeviceCount(int *count) {
    STAND_IN_STEP();
    *count = 1;
    return hipSuccess;
}

hipError_t hipGetDevice(int *device) {
    STAND_IN_STEP();
    *device = 0;
    return hipSuccess;
}

hipError_t hipSetDevice(int device) {
    STAND_IN_STEP();
    return device == 0 ? hipSuccess : hipErrorInvalidDevice;
}

const char *hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "stand-in device error"; }

hipError_t hipGetLastError(void) { return hipSuccess; }

hipError_t hipMalloc(void **ptr, size_t size) {
    STAND_IN_STEP();
    const size_t bytes = (size + 255) / 256 * 256;
    void *p = nullptr;
    if (posix_memalign(&p, 256, bytes == 0 ? 256 : bytes) != 0)
        return hipErrorOutOfMemory;
    std::memset(p, 0, bytes == 0 ? 256 : bytes);
    ++g_live;
    ++g_alloc_calls;
    *ptr = p;
    return hipSuccess;
}

hipError_t hipFree(void *ptr) {
    ++g_alloc_calls;
    if (ptr) {
        --g_live;
        std::free(ptr);
    }
    STAND_IN_STEP();
    return hipSuccess;
}

hipError_t hipMemcpyAsync(void *dst, const void *src, size_t bytes, hipMemcpyKind, hipStream_t) {
    STAND_IN_STEP();
    std::memmove(dst, src, bytes);
    return hipSuccess;
}

hipError_t hipMemcpy2DAsync(void *dst, size_t dpitch, const void *src, size_t spitch, size_t width, size_t height,
                            hipMemcpyKind, hipStream_t) {
    STAND_IN_STEP();
    for (size_t r = 0; r < height; ++r)
        std::memmove(static_cast<char *>(dst) + r * dpitch, static_cast<const char *>(src) + r * spitch, width);
    return hipSuccess;
}

hipError_t hipStreamCreate(hipStream_t *s) {
    STAND_IN_STEP();
    *s = token<hipStream_t>();
    return hipSuccess;
}

hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned int) {
    STAND_IN_STEP();
    *s = token<hipStream_t>();
    return hipSuccess;
}

hipError_t hipStreamDestroy(hipStream_t s) {
    release(s);
    STAND_IN_STEP();
    return hipSuccess;
}

hipError_t hipStreamSynchronize(hipStream_t) {
    STAND_IN_STEP();
    return hipSuccess;
}

hipError_t hipEventCreate(hipEvent_t *e) {
    STAND_IN_STEP();
    *e = token<hipEvent_t>();
    return hipSuccess;
}

hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) {
    STAND_IN_STEP();
    *e = token<hipEvent_t>();
    return hipSuccess;
}

hipError_t hipEventDestroy(hipEvent_t e) {
    release(e);
    STAND_IN_STEP();
    return hipSuccess;
}

hipError_t hipEventRecord(hipEvent_t, hipStream_t) {
    STAND_IN_STEP();
    return hipSuccess;
}

hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t) {
    STAND_IN_STEP();
    *ms = 0.001f;
    return hipSuccess;
}

hipError_t hipStreamIsCapturing(hipStream_t, hipStreamCaptureStatus *status) {
    STAND_IN_STEP();
    *status = g_capturing ? hipStreamCaptureStatusActive : hipStreamCaptureStatusNone;
    return hipSuccess;
}

hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) {
    STAND_IN_STEP();
    g_capturing = true;
    return hipSuccess;
}

hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *graph) {
    g_capturing = false;
    STAND_IN_STEP();
    *graph = token<hipGraph_t>();
    return hipSuccess;
}

hipError_t hipGraphInstantiate(hipGraphExec_t *exec, hipGraph_t, hipGraphNode_t *, char *, size_t) {
    STAND_IN_STEP();
    *exec = token<hipGraphExec_t>();
    return hipSuccess;
}

hipError_t hipGraphDestroy(hipGraph_t graph) {
    release(graph);
    STAND_IN_STEP();
    return hipSuccess;
}

hipError_t hipGraphExecDestroy(hipGraphExec_t exec) {
    release(exec);
    STAND_IN_STEP();
    return hipSuccess;
}

hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) {
    STAND_IN_STEP();
    return hipSuccess;
}
