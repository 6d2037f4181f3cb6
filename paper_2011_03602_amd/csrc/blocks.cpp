// C interface of the function-block routines (Sec. 3.2.2, Sec. 4.2.1): the
// GPU routines a recognised host function block is replaced with. Argument
// checks live here; the kernels are in gemm.hip.
#include "abi_util.hpp"
#include "ofl_internal.hpp"

extern "C" int ofl_gemm_f32(int M, int N, int K, const float *A, int lda, const float *B, int ldb, float *C,
                            int ldc, void *stream) {
    return ofl::guarded(nullptr, [&] {
        if (M < 0 || N < 0 || K < 0)
            ofl::fail(OFL_EINVAL, "negative matrix size");
        if (lda < K || ldb < N || ldc < N || lda < 0 || ldb < 0 || ldc < 0)
            ofl::fail(OFL_EINVAL, "a row stride is shorter than its row");
        if ((M + 127) / 128 > 65535)
            ofl::fail(OFL_EINVAL, "M above 65535 * 128 rows");
        if (M == 0 || N == 0)
            return;
        if (!C || (K > 0 && (!A || !B)))
            ofl::fail(OFL_EINVAL, "NULL pointer to an operand the product uses");
        ofl::launch_gemm_f32(M, N, K, A, lda, B, ldb, C, ldc, static_cast<hipStream_t>(stream));
    });
}
