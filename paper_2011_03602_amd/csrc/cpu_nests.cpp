// The CPU side of the offload gene: the three loop nests as the original CPU
// program runs them (gene bit 0, paper Sec. 3.2.1), in FP32 on the caller's
// unpadded host arrays (linear index i + I*(j + J*k)). These are not a
// fallback: a nest runs here only when its gene bit says CPU, and a GPU bit
// never lands here. The k-planes are split into contiguous ranges over host
// threads; the residual adds per-plane sums in plane order, so its result does
// not depend on the thread count.
#include "cpu_nests.hpp"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <vector>

namespace ofl {

int cpu_threads() {
    for (const char *name : {"OFL_CPU_THREADS", "OMP_NUM_THREADS"}) {
        const char *v = std::getenv(name);
        if (v && std::atoi(v) > 0)
            return std::atoi(v);
    }
    const unsigned hw = std::thread::hardware_concurrency();
    return hw ? static_cast<int>(hw) : 1;
}

// Starting a thread costs tens of microseconds: below this many points per
// thread a small grid runs faster on fewer threads (or on the caller's).
constexpr long long kMinPointsPerThread = 1 << 14;

// f(k) for k in [lo, hi), split into contiguous ranges over the host threads;
// each index stands for `work` points.
template <class F>
void parallel_planes(int lo, int hi, long long work, F &&f) {
    const int n = hi - lo;
    const long long by_work = std::max<long long>(1, static_cast<long long>(n) * work / kMinPointsPerThread);
    const int nt = static_cast<int>(std::max<long long>(1, std::min<long long>({cpu_threads(), n, by_work})));
    if (nt == 1) {
        for (int k = lo; k < hi; ++k)
            f(k);
        return;
    }
    std::vector<std::thread> pool;
    pool.reserve(static_cast<size_t>(nt));
    for (int t = 0; t < nt; ++t) {
        const int a = lo + static_cast<int>(static_cast<long long>(n) * t / nt);
        const int b = lo + static_cast<int>(static_cast<long long>(n) * (t + 1) / nt);
        pool.emplace_back([a, b, &f] {
            for (int k = a; k < b; ++k)
                f(k);
        });
    }
    for (auto &th : pool)
        th.join();
}

float bf16_bits_to_f32(uint16_t q) {
    const uint32_t u = static_cast<uint32_t>(q) << 16;
    float f;
    std::memcpy(&f, &u, sizeof f);
    return f;
}

uint16_t f32_to_bf16_rne(float x) {
    uint32_t u;
    std::memcpy(&u, &x, sizeof u);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu) != 0)
        return static_cast<uint16_t>((u >> 16) | 0x0040u);  // keep NaN, quietened
    // Adding 0x7fff plus the lowest kept bit rounds to nearest, ties to even.
    u += 0x7fffu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}

namespace {

struct CoefF32 {
    const float *c[12];
    float at(int n, ptrdiff_t idx) const { return c[n][idx]; }
};

struct CoefBF16 {
    const uint16_t *c[12];
    float bias[12];
    float at(int n, ptrdiff_t idx) const { return bias[n] + bf16_bits_to_f32(c[n][idx]); }
};

template <class Co>
void sweep_impl(int I, int J, int K, const Co &co, const float *p, float *wrk2, float omega) {
    const ptrdiff_t dj = I;                        // offset of the j+1 neighbour
    const ptrdiff_t dk = static_cast<ptrdiff_t>(I) * J;  // offset of the k+1 neighbour
    parallel_planes(1, K - 1, static_cast<long long>(I) * J, [&](int k) {
        for (int j = 1; j < J - 1; ++j) {
            for (int i = 1; i < I - 1; ++i) {
                const ptrdiff_t c = i + dj * j + dk * k;
                const float *q = p + c;
                float s0 = co.at(0, c) * q[1] + co.at(1, c) * q[dj] + co.at(2, c) * q[dk];
                s0 += co.at(4, c) * ((q[1 + dj] - q[1 - dj]) - (q[dj - 1] - q[-1 - dj]));
                s0 += co.at(5, c) * ((q[dj + dk] - q[dk - dj]) - (q[dj - dk] - q[-dj - dk]));
                s0 += co.at(6, c) * ((q[1 + dk] - q[dk - 1]) - (q[1 - dk] - q[-1 - dk]));
                s0 += co.at(7, c) * q[-1] + co.at(8, c) * q[-dj] + co.at(9, c) * q[-dk] + co.at(11, c);
                const float ss = (co.at(3, c) * s0 - q[0]) * co.at(10, c);
                wrk2[c] = q[0] + omega * ss;
            }
        }
    });
}

}  // namespace

void cpu_sweep_f32(int I, int J, int K, const float *const coef[12], const float *p, float *wrk2, float omega) {
    CoefF32 co;
    for (int n = 0; n < 12; ++n)
        co.c[n] = coef[n];
    sweep_impl(I, J, K, co, p, wrk2, omega);
}

void cpu_sweep_bf16(int I, int J, int K, const uint16_t *const coef[12], const float bias[12], const float *p,
                    float *wrk2, float omega) {
    CoefBF16 co;
    for (int n = 0; n < 12; ++n) {
        co.c[n] = coef[n];
        co.bias[n] = bias[n];
    }
    sweep_impl(I, J, K, co, p, wrk2, omega);
}

double cpu_residual(int I, int J, int K, const float *p, const float *wrk2, float omega) {
    const size_t sI = static_cast<size_t>(I);
    const size_t sIJ = sI * static_cast<size_t>(J);
    std::vector<double> plane(static_cast<size_t>(K), 0.0);
    parallel_planes(1, K - 1, static_cast<long long>(I) * J, [&](int k) {
        double acc = 0.0;
        for (int j = 1; j < J - 1; ++j)
            for (int i = 1; i < I - 1; ++i) {
                const size_t c = static_cast<size_t>(i) + sI * j + sIJ * k;
                const double d = static_cast<double>(wrk2[c] - p[c]);
                acc += d * d;
            }
        plane[static_cast<size_t>(k)] = acc;
    });
    double total = 0.0;
    for (int k = 1; k < K - 1; ++k)
        total += plane[static_cast<size_t>(k)];
    const double om = static_cast<double>(omega);
    return total / (om * om);
}

void cpu_copyback(int I, int J, int K, const float *wrk2, float *p) {
    const size_t sI = static_cast<size_t>(I);
    const size_t sIJ = sI * static_cast<size_t>(J);
    parallel_planes(1, K - 1, static_cast<long long>(I) * J, [&](int k) {
        for (int j = 1; j < J - 1; ++j) {
            const size_t c = 1 + sI * j + sIJ * k;
            std::memcpy(p + c, wrk2 + c, sizeof(float) * static_cast<size_t>(I - 2));
        }
    });
}

void cpu_encode_bf16(const float *x, size_t n, float bias, uint16_t *q) {
    const int nt = static_cast<int>(std::max<size_t>(1, std::min<size_t>(static_cast<size_t>(cpu_threads()), n / 65536 + 1)));
    parallel_planes(0, nt, static_cast<long long>(n / static_cast<size_t>(nt)), [&](int t) {
        const size_t a = n * static_cast<size_t>(t) / static_cast<size_t>(nt);
        const size_t b = n * static_cast<size_t>(t + 1) / static_cast<size_t>(nt);
        for (size_t u = a; u < b; ++u)
            q[u] = f32_to_bf16_rne(x[u] - bias);
    });
}

}  // namespace ofl
