// CPU loop nests (gene bit 0) and the host-side bfloat16 encoder.
#pragma once

#include <cstddef>
#include <cstdint>

namespace ofl {

float bf16_bits_to_f32(uint16_t q);
uint16_t f32_to_bf16_rne(float x);

void cpu_sweep_f32(int I, int J, int K, const float *const coef[12], const float *p, float *wrk2, float omega);
void cpu_sweep_bf16(int I, int J, int K, const uint16_t *const coef[12], const float bias[12], const float *p,
                    float *wrk2, float omega);
double cpu_residual(int I, int J, int K, const float *p, const float *wrk2, float omega);
void cpu_copyback(int I, int J, int K, const float *wrk2, float *p);
// q[t] = bfloat16(fl32(x[t] - bias)), round to nearest even.
void cpu_encode_bf16(const float *x, size_t n, float bias, uint16_t *q);
int cpu_threads();

}  // namespace ofl
