// Test fixture, not part of the library: runs single MFMA instructions on operands the test
// chooses lane by lane, so that a test can compare their results with exact arithmetic.  It
// pins the rounding behaviour that the library's error bound for the FP32 contraction
// assumes (one rounding step per half of a BF16 MFMA's K range, two per FP32 MFMA).
//
// Layout (one wave of 64 lanes per case, lane l, h = l / 32):
//   32x32x16 BF16: lane l holds A[l % 32][8 h + t] and B[8 h + t][l % 32], t = 0..7, as 8 BF16
//                  values in 4 dwords (value t in the low half of dword t / 2 when t is even);
//   32x32x2 FP32:  lane l holds A[l % 32][h] and B[h][l % 32];
//   accumulator:   register r of lane l is D[8 (r / 4) + 4 h + r % 4][l % 32].
// Buffers: A and B `cases` x 64 lanes (uint4 for BF16, float for FP32), C and D `cases` x 64 x 16
// floats, all device pointers.  The grid has exactly `cases` workgroups of one wave, so every
// access is in bounds.
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;

__global__ __launch_bounds__(64) void probe_bf16_kernel(const uint4* A, const uint4* B, const float* C, float* D) {
    const size_t c = blockIdx.x, l = threadIdx.x;
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = C[(c * 64 + l) * 16 + r];
    const bf16x8 a = __builtin_bit_cast(bf16x8, A[c * 64 + l]);
    const bf16x8 b = __builtin_bit_cast(bf16x8, B[c * 64 + l]);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 16; ++r) D[(c * 64 + l) * 16 + r] = acc[r];
}

__global__ __launch_bounds__(64) void probe_f32_kernel(const float* A, const float* B, const float* C, float* D) {
    const size_t c = blockIdx.x, l = threadIdx.x;
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = C[(c * 64 + l) * 16 + r];
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(A[c * 64 + l], B[c * 64 + l], acc, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 16; ++r) D[(c * 64 + l) * 16 + r] = acc[r];
}

extern "C" int rr_probe_mfma_bf16(const void* A, const void* B, const void* C, void* D, int cases, void* stream) {
    if (cases <= 0 || !A || !B || !C || !D) return 1;
    hipLaunchKernelGGL(probe_bf16_kernel, dim3(cases), dim3(64), 0, (hipStream_t)stream, (const uint4*)A,
                       (const uint4*)B, (const float*)C, (float*)D);
    return hipGetLastError() == hipSuccess ? 0 : 2;
}

extern "C" int rr_probe_mfma_f32(const void* A, const void* B, const void* C, void* D, int cases, void* stream) {
    if (cases <= 0 || !A || !B || !C || !D) return 1;
    hipLaunchKernelGGL(probe_f32_kernel, dim3(cases), dim3(64), 0, (hipStream_t)stream, (const float*)A,
                       (const float*)B, (const float*)C, (float*)D);
    return hipGetLastError() == hipSuccess ? 0 : 2;
}
