// Achievable-peak probes: what this device sustains on the matrix cores and
// on HBM, so that measured kernels can be reported against the device's own
// ceiling as well as the published one.
//
// * mfma16_probe: each wave issues back-to-back independent
//   v_mfma_f32_16x16x32_f16 (four accumulator chains, operands in
//   registers), the instruction the 16-bit assembly runs on.
// * mfma64_probe: the same with v_mfma_f64_16x16x4_f64 (FP64 assembly, J).
// * copy_probe: a 16-byte-per-lane streaming copy, bytes read + written.
#include "tai_internal.h"

namespace tai {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));

// independent accumulator chains per wave (two waves per SIMD); each chain
// has its own A operand
constexpr int kChains16 = 4, kChains64 = 8;

__global__ void __launch_bounds__(256) mfma16_probe(int iters, float* out) {
  const int lane = threadIdx.x & 63;
  v8h a[kChains16], b;
#pragma unroll
  for (int i = 0; i < 8; ++i) b[i] = (_Float16)(0.001f * (float)((lane * 3 + i) & 7));
#pragma unroll
  for (int c = 0; c < kChains16; ++c)
#pragma unroll
    for (int i = 0; i < 8; ++i) a[c][i] = (_Float16)(0.001f * (float)((lane + i + c) & 7));
  v4f acc[kChains16];
#pragma unroll
  for (int c = 0; c < kChains16; ++c) acc[c] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < kChains16; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[c], b, acc[c], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kChains16; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void __launch_bounds__(256) mfma64_probe(int iters, float* out) {
  const int lane = threadIdx.x & 63;
  const double b = 0.001 * (double)((lane * 3) & 7);
  double a[kChains64];
#pragma unroll
  for (int c = 0; c < kChains64; ++c) a[c] = 0.001 * (double)((lane + c) & 7);
  v4d acc[kChains64];
#pragma unroll
  for (int c = 0; c < kChains64; ++c) acc[c] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < kChains64; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[c], b, acc[c], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < kChains64; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[blockIdx.x * blockDim.x + threadIdx.x] = (float)s;
}

__global__ void __launch_bounds__(256) copy_probe(const uint4* __restrict__ src, uint4* __restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

}  // namespace

hipError_t launch_probe(int what, int cus, float* out, const void* src, void* dst, int64_t n16, int iters,
                        hipStream_t s) {
  if (what == 0) {
    hipLaunchKernelGGL(mfma16_probe, dim3(2 * cus), dim3(256), 0, s, iters, out);
  } else if (what == 1) {
    hipLaunchKernelGGL(mfma64_probe, dim3(2 * cus), dim3(256), 0, s, iters, out);
  } else {
    hipLaunchKernelGGL(copy_probe, dim3(8 * cus), dim3(256), 0, s, static_cast<const uint4*>(src),
                       static_cast<uint4*>(dst), n16);
  }
  return hipGetLastError();
}

double probe_work(int what, int cus, int64_t n16, int iters) {
  const double waves = 2.0 * cus * 4.0;
  if (what == 0) return waves * iters * kChains16 * (2.0 * 16 * 16 * 32);  // flops
  if (what == 1) return waves * iters * kChains64 * (2.0 * 16 * 16 * 4);   // flops
  return 2.0 * 16.0 * (double)n16;                                       // bytes read + written
}

}  // namespace tai
