// Ceiling microbenchmarks for the roofline of the interpolation kernels:
// vector FMA issue rate, v_exp_f32 rate, a 1 exp : 4 FMA mix, and an HBM
// copy.  Built into libgmmpeak.so (measurement tooling, not part of the
// interpolation ABI); bench.py times the launches with events.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int kIters = 4096;

// 8 independent FMA chains per lane: kIters * 8 FMAs per lane
__global__ __launch_bounds__(256) void k_fma(float* out, float a, float b) {
  float x[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) x[i] = threadIdx.x * 0.001f + i;
  for (int it = 0; it < kIters; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i] = __builtin_fmaf(x[i], a, b);
  }
  float s = 0.0f;
#pragma unroll
  for (int i = 0; i < 8; ++i) s += x[i];
  if (s == 1.2345f) out[blockIdx.x] = s;  // keeps the work alive
}

// 8 independent exp2 chains per lane: kIters * 8 v_exp_f32 per lane
__global__ __launch_bounds__(256) void k_exp(float* out, float a) {
  (void)a;
  float x[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) x[i] = -(threadIdx.x & 7) * 0.01f - i * 0.1f;
  for (int it = 0; it < kIters; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i] = __builtin_amdgcn_exp2f(x[i]);
  }
  float s = 0.0f;
#pragma unroll
  for (int i = 0; i < 8; ++i) s += x[i];
  if (s == 1.2345f) out[blockIdx.x] = s;
}

// per iteration and chain: 1 exp2, 1 mul, 4 FMAs (the shape of the gather's
// per-pair work for a few channels)
__global__ __launch_bounds__(256) void k_mix(float* out, float a, float b) {
  float x[4], y[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    x[i] = -(threadIdx.x & 7) * 0.01f - i * 0.1f;
#pragma unroll
    for (int k = 0; k < 4; ++k) y[i][k] = 0.0f;
  }
  for (int it = 0; it < kIters; ++it) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float w = __builtin_amdgcn_exp2f(x[i] * a);
#pragma unroll
      for (int k = 0; k < 4; ++k) y[i][k] = __builtin_fmaf(w, b, y[i][k]);
      x[i] = y[i][0] * -1e-6f;
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int k = 0; k < 4; ++k) s += y[i][k];
  if (s == 1.2345f) out[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_copy(const float4* __restrict__ src, float4* __restrict__ dst,
                                              long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] = src[i];
}

// Streaming copy: each workgroup moves one contiguous span of kSpan float4s
// per trip, four loads of a thread in flight before its four stores, with
// non-temporal hints (the data is touched once).  n must be a multiple of
// 4 * 256 float4s.
constexpr int kSpan = 4 * 256;
typedef float f4v __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_copy_stream(const f4v* __restrict__ src,
                                                     f4v* __restrict__ dst, long long n) {
  for (long long base = (long long)blockIdx.x * kSpan; base < n; base += (long long)gridDim.x * kSpan) {
    f4v r[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) r[k] = __builtin_nontemporal_load(src + base + k * 256 + threadIdx.x);
#pragma unroll
    for (int k = 0; k < 4; ++k) __builtin_nontemporal_store(r[k], dst + base + k * 256 + threadIdx.x);
  }
}

// Read-only stream (a sum per thread; one store per workgroup keeps it alive).
__global__ __launch_bounds__(256) void k_read_stream(const f4v* __restrict__ src, float* out,
                                                     long long n) {
  f4v acc = {0.0f, 0.0f, 0.0f, 0.0f};
  for (long long base = (long long)blockIdx.x * kSpan; base < n; base += (long long)gridDim.x * kSpan) {
    f4v r[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) r[k] = __builtin_nontemporal_load(src + base + k * 256 + threadIdx.x);
#pragma unroll
    for (int k = 0; k < 4; ++k) acc += r[k];
  }
  const float s = acc.x + acc.y + acc.z + acc.w;
  if (s == 1.2345f) out[blockIdx.x & 1023] = s;
}

}  // namespace

extern "C" {

// which: 0 fma, 1 exp, 2 mix, 3 copy (grid-stride), 4 streaming copy,
// 5 streaming read.  blocks: workgroups of 256 threads (0 picks 8 per compute
// unit).  For the copies, n_float4 elements are copied from src to dst (4, 5:
// n_float4 a multiple of 1024).  Returns the number of lane operations (0-2)
// or bytes moved (3-5) one launch performs, or -1 on a launch error.
double gmm_peak_launch(int which, int blocks, void* out, const void* src, void* dst,
                       long long n_float4, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (blocks <= 0) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return -1.0;
    blocks = cus * 8;
  }
  const double lanes = (double)blocks * 256.0;
  switch (which) {
    case 0:
      hipLaunchKernelGGL(k_fma, dim3(blocks), dim3(256), 0, st, (float*)out, 0.999f, 0.001f);
      return hipGetLastError() == hipSuccess ? lanes * kIters * 8 : -1.0;
    case 1:
      hipLaunchKernelGGL(k_exp, dim3(blocks), dim3(256), 0, st, (float*)out, 0.5f);
      return hipGetLastError() == hipSuccess ? lanes * kIters * 8 : -1.0;
    case 2:
      hipLaunchKernelGGL(k_mix, dim3(blocks), dim3(256), 0, st, (float*)out, 0.5f, 0.25f);
      // per chain and iteration: mul + exp + 4 FMA + mul = 7 VALU instructions, 1 of them exp
      return hipGetLastError() == hipSuccess ? lanes * kIters * 4 : -1.0;
    case 3:
      hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, st, (const float4*)src, (float4*)dst,
                         n_float4);
      return hipGetLastError() == hipSuccess ? 32.0 * (double)n_float4 : -1.0;
    case 4:
      if (n_float4 % kSpan) return -1.0;
      hipLaunchKernelGGL(k_copy_stream, dim3(blocks), dim3(256), 0, st, (const f4v*)src,
                         (f4v*)dst, n_float4);
      return hipGetLastError() == hipSuccess ? 32.0 * (double)n_float4 : -1.0;
    case 5:
      if (n_float4 % kSpan) return -1.0;
      hipLaunchKernelGGL(k_read_stream, dim3(blocks), dim3(256), 0, st, (const f4v*)src,
                         (float*)out, n_float4);
      return hipGetLastError() == hipSuccess ? 16.0 * (double)n_float4 : -1.0;
    default:
      return -1.0;
  }
}

}  // extern "C"
