// Backward (adjoint) of the Gaussian-mixture interpolation.  The paper has a
// hand-written backward kernel for its point-position optimisation (Section
// 3.3) but does not write the formulas out; they follow from Eq. 1 by the
// quotient rule.  With G = dL/dout, alpha_i = 1/Z_i, beta_i = alpha_i
// sum_k G_ik out_ik and A_ij = alpha_i sum_k G_ik c_jk - beta_i:
//   dL/dc_jk     = sum_i w_ij alpha_i G_ik
//   dL/dx_j      = sum_i A_ij w_ij (u_i - x_j) / sigma_j^2      (y likewise)
//   dL/dsigma_j  = sum_i A_ij w_ij d2_ij / sigma_j^3
// over the pixels i inside the radius of point j.
//
//   k_bwd_pixel   per pixel: G'_ik = G_ik / Z_i and beta_i, packed per pixel
//                 so the point loop reads one record per pixel
//   k_bwd_point   one thread per point (bin-sorted order, so neighbouring
//                 lanes read neighbouring pixels): walks the bounding box of its
//                 disk, repeats the forward's radius test exactly, recomputes
//                 w_ij instead of storing it, accumulates in registers and
//                 writes the gradients at the point's original index (no
//                 atomics, deterministic)
//   k_bwd_sigma_sum  shared sigma: fixed-order sum of the per-workgroup partial
//                 sums of dL/dsigma_j
#include "common.hpp"

namespace gmm {
namespace {

template <int CT>
__global__ __launch_bounds__(256) void k_bwd_pixel(const float* __restrict__ Z,
                                                   const float* __restrict__ out,
                                                   const float* __restrict__ G, int C, int HW,
                                                   long long total, float* __restrict__ prec) {
  constexpr int CP = (CT + 1 + 3) / 4 * 4;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const long long b = i / HW;
  const long long pix = i - b * HW;
  const float z = Z[i];
  float rec[CP];
#pragma unroll
  for (int k = 0; k < CP; ++k) rec[k] = 0.0f;
  if (z > 0.0f) {
    const float a = 1.0f / z;
    float beta = 0.0f;
#pragma unroll
    for (int k = 0; k < CT; ++k) {
      if (k < C) {
        const size_t idx = ((size_t)b * C + k) * HW + pix;
        const float gk = G[idx];
        rec[k] = gk * a;
        beta = __builtin_fmaf(gk, out[idx], beta);
      }
    }
    rec[CT] = beta * a;
  }
  float4* dst = reinterpret_cast<float4*>(prec + (size_t)i * CP);
#pragma unroll
  for (int q = 0; q < CP / 4; ++q)
    dst[q] = make_float4(rec[4 * q], rec[4 * q + 1], rec[4 * q + 2], rec[4 * q + 3]);
}

template <int CT>
__global__ __launch_bounds__(256) void k_bwd_point(
    const float4* __restrict__ geo, const float* __restrict__ col, const int* __restrict__ perm,
    const float* __restrict__ sigma, const float* __restrict__ prec, int N, int C, int H, int W,
    int per_point, float radius, float* __restrict__ grad_pos, float* __restrict__ grad_sigma,
    float* __restrict__ grad_values, float* __restrict__ gpart) {
  constexpr int CS = CT < 4 ? 4 : CT;
  constexpr int CP = (CT + 1 + 3) / 4 * 4;
  __shared__ float red[4];
  const int b = blockIdx.y;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  float gsig = 0.0f;
  if (t < N) {
    const size_t gt = (size_t)b * N + t;
    const float4 g = geo[gt];
    float cc[CT];
#pragma unroll
    for (int k = 0; k < CT; ++k) cc[k] = col[gt * CS + k];
    const int j = perm[gt];
    const size_t gj = (size_t)b * N + j;
    const float sg = per_point ? sigma[gj] : sigma[b];
    const float rs = __fmul_rn(radius, sg);
    const float Rh = rs * (1.0f + 0x1p-10f) + 0x1p-6f;
    // bounding box of the disk, clipped to the image (float clamps drop NaN)
    const float fulo = fminf(fmaxf(ceilf(g.x - Rh), 0.0f), (float)W);
    const float fuhi = fmaxf(fminf(floorf(g.x + Rh), (float)(W - 1)), -1.0f);
    const float fvlo = fminf(fmaxf(ceilf(g.y - Rh), 0.0f), (float)H);
    const float fvhi = fmaxf(fminf(floorf(g.y + Rh), (float)(H - 1)), -1.0f);
    const int ulo = (int)fulo, uhi = (int)fuhi, vlo = (int)fvlo, vhi = (int)fvhi;
    float gx = 0.0f, gy = 0.0f, gs = 0.0f;
    float gc[CT];
#pragma unroll
    for (int k = 0; k < CT; ++k) gc[k] = 0.0f;
    const float* pb = prec + (size_t)b * H * W * CP;
    for (int v = vlo; v <= vhi; ++v) {
      const float dy = (float)v - g.y;
      const float dyy = dy * dy;
      const float* prow = pb + (size_t)v * W * CP;
      for (int u = ulo; u <= uhi; ++u) {
        const float dx = (float)u - g.x;
        const float d2 = dx * dx + dyy;
        if (d2 <= g.w) {
          const float w = __builtin_amdgcn_exp2f(d2 * g.z);
          const float4* rp = reinterpret_cast<const float4*>(prow + (size_t)u * CP);
          float rec[CP];
#pragma unroll
          for (int q = 0; q < CP / 4; ++q) {
            const float4 r4 = rp[q];
            rec[4 * q] = r4.x; rec[4 * q + 1] = r4.y; rec[4 * q + 2] = r4.z; rec[4 * q + 3] = r4.w;
          }
          float A = -rec[CT];
#pragma unroll
          for (int k = 0; k < CT; ++k) {
            A = __builtin_fmaf(rec[k], cc[k], A);
            gc[k] = __builtin_fmaf(w, rec[k], gc[k]);
          }
          const float tA = A * w;
          gx = __builtin_fmaf(tA, dx, gx);
          gy = __builtin_fmaf(tA, dy, gy);
          gs = __builtin_fmaf(tA, d2, gs);
        }
      }
    }
    const float inv_s2 = 1.0f / (sg * sg);
    if (grad_pos) {
      reinterpret_cast<float2*>(grad_pos)[gj] = make_float2(gx * inv_s2, gy * inv_s2);
    }
    gsig = gs * inv_s2 / sg;
    if (grad_sigma && per_point) grad_sigma[gj] = gsig;
    if (grad_values) {
#pragma unroll
      for (int k = 0; k < CT; ++k)
        if (k < C) grad_values[gj * C + k] = gc[k];
    }
  }
  if (!per_point && grad_sigma) {
    // fixed-order workgroup sum of dL/dsigma_j
    for (int o = 32; o > 0; o >>= 1) gsig += __shfl_xor(gsig, o);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = gsig;
    __syncthreads();
    if (threadIdx.x == 0)
      gpart[(size_t)b * gridDim.x + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
  }
}

__global__ __launch_bounds__(256) void k_bwd_sigma_sum(const float* __restrict__ gpart, int groups,
                                                       float* __restrict__ grad_sigma) {
  __shared__ float red[4];
  const int b = blockIdx.x;
  float s = 0.0f;
  for (int i = threadIdx.x; i < groups; i += 256) s += gpart[(size_t)b * groups + i];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = s;
  __syncthreads();
  if (threadIdx.x == 0) grad_sigma[b] = (red[0] + red[1]) + (red[2] + red[3]);
}

template <int CT>
hipError_t launch_backward_t(const Geometry& g, const float* sigma, const float* out,
                             const float* grad_out, float* grad_pos, float* grad_sigma,
                             float* grad_values, const Views& v, hipStream_t st) {
  const long long total = (long long)g.B * g.H * g.W;
  hipLaunchKernelGGL(k_bwd_pixel<CT>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, v.Z,
                     out, grad_out, g.C, g.H * g.W, total, v.prec);
  const int groups = bwd_groups_per_image(g);
  if (g.N > 0) {
    hipLaunchKernelGGL(k_bwd_point<CT>, dim3(groups, g.B), dim3(256), 0, st, v.geo, v.col, v.perm,
                       sigma, v.prec, g.N, g.C, g.H, g.W, g.per_point, g.radius, grad_pos,
                       grad_sigma, grad_values, v.gpart);
  }
  if (!g.per_point && grad_sigma) {
    // with N = 0 there are no partial sums and the kernel writes zeros
    hipLaunchKernelGGL(k_bwd_sigma_sum, dim3(g.B), dim3(256), 0, st, v.gpart,
                       g.N > 0 ? groups : 0, grad_sigma);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_backward(const Geometry& g, const float* sigma, const float* out,
                           const float* grad_out, float* grad_pos, float* grad_sigma,
                           float* grad_values, const Views& v, hipStream_t st) {
  switch (g.CT) {
#define GMM_CASE(n) \
    case n: return launch_backward_t<n>(g, sigma, out, grad_out, grad_pos, grad_sigma, grad_values, v, st);
    GMM_CASE(1) GMM_CASE(2) GMM_CASE(3) GMM_CASE(4) GMM_CASE(8) GMM_CASE(16) GMM_CASE(32)
#undef GMM_CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace gmm
