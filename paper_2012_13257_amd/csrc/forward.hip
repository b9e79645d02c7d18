// Forward gather (paper, Section 2, Eq. 1 and Eq. 2): every output pixel is
// the weighted mean of the values of the points within radius*sigma_j of it.
//
// Work decomposition: one wavefront owns an 8x8 block of output pixels (one
// pixel per lane); a 256-thread workgroup covers 2x2 blocks.  The wavefront
// walks the bins that can hold points reaching its block (one contiguous
// range of the bin-sorted records per bin row), 64 candidates at a time:
// each lane tests one candidate's disk against the block, a ballot collects
// the hits, and the hits are then consumed one by one with the candidate's
// record held in scalar registers (uniform loads), every lane evaluating the
// radius test and the weight for its own pixel.  Accumulation is float32 in
// the fixed bin/record order, so the result is deterministic.  There is no
// dense contraction here, so no matrix cores are used; the loop is bound by
// vector ALU issue (the exp2 and the per-channel FMAs).
#include "common.hpp"

namespace gmm {
namespace {

__device__ inline int bin_coord(float c, float inv_tile, int nmax) {
  float f = floorf(c * inv_tile);
  if (!(f >= 0.0f)) return 0;
  if (f >= (float)(nmax - 1)) return nmax - 1;
  return (int)f;
}

// Workgroups are dispatched round-robin over the 8 XCDs; give every XCD a
// contiguous range of tiles so that neighbouring tiles (which read the same
// halo records) share one L2.
__device__ inline int xcd_remap(int bid, int nblocks) {
  const int xcd = bid & 7, idx = bid >> 3;
  const int per = nblocks >> 3, rem = nblocks & 7;
  return xcd * per + min(xcd, rem) + idx;
}

template <int CT>
__global__ __launch_bounds__(256) void k_forward(
    const float4* __restrict__ geo, const float* __restrict__ col, const int* __restrict__ offset,
    const float* __restrict__ reach, int N, int C, int H, int W, float inv_tile, int nbx, int nby,
    int nb, int wgx, int wg_per_image, int total_wg, float* __restrict__ out,
    float* __restrict__ Zout) {
  constexpr int CS = CT < 4 ? 4 : CT;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int tile = xcd_remap(blockIdx.x, total_wg);
  const int b = tile / wg_per_image;
  const int rem = tile - b * wg_per_image;
  const int ty = rem / wgx, tx = rem - ty * wgx;
  const int u0 = (2 * tx + (wid & 1)) * kBlockSide;
  const int v0 = (2 * ty + (wid >> 1)) * kBlockSide;
  if (u0 >= W || v0 >= H) return;
  const int ue = min(u0 + kBlockSide - 1, W - 1);
  const int ve = min(v0 + kBlockSide - 1, H - 1);
  const int u = u0 + (lane & 7), v = v0 + (lane >> 3);
  const float fu = (float)u, fv = (float)v;

  // conservative reach of any point of this image (see the design notes:
  // covers the float32 rounding of the radius test and of the bin bounds)
  // (float math runs on the vector ALU; readfirstlane moves the wave-uniform
  // results to scalar registers so the record loads below are scalar loads)
  const float Rh = reach[b] * (1.0f + 0x1p-10f) + 0x1p-6f;
  const int bx_lo = __builtin_amdgcn_readfirstlane(bin_coord((float)u0 - Rh, inv_tile, nbx));
  const int bx_hi = __builtin_amdgcn_readfirstlane(bin_coord((float)ue + Rh, inv_tile, nbx));
  const int by_lo = __builtin_amdgcn_readfirstlane(bin_coord((float)v0 - Rh, inv_tile, nby));
  const int by_hi = __builtin_amdgcn_readfirstlane(bin_coord((float)ve + Rh, inv_tile, nby));
  const int* ob = offset + (size_t)b * (nb + 1);
  const size_t gbase = (size_t)b * N;
  const float4* gb = geo + gbase;
  const float* cb = col + gbase * CS;

  float Z = 0.0f;
  float acc[CT];
#pragma unroll
  for (int k = 0; k < CT; ++k) acc[k] = 0.0f;

  for (int by = by_lo; by <= by_hi; ++by) {
    const int s = __builtin_amdgcn_readfirstlane(ob[by * nbx + bx_lo]);
    const int e = __builtin_amdgcn_readfirstlane(ob[by * nbx + bx_hi + 1]);
    for (int c0 = s; c0 < e; c0 += 64) {
      const int jc = c0 + lane;
      bool hit = false;
      if (jc < e) {
        const float4 g = gb[jc];
        const float ex = fmaxf(fmaxf((float)u0 - g.x, g.x - (float)ue), 0.0f);
        const float ey = fmaxf(fmaxf((float)v0 - g.y, g.y - (float)ve), 0.0f);
        hit = ex * ex + ey * ey <= g.w * 1.001f + 1e-6f;
      }
      unsigned long long mask = __ballot(hit);
      while (mask) {
        const int bit = __builtin_ctzll(mask);
        mask &= mask - 1;
        const int j = __builtin_amdgcn_readfirstlane(c0 + bit);
        const float4 g = gb[j];
        float cc[CT];
        if constexpr (CT == 1) {
          cc[0] = cb[(size_t)j * CS];
        } else if constexpr (CT == 2) {
          const float2 t = *reinterpret_cast<const float2*>(cb + (size_t)j * CS);
          cc[0] = t.x; cc[1] = t.y;
        } else {
          const float4* cp = reinterpret_cast<const float4*>(cb + (size_t)j * CS);
#pragma unroll
          for (int q = 0; q < (CT + 3) / 4; ++q) {
            const float4 t = cp[q];
            cc[4 * q] = t.x;
            if (4 * q + 1 < CT) cc[4 * q + 1] = t.y;
            if (4 * q + 2 < CT) cc[4 * q + 2] = t.z;
            if (4 * q + 3 < CT) cc[4 * q + 3] = t.w;
          }
        }
        // radius test exactly as specified: float32, every operation rounded
        const float dx = fu - g.x;
        const float dy = fv - g.y;
        const float d2 = dx * dx + dy * dy;
        float w = __builtin_amdgcn_exp2f(d2 * g.z);
        w = (d2 <= g.w) ? w : 0.0f;
        Z += w;
#pragma unroll
        for (int k = 0; k < CT; ++k) acc[k] = __builtin_fmaf(w, cc[k], acc[k]);
      }
    }
  }

  if (u <= ue && v <= ve) {
    const size_t HW = (size_t)H * W;
    const size_t pix = (size_t)v * W + u;
    float* ob_out = out + (size_t)b * C * HW + pix;
#pragma unroll
    for (int k = 0; k < CT; ++k) {
      if (k < C) ob_out[k * HW] = Z > 0.0f ? acc[k] / Z : 0.0f;
    }
    if (Zout) Zout[(size_t)b * HW + pix] = Z;
  }
}

template <int CT>
hipError_t launch_forward_t(const Geometry& g, const Views& v, float* out, hipStream_t st) {
  const int wgx = (g.bx_blocks + 1) / 2;
  const int wgy = (g.by_blocks + 1) / 2;
  const int per_image = wgx * wgy;
  const long long total = (long long)per_image * g.B;
  if (total >= (1LL << 31)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_forward<CT>, dim3((unsigned)total), dim3(256), 0, st, v.geo, v.col,
                     v.offset, v.reach, g.N, g.C, g.H, g.W, 1.0f / (float)g.T, g.nbx, g.nby, g.nb,
                     wgx, per_image, (int)total, out, v.Z);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_forward(const Geometry& g, const Views& v, float* out, hipStream_t st) {
  switch (g.CT) {
    case 1: return launch_forward_t<1>(g, v, out, st);
    case 2: return launch_forward_t<2>(g, v, out, st);
    case 3: return launch_forward_t<3>(g, v, out, st);
    case 4: return launch_forward_t<4>(g, v, out, st);
    case 8: return launch_forward_t<8>(g, v, out, st);
    case 16: return launch_forward_t<16>(g, v, out, st);
    case 32: return launch_forward_t<32>(g, v, out, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace gmm
