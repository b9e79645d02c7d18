// Spatial binning of the points: the counting sort that lets each output
// block find the points that can be "close enough" to it (paper, Section 2,
// the sentence after Eq. 2: only near points take part).
//
//   k_bin_zero        clear the per-bin counters and the per-image reach
//   k_bin_count       bin of every point, its arrival rank in the bin (atomic),
//                     per-image maximum of f32(radius*sigma)
//   k_bin_scan        exclusive prefix sum of the counts -> bin offsets
//   k_bin_scatter     every point index into its bin's segment (arrival order)
//   k_bin_sort_gather each bin's segment sorted by point index (so the order is
//                     the stable counting-sort order and does not depend on
//                     atomic timing), then the sorted point records
//                     (x, y, k = -log2(e)/(2 sigma^2), R2 = f32(f32(r sigma)^2))
//                     and values are gathered into bin order.
#include <climits>

#include "common.hpp"

namespace gmm {
namespace {

constexpr float kLog2e = 1.4426950408889634f;

__global__ void k_bin_zero(int* __restrict__ count, long long n, float* __restrict__ reach, int B) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long stride = (long long)gridDim.x * blockDim.x;
  for (long long t = i; t < n; t += stride) count[t] = 0;
  if (i < B) reach[i] = 0.0f;
}

__device__ inline int bin_coord(float c, float inv_tile, int nmax) {
  // floor(c / tile) clamped to [0, nmax-1]; c * (1/tile) is exact for a
  // power-of-two tile.  NaN and negative values land in bin 0.
  float f = floorf(c * inv_tile);
  if (!(f >= 0.0f)) return 0;
  if (f >= (float)(nmax - 1)) return nmax - 1;
  return (int)f;
}

__global__ __launch_bounds__(256) void k_bin_count(
    const float2* __restrict__ pos, const float* __restrict__ sigma, int N, int per_point,
    float radius, float inv_tile, int nbx, int nby, int nb, int* __restrict__ count,
    int* __restrict__ slot, int* __restrict__ binof, float* __restrict__ reach) {
  const int b = blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  float rs = 0.0f;
  if (j < N) {
    const size_t gj = (size_t)b * N + j;
    float2 p = pos[gj];
    int bx = bin_coord(p.x, inv_tile, nbx);
    int by = bin_coord(p.y, inv_tile, nby);
    int bin = by * nbx + bx;
    binof[gj] = bin;
    slot[gj] = atomicAdd(&count[(size_t)b * nb + bin], 1);
    float s = per_point ? sigma[gj] : sigma[b];
    rs = __fmul_rn(radius, s);
    if (!(rs >= 0.0f)) rs = 0.0f;  // caller contract violated; keep the reach sane
  }
  // wave maximum, then one atomic per wave (max of non-negative floats is an
  // unsigned max of their bit patterns)
  for (int o = 32; o > 0; o >>= 1) rs = fmaxf(rs, __shfl_xor(rs, o));
  if ((threadIdx.x & 63) == 0 && rs > 0.0f)
    atomicMax(reinterpret_cast<unsigned int*>(reach) + b, __float_as_uint(rs));
}

// One workgroup of 1024 threads per image: exclusive scan of count[b, 0..nb)
// into offset[b, 0..nb], processed in tiles of 4096 counts (int4 per thread).
__global__ __launch_bounds__(1024) void k_bin_scan(const int* __restrict__ count, int nb,
                                                   int* __restrict__ offset) {
  __shared__ int wsum[16];
  __shared__ int carry_s;
  const int b = blockIdx.x;
  const int* c = count + (size_t)b * nb;
  int* o = offset + (size_t)b * (nb + 1);
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  int carry = 0;
  for (int base = 0; base < nb; base += 4096) {
    int v[4];
    int i0 = base + tid * 4;
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = (i0 + q < nb) ? c[i0 + q] : 0;
    int local = v[0] + v[1] + v[2] + v[3];
    // inclusive wave scan of the per-thread sums
    int incl = local;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      int t = __shfl_up(incl, d);
      if (lane >= d) incl += t;
    }
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    if (wid == 0) {
      int s = lane < 16 ? wsum[lane] : 0;
      int si = s;
#pragma unroll
      for (int d = 1; d < 16; d <<= 1) {
        int t = __shfl_up(si, d);
        if (lane >= d) si += t;
      }
      if (lane < 16) wsum[lane] = si - s;  // exclusive prefix of wave sums
      if (lane == 15) carry_s = si;        // tile total
    }
    __syncthreads();
    int run = carry + wsum[wid] + incl - local;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (i0 + q < nb) o[i0 + q] = run;
      run += v[q];
    }
    carry += carry_s;
    __syncthreads();
  }
  if (tid == 0) o[nb] = carry;
}

__global__ __launch_bounds__(256) void k_bin_scatter(const int* __restrict__ binof,
                                                     const int* __restrict__ slot,
                                                     const int* __restrict__ offset, int N, int nb,
                                                     int* __restrict__ tmp) {
  const int b = blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const size_t gj = (size_t)b * N + j;
  int dest = offset[(size_t)b * (nb + 1) + binof[gj]] + slot[gj];
  tmp[(size_t)b * N + dest] = j;
}

// ---------------------------------------------------------------------------
// Per-bin sort (one wavefront per bin) and record gather
// ---------------------------------------------------------------------------

constexpr int kLdsSort = 2048;  // ints of LDS per wavefront for in-LDS sorting

// Orders the LDS and global accesses of one wavefront's lanes (the sort
// exchanges data between lanes through LDS and through global memory).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Bitonic sort of 64 values held one per lane, ascending by lane.
__device__ inline int wave_sort64(int v, int lane) {
#pragma unroll
  for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      int other = __shfl_xor(v, j);
      bool asc = (lane & k) == 0;
      bool lower = (lane & j) == 0;
      v = (lower == asc) ? min(v, other) : max(v, other);
    }
  }
  return v;
}

// Bitonic sort of p (power of two, <= kLdsSort) ints in LDS by one wavefront.
__device__ inline void lds_bitonic(int* a, int p, int lane) {
  for (int k = 2; k <= p; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      const int jl = __builtin_ctz(j);
      for (int t = lane; t < (p >> 1); t += 64) {
        int i = ((t >> jl) << (jl + 1)) | (t & (j - 1));
        int l = i + j;
        int ai = a[i], al = a[l];
        bool asc = (i & k) == 0;
        if ((ai > al) == asc) { a[i] = al; a[l] = ai; }
      }
      wave_sync();
    }
  }
}

// Sorts seg[0..n) ascending, leaving the result in dst[0..n).  seg is used as
// scratch.  Values are distinct point indices.
__device__ void wave_sort_segment(int* seg, int* dst, int n, int* lds, int lane) {
  if (n <= 64) {
    int v = lane < n ? seg[lane] : INT_MAX;
    v = wave_sort64(v, lane);
    if (lane < n) dst[lane] = v;
    return;
  }
  // 1) sort runs of kLdsSort in LDS, written back in place to seg
  for (int r0 = 0; r0 < n; r0 += kLdsSort) {
    int m = min(kLdsSort, n - r0);
    int p = 64;
    while (p < m) p <<= 1;
    for (int i = lane; i < p; i += 64) lds[i] = i < m ? seg[r0 + i] : INT_MAX;
    wave_sync();
    lds_bitonic(lds, p, lane);
    int* out = (n <= kLdsSort) ? dst : seg;
    for (int i = lane; i < m; i += 64) out[r0 + i] = lds[i];
    __threadfence_block();
    wave_sync();
  }
  if (n <= kLdsSort) return;
  // 2) merge runs pairwise in global memory (merge by rank: the destination of
  //    an element is its index in its run plus its rank in the other run)
  int* src = seg;
  int* out = dst;
  for (int run = kLdsSort; run < n; run <<= 1) {
    for (int a0 = 0; a0 < n; a0 += 2 * run) {
      int alen = min(run, n - a0);
      int b0 = a0 + alen;
      int blen = min(run, n - b0);
      if (blen <= 0) {
        for (int i = lane; i < alen; i += 64) out[a0 + i] = src[a0 + i];
        continue;
      }
      for (int i = lane; i < alen + blen; i += 64) {
        bool inA = i < alen;
        int v = inA ? src[a0 + i] : src[b0 + i - alen];
        const int* other = inA ? src + b0 : src + a0;
        int olen = inA ? blen : alen;
        int lo = 0, hi = olen;  // count of other-run elements < v
        while (lo < hi) {
          int mid = (lo + hi) >> 1;
          if (other[mid] < v) lo = mid + 1; else hi = mid;
        }
        int idx = inA ? i : i - alen;
        out[a0 + idx + lo] = v;
      }
    }
    __threadfence_block();
    wave_sync();
    int* t = src; src = out; out = t;
  }
  if (src != dst) {
    for (int i = lane; i < n; i += 64) dst[i] = src[i];
  }
}

__global__ __launch_bounds__(256) void k_bin_sort_gather(
    const float2* __restrict__ pos, const float* __restrict__ sigma, const float* __restrict__ values,
    int B, int N, int C, int CS, int nb, int per_point, float radius,
    const int* __restrict__ offset, int* __restrict__ tmp, int* __restrict__ perm,
    float4* __restrict__ geo, float* __restrict__ col) {
  __shared__ int lds_all[4][kLdsSort];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const long long gbin = (long long)blockIdx.x * 4 + wid;
  if (gbin >= (long long)B * nb) return;
  const int b = (int)(gbin / nb);
  const int k = (int)(gbin % nb);
  const int* ob = offset + (size_t)b * (nb + 1);
  const int s = ob[k];
  const int n = ob[k + 1] - s;
  if (n <= 0) return;
  const size_t base = (size_t)b * N + s;
  wave_sort_segment(tmp + base, perm + base, n, lds_all[wid], lane);
  __threadfence_block();
  wave_sync();
  const float* vb = values + (size_t)b * N * C;
  for (int i = lane; i < n; i += 64) {
    const int j = perm[base + i];
    const size_t gj = (size_t)b * N + j;
    float2 p = pos[gj];
    float sg = per_point ? sigma[gj] : sigma[b];
    float rs = __fmul_rn(radius, sg);
    float R2 = __fmul_rn(rs, rs);
    float kk = -0.5f * kLog2e / __fmul_rn(sg, sg);
    geo[base + i] = make_float4(p.x, p.y, kk, R2);
    float* cd = col + (base + i) * CS;
    const float* cs = vb + (size_t)j * C;
    for (int c = 0; c < CS; ++c) cd[c] = c < C ? cs[c] : 0.0f;
  }
}

inline unsigned grid1(long long n, int block) { return (unsigned)((n + block - 1) / block); }

}  // namespace

hipError_t launch_binning(const Geometry& g, const float* pos, const float* sigma,
                          const float* values, const Views& v, hipStream_t st) {
  const long long ncount = (long long)g.B * g.nb;
  {
    long long n = ncount > g.B ? ncount : g.B;
    unsigned blocks = grid1(n, 256);
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_bin_zero, dim3(blocks), dim3(256), 0, st, v.count, ncount, v.reach, g.B);
  }
  const float inv_tile = 1.0f / (float)g.T;
  if (g.N > 0) {
    hipLaunchKernelGGL(k_bin_count, dim3(grid1(g.N, 256), g.B), dim3(256), 0, st,
                       reinterpret_cast<const float2*>(pos), sigma, g.N, g.per_point, g.radius,
                       inv_tile, g.nbx, g.nby, g.nb, v.count, v.slot, v.binof, v.reach);
  }
  hipLaunchKernelGGL(k_bin_scan, dim3(g.B), dim3(1024), 0, st, v.count, g.nb, v.offset);
  if (g.N > 0) {
    hipLaunchKernelGGL(k_bin_scatter, dim3(grid1(g.N, 256), g.B), dim3(256), 0, st, v.binof,
                       v.slot, v.offset, g.N, g.nb, v.tmp);
    hipLaunchKernelGGL(k_bin_sort_gather, dim3(grid1(ncount, 4)), dim3(256), 0, st,
                       reinterpret_cast<const float2*>(pos), sigma, values, g.B, g.N, g.C, g.CS,
                       g.nb, g.per_point, g.radius, v.offset, v.tmp, v.perm, v.geo, v.col);
  }
  return hipGetLastError();
}

}  // namespace gmm
