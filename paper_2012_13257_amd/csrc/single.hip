// Single-call path: one launch per phase over every image of one problem
// (grid.y = image, or a flattened XCD-aware grid for the forward gather).
#include <algorithm>

#include "kernels.hpp"

namespace gmm {
namespace {

// Radix tiles are dealt to workgroups XCD by XCD: workgroup i runs on XCD
// i % 8 and takes tile (i % 8) * per8 + i / 8 (per8 = ceil(ntiles / 8)), so
// each XCD covers one contiguous eighth of the tiles.  Neighbouring tiles
// write neighbouring words of the digit histograms and neighbouring runs of
// the scatter's output; on one XCD those shared cache lines are merged in its
// L2 instead of being written back in parts by two (the scatter is ~10%
// faster, the key pass ~10%).
__device__ inline int xcd_tile(int per8) { return (blockIdx.x & 7) * per8 + (blockIdx.x >> 3); }

template <int ST>
__global__ __launch_bounds__(256) void k_bin_keys(ImageView v0, int per8) {
  __shared__ float red4[4];
  __shared__ int lh[kMaxDigits];
  const int tile = xcd_tile(per8);
  if (tile >= v0.ntiles) return;
  dev::bin_keys<ST>(image_of(v0, blockIdx.y), tile, red4, lh);
}

__global__ __launch_bounds__(256) void k_radix_hist(ImageView v0, int p, int per8) {
  __shared__ int lh[256];
  const int tile = xcd_tile(per8);
  if (tile >= v0.ntiles) return;
  dev::radix_hist(image_of(v0, blockIdx.y), p, tile, lh);
}

__global__ __launch_bounds__(256) void k_radix_scan(ImageView v0, int p) {
  __shared__ int tmp4[4];
  dev::radix_scan_digit(image_of(v0, blockIdx.y), p, blockIdx.x, tmp4);
}

__global__ __launch_bounds__(256) void k_radix_scan_small(ImageView v0, int p) {
  dev::radix_scan_digits_small(image_of(v0, blockIdx.y), p, blockIdx.x);
}

template <bool kWide, int ST, int kDig>
__global__ __launch_bounds__(256) void k_radix_scatter(ImageView v0, int p, int per8) {
  __shared__ int lds[dev::radix_scatter_lds_ints<kDig>()];
  const int tile = xcd_tile(per8);
  if (tile >= v0.ntiles) return;
  dev::radix_scatter<kWide, ST, kDig>(image_of(v0, blockIdx.y), p, tile, lds);
}

template <int ST>
__global__ __launch_bounds__(256) void k_place_wide(ImageView v0) {
  dev::place_wide<ST>(image_of(v0, blockIdx.y), blockIdx.x);
}

// also clears the counters of the forward's work order (fplan, 64 ints)
__global__ __launch_bounds__(256) void k_bin_finish(ImageView v0, int* fplan) {
  __shared__ float red4[4];
  if (fplan && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x < 64) fplan[threadIdx.x] = 0;
  dev::bin_finish(image_of(v0, blockIdx.y), blockIdx.x, red4);
}

// Work order of the forward, heaviest first.  A heavy unit (unit_is_heavy) is
// split into two work items (blocks 0-1 and 2-3, two wavefronts per block),
// any other unit is one item (one wavefront per block).  Item number = (image * units + unit) * 4 + mode;
// each item goes to the list of its cost class (floor(log2) + 1 of its
// candidate count, 0 for none).  fplan[0..31]: list sizes, lists from
// fplan + 64 (kPlanBuckets x 2 * total).  A workgroup ranks its items per
// class in LDS and reserves each class's slots with one global atomic.  The
// order inside a list follows the atomics and varies from run to run; the
// results do not depend on it (each item computes its pixels on its own).
__device__ inline int cost_class(int cost) {
  return cost == 0 ? 0 : min(kPlanBuckets - 1, 32 - __clz(cost));
}
// Four threads per unit (one per block, lanes 4u .. 4u+3 of a wavefront),
// 64 units per workgroup; the first thread of a unit classifies it.
__global__ __launch_bounds__(256) void k_fwd_plan(ImageView v0, int units, int total, int* fplan) {
  __shared__ int cnt[kPlanBuckets], base[kPlanBuckets];
  const int id = blockIdx.x * 64 + (threadIdx.x >> 2), sb = threadIdx.x & 3;
  if (threadIdx.x < kPlanBuckets) cnt[threadIdx.x] = 0;
  __syncthreads();
  int mine = 0;
  if (id < total) {
    const int b = id / units;
    mine = dev::block_candidates(image_of(v0, b), id - b * units, sb);
  }
  // the unit's four counts in every one of its threads (id is the same for
  // the four lanes, so all four take part in the shuffles)
  int c[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) c[k] = __shfl(mine, (threadIdx.x & 63 & ~3) + k);
  int cls[2] = {-1, -1}, rank[2] = {0, 0}, item[2] = {0, 0};
  if (id < total && sb == 0) {
    const int sum = c[0] + c[1] + c[2] + c[3];
    if (dev::unit_is_heavy(c)) {
      cls[0] = cost_class(c[0] + c[1]);
      cls[1] = cost_class(c[2] + c[3]);
      item[0] = id * 4 + 1;
      item[1] = id * 4 + 2;
    } else {
      cls[0] = cost_class(sum);
      item[0] = id * 4;
    }
    for (int k = 0; k < 2; ++k)
      if (cls[k] >= 0) rank[k] = atomicAdd(&cnt[cls[k]], 1);
  }
  __syncthreads();
  if (threadIdx.x < kPlanBuckets && cnt[threadIdx.x] > 0)
    base[threadIdx.x] = atomicAdd(&fplan[threadIdx.x], cnt[threadIdx.x]);
  __syncthreads();
  for (int k = 0; k < 2; ++k)
    if (cls[k] >= 0) fplan[64 + (size_t)cls[k] * 2 * total + base[cls[k]] + rank[k]] = item[k];
}

// Forward gather.  Up to 4 channels: workgroup i takes the i-th unit of the
// plan's work order, so the dispatcher starts the heaviest units first and
// fills in the light ones as compute units free up (a unit's result does not
// depend on which workgroup computes it or when).  More channels: one
// workgroup per 16x16 tile, a wavefront per 8x8 block.
template <int CT, int KV, int ST>
__global__ __launch_bounds__(256) void k_forward_lpt(ImageView v0, int units, int total,
                                                     const int* fplan) {
  __shared__ float4 s_rec[dev::fwd_quarter_lds_f4<CT>()];
  const int lane = threadIdx.x & 63;
  // lane l < 32: work items in the classes 31 .. 31 - l (heaviest first)
  int incl = lane < kPlanBuckets ? fplan[kPlanBuckets - 1 - lane] : 0;
#pragma unroll
  for (int o = 1; o < 32; o <<= 1) {
    const int y = __shfl_up(incl, o);
    if (lane >= o) incl += y;
  }
  const int w = blockIdx.x;
  if (w >= __shfl(incl, kPlanBuckets - 1)) return;  // fewer items than the grid's upper bound
  const unsigned long long m = __ballot(lane < kPlanBuckets && w < incl);
  // k and before are wave-uniform: taken into scalar registers, the item is a
  // scalar load and the whole block walk below runs on scalar control flow
  const int k = __builtin_amdgcn_readfirstlane(__ffsll((long long)m) - 1);  // class of item w
  const int before = __builtin_amdgcn_readfirstlane(k > 0 ? __shfl(incl, k - 1) : 0);
  const int item = fplan[64 + (size_t)(kPlanBuckets - 1 - k) * 2 * total + (w - before)];
  const int id = item >> 2;
  const int b = id / units;
  dev::forward_block_q<CT, KV, ST>(image_of(v0, b), id - b * units, item & 3, s_rec);
}

template <int CT, int KV, int ST>
__global__ __launch_bounds__(256) void k_forward(ImageView v0, int tiles_per_image) {
  __shared__ float4 s_geo[4 * 64];
  __shared__ float4 s_col[4 * 64 * (CT / 4)];
  const int t = blockIdx.x;
  const int b = t / tiles_per_image;
  dev::forward_tile<CT, KV, ST>(image_of(v0, b), t - b * tiles_per_image, s_geo, s_col);
}

template <int NP, int ST, bool kPlanar>
__global__ __launch_bounds__(256) void k_bwd_pixel(ImageView v0) {
  dev::bwd_pixel<NP, ST, kPlanar>(image_of(v0, blockIdx.y), blockIdx.x);
}

// The dispatcher hands workgroup i to XCD i % 8; units of 256 sorted points
// are assigned so that each XCD walks one contiguous eighth of the sorted
// order -- a band of the image whose pixel records stay in that XCD's L2 --
// instead of every XCD touching the whole image.  per8 = ceil(units / 8).
template <int CT, int KV, int ST>
__global__ __launch_bounds__(256) void k_bwd_point(ImageView v0, int per8) {
  __shared__ float red4[4];
  __shared__ int lds[256 + 64];
  __shared__ float4 stage[dev::kBwdStageF4];
  const int unit = (blockIdx.x & 7) * per8 + (blockIdx.x >> 3);
  if ((int)(blockIdx.x >> 3) >= per8 || unit >= v0.units256) return;
  dev::bwd_point<CT, KV, ST>(image_of(v0, blockIdx.y), unit, red4, lds, stage);
}

template <int CT, int KV, int ST>
__global__ __launch_bounds__(256) void k_bwd_point_wide(ImageView v0, int per8) {
  __shared__ float red4[4];
  __shared__ float gs_l[256], gs2_l[256];
  __shared__ int cls_l[256], order[256];
  const int unit = (blockIdx.x & 7) * per8 + (blockIdx.x >> 3);
  if ((int)(blockIdx.x >> 3) >= per8 || unit >= v0.units256) return;
  dev::bwd_point_wide<CT, KV, ST>(image_of(v0, blockIdx.y), unit, red4, gs_l, gs2_l, cls_l, order);
}

__global__ __launch_bounds__(256) void k_bwd_sigma_sum(ImageView v0) {
  __shared__ float red4[4];
  dev::bwd_sigma_sum(image_of(v0, blockIdx.x), red4);
}

__global__ __launch_bounds__(256) void k_debug_count(ImageView v0, int* count) {
  const ImageView v = image_of(v0, blockIdx.y);
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k < v.nb) count[(size_t)blockIdx.y * v.nb + k] = v.offset[k + 1] - v.offset[k];
}

inline unsigned cdiv(long long n, int d) { return (unsigned)((n + d - 1) / d); }

template <int CT, int KV, int ST>
hipError_t launch_forward_t(const Geometry& g, const ImageView& v0, int* fplan, hipStream_t st) {
  if constexpr (CT <= 4) {
    const int total = g.fwd_units * g.B;  // checked against 2^31 / kPlanBuckets
    {
      ProfRange pr_("fwd_plan", st);
      hipLaunchKernelGGL(k_fwd_plan, dim3(cdiv(total, 64)), dim3(256), 0, st, v0, g.fwd_units,
                         total, fplan);
    }
    ProfRange pr_("forward", st);
    hipLaunchKernelGGL((k_forward_lpt<CT, KV, ST>), dim3((unsigned)(2 * total)), dim3(256), 0, st, v0,
                       g.fwd_units, total, fplan);
  } else {
    const int per = dev::fwd_tiles(g.bx_blocks, g.by_blocks);
    const long long total = (long long)per * g.B;
    if (total >= (1LL << 31)) return hipErrorInvalidValue;
    ProfRange pr_("forward", st);
    hipLaunchKernelGGL((k_forward<CT, KV, ST>), dim3((unsigned)total), dim3(256), 0, st, v0, per);
  }
  return hipSuccess;
}

template <int CT, int KV, int ST>
hipError_t launch_backward_t(const Geometry& g, const ImageView& v0, hipStream_t st) {
  {
    ProfRange pr_("bwd_pixel", st);
    // planar records for the eight-lanes-per-point adjoint of CT >= 8
    hipLaunchKernelGGL((k_bwd_pixel<CT, ST, (CT >= 8)>), dim3(cdiv((long long)g.H * g.W, 256), g.B),
                       dim3(256), 0, st, v0);
  }
  if (g.N > 0) {
    ProfRange pr_("bwd_point", st);
    const int per8 = (g.units256 + 7) / 8;
    if constexpr (CT >= 8)
      hipLaunchKernelGGL((k_bwd_point_wide<CT, KV, ST>), dim3(8 * per8, g.B), dim3(256), 0, st, v0,
                         per8);
    else
      hipLaunchKernelGGL((k_bwd_point<CT, KV, ST>), dim3(8 * per8, g.B), dim3(256), 0, st, v0,
                         per8);
  }
  if (!g.per_point && v0.grad_sigma) {
    ProfRange pr_("bwd_sigma_sum", st);
    hipLaunchKernelGGL(k_bwd_sigma_sum, dim3(g.B), dim3(256), 0, st, v0);
  }
  return hipSuccess;
}

// Channel-count dispatch of one kernel variant.
template <int KV, int ST>
hipError_t launch_forward_kv(const Geometry& g, const ImageView& v0, int* fplan, hipStream_t st) {
  switch (g.CT) {
    case 1: return launch_forward_t<1, KV, ST>(g, v0, fplan, st);
    case 2: return launch_forward_t<2, KV, ST>(g, v0, fplan, st);
    case 3: return launch_forward_t<3, KV, ST>(g, v0, fplan, st);
    case 4: return launch_forward_t<4, KV, ST>(g, v0, fplan, st);
    case 8: return launch_forward_t<8, KV, ST>(g, v0, fplan, st);
    case 16: return launch_forward_t<16, KV, ST>(g, v0, fplan, st);
    case 32: return launch_forward_t<32, KV, ST>(g, v0, fplan, st);
  }
  return hipErrorInvalidValue;
}

template <int KV, int ST>
hipError_t launch_backward_kv(const Geometry& g, const ImageView& v0, hipStream_t st) {
  switch (g.CT) {
    case 1: return launch_backward_t<1, KV, ST>(g, v0, st);
    case 2: return launch_backward_t<2, KV, ST>(g, v0, st);
    case 3: return launch_backward_t<3, KV, ST>(g, v0, st);
    case 4: return launch_backward_t<4, KV, ST>(g, v0, st);
    case 8: return launch_backward_t<8, KV, ST>(g, v0, st);
    case 16: return launch_backward_t<16, KV, ST>(g, v0, st);
    case 32: return launch_backward_t<32, KV, ST>(g, v0, st);
  }
  return hipErrorInvalidValue;
}

// Binning (a1-a5) for values stored as ST.
template <int ST>
hipError_t launch_binning(const Geometry& g0, const ImageView& v00, int* fplan, hipStream_t st) {
  // Keys of 9 or 10 bits take one radix pass over up to kMaxDigits digits
  // here instead of two of at most 256 (the serving path keeps the latter):
  // the same stable order, one histogram, scan and scatter fewer.
  Geometry g = g0;
  ImageView v0 = v00;
  if (g.kbits > 8 && g.kbits <= 10) {
    g.npass = 1;
    g.dbits = g.kbits;
    v0.npass = 1;
    v0.dbits = g.kbits;
  }
  const bool wide_digits = g.npass == 1 && g.dbits > 8;
  const int per8 = (g.ntiles + 7) / 8;  // radix tiles per XCD
  if (g.N > 0) {
    ProfRange pr_("bin_keys", st);
    hipLaunchKernelGGL((k_bin_keys<ST>), dim3(8 * per8, g.B), dim3(256), 0, st, v0, per8);
  }
  for (int p = 0; p < g.npass && g.N > 0; ++p) {
    if (p > 0) {
      ProfRange pr_("radix_hist", st);
      hipLaunchKernelGGL(k_radix_hist, dim3(8 * per8, g.B), dim3(256), 0, st, v0, p, per8);
    }
    {
      ProfRange pr_("radix_scan", st);
      const int width = std::min(g.dbits, g.kbits - p * g.dbits);
      if (g.ntiles <= 64)
        hipLaunchKernelGGL(k_radix_scan_small, dim3(((1u << width) + 3) / 4, g.B), dim3(256), 0, st,
                           v0, p);
      else
        hipLaunchKernelGGL(k_radix_scan, dim3(1u << width, g.B), dim3(256), 0, st, v0, p);
    }
    {
      ProfRange pr_("radix_scatter", st);
      if (wide_digits) {
        if (g.CS > 4)
          hipLaunchKernelGGL((k_radix_scatter<true, ST, kMaxDigits>), dim3(8 * per8, g.B), dim3(256),
                             0, st, v0, p, per8);
        else
          hipLaunchKernelGGL((k_radix_scatter<false, ST, kMaxDigits>), dim3(8 * per8, g.B),
                             dim3(256), 0, st, v0, p, per8);
      } else if (g.CS > 4) {
        hipLaunchKernelGGL((k_radix_scatter<true, ST, 256>), dim3(8 * per8, g.B), dim3(256), 0, st,
                           v0, p, per8);
      } else {
        hipLaunchKernelGGL((k_radix_scatter<false, ST, 256>), dim3(8 * per8, g.B), dim3(256), 0,
                           st, v0, p, per8);
      }
    }
  }
  if (g.CS > 4 && g.npass > 0 && g.N > 0) {
    ProfRange pr_("place_wide", st);
    hipLaunchKernelGGL((k_place_wide<ST>), dim3(cdiv(g.N, 64), g.B), dim3(256), 0, st, v0);
  }
  {
    ProfRange pr_("bin_finish", st);
    hipLaunchKernelGGL(k_bin_finish, dim3(dev::finish_units(g.N), g.B), dim3(256), 0, st, v0,
                       fplan);
  }
  return hipGetLastError();
}

}  // namespace

// Kernel variants take float32 storage; the default kernel any storage.
hipError_t launch_forward_all(const Geometry& g, const ImageView& v0, int* fplan, hipStream_t st) {
  hipError_t e;
  switch (g.st) {
    case INTERP_STORAGE_F32: e = launch_binning<INTERP_STORAGE_F32>(g, v0, fplan, st); break;
    case INTERP_STORAGE_BF16: e = launch_binning<INTERP_STORAGE_BF16>(g, v0, fplan, st); break;
    case INTERP_STORAGE_F16: e = launch_binning<INTERP_STORAGE_F16>(g, v0, fplan, st); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  if (g.st == INTERP_STORAGE_BF16) {
    e = launch_forward_kv<0, INTERP_STORAGE_BF16>(g, v0, fplan, st);
  } else if (g.st == INTERP_STORAGE_F16) {
    e = launch_forward_kv<0, INTERP_STORAGE_F16>(g, v0, fplan, st);
  } else {
    switch (g.kern) {
      case 0: e = launch_forward_kv<0, 0>(g, v0, fplan, st); break;
      case 1: e = launch_forward_kv<1, 0>(g, v0, fplan, st); break;
      case 2: e = launch_forward_kv<2, 0>(g, v0, fplan, st); break;
      case 3: e = launch_forward_kv<3, 0>(g, v0, fplan, st); break;
      default: return hipErrorInvalidValue;
    }
  }
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t launch_backward_all(const Geometry& g, const ImageView& v0, hipStream_t st) {
  hipError_t e;
  if (g.st == INTERP_STORAGE_BF16) {
    e = launch_backward_kv<0, INTERP_STORAGE_BF16>(g, v0, st);
  } else if (g.st == INTERP_STORAGE_F16) {
    e = launch_backward_kv<0, INTERP_STORAGE_F16>(g, v0, st);
  } else {
    switch (g.kern) {
      case 0: e = launch_backward_kv<0, 0>(g, v0, st); break;
      case 1: e = launch_backward_kv<1, 0>(g, v0, st); break;
      case 2: e = launch_backward_kv<2, 0>(g, v0, st); break;
      case 3: e = launch_backward_kv<3, 0>(g, v0, st); break;
      default: return hipErrorInvalidValue;
    }
  }
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t launch_debug_count(const Geometry& g, const ImageView& v0, int* count, hipStream_t st) {
  hipLaunchKernelGGL(k_debug_count, dim3(cdiv(g.nb, 256), g.B), dim3(256), 0, st, v0, count);
  return hipGetLastError();
}

}  // namespace gmm
