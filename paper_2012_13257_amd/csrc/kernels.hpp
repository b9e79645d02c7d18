// Kernel bodies of the Gaussian-mixture interpolation, as device functions on
// one ImageView.  The single-call path (single.hip) and the serving job-table
// path (server.hip) wrap the same functions, so a request computes exactly
// the same bits alone and inside a batch.
//
// Method (paper, Section 2, Eq. 1 and Eq. 2): out_i = sum_j w_ij c_j / Z_i,
// Z_i = sum_j w_ij, w_ij = exp(-|g_i - p_j|^2 / (2 sigma_j^2)), summed over the
// points close enough to pixel i (radius * sigma_j, inclusive, float32 test
// without FMA); every channel on its own.
//
// Phases of one forward:
//   bin_keys       bin key of every point; partial maxima of radius*sigma;
//                  digit histograms of the first radix pass
//   radix_hist / radix_scan / radix_scatter   (x npass; no radix_hist in
//                  the first pass)
//                  stable LSD radix sort of (key, point index, record)
//                  -> the counting-sort order by bin, ties by point index,
//                  and the point records (x, y, k, R2, values) in that order
//   bin_finish     bin offsets from the sorted keys; per-image reach
//   fwd_plan       (single-call path) cost class of every forward unit, for
//                  a heaviest-first launch order
//   forward        the gather: per 8x8 pixel block, candidates from the bins
//                  within reach, culled per 4x4 quarter of the block, hits
//                  evaluated per pixel
// Backward (quotient rule on Eq. 1; formulas in include/gmminterp.h):
//   bwd_pixel      G'_ik = G_ik / Z_i and beta_i per pixel
//   bwd_point      per point: walk its disk's bounding box, recompute w_ij,
//                  accumulate the gradients in registers (no atomics)
//   bwd_sigma_sum  shared sigma: fixed-order sum of the per-point dL/dsigma
#pragma once

#include <climits>
#include <type_traits>

#include "common.hpp"

namespace gmm {
namespace dev {

constexpr float kLog2e = 1.4426950408889634f;

__device__ inline int bin_coord(float c, float inv_tile, int nmax) {
  // floor(c / tile) clamped to [0, nmax-1]; c * (1/tile) is exact for a
  // power-of-two tile.  NaN and negative values land in bin 0.
  const float f = floorf(c * inv_tile);
  if (!(f >= 0.0f)) return 0;
  if (f >= (float)(nmax - 1)) return nmax - 1;
  return (int)f;
}

// (sigma_x, sigma_y) of point j: the isotropic kernel's sigma twice, or the
// diagonal kernel's pair.
__device__ inline float2 sigma2_of(const ImageView& v, int j) {
  const float* s = v.per_point ? v.sigma + (size_t)j * v.nsig : v.sigma;
  return v.nsig == 2 ? make_float2(s[0], s[1]) : make_float2(s[0], s[0]);
}

// The sorted point record.  Isotropic kernel: x, y, the exp2 scale
// k = -log2(e)/(2 sigma^2) and the squared radius R2 = f32(f32(radius*sigma)^2)
// of the radius test.  Diagonal kernel: x, y and the inverse sigmas
// ix = 1/sigma_x, iy = 1/sigma_y of the Mahalanobis test (correctly rounded
// divisions, as the test specifies).
__device__ inline float4 make_geo(float2 p, float2 sg, float radius, bool diag) {
  if (diag) return make_float4(p.x, p.y, __fdiv_rn(1.0f, sg.x), __fdiv_rn(1.0f, sg.y));
  const float rs = __fmul_rn(radius, sg.x);
  const float R2 = __fmul_rn(rs, rs);
  const float kk = -0.5f * kLog2e / __fmul_rn(sg.x, sg.x);
  return make_float4(p.x, p.y, kk, R2);
}

// The point's sigma (sigma_x, sigma_y) recovered from its sorted record, for
// the adjoint's disk extent and chain rule: reading sigma at the point's
// original index would be a gather with a dependent address.  Isotropic:
// sigma^2 = -log2(e) / (2 k); diagonal: sigma = 1 / (1/sigma).  Within a few
// float32 roundings of the input sigma, which moves the gradients' scale
// factors by a few parts in 1e7 and stays far inside the extents' margins.
template <bool kDiag>
__device__ inline float2 record_sigma(float4 g) {
  if constexpr (kDiag) {
    return make_float2(1.0f / g.z, 1.0f / g.w);
  } else {
    const float s = __builtin_sqrtf(-0.5f * kLog2e / g.z);
    return make_float2(s, s);
  }
}

// The normal density's factor 1/(2 pi sigma_x sigma_y) of a normalised
// kernel, from the point's record: the isotropic record holds
// k = -log2(e) / (2 sigma^2), so the factor is k * (-1 / (pi log2(e)));
// the diagonal record holds 1/sigma_x and 1/sigma_y.  (A few float32
// roundings from the exact factor: far inside the outputs' tolerance.)
template <bool kDiag>
__device__ inline float record_density(float4 g) {
  if constexpr (kDiag) return (g.z * g.w) * 0.159154943091895336f;  // 1 / (2 pi)
  else return g.z * -0.220635600152651643f;                        // -1 / (pi log2(e))
}

// Truncation radius (pixels) of a point along its longer axis.
__device__ inline float point_reach(float2 sg, float radius) {
  return __fmul_rn(radius, fmaxf(sg.x, sg.y));
}

// Conservative reach (pixels) of a point set whose largest radius*sigma is
// rs: covers the float32 rounding of the radius test and of the bin bounds.
__device__ inline float conservative_reach(float rs) { return rs * (1.0f + 0x1p-10f) + 0x1p-6f; }

__device__ inline float block_max(float x, float* red4) {
  for (int o = 32; o > 0; o >>= 1) x = fmaxf(x, __shfl_xor(x, o));
  if ((threadIdx.x & 63) == 0) red4[threadIdx.x >> 6] = x;
  __syncthreads();
  const float m = fmaxf(fmaxf(red4[0], red4[1]), fmaxf(red4[2], red4[3]));
  __syncthreads();
  return m;
}

// Fixed-order sum over a 256-thread block (xor tree, then the four waves in order).
__device__ inline float block_sum(float x, float* red4) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  if ((threadIdx.x & 63) == 0) red4[threadIdx.x >> 6] = x;
  __syncthreads();
  const float s = (red4[0] + red4[1]) + (red4[2] + red4[3]);
  __syncthreads();
  return s;
}

// Orders one wavefront's LDS writes before its lanes read each other's data.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Storage of the value arrays (values, out, grad_out, grad_values and the
// sorted value records): float32, bfloat16 or half.  Elements are widened
// to float32 on load (exact) and rounded to nearest even on store.
template <int ST> struct Val;
template <> struct Val<INTERP_STORAGE_F32> {
  __device__ static float load(const float* p, size_t i) { return p[i]; }
  __device__ static void store(float* p, size_t i, float x) { p[i] = x; }
  // elements 4g .. 4g+3
  __device__ static float4 load4(const float* p, size_t g) {
    return reinterpret_cast<const float4*>(p)[g];
  }
  __device__ static void store4(float* p, size_t g, float4 x) { reinterpret_cast<float4*>(p)[g] = x; }
};
__device__ inline float bf16_widen(unsigned h) { return __uint_as_float(h << 16); }
__device__ inline unsigned bf16_round(float x) {
  const unsigned u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;  // NaN stays NaN
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}
template <> struct Val<INTERP_STORAGE_BF16> {
  __device__ static float load(const float* p, size_t i) {
    return bf16_widen(reinterpret_cast<const unsigned short*>(p)[i]);
  }
  __device__ static void store(float* p, size_t i, float x) {
    reinterpret_cast<unsigned short*>(p)[i] = (unsigned short)bf16_round(x);
  }
  __device__ static float4 load4(const float* p, size_t g) {
    const uint2 q = reinterpret_cast<const uint2*>(p)[g];
    return make_float4(bf16_widen(q.x & 0xffffu), bf16_widen(q.x >> 16), bf16_widen(q.y & 0xffffu),
                       bf16_widen(q.y >> 16));
  }
  __device__ static void store4(float* p, size_t g, float4 x) {
    reinterpret_cast<uint2*>(p)[g] = make_uint2(bf16_round(x.x) | (bf16_round(x.y) << 16),
                                                bf16_round(x.z) | (bf16_round(x.w) << 16));
  }
};
template <> struct Val<INTERP_STORAGE_F16> {
  __device__ static float load(const float* p, size_t i) {
    return (float)reinterpret_cast<const _Float16*>(p)[i];
  }
  __device__ static void store(float* p, size_t i, float x) {
    reinterpret_cast<_Float16*>(p)[i] = (_Float16)x;
  }
  __device__ static float4 load4(const float* p, size_t g) {
    const uint2 q = reinterpret_cast<const uint2*>(p)[g];
    _Float16 e[4];
    __builtin_memcpy(e, &q, 8);
    return make_float4((float)e[0], (float)e[1], (float)e[2], (float)e[3]);
  }
  __device__ static void store4(float* p, size_t g, float4 x) {
    _Float16 e[4] = {(_Float16)x.x, (_Float16)x.y, (_Float16)x.z, (_Float16)x.w};
    uint2 q;
    __builtin_memcpy(&q, e, 8);
    reinterpret_cast<uint2*>(p)[g] = q;
  }
};

// ---------------------------------------------------------------------------
// Binning: stable LSD radix sort of the bin keys (no global atomics)
// ---------------------------------------------------------------------------

// The record of point j: geo (make_geo) and its values padded to CS.
__device__ inline float4 point_geo(const ImageView& v, int j) {
  return make_geo(v.pos[j], sigma2_of(v, j), v.radius, v.nsig == 2);
}
template <int ST = INTERP_STORAGE_F32>
__device__ inline float4 point_values4(const ImageView& v, int j, int c) {
  const size_t base = (size_t)j * v.C;
  float q[4];
  if (v.values_vec4 && c < v.C) {  // four values in one load
    const float4 x = Val<ST>::load4(v.values, (base + c) / 4);
    q[0] = x.x; q[1] = x.y; q[2] = x.z; q[3] = x.w;
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i) q[i] = c + i < v.C ? Val<ST>::load(v.values, base + c + i) : 0.0f;
  }
  return make_float4(q[0], q[1], q[2], q[3]);
}

// unit = one radix tile of kRadixTile points: bin key of every point, the
// tile's maximum of radius*sigma and -- the first radix pass needs it -- the
// tile's histogram of the lowest key digit.  lh: kMaxDigits ints of LDS.  With a
// single bin (no radix pass) the point order is already sorted and the
// sorted records are written here.
template <int ST = INTERP_STORAGE_F32>
__device__ inline void bin_keys(const ImageView& v, int tile, float* red4, int* lh) {
  const int t = threadIdx.x;
  const int width0 = v.npass > 0 ? min(v.dbits, v.kbits) : 0;
  const int mask0 = (1 << width0) - 1;
  const int j0 = tile * kRadixTile + t;
  float2 p[kRadixItems], sg[kRadixItems];
#pragma unroll
  for (int r = 0; r < kRadixItems; ++r) {
    const int jc = min(j0 + r * 256, v.N - 1);  // clamped: no load behind a branch
    p[r] = v.pos[jc];
    sg[r] = sigma2_of(v, jc);
  }
  for (int d = t; d < kMaxDigits; d += 256) lh[d] = 0;
  __syncthreads();
  float rmax = 0.0f;
#pragma unroll
  for (int r = 0; r < kRadixItems; ++r) {
    const int j = j0 + r * 256;
    if (j < v.N) {
      const int key =
          bin_coord(p[r].y, v.inv_tile, v.nby) * v.nbx + bin_coord(p[r].x, v.inv_tile, v.nbx);
      v.binof[j] = key;
      if (v.npass > 0) atomicAdd(&lh[key & mask0], 1);
      float rs = point_reach(sg[r], v.radius);
      if (!(rs >= 0.0f)) rs = 0.0f;  // caller contract violated; keep the reach sane
      rmax = fmaxf(rmax, rs);
    }
  }
  if (v.npass == 0) {
    for (int r = 0; r < kRadixItems; ++r) {
      const int j = j0 + r * 256;
      if (j >= v.N) continue;
      v.keysF[j] = 0;
      v.perm[j] = j;
      v.geo[j] = make_geo(p[r], sg[r], v.radius, v.nsig == 2);
      for (int c = 0; c < v.CS; c += 4)
        Val<ST>::store4(v.col, (size_t)j * (v.CS / 4) + c / 4, point_values4<ST>(v, j, c));
    }
  }
  __syncthreads();
  if (v.npass > 0)
    for (int d = t; d <= mask0; d += 256) v.hist[d * v.ntiles + tile] = lh[d];
  const float m = block_max(rmax, red4);
  if (t == 0) v.rpart[tile] = m;
}

__device__ inline void radix_pass_bits(const ImageView& v, int p, int* shift, int* width) {
  *shift = p * v.dbits;
  *width = min(v.dbits, v.kbits - *shift);
}

// unit = one tile of kRadixTile keys: digit histogram of the tile (passes
// after the first; bin_keys counts the first)
__device__ inline void radix_hist(const ImageView& v, int p, int tile, int* lh) {
  int shift, width;
  radix_pass_bits(v, p, &shift, &width);
  const int ndig = 1 << width, mask = ndig - 1;
  const int* kin = ((p - 1) & 1) == 0 ? v.kA : v.kB;
  lh[threadIdx.x] = 0;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRadixItems; ++r) {
    const int idx = tile * kRadixTile + r * 256 + threadIdx.x;
    if (idx < v.N) atomicAdd(&lh[(kin[idx] >> shift) & mask], 1);
  }
  __syncthreads();
  if (threadIdx.x < ndig) v.hist[threadIdx.x * v.ntiles + tile] = lh[threadIdx.x];
  __syncthreads();
}

// Exclusive scan of x over the 256 threads of a block (wave scans, then the
// four wave totals in order).  tmp4: 4 ints of LDS.
__device__ inline int block_exclusive_scan256(int x, int* tmp4) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int incl = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(incl, o);
    if (lane >= o) incl += y;
  }
  if (lane == 63) tmp4[wid] = incl;
  __syncthreads();
  int pre = 0;
  for (int w = 0; w < wid; ++w) pre += tmp4[w];
  __syncthreads();
  return pre + incl - x;
}

// unit = one digit: exclusive scan of the digit's per-tile counts over the
// tiles, in place, and the digit's total.  tmp4: 4 ints of LDS.
__device__ inline void radix_scan_digit(const ImageView& v, int p, int d, int* tmp4) {
  int shift, width;
  radix_pass_bits(v, p, &shift, &width);
  if (d >= (1 << width)) return;
  int* row = v.hist + (size_t)d * v.ntiles;
  int carry = 0;
  for (int seg = 0; seg < v.ntiles; seg += 256 * 8) {
    const int i0 = seg + threadIdx.x * 8;
    int x[8], sum = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      x[k] = i0 + k < v.ntiles ? row[i0 + k] : 0;
      sum += x[k];
    }
    int pre = block_exclusive_scan256(sum, tmp4) + carry;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (i0 + k < v.ntiles) row[i0 + k] = pre;
      pre += x[k];
    }
    // the segment total: the last thread's running prefix
    if (threadIdx.x == 255) tmp4[0] = pre;
    __syncthreads();
    carry = tmp4[0];
    __syncthreads();
  }
  if (threadIdx.x == 0) v.dtot[d] = carry;
}

// The same for four digits per 256-thread block, one wavefront per digit,
// when a pass has at most 64 tiles (a block per digit would spend its time
// being dispatched).  unit = a group of four digits.
__device__ inline void radix_scan_digits_small(const ImageView& v, int p, int unit) {
  int shift, width;
  radix_pass_bits(v, p, &shift, &width);
  const int lane = threadIdx.x & 63;
  const int d = unit * 4 + (int)(threadIdx.x >> 6);
  if (d >= (1 << width)) return;
  int* row = v.hist + (size_t)d * v.ntiles;
  const int x = lane < v.ntiles ? row[lane] : 0;
  int incl = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(incl, o);
    if (lane >= o) incl += y;
  }
  if (lane < v.ntiles) row[lane] = incl - x;
  if (lane == 63) v.dtot[d] = incl;
}

// LDS ints radix_scatter<kDig> needs: wrun[4][kDig], base[kDig], tstart[kDig],
// tmp4, and the tile's keys and source slots in digit order.  kDig: the
// digits a pass may have (256, or kMaxDigits for the single-call path's one
// pass over keys of 9 or 10 bits).
template <int kDig = 256>
__host__ __device__ constexpr int radix_scatter_lds_ints() { return 6 * kDig + 4 + 2 * kRadixTile; }

// unit = one tile: stable scatter of the tile's (key, point index) pairs by
// the pass's digit.  Each wavefront ranks the kRadixTile / 4 consecutive keys
// it owns in rounds of 64 (equal digits by ballot -- multisplit -- and a
// per-wavefront running count per digit in LDS); the wavefronts' counts then
// give every key its place in a digit-ordered list of the tile in LDS
// (wavefronts in index order, so equal digits keep their input order), which
// is written out so that every digit's entries form one contiguous run in the
// output.  The last pass writes the sorted keys, the permutation and the
// sorted point records (x, y, k, R2 and the values padded to CS).
// kWide: the records carry more than four values (CS > 4).
template <bool kWide = false, int ST = INTERP_STORAGE_F32, int kDig = 256>
__device__ inline void radix_scatter(const ImageView& v, int p, int tile, int* lds) {
  static_assert(kDig % 256 == 0 && kDig <= kMaxDigits, "digits per thread");
  constexpr int DPT = kDig / 256;  // digits per thread (thread t owns [t DPT, t DPT + DPT))
  int* wrun = lds;                 // [4][kDig]
  int* base = lds + 4 * kDig;      // [kDig]
  int* tstart = base + kDig;       // [kDig]
  int* tmp4 = tstart + kDig;       // [4]
  int* skey = tmp4 + 4;            // [kRadixTile]
  int* ssrc = skey + kRadixTile;   // [kRadixTile] slot of the entry in the tile's input
  int shift, width;
  radix_pass_bits(v, p, &shift, &width);
  const int ndig = 1 << width, mask = ndig - 1;
  const bool first = p == 0, last = p == v.npass - 1;
  const bool in_a = ((p - 1) & 1) == 0, out_a = (p & 1) == 0;
  // buffer choice by value (selecting between fields through the view would
  // make the compiler copy the view to scratch memory)
  int* const kA = v.kA; int* const kB = v.kB; int* const vA = v.vA; int* const vB = v.vB;
  const int* kin = first ? v.binof : (in_a ? kA : kB);
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const int t0 = tile * kRadixTile;
  const int tn = min(kRadixTile, v.N - t0);
  // every global load of the ranking is issued up front (the LDS fences
  // below would otherwise hold each one back until it is needed; indices
  // are clamped into the array so that no load sits behind a branch)
  int key[kRadixItems], rk[kRadixItems];
  const int s0 = wid * (kRadixTile / 4) + lane;  // this lane's first slot in the tile
#pragma unroll
  for (int r = 0; r < kRadixItems; ++r) key[r] = kin[min(t0 + s0 + r * 64, v.N - 1)];
  // global start of each digit for this tile: digit base + tile offset
  {
    int dt[DPT], th[DPT], sum = 0;
#pragma unroll
    for (int i = 0; i < DPT; ++i) {
      const int d = t * DPT + i;
      dt[i] = d < ndig ? v.dtot[d] : 0;
      th[i] = d < ndig ? v.hist[d * v.ntiles + tile] : 0;
      sum += dt[i];
    }
    int pre = block_exclusive_scan256(sum, tmp4);
#pragma unroll
    for (int i = 0; i < DPT; ++i) {
      base[t * DPT + i] = pre + th[i];
      pre += dt[i];
    }
#pragma unroll
    for (int i = 0; i < 4 * DPT; ++i) wrun[i * 256 + t] = 0;
  }
  __syncthreads();
  // 1) rank of every key among the equal digits of its wavefront's keys
  const unsigned long long below = (1ull << lane) - 1ull;
  int* myrun = wrun + wid * kDig;
#pragma unroll
  for (int r = 0; r < kRadixItems; ++r) {
    const bool valid = s0 + r * 64 < tn;
    const int d = (key[r] >> shift) & mask;
    unsigned long long peers = __ballot(valid);
    for (int bit = 0; bit < width; ++bit) {
      const bool on = (d >> bit) & 1;
      const unsigned long long m = __ballot(on);
      peers &= on ? m : ~m;
    }
    const int rank = __popcll(peers & below);
    const int prior = myrun[d];
    rk[r] = valid ? prior + rank : -1;
    wave_lds_sync();
    if (valid && rank == 0) myrun[d] = prior + __popcll(peers);
    wave_lds_sync();
  }
  __syncthreads();
  // 2) per digit: start of each wavefront's keys and of the digit in the tile
  {
    int tot[DPT], sum = 0;
#pragma unroll
    for (int i = 0; i < DPT; ++i) {
      const int d = t * DPT + i;
      tot[i] = 0;
      if (d < ndig) {
        const int c0 = wrun[d], c1 = wrun[kDig + d], c2 = wrun[2 * kDig + d], c3 = wrun[3 * kDig + d];
        wrun[d] = 0;
        wrun[kDig + d] = c0;
        wrun[2 * kDig + d] = c0 + c1;
        wrun[3 * kDig + d] = c0 + c1 + c2;
        tot[i] = c0 + c1 + c2 + c3;
      }
      sum += tot[i];
    }
    int pre = block_exclusive_scan256(sum, tmp4);
#pragma unroll
    for (int i = 0; i < DPT; ++i) {
      tstart[t * DPT + i] = pre;
      pre += tot[i];
    }
  }
  __syncthreads();
  // 3) the tile in digit order in LDS: key and input slot
#pragma unroll
  for (int r = 0; r < kRadixItems; ++r) {
    if (rk[r] >= 0) {
      const int d = (key[r] >> shift) & mask;
      const int lpos = tstart[d] + myrun[d] + rk[r];
      skey[lpos] = key[r];
      ssrc[lpos] = s0 + r * 64;
    }
  }
  __syncthreads();
  // 4) write out: consecutive entries of one digit go to consecutive places;
  // all loads of this thread's entries first, then the stores.  Narrow
  // records (CS = 4) travel with their keys through every pass: the first
  // pass builds them from the inputs (coalesced reads of the tile's points)
  // and the last leaves them in bin order.  Wide records (more than four
  // values) cost more to move in every pass than to read once: the passes
  // before the last move only (key, point index), and the last pass reads
  // each entry's record from the inputs at its point index.
  int* const keysF = v.keysF; int* const perm = v.perm;
  float4* const geo = v.geo; float* const col = v.col;
  float4* const geoA = v.geoA; float4* const geoB = v.geoB;
  float4* const colA = v.colA; float4* const colB = v.colB;
  const int* jin = in_a ? vA : vB;
  int ek[kRadixItems], ej[kRadixItems], epos[kRadixItems];
  float4 eg[kRadixItems], ec[kRadixItems];
#pragma unroll
  for (int q = 0; q < kRadixItems; ++q) {
    const int e = min(t + q * 256, tn - 1);
    ek[q] = skey[e];
    const int src = t0 + ssrc[e];
    const int d = (ek[q] >> shift) & mask;
    epos[q] = base[d] + e - tstart[d];
    ej[q] = first ? src : jin[src];
    if constexpr (!kWide) {
      if (first) {
        eg[q] = point_geo(v, src);
        ec[q] = point_values4<ST>(v, src, 0);
      } else {
        eg[q] = (in_a ? geoA : geoB)[src];
        ec[q] = (in_a ? colA : colB)[src];
      }
    }
  }
  if (kWide && last) {
    // wide records are placed afterwards by place_wide, which reads the
    // inputs in point order: here the inverse permutation, in the index
    // buffer this pass does not use
    int* const iperm = out_a ? vA : vB;
#pragma unroll
    for (int q = 0; q < kRadixItems; ++q) {
      if (t + q * 256 < tn) {
        const int g = epos[q];
        keysF[g] = ek[q];
        perm[g] = ej[q];
        iperm[ej[q]] = g;
      }
    }
  } else if (last) {
#pragma unroll
    for (int q = 0; q < kRadixItems; ++q) {
      if (t + q * 256 < tn) {
        const int g = epos[q];
        keysF[g] = ek[q];
        perm[g] = ej[q];
        geo[g] = eg[q];
        Val<ST>::store4(col, (size_t)g * (v.CS / 4), ec[q]);
      }
    }
  } else {
    int* kout = out_a ? kA : kB;
    int* jout = out_a ? vA : vB;
#pragma unroll
    for (int q = 0; q < kRadixItems; ++q) {
      if (t + q * 256 < tn) {
        kout[epos[q]] = ek[q];
        jout[epos[q]] = ej[q];
        if constexpr (!kWide) {
          (out_a ? geoA : geoB)[epos[q]] = eg[q];
          (out_a ? colA : colB)[epos[q]] = ec[q];
        }
      }
    }
  }
  __syncthreads();
}

// unit = 256 points in point order, after the last radix pass of wide
// records: each point's sorted record (geo, and the values padded to CS) is
// built from coalesced reads of the inputs and written to its sorted place
// (iperm: the inverse permutation the last pass left in the index buffer it
// did not use).  Gathering the records in sorted order instead reads every
// point's inputs from a random place, a cache line per piece.
// unit = 64 points, four lanes per point: lane k of a point writes its
// values' groups of four k, k + 4, ..., so that one store instruction writes
// whole 64-byte pieces of the sorted records.
template <int ST = INTERP_STORAGE_F32>
__device__ inline void place_wide(const ImageView& v, int unit) {
  const int j = unit * 64 + (threadIdx.x >> 2), k = threadIdx.x & 3;
  if (j >= v.N) return;
  const int* iperm = ((v.npass - 1) & 1) == 0 ? v.vA : v.vB;
  const int g = iperm[j];
  if (k == 0) v.geo[g] = point_geo(v, j);
  for (int c = 4 * k; c < v.CS; c += 16)
    Val<ST>::store4(v.col, (size_t)g * (v.CS / 4) + c / 4, point_values4<ST>(v, j, c));
}

// unit = 256 sorted positions (N + 1 positions in all): bin offsets from the
// sorted keys -- position i opens every bin in (key[i-1], key[i]]; position N
// closes the rest.  Unit 0 also reduces the per-image reach.
__device__ inline void bin_finish(const ImageView& v, int unit, float* red4) {
  const int i = unit * 256 + threadIdx.x;
  if (i <= v.N) {
    const int kcur = i < v.N ? v.keysF[i] : v.nb;
    const int kprev = i > 0 ? v.keysF[i - 1] : -1;
    for (int k = kprev + 1; k <= kcur; ++k) v.offset[k] = i;
  }
  if (unit == 0) {
    float m = 0.0f;
    for (int q = threadIdx.x; q < v.ntiles; q += 256) m = fmaxf(m, v.rpart[q]);
    m = block_max(m, red4);
    if (threadIdx.x == 0) v.reach[0] = m;
  }
}

// number of positions bin_finish covers, in units of 256
__host__ __device__ inline int finish_units(int N) { return (N + 1 + 255) / 256; }

// ---------------------------------------------------------------------------
// Forward gather
// ---------------------------------------------------------------------------

// Kernel variants (template parameter KV: INTERP_KERNEL_* flags).
template <int KV> constexpr bool kDiagonal = (KV & INTERP_KERNEL_DIAGONAL) != 0;
template <int KV> constexpr bool kNormalized = (KV & INTERP_KERNEL_NORMALIZED) != 0;
constexpr float kHalfLog2e = -0.5f * kLog2e;  // exp(-m/2) = exp2(m * kHalfLog2e)

// The weight of pixel (fu, fv) for sorted record r, zero outside the
// truncation radius: the specified float32 test, every operation rounded.
// Isotropic: d2 = dx*dx + dy*dy, include iff d2 <= R2, w = exp2(d2 * k).
// Diagonal: qx = dx*ix, qy = dy*iy, m2 = qx*qx + qy*qy, include iff
// m2 <= r2, w = exp2(m2 * (-log2(e)/2)).
template <int KV>
__device__ inline float pair_weight(float fu, float fv, float4 r, float r2) {
  const float dx = fu - r.x;
  const float dy = fv - r.y;
  if constexpr (kDiagonal<KV>) {
    const float qx = dx * r.z;
    const float qy = dy * r.w;
    const float m2 = qx * qx + qy * qy;
    const float w = __builtin_amdgcn_exp2f(m2 * kHalfLog2e);
    return (m2 <= r2) ? w : 0.0f;
  } else {
    const float d2 = dx * dx + dy * dy;
    const float w = __builtin_amdgcn_exp2f(d2 * r.z);
    return (d2 <= r.w) ? w : 0.0f;
  }
}

// Conservative test: can record g reach a box whose nearest point is ex, ey
// (>= 0) away from it along x and y?
template <int KV>
__device__ inline float box_sq(float e, float inv) {
  if constexpr (kDiagonal<KV>) { const float a = e * inv; return a * a; }
  else return e * e;
}
template <int KV>
__device__ inline float reach_lim(float4 g, float r2) {
  if constexpr (kDiagonal<KV>) return r2 * 1.001f + 1e-6f;
  else return g.w * 1.001f + 1e-6f;
}


__host__ __device__ inline int fwd_tiles_x(int bx_blocks) { return (bx_blocks + 1) / 2; }
__host__ __device__ inline int fwd_tiles(int bx_blocks, int by_blocks) {
  return ((bx_blocks + 1) / 2) * ((by_blocks + 1) / 2);
}

// One 256-thread block = one 16x16 pixel tile; wavefront w owns the 8x8
// block (w & 1, w >> 1) of it, one pixel per lane.  Candidates are the
// records of the bins within reach of the block (one contiguous range per
// bin row), taken 64 at a time: each lane tests one candidate's disk against
// the block, the hits are compacted in candidate order into the wavefront's
// LDS list, and every lane then evaluates each hit for its pixel.
template <int CT, int KV = 0, int ST = INTERP_STORAGE_F32>
__device__ inline void forward_tile(const ImageView& v, int tile, float4* s_geo /*[4][64]*/,
                                    float4* s_col /*[4][64*CS/4]*/) {
  constexpr int CS = CT < 4 ? 4 : CT;
  constexpr int NC = CT;
  const float r2 = v.r2;
  const int lane = threadIdx.x & 63, wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wgx = fwd_tiles_x(v.bx_blocks);
  const int ty = tile / wgx, tx = tile - ty * wgx;
  const int u0 = (2 * tx + (wid & 1)) * kBlockSide;
  const int v0 = (2 * ty + (wid >> 1)) * kBlockSide;
  if (u0 >= v.W || v0 >= v.H) return;
  const int ue = min(u0 + kBlockSide - 1, v.W - 1);
  const int ve = min(v0 + kBlockSide - 1, v.H - 1);
  const int u = u0 + (lane & 7), vv = v0 + (lane >> 3);
  const float fu = (float)u, fv = (float)vv;

  // float math runs on the vector ALU; readfirstlane keeps the wave-uniform
  // loop bounds in scalar registers
  const float Rh = conservative_reach(v.reach[0]);
  const int bx_lo = __builtin_amdgcn_readfirstlane(bin_coord((float)u0 - Rh, v.inv_tile, v.nbx));
  const int bx_hi = __builtin_amdgcn_readfirstlane(bin_coord((float)ue + Rh, v.inv_tile, v.nbx));
  const int by_lo = __builtin_amdgcn_readfirstlane(bin_coord((float)v0 - Rh, v.inv_tile, v.nby));
  const int by_hi = __builtin_amdgcn_readfirstlane(bin_coord((float)ve + Rh, v.inv_tile, v.nby));
  const float4* gb = v.geo;
  const float* cb = v.col;

  float Z = 0.0f;
  float acc[CT];
#pragma unroll
  for (int k = 0; k < CT; ++k) acc[k] = 0.0f;

  float4* lgeo = s_geo + wid * 64;
  float4* lcol = s_col + wid * 64 * (CS / 4);

  for (int by = by_lo; by <= by_hi; ++by) {
    const int s = __builtin_amdgcn_readfirstlane(v.offset[by * v.nbx + bx_lo]);
    const int e = __builtin_amdgcn_readfirstlane(v.offset[by * v.nbx + bx_hi + 1]);
    for (int c0 = s; c0 < e; c0 += 64) {
      const int jc = c0 + lane;
      bool hit = false;
      float4 g = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      if (jc < e) {
        g = gb[jc];
        const float ex = fmaxf(fmaxf((float)u0 - g.x, g.x - (float)ue), 0.0f);
        const float ey = fmaxf(fmaxf((float)v0 - g.y, g.y - (float)ve), 0.0f);
        hit = box_sq<KV>(ex, g.z) + box_sq<KV>(ey, g.w) <= reach_lim<KV>(g, r2);
      }
      const unsigned long long mask = __ballot(hit);
      if (mask == 0) continue;
      if (hit) {
        const int slot = __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                                   __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0));
        lgeo[slot] = g;
#pragma unroll
        for (int q = 0; q < CS / 4; ++q)
          lcol[slot * (CS / 4) + q] = Val<ST>::load4(cb, (size_t)jc * (CS / 4) + q);
      }
      wave_lds_sync();
      const int nh = __popcll(mask);
      for (int i = 0; i < nh; ++i) {
        const float4 r = lgeo[i];
        float cc[CS];
#pragma unroll
        for (int q = 0; q < CS / 4; ++q) {
          const float4 tq = lcol[i * (CS / 4) + q];
          cc[4 * q] = tq.x; cc[4 * q + 1] = tq.y; cc[4 * q + 2] = tq.z; cc[4 * q + 3] = tq.w;
        }
        float w = pair_weight<KV>(fu, fv, r, r2);
        if constexpr (kNormalized<KV>) w *= record_density<kDiagonal<KV>>(r);
        Z += w;
#pragma unroll
        for (int k = 0; k < NC; ++k) acc[k] = __builtin_fmaf(w, cc[k], acc[k]);
      }
      wave_lds_sync();
    }
  }

  if (u <= ue && vv <= ve) {
    const size_t HW = (size_t)v.H * v.W;
    const size_t pix = (size_t)vv * v.W + u;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      if (k < v.C) Val<ST>::store(v.out, k * HW + pix, Z > 0.0f ? acc[k] / Z : 0.0f);
    }
    v.Z[pix] = Z;
  }
}

// Forward gather for up to 4 channels.  A wavefront evaluates one 8x8 pixel
// block; a block's candidates are the records of the bins within reach --
// one contiguous range of the sorted order per bin row -- taken 64 records
// of one row at a time; when two wavefronts share a block they take
// alternate chunks (a dense block is spread over two SIMDs).  Within a
// wavefront the block is cut into four 4x4 quarters: each candidate is tested against every quarter and appended to
// the LDS list of each quarter its disk reaches, and a quarter's list is
// evaluated four candidates at a time -- lane group g = lane / 16 takes list
// entries g, g+4, ... for pixel lane % 16 of the quarter (lists are padded to
// a multiple of four with a null record that fails the radius test: w = 0,
// values 0).  The next chunk's
// records are loaded while the current one is processed.  Partial sums are
// combined in a fixed order: the lane groups of a quarter as (g0 + g1) +
// (g2 + g3), then the two wavefronts of a block (if split) in order.
// A chunk has at most 64 candidates, so a list of n <= 64 hits padded to a
// multiple of four never exceeds 64 entries.  An entry is the 16-byte
// position record and the record's CT values (kept apart, so that the lists
// of C = 3 take 64 x 28 B x 4 quarters x 4 wavefronts = 28 KB per workgroup:
// five workgroups then fit a compute unit, where 32-byte entries left room
// for four -- 7% faster on the 1024^2 workload).
constexpr int kQuarterList = 64;
static_assert(kQuarterList >= 64 && kQuarterList % 4 == 0, "a list holds a whole padded chunk");
template <int CT>
__host__ __device__ inline constexpr int fwd_quarter_lds_f4() {
  // per wavefront: 4 x kQuarterList position records, then CT values each
  return 4 * (4 * kQuarterList + (4 * kQuarterList * CT + 3) / 4);
}

__host__ __device__ inline int fwd_units(int bx_blocks, int by_blocks) {
  return FwdUnits(bx_blocks, by_blocks).count();
}

// Bins whose records can reach pixels of the box [u0, ue] x [v0, ve]: the
// bin columns [*bx_lo, *bx_hi] of the bin rows [*by_lo, *by_hi].
__device__ inline void box_bins(const ImageView& v, int u0, int ue, int v0, int ve, int* bx_lo,
                                int* bx_hi, int* by_lo, int* by_hi) {
  const float Rh = conservative_reach(v.reach[0]);
  *bx_lo = bin_coord((float)u0 - Rh, v.inv_tile, v.nbx);
  *bx_hi = bin_coord((float)ue + Rh, v.inv_tile, v.nbx);
  *by_lo = bin_coord((float)v0 - Rh, v.inv_tile, v.nby);
  *by_hi = bin_coord((float)ve + Rh, v.inv_tile, v.nby);
}

// Pixel box of block (bxb, byb): [u0, ue] x [v0, ve]
__device__ inline void block_box(const ImageView& v, int bxb, int byb, int* u0, int* ue, int* v0,
                                 int* ve) {
  *u0 = bxb * kBlockSide;
  *v0 = byb * kBlockSide;
  *ue = min(*u0 + kBlockSide - 1, v.W - 1);
  *ve = min(*v0 + kBlockSide - 1, v.H - 1);
}

// Candidate records of block sb (0..3) of a forward unit (the cost estimate
// of the plan); 0 for blocks outside the image and for padding units.
__device__ inline int block_candidates(const ImageView& v, int unit, int sb) {
  int ucx, ucy;
  const bool in_grid = FwdUnits(v.bx_blocks, v.by_blocks).coords(unit, &ucx, &ucy);
  const int bxb = ucx * 2 + (sb & 1), byb = ucy * 2 + (sb >> 1);
  if (!in_grid || bxb >= v.bx_blocks || byb >= v.by_blocks) return 0;
  int u0, ue, v0, ve, bx_lo, bx_hi, by_lo, by_hi;
  block_box(v, bxb, byb, &u0, &ue, &v0, &ve);
  box_bins(v, u0, ue, v0, ve, &bx_lo, &bx_hi, &by_lo, &by_hi);
  int cost = 0;
  for (int r = by_lo; r <= by_hi; ++r)
    cost += v.offset[r * v.nbx + bx_hi + 1] - v.offset[r * v.nbx + bx_lo];
  return cost;
}
__device__ inline void unit_candidates(const ImageView& v, int unit, int cost[4]) {
  for (int sb = 0; sb < 4; ++sb) cost[sb] = block_candidates(v, unit, sb);
}

// A unit whose blocks hold kHeavyUnit or more candidate records is evaluated
// as two halves (modes 1 and 2), any other unit whole (mode 0).  Both paths
// take this decision the same way, so a pixel's sum is taken in the same
// order alone and in a batch.
constexpr int kHeavyUnit = 8192;
__device__ inline bool unit_is_heavy(const int cost[4]) {
  return cost[0] + cost[1] + cost[2] + cost[3] >= kHeavyUnit;
}

// mode 0: the whole unit, wavefront w on block w; mode 1 / 2: blocks 0-1 /
// 2-3, wavefronts 2b and 2b+1 on the b-th of them.
template <int CT, int KV = 0, int ST = INTERP_STORAGE_F32>
__device__ inline void forward_block_q(const ImageView& v, int unit, int mode, float4* s_rec) {
  static_assert(CT <= 4, "the quarter lists hold the values of a record in one float4");
  constexpr int NC = CT;
  const float r2 = v.r2;
  const int lane = threadIdx.x & 63, wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int grp = lane >> 4, p = lane & 15;
  const int split = mode == 0 ? 1 : 2;                         // wavefronts per block
  const int sb = mode == 0 ? wid : 2 * (mode - 1) + (wid >> 1);  // this wavefront's block
  const int phase = mode == 0 ? 0 : (wid & 1);
  int ucx, ucy;
  const bool in_grid = FwdUnits(v.bx_blocks, v.by_blocks).coords(unit, &ucx, &ucy);
  const int bxb = ucx * 2 + (sb & 1), byb = ucy * 2 + (sb >> 1);
  const bool active = in_grid && bxb < v.bx_blocks && byb < v.by_blocks;
  int u0, ue, v0, ve;
  block_box(v, active ? bxb : 0, active ? byb : 0, &u0, &ue, &v0, &ve);

  // quarter boxes: columns [u0, ul] and [u0 + 4, ur], rows [v0, vt] and [v0 + 4, vb]
  const float fu0 = (float)u0, fv0 = (float)v0;
  const float ful = (float)min(u0 + 3, ue), fur0 = (float)(u0 + 4), fure = (float)ue;
  const float fvt = (float)min(v0 + 3, ve), fvb0 = (float)(v0 + 4), fvbe = (float)ve;
  const bool has_r = u0 + 4 <= ue, has_b = v0 + 4 <= ve;
  // this lane's pixel in quarter q: (u0 + 4 (q & 1) + p % 4, v0 + 4 (q >> 1) + p / 4)
  const float pu = fu0 + (float)(p & 3), pv = fv0 + (float)(p >> 2);

  int bb[4];
  box_bins(v, u0, ue, v0, ve, &bb[0], &bb[1], &bb[2], &bb[3]);
  const int bx_lo = __builtin_amdgcn_readfirstlane(bb[0]);
  const int bx_hi = __builtin_amdgcn_readfirstlane(bb[1]);
  const int by_lo = __builtin_amdgcn_readfirstlane(bb[2]);
  const int by_hi = active ? __builtin_amdgcn_readfirstlane(bb[3]) : by_lo - 1;
  const float4* gb = v.geo;
  const float* cb = v.col;  // one group of four stored values per record

  float Z[4], acc[4][CT];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    Z[q] = 0.0f;
#pragma unroll
    for (int k = 0; k < CT; ++k) acc[q][k] = 0.0f;
  }

  constexpr int kWaveF4 = fwd_quarter_lds_f4<CT>() / 4;
  static_assert((CT + 1) * 256 <= 4 * fwd_quarter_lds_f4<CT>(), "the halves' sums fit the lists");
  float4* lst = s_rec + wid * kWaveF4;                               // [4][kQuarterList] records
  float* lcv = reinterpret_cast<float*>(lst + 4 * kQuarterList);     // [4][kQuarterList][CT] values
  // the padding record fails every kernel's radius test: its NaN position
  // makes d2 (or m2) NaN, and NaN <= anything is false (w = 0)
  const float4 null_geo = make_float4(__builtin_nanf(""), __builtin_nanf(""), 0.0f, -1.0f);
  const float4 zero4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);

  // bin rows in groups of 64 (one row per lane)
  for (int rg = by_lo; rg <= by_hi; rg += 64) {
    const int nr = min(64, by_hi - rg + 1);
    int s_r = 0, len = 0;
    if (lane < nr) {
      const int* o = v.offset + (size_t)(rg + lane) * v.nbx;
      s_r = o[bx_lo];
      len = o[bx_hi + 1] - s_r;
    }
    // Chunk cursor (wave-uniform): row r of the group, offset c in it, the
    // row's first record rs and length rn.  Chunks are 64 records of one row;
    // when two wavefronts share the block they take alternate chunks.
    struct Cursor {
      int r, c, rs, rn;
    };
    auto advance = [&](Cursor& k) {
      k.c += 64;
      while (k.c >= k.rn) {
        if (++k.r >= nr) return;
        k.c = 0;
        k.rs = __builtin_amdgcn_readlane(s_r, k.r);
        k.rn = __builtin_amdgcn_readlane(len, k.r);
      }
    };
    Cursor cur{-1, -64, 0, 0};
    advance(cur);
    if (phase) advance(cur);
    float4 g_n = zero4, c_n = zero4;
    if (cur.r < nr && cur.c + lane < cur.rn) {
      g_n = gb[cur.rs + cur.c + lane];
      c_n = Val<ST>::load4(cb, cur.rs + cur.c + lane);
    }
    while (cur.r < nr) {
      const bool in = cur.c + lane < cur.rn;
      const float4 g = g_n, c = c_n;
      Cursor nxt = cur;
      advance(nxt);
      if (split == 2) advance(nxt);
      if (nxt.r < nr && nxt.c + lane < nxt.rn) {
        g_n = gb[nxt.rs + nxt.c + lane];
        c_n = Val<ST>::load4(cb, nxt.rs + nxt.c + lane);
      }
      cur = nxt;
      // disk of the candidate against the box of each quarter (conservative)
      const float lim = reach_lim<KV>(g, r2);
      const float exl = fmaxf(fmaxf(fu0 - g.x, g.x - ful), 0.0f);
      const float exr = fmaxf(fmaxf(fur0 - g.x, g.x - fure), 0.0f);
      const float eyt = fmaxf(fmaxf(fv0 - g.y, g.y - fvt), 0.0f);
      const float eyb = fmaxf(fmaxf(fvb0 - g.y, g.y - fvbe), 0.0f);
      const float xl = box_sq<KV>(exl, g.z), xr = box_sq<KV>(exr, g.z);
      const float yt = box_sq<KV>(eyt, g.w), yb = box_sq<KV>(eyb, g.w);
      const bool h[4] = {in && xl + yt <= lim, in && has_r && xr + yt <= lim,
                         in && has_b && xl + yb <= lim, in && has_r && has_b && xr + yb <= lim};
      unsigned long long m[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) m[q] = __ballot(h[q]);
      if ((m[0] | m[1] | m[2] | m[3]) == 0) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int slot = __builtin_amdgcn_mbcnt_hi((unsigned)(m[q] >> 32),
                                                   __builtin_amdgcn_mbcnt_lo((unsigned)m[q], 0));
        if (h[q]) {
          lst[q * kQuarterList + slot] = g;
          float* dv = lcv + (q * kQuarterList + slot) * CT;
          const float cx[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
          for (int k = 0; k < CT; ++k) dv[k] = cx[k];
        }
      }
      int nit[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int n = __popcll(m[q]);
        const int pad = (-n) & 3;
        if (lane < pad) {
          lst[q * kQuarterList + n + lane] = null_geo;
          float* dv = lcv + (q * kQuarterList + n + lane) * CT;
#pragma unroll
          for (int k = 0; k < CT; ++k) dv[k] = 0.0f;
        }
        nit[q] = (n + 3) >> 2;
      }
      wave_lds_sync();
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float fu = pu + (float)(4 * (q & 1)), fv = pv + (float)(4 * (q >> 1));
        const float4* L = lst + q * kQuarterList + grp;
        const float* LV = lcv + (q * kQuarterList + grp) * CT;
        for (int i = 0; i < nit[q]; ++i) {
          const float4 r = L[4 * i];
          float cc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
          for (int k = 0; k < CT; ++k) cc[k] = LV[4 * CT * i + k];
          float w = pair_weight<KV>(fu, fv, r, r2);
          if constexpr (kNormalized<KV>) w *= record_density<kDiagonal<KV>>(r);
          Z[q] += w;
#pragma unroll
          for (int k = 0; k < NC; ++k) acc[q][k] = __builtin_fmaf(w, cc[k], acc[q][k]);
        }
      }
      wave_lds_sync();
    }
  }

  // lane groups: (g0 + g1) + (g2 + g3) per quarter; lane group q keeps quarter q
  float part[CT + 1];
#pragma unroll
  for (int k = 0; k <= CT; ++k) part[k] = 0.0f;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
#pragma unroll
    for (int k = 0; k <= CT; ++k) {
      float a = k < CT ? acc[q][k] : Z[q];
      a += __shfl_xor(a, 16);
      a += __shfl_xor(a, 32);
      part[k] = grp == q ? a : part[k];
    }
  }
  // the two wavefronts of a block (halves), through the (now free) list memory
  if (mode != 0) {
    __syncthreads();
    float* red = reinterpret_cast<float*>(s_rec);
#pragma unroll
    for (int k = 0; k <= CT; ++k) red[(k * 4 + wid) * 64 + lane] = part[k];
    __syncthreads();
    const float* r0 = red + (wid & ~1) * 64 + lane;
#pragma unroll
    for (int k = 0; k <= CT; ++k) part[k] = r0[k * 256] + r0[k * 256 + 64];
  }
  const float Zo = part[CT];
  const int u = u0 + 4 * (grp & 1) + (p & 3), vv = v0 + 4 * (grp >> 1) + (p >> 2);
  if (active && phase == 0 && u <= ue && vv <= ve) {
    const size_t HW = (size_t)v.H * v.W;
    const size_t pix = (size_t)vv * v.W + u;
#pragma unroll
    for (int k = 0; k < CT; ++k) {
      if (k < v.C) Val<ST>::store(v.out, k * HW + pix, Zo > 0.0f ? part[k] / Zo : 0.0f);
    }
    v.Z[pix] = Zo;
  }
}

// ---------------------------------------------------------------------------
// Backward
// ---------------------------------------------------------------------------

// unit = 256 pixels: G'_ik = G_ik / Z_i and beta_i = sum_k G_ik out_ik / Z_i.
// Interleaved ([H*W][CP]: G'_0 .. G'_{CT-1}, beta, zero padding) for the
// one-lane-per-point adjoint; planar for the eight-lanes-per-point adjoint of
// many channels (CT a multiple of four): [CT/4][H*W] groups of four G' values,
// then [H*W] betas (a plane of its own, so that reading beta costs 4 bytes,
// not a padded group of 16).
template <int CT, int ST = INTERP_STORAGE_F32, bool kPlanar = false>
__device__ inline void bwd_pixel(const ImageView& v, int unit) {
  constexpr int CP = (CT + 1 + 3) / 4 * 4;
  const int HW = v.H * v.W;
  const int i = unit * 256 + threadIdx.x;
  if (i >= HW) return;
  const float z = v.Z[i];
  float rec[CP];
#pragma unroll
  for (int k = 0; k < CP; ++k) rec[k] = 0.0f;
  if (z > 0.0f) {
    const float a = 1.0f / z;
    float beta = 0.0f;
#pragma unroll
    for (int k = 0; k < CT; ++k) {
      if (k < v.C) {
        const size_t idx = (size_t)k * HW + i;
        const float gk = Val<ST>::load(v.grad_out, idx);
        rec[k] = gk * a;
        beta = __builtin_fmaf(gk, Val<ST>::load(v.out, idx), beta);
      }
    }
    rec[CT] = beta * a;
  }
  if constexpr (kPlanar) {
    static_assert(CT % 4 == 0, "planar records: whole groups of four values");
    float4* dst = reinterpret_cast<float4*>(v.prec) + i;
#pragma unroll
    for (int q = 0; q < CT / 4; ++q)
      dst[(size_t)q * HW] = make_float4(rec[4 * q], rec[4 * q + 1], rec[4 * q + 2], rec[4 * q + 3]);
    reinterpret_cast<float*>(reinterpret_cast<float4*>(v.prec) + (size_t)(CT / 4) * HW)[i] = rec[CT];
  } else {
    float4* dst = reinterpret_cast<float4*>(v.prec + (size_t)i * CP);
#pragma unroll
    for (int q = 0; q < CP / 4; ++q)
      dst[q] = make_float4(rec[4 * q], rec[4 * q + 1], rec[4 * q + 2], rec[4 * q + 3]);
  }
}

// Pixel records a workgroup of the adjoint can stage in LDS (36 KB).
constexpr int kBwdStageF4 = 2304;
// The adjoint walks each row of a disk in whole groups of kBwdGroup pixels
// (padding pixels get w = 0).  Groups of 2 pad fewer pixels on the short
// chords of small disks but measured slower than groups of 4, whose four
// independent weights keep more work in flight per loop trip.
constexpr int kBwdGroup = 4;

// unit = 256 points in sorted order.  When the unit's points lie in one bin
// row and the pixel records they can reach fit in kBwdStageF4 float4s, the
// block first copies that window of records to LDS (one coalesced pass)
// and the walk below reads LDS; otherwise it reads the records from global
// memory.  The block then regroups its points by the size of their disk (so
// the lanes of a wavefront loop over similar extents); each thread walks its
// point's disk row by row -- the columns of a row bounded by a conservative
// chord and visited without branching (pixels outside the radius get w = 0,
// so the loads can be issued ahead), the forward's radius test repeated bit
// for bit -- recomputes w_ij and accumulates in registers; results go to the
// point's own index.  A point's result does not depend on which lane
// computes it, and the shared-sigma partial sum is taken in the original
// point order: the output is deterministic.  lds: 256 + 32 ints; stage:
// kBwdStageF4 float4s.
template <int CT, int KV = 0, int ST = INTERP_STORAGE_F32>
__device__ inline void bwd_point(const ImageView& v, int unit, float* red4, int* lds,
                                 float4* stage) {
  constexpr int CS = CT < 4 ? 4 : CT;
  constexpr bool kD = kDiagonal<KV>, kN = kNormalized<KV>;
  constexpr int NC = CT;
  constexpr int CP = (NC + 1 + 3) / 4 * 4;  // pixel record: G'_0..G'_{NC-1}, beta
  constexpr int CP4 = CP / 4;
  int* order = lds;            // [256] local point index by regrouped slot
  int* cls_n = lds + 256;      // [32]
  float* gs_l = reinterpret_cast<float*>(lds);
  const int base = unit * 256;
  // the window of pixel records the unit's points can reach: bin columns
  // [first, last] of one bin row, widened by the image's reach and by
  // kBwdGroup - 1 pixels for the groups below
  // (bins recomputed from the saved sorted positions, as bin_keys made them)
  int rx0 = 0, rx1 = -1, ry0 = 0, ry1 = -1;
  {
    const float4 gf = v.geo[base], gl = v.geo[min(base + 255, v.N - 1)];
    const int byf = bin_coord(gf.y, v.inv_tile, v.nby), byl = bin_coord(gl.y, v.inv_tile, v.nby);
    if (byf == byl) {
      const int bxf = bin_coord(gf.x, v.inv_tile, v.nbx), bxl = bin_coord(gl.x, v.inv_tile, v.nbx);
      const float Rh = conservative_reach(v.reach[0]);
      const float T = (float)v.T;
      const float x0 = floorf((float)bxf * T - Rh) - (float)(kBwdGroup - 1);
      const float x1 = ceilf((float)(bxl + 1) * T + Rh) + (float)(kBwdGroup - 1);
      const float y0 = floorf((float)byf * T - Rh), y1 = ceilf((float)(byf + 1) * T + Rh);
      rx0 = (int)fmaxf(x0, 0.0f);
      rx1 = (int)fminf(x1, (float)(v.W - 1));
      ry0 = (int)fmaxf(y0, 0.0f);
      ry1 = (int)fminf(y1, (float)(v.H - 1));
    }
  }
  const int rw = rx1 - rx0 + 1, rh = ry1 - ry0 + 1;
  const bool staged = rw > 0 && rh > 0 && rw * rh * CP4 <= kBwdStageF4;
  if (staged) {
    const int rowf4 = rw * CP4;
    for (int i = threadIdx.x; i < rh * rowf4; i += 256) {
      const int r = i / rowf4, c = i - r * rowf4;
      stage[i] = reinterpret_cast<const float4*>(v.prec)[((size_t)(ry0 + r) * v.W + rx0) * CP4 + c];
    }
  }
  {
    const int tt = base + threadIdx.x;
    int cls = 0;
    if (tt < v.N) {
      const float4 gg = v.geo[tt];
      const float ext = kD ? v.radius / fmaxf(fminf(gg.z, gg.w), 1e-30f) : sqrtf(fmaxf(gg.w, 0.0f));
      cls = min(31, 1 + (int)fminf(2.0f * ext, 30.0f));
    }
    if (threadIdx.x < 32) cls_n[threadIdx.x] = 0;
    __syncthreads();
    const int slot = atomicAdd(&cls_n[cls], 1);
    __syncthreads();
    if (threadIdx.x == 0) {
      int run = 0;
      for (int c = 0; c < 32; ++c) { const int n = cls_n[c]; cls_n[c] = run; run += n; }
    }
    __syncthreads();
    order[cls_n[cls] + slot] = threadIdx.x;
    __syncthreads();
  }
  const int lp = order[threadIdx.x];
  const int t = base + lp;
  float gsig = 0.0f, gsig2 = 0.0f;
  if (t < v.N) {
    const float4 g = v.geo[t];
    float cc[CT];
#pragma unroll
    for (int k = 0; k < CT; ++k) cc[k] = Val<ST>::load(v.col, (size_t)t * CS + k);
    const float zeta = kN ? record_density<kD>(g) : 1.0f;
    const int j = v.perm[t];
    const float2 sg = record_sigma<kD>(g);
    const float Rhx = conservative_reach(__fmul_rn(v.radius, sg.x));
    const float Rh = conservative_reach(__fmul_rn(v.radius, sg.y));  // along y
    // bounding box of the disk (ellipse), clipped to the image (the float
    // clamps also drop NaN and keep the conversions in range)
    const float fvlo = fminf(fmaxf(ceilf(g.y - Rh), 0.0f), (float)v.H);
    const float fvhi = fmaxf(fminf(floorf(g.y + Rh), (float)(v.H - 1)), -1.0f);
    int vlo = (int)fvlo, vhi = (int)fvhi;
    if (staged) {  // a point of the unit never leaves the window; invalid inputs are cut to it
      vlo = max(vlo, ry0);
      vhi = min(vhi, ry1);
    }
    float gx = 0.0f, gy = 0.0f, gs = 0.0f, gs2 = 0.0f, ga = 0.0f;
    float gc[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) gc[k] = 0.0f;
    // squared radius of the chord computation, a little beyond the test's
    const float R2m = (kD ? v.r2 : g.w) * (1.0f + 0x1p-20f);
    // the disk walk; rec(py, px, q) returns float4 q of pixel (py, px)'s record
    // interior: the disk's box, widened by G - 1 pixels for the groups of G,
    // lies inside the image (and the staged window) for every lane of the
    // wavefront, so the rows need no clamping
    constexpr int G = kBwdGroup;
    const bool interior_lane = !(t < v.N) || (g.x - Rhx >= (float)max(rx0 * staged, 0) &&
                                              g.x + Rhx + (float)(G - 1) <=
                                                  (float)(staged ? rx1 : v.W - 1) &&
                                              g.y - Rh >= 0.0f && g.y + Rh <= (float)(v.H - 1));
    const bool interior = __ballot(!interior_lane) == 0;
    auto walk = [&](auto rec_of, auto interior_tag) {
      constexpr bool kInterior = decltype(interior_tag)::value;
      for (int py = vlo; py <= vhi; ++py) {
        const float dy = (float)py - g.y;
        // the row's term of the test: dy^2, or qy^2 = (dy / sigma_y)^2
        const float qy = kD ? dy * g.w : dy;
        const float dyy = qy * qy;
        // conservative chord of the disk on this row (v_sqrt_f32's error is
        // far inside the margin), widened to a multiple of G pixels inside the
        // image so that every row runs whole groups; every pixel is visited
        // without branching (pixels outside the radius get w = 0)
        const float rr = __builtin_amdgcn_sqrtf(fmaxf(R2m - dyy, 0.0f)) * (kD ? sg.x : 1.0f) *
                             (1.0f + 0x1p-10f) + 0x1p-10f;
        int ulo, uhi;
        if constexpr (kInterior) {
          ulo = (int)ceilf(g.x - rr);
          uhi = (int)floorf(g.x + rr);
        } else {
          ulo = (int)fminf(fmaxf(ceilf(g.x - rr), 0.0f), (float)v.W);
          uhi = (int)fmaxf(fminf(floorf(g.x + rr), (float)(v.W - 1)), -1.0f);
        }
        // px is the pixel column and fpx the same integer as a float (exact:
        // columns stay far below 2^24), so no conversion per pixel
        auto pixel = [&](int px, float fpx) {
          const float dx = fpx - g.x;
          // the forward's test and weight, bit for bit (pair_weight)
          const float qx = kD ? dx * g.z : dx;
          const float qxx = qx * qx;
          const float d2 = qxx + dyy;
          float rec[CP];
#pragma unroll
          for (int q = 0; q < CP4; ++q) {
            const float4 r4 = rec_of(py, px, q);
            rec[4 * q] = r4.x; rec[4 * q + 1] = r4.y; rec[4 * q + 2] = r4.z; rec[4 * q + 3] = r4.w;
          }
          float w = __builtin_amdgcn_exp2f(d2 * (kD ? kHalfLog2e : g.z));
          w = (d2 <= (kD ? v.r2 : g.w)) ? w : 0.0f;
          if constexpr (kN) w *= zeta;
          float A = -rec[NC];
#pragma unroll
          for (int k = 0; k < NC; ++k) A = __builtin_fmaf(rec[k], cc[k], A);
#pragma unroll
          for (int k = 0; k < NC; ++k) gc[k] = __builtin_fmaf(w, rec[k], gc[k]);
          const float tA = A * w;
          gx = __builtin_fmaf(tA, qx, gx);
          gy = __builtin_fmaf(tA, qy, gy);
          if constexpr (kD) {
            gs = __builtin_fmaf(tA, qxx, gs);
            gs2 = __builtin_fmaf(tA, dyy, gs2);
          } else {
            gs = __builtin_fmaf(tA, d2, gs);
          }
          if constexpr (kN) ga += tA;
        };
        auto groups = [&](int lo, int n) {  // n: a multiple of G
          float fpx = (float)lo;
          for (int px = lo; px < lo + n; px += G) {
#pragma unroll
            for (int i = 0; i < G; ++i) pixel(px + i, fpx + (float)i);
            fpx += (float)G;
          }
        };
        const int ng = (uhi - ulo + G) & ~(G - 1);
        if constexpr (kInterior) {
          groups(ulo, ng);  // the chord (ng = 0 when it is empty) and its padding are inside
        } else if (uhi >= ulo && ng <= v.W) {
          // whole groups of G pixels, the window moved inside the image
          ulo = min(ulo, v.W - ng);
          if (staged && (ulo < rx0 || ulo + ng - 1 > rx1)) continue;  // only for invalid inputs
          groups(ulo, ng);
        } else {
          if (staged) {
            ulo = max(ulo, rx0);
            uhi = min(uhi, rx1);
          }
          for (int px = ulo; px <= uhi; ++px) pixel(px, (float)px);
        }
      }
    };
    auto from_stage = [&](int py, int px, int q) {
      return stage[((py - ry0) * rw + (px - rx0)) * CP4 + q];
    };
    const float4* prec4 = reinterpret_cast<const float4*>(v.prec);
    auto from_global = [&](int py, int px, int q) {
      return prec4[((size_t)py * v.W + px) * CP4 + q];
    };
    using Yes = std::integral_constant<bool, true>;
    using No = std::integral_constant<bool, false>;
    if (staged) {
      if (interior) walk(from_stage, Yes{}); else walk(from_stage, No{});
    } else {
      if (interior) walk(from_global, Yes{}); else walk(from_global, No{});
    }
    // chain rule through the weight: d w / d x = w dx / sigma^2 (isotropic)
    // or w qx / sigma_x (diagonal); d w / d sigma = w d2 / sigma^3 or
    // w qx^2 / sigma_x; a normalised kernel's factor adds -2 w / sigma or
    // -w / sigma_x
    float2 gp;
    if constexpr (kD) {
      gp = make_float2(gx * g.z, gy * g.w);
      gsig = (kN ? gs - ga : gs) * g.z;
      gsig2 = (kN ? gs2 - ga : gs2) * g.w;
    } else {
      const float inv_s2 = 1.0f / (sg.x * sg.x);
      gp = make_float2(gx * inv_s2, gy * inv_s2);
      gsig = gs * inv_s2 / sg.x;
      if constexpr (kN) gsig -= 2.0f * ga / sg.x;
    }
    if (v.grad_pos) reinterpret_cast<float2*>(v.grad_pos)[j] = gp;
    if (v.grad_sigma && v.per_point) {
      if constexpr (kD) reinterpret_cast<float2*>(v.grad_sigma)[j] = make_float2(gsig, gsig2);
      else v.grad_sigma[j] = gsig;
    }
    if (v.grad_values) {
      // the point's values' gradient is one scattered store where it can be
      // (a float32 vector of C = 2..4 elements needs only 4-byte alignment)
      if constexpr (ST == INTERP_STORAGE_F32 && NC >= 2 && NC <= 4) {
        typedef float vnu __attribute__((ext_vector_type(NC), aligned(4)));
        if (v.C == NC) {
          vnu x;
#pragma unroll
          for (int k = 0; k < NC; ++k) x[k] = gc[k];
          *reinterpret_cast<vnu*>(v.grad_values + (size_t)j * NC) = x;
        } else {
#pragma unroll
          for (int k = 0; k < NC; ++k)
            if (k < v.C) v.grad_values[(size_t)j * v.C + k] = gc[k];
        }
      } else {
#pragma unroll
        for (int k = 0; k < NC; ++k)
          if (k < v.C) Val<ST>::store(v.grad_values, (size_t)j * v.C + k, gc[k]);
      }
    }
  }
  if (!v.per_point && v.grad_sigma) {
    // the shared sigma's derivative: per-unit partial sums in point order
    __syncthreads();
    gs_l[lp] = gsig;
    __syncthreads();
    const float s = block_sum(gs_l[threadIdx.x], red4);
    if (threadIdx.x == 0) v.gpart[2 * unit] = s;
    if constexpr (kD) {
      gs_l[lp] = gsig2;
      __syncthreads();
      const float s2 = block_sum(gs_l[threadIdx.x], red4);
      if (threadIdx.x == 0) v.gpart[2 * unit + 1] = s2;
    }
  }
}

// Adjoint for eight or more value slots (CT >= 8).  One lane per point
// would read a whole pixel record (CP values) per pixel from a different
// place in every lane; here eight lanes share a point instead: a wavefront
// takes eight points at a time, lane group g = lane / 8 on one point and
// lane l = lane % 8 on columns l, l + 8, ... of each row of its disk, so
// that the group reads eight neighbouring pixels -- one 128-byte line per
// group of four values of the planar pixel records.  A round of the
// workgroup takes 32 consecutive points of the unit (in sorted order, so
// their disks overlap and share records in the caches), ordered by disk
// size among themselves; rows are walked in pairs, one pixel of each per
// trip, for two independent chains per lane.  The test and the
// weight per pixel are the one-lane kernel's, bit for bit; a group's partial
// sums are combined by an xor butterfly over its eight lanes (every lane
// ends with the same bits) and its lanes write the point's results.  gs_l,
// gs2_l: 256 floats each.
template <int CT, int KV = 0, int ST = INTERP_STORAGE_F32>
__device__ inline void bwd_point_wide(const ImageView& v, int unit, float* red4, float* gs_l,
                                      float* gs2_l, int* cls_l, int* order) {
  static_assert(CT >= 8, "eight lanes per point pay off for wide records only");
  constexpr int CS = CT;
  constexpr bool kD = kDiagonal<KV>, kN = kNormalized<KV>;
  constexpr int NC = CT;
  const int base = unit * 256;
  // within each round of 32 consecutive points, the points in order of disk
  // size (class of half a pixel of extent, ties by position), so that the
  // eight points of a wavefront loop over similar extents
  {
    const int tt = base + threadIdx.x;
    int cls = 0;
    if (tt < v.N) {
      const float4 gg = v.geo[tt];
      const float ext = kD ? v.radius / fmaxf(fminf(gg.z, gg.w), 1e-30f) : sqrtf(fmaxf(gg.w, 0.0f));
      cls = (int)fminf(2.0f * ext, 1e6f);
    }
    cls_l[threadIdx.x] = cls;
    __syncthreads();
    const int r0 = threadIdx.x & ~31, me = threadIdx.x & 31;
    int rank = 0;
    for (int k = 0; k < 32; ++k) {
      const int ck = cls_l[r0 + k];
      rank += (ck < cls || (ck == cls && k < me)) ? 1 : 0;
    }
    order[r0 + rank] = threadIdx.x;
    __syncthreads();
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int grp = lane >> 3, l = lane & 7;
  const size_t HW = (size_t)v.H * v.W;
  const float4* prec4 = reinterpret_cast<const float4*>(v.prec);
  const float* betap = reinterpret_cast<const float*>(prec4 + (size_t)(NC / 4) * HW);
  for (int r = 0; r < 8; ++r) {
    const int lp = order[r * 32 + wid * 8 + grp];
    const int t = base + lp;
    if (t >= v.N) continue;
    const float4 g = v.geo[t];
    float cc[CT];
#pragma unroll
    for (int q = 0; q < CT / 4; ++q) {
      const float4 c4 = Val<ST>::load4(v.col, (size_t)t * (CS / 4) + q);
      cc[4 * q] = c4.x; cc[4 * q + 1] = c4.y; cc[4 * q + 2] = c4.z; cc[4 * q + 3] = c4.w;
    }
    const float zeta = kN ? record_density<kD>(g) : 1.0f;
    const int j = v.perm[t];
    const float2 sg = record_sigma<kD>(g);
    const float Rh = conservative_reach(__fmul_rn(v.radius, sg.y));  // along y
    const float fvlo = fminf(fmaxf(ceilf(g.y - Rh), 0.0f), (float)v.H);
    const float fvhi = fmaxf(fminf(floorf(g.y + Rh), (float)(v.H - 1)), -1.0f);
    const int vlo = (int)fvlo, vhi = (int)fvhi;
    float gx = 0.0f, gy = 0.0f, gs = 0.0f, gs2 = 0.0f, ga = 0.0f;
    float gc[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) gc[k] = 0.0f;
    const float R2m = (kD ? v.r2 : g.w) * (1.0f + 0x1p-20f);
    // the chord of row py: columns [ulo, uhi] (conservative: the radius
    // test decides), clipped to the image
    auto chord = [&](int py, float* dyy_o, float* qy_o, int* ulo_o, int* uhi_o) {
      const float dy = (float)py - g.y;
      const float qy = kD ? dy * g.w : dy;
      const float dyy = qy * qy;
      const float rr = __builtin_amdgcn_sqrtf(fmaxf(R2m - dyy, 0.0f)) * (kD ? sg.x : 1.0f) *
                           (1.0f + 0x1p-10f) + 0x1p-10f;
      *ulo_o = (int)fminf(fmaxf(ceilf(g.x - rr), 0.0f), (float)v.W);
      *uhi_o = (int)fmaxf(fminf(floorf(g.x + rr), (float)(v.W - 1)), -1.0f);
      *dyy_o = dyy;
      *qy_o = qy;
    };
    // pixel (px, py) with its record read at column pxc of the row (pxc is
    // px inside the chord; w = 0 when px is not)
    auto pixel = [&](int py, int px, bool inside, int pxc, float dyy, float qy) {
      const float4* rowp = prec4 + (size_t)py * v.W;
      float rec[NC + 1];
#pragma unroll
      for (int q = 0; q < NC / 4; ++q) {
        const float4 r4 = rowp[(size_t)q * HW + pxc];
        rec[4 * q] = r4.x; rec[4 * q + 1] = r4.y; rec[4 * q + 2] = r4.z; rec[4 * q + 3] = r4.w;
      }
      rec[NC] = betap[(size_t)py * v.W + pxc];
      const float dx = (float)px - g.x;
      const float qx = kD ? dx * g.z : dx;
      const float qxx = qx * qx;
      const float d2 = qxx + dyy;
      float w = __builtin_amdgcn_exp2f(d2 * (kD ? kHalfLog2e : g.z));
      w = (inside && d2 <= (kD ? v.r2 : g.w)) ? w : 0.0f;
      if constexpr (kN) w *= zeta;
      // A in four partial chains (a 16-deep chain of dependent FMAs would
      // leave the lane waiting on each result)
      float Ap[4] = {-rec[NC], 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int k = 0; k < NC; ++k) Ap[k & 3] = __builtin_fmaf(rec[k], cc[k], Ap[k & 3]);
      const float A = (Ap[0] + Ap[1]) + (Ap[2] + Ap[3]);
#pragma unroll
      for (int k = 0; k < NC; ++k) gc[k] = __builtin_fmaf(w, rec[k], gc[k]);
      const float tA = A * w;
      gx = __builtin_fmaf(tA, qx, gx);
      gy = __builtin_fmaf(tA, qy, gy);
      if constexpr (kD) {
        gs = __builtin_fmaf(tA, qxx, gs);
        gs2 = __builtin_fmaf(tA, dyy, gs2);
      } else {
        gs = __builtin_fmaf(tA, d2, gs);
      }
      if constexpr (kN) ga += tA;
    };
    // rows in pairs: every trip evaluates one pixel of each row (two
    // independent chains per lane) over the union of the two chords
    for (int py = vlo; py <= vhi; py += 2) {
      float dyyA, qyA, dyyB = 0.0f, qyB = 0.0f;
      int uloA, uhiA, uloB = 1, uhiB = 0;
      chord(py, &dyyA, &qyA, &uloA, &uhiA);
      const bool hasB = py + 1 <= vhi;
      if (hasB) chord(py + 1, &dyyB, &qyB, &uloB, &uhiB);
      // an empty chord takes the other's start (no pixel of it is inside)
      if (uloB > uhiB) { uloB = uloA; uhiB = uloA - 1; }
      if (uloA > uhiA) { uloA = uloB; uhiA = uloB - 1; }
      const int lo = min(uloA, uloB), hi = max(uhiA, uhiB);
      const int rowB = hasB ? py + 1 : py;
      for (int s0 = lo; s0 <= hi; s0 += 8) {
        const int px = s0 + l;
        const bool inA = px >= uloA && px <= uhiA, inB = px >= uloB && px <= uhiB;
        // load columns inside the image: the chord's (or its start's)
        const int pA = min(min(max(px, uloA), max(uhiA, uloA)), v.W - 1);
        const int pB = min(min(max(px, uloB), max(uhiB, uloB)), v.W - 1);
        pixel(py, px, inA, pA, dyyA, qyA);
        pixel(rowB, px, inB, pB, dyyB, qyB);
      }
    }
    // the group's sums (xor butterfly: every lane of the group ends with the
    // same bits)
    auto gsum = [](float x) {
      x += __shfl_xor(x, 1);
      x += __shfl_xor(x, 2);
      x += __shfl_xor(x, 4);
      return x;
    };
#pragma unroll
    for (int k = 0; k < NC; ++k) gc[k] = gsum(gc[k]);
    gx = gsum(gx);
    gy = gsum(gy);
    gs = gsum(gs);
    if constexpr (kD) gs2 = gsum(gs2);
    if constexpr (kN) ga = gsum(ga);
    float2 gp;
    float gsig, gsig2 = 0.0f;
    if constexpr (kD) {
      gp = make_float2(gx * g.z, gy * g.w);
      gsig = (kN ? gs - ga : gs) * g.z;
      gsig2 = (kN ? gs2 - ga : gs2) * g.w;
    } else {
      const float inv_s2 = 1.0f / (sg.x * sg.x);
      gp = make_float2(gx * inv_s2, gy * inv_s2);
      gsig = gs * inv_s2 / sg.x;
      if constexpr (kN) gsig -= 2.0f * ga / sg.x;
    }
    if (l == 0) {
      if (v.grad_pos) reinterpret_cast<float2*>(v.grad_pos)[j] = gp;
      if (v.grad_sigma && v.per_point) {
        if constexpr (kD) reinterpret_cast<float2*>(v.grad_sigma)[j] = make_float2(gsig, gsig2);
        else v.grad_sigma[j] = gsig;
      }
      gs_l[lp] = gsig;
      gs2_l[lp] = gsig2;
    }
    if (v.grad_values) {
      // lane l writes channels l, l + 8, ...: eight consecutive values of
      // the point per store
#pragma unroll
      for (int m = 0; m < (NC + 7) / 8; ++m) {
        float x = gc[8 * m];
#pragma unroll
        for (int kk = 1; kk < 8; ++kk)
          if (8 * m + kk < NC) x = l == kk ? gc[8 * m + kk] : x;
        const int k = 8 * m + l;
        if (k < NC && k < v.C) Val<ST>::store(v.grad_values, (size_t)j * v.C + k, x);
      }
    }
  }
  if (!v.per_point && v.grad_sigma) {
    // the shared sigma's derivative: per-unit partial sums in point order
    // (points beyond N contribute nothing)
    __syncthreads();
    const bool own = base + (int)threadIdx.x < v.N;
    const float s = block_sum(own ? gs_l[threadIdx.x] : 0.0f, red4);
    if (threadIdx.x == 0) v.gpart[2 * unit] = s;
    if constexpr (kD) {
      const float s2 = block_sum(own ? gs2_l[threadIdx.x] : 0.0f, red4);
      if (threadIdx.x == 0) v.gpart[2 * unit + 1] = s2;
    }
  }
}

// one 256-thread block per image: grad_sigma = fixed-order sum of gpart
// (one value per sigma component)
__device__ inline void bwd_sigma_sum(const ImageView& v, float* red4) {
  for (int a = 0; a < v.nsig; ++a) {
    float s = 0.0f;
    for (int q = threadIdx.x; q < v.units256; q += 256) s += v.gpart[2 * q + a];
    s = block_sum(s, red4);
    if (threadIdx.x == 0) v.grad_sigma[a] = s;
  }
}

}  // namespace dev
}  // namespace gmm
