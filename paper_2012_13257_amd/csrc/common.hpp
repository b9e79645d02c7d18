// Shared host/device definitions of libgmminterp: problem geometry, buffer
// layouts of the saved state and the workspace, and launch helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "gmminterp.h"

namespace gmm {

constexpr int kBlockSide = 8;          // one wavefront owns an 8x8 pixel block
constexpr int kWave = 64;
constexpr int kMaxChannels = 32;
constexpr float kMaxRadius = 12.0f;    // exp2 of -r^2/2*log2(e) stays a normal float
constexpr size_t kAlign = 256;

inline size_t align_up(size_t x, size_t a = kAlign) { return (x + a - 1) / a * a; }

// Channel count the kernels are instantiated for: the smallest of
// {1,2,3,4,8,16,32} that is >= C.  Extra channels are zero padding.
inline int channel_template(int C) {
  if (C <= 4) return C;
  if (C <= 8) return 8;
  if (C <= 16) return 16;
  return 32;
}
// Floats per sorted point record of values (16-byte multiple).
inline int col_stride(int C) { int t = channel_template(C); return t < 4 ? 4 : t; }
// Floats per backward pixel record (G'_0..G'_{CT-1}, beta), 16-byte multiple.
inline int pix_stride(int C) { return (channel_template(C) + 1 + 3) / 4 * 4; }

struct Geometry {
  int B, N, C, H, W, T;
  int nbx, nby, nb;
  int CT, CS, CP;
  float radius;
  int per_point;
  int bx_blocks, by_blocks;            // 8x8 pixel blocks per image row / column
};

// Byte offsets of every array inside the saved buffer and the workspace.
struct Layout {
  // saved
  size_t Z, reach, offset, perm, geo, col, saved_bytes;
  // workspace
  size_t count, slot, binof, tmp, prec, gpart, work_bytes;
};

inline int bwd_groups_per_image(const Geometry& g) { return (g.N + 255) / 256; }

inline Layout make_layout(const Geometry& g) {
  Layout L{};
  size_t o = 0;
  const size_t B = g.B, N = g.N, HW = size_t(g.H) * g.W;
  L.Z = o;      o = align_up(o + B * HW * 4);
  L.reach = o;  o = align_up(o + B * 4);
  L.offset = o; o = align_up(o + B * (size_t(g.nb) + 1) * 4);
  L.perm = o;   o = align_up(o + B * N * 4);
  L.geo = o;    o = align_up(o + B * N * 16);
  L.col = o;    o = align_up(o + B * N * size_t(g.CS) * 4);
  L.saved_bytes = o;
  o = 0;
  L.count = o;  o = align_up(o + B * size_t(g.nb) * 4);
  L.slot = o;   o = align_up(o + B * N * 4);
  L.binof = o;  o = align_up(o + B * N * 4);
  L.tmp = o;    o = align_up(o + B * N * 4);
  L.prec = o;   o = align_up(o + B * HW * size_t(g.CP) * 4);
  L.gpart = o;  o = align_up(o + B * size_t(bwd_groups_per_image(g)) * 4 + 4);
  L.work_bytes = o;
  return L;
}

// Validates the problem; fills g and returns "" or an error message.
inline std::string make_geometry(const interp_problem* p, Geometry* g) {
  if (!p) return "problem is NULL";
  if (p->B < 1) return "B must be >= 1";
  if (p->N < 0) return "N must be >= 0";
  if (p->C < 1 || p->C > kMaxChannels) return "C must be in [1, 32]";
  if (p->H < 1 || p->W < 1 || p->H > 32768 || p->W > 32768) return "H and W must be in [1, 32768]";
  if (!(p->radius > 0.0f) || !(p->radius <= kMaxRadius)) return "radius must be in (0, 12]";
  if (p->sigma_per_point != 0 && p->sigma_per_point != 1) return "sigma_per_point must be 0 or 1";
  int T = p->tile == 0 ? 8 : p->tile;
  if (T != 4 && T != 8 && T != 16 && T != 32 && T != 64) return "tile must be 0, 4, 8, 16, 32 or 64";
  const long long BN = (long long)p->B * p->N;
  const long long BHW = (long long)p->B * p->H * p->W;
  if (BN >= (1LL << 31)) return "B*N must be below 2^31";
  if (BHW >= (1LL << 31)) return "B*H*W must be below 2^31";
  if ((long long)p->B * p->N * channel_template(p->C) >= (1LL << 31)) return "B*N*C must be below 2^31";
  if (BHW * pix_stride(p->C) >= (1LL << 31)) return "B*H*W*(C+1) must be below 2^31";
  g->B = p->B; g->N = p->N; g->C = p->C; g->H = p->H; g->W = p->W; g->T = T;
  g->nbx = (p->W + T - 1) / T;
  g->nby = (p->H + T - 1) / T;
  g->nb = g->nbx * g->nby;
  g->CT = channel_template(p->C);
  g->CS = col_stride(p->C);
  g->CP = pix_stride(p->C);
  g->radius = p->radius;
  g->per_point = p->sigma_per_point;
  g->bx_blocks = (p->W + kBlockSide - 1) / kBlockSide;
  g->by_blocks = (p->H + kBlockSide - 1) / kBlockSide;
  return "";
}

// Device view of the saved state and the workspace.
struct Views {
  float* Z;
  float* reach;      // per image: conservative neighbour reach in pixels
  int* offset;       // [B, nb+1]
  int* perm;         // [B, N]
  float4* geo;       // [B, N] sorted (x, y, k, R2), k = -log2(e)/(2 sigma^2)
  float* col;        // [B, N, CS] sorted values
  int* count;        // [B, nb]
  int* slot;         // [B, N]
  int* binof;        // [B, N]
  int* tmp;          // [B, N]
  float* prec;       // [B, H, W, CP]
  float* gpart;      // [B, groups]
};

inline Views make_views(const Layout& L, void* saved, void* work) {
  char* s = static_cast<char*>(saved);
  char* w = static_cast<char*>(work);
  Views v;
  v.Z = reinterpret_cast<float*>(s + L.Z);
  v.reach = reinterpret_cast<float*>(s + L.reach);
  v.offset = reinterpret_cast<int*>(s + L.offset);
  v.perm = reinterpret_cast<int*>(s + L.perm);
  v.geo = reinterpret_cast<float4*>(s + L.geo);
  v.col = reinterpret_cast<float*>(s + L.col);
  v.count = reinterpret_cast<int*>(w + L.count);
  v.slot = reinterpret_cast<int*>(w + L.slot);
  v.binof = reinterpret_cast<int*>(w + L.binof);
  v.tmp = reinterpret_cast<int*>(w + L.tmp);
  v.prec = reinterpret_cast<float*>(w + L.prec);
  v.gpart = reinterpret_cast<float*>(w + L.gpart);
  return v;
}

// Kernel launch entry points (defined in the kernel translation units).
hipError_t launch_binning(const Geometry& g, const float* pos, const float* sigma,
                          const float* values, const Views& v, hipStream_t st);
hipError_t launch_forward(const Geometry& g, const Views& v, float* out, hipStream_t st);
hipError_t launch_backward(const Geometry& g, const float* sigma, const float* out,
                           const float* grad_out, float* grad_pos, float* grad_sigma,
                           float* grad_values, const Views& v, hipStream_t st);

}  // namespace gmm
