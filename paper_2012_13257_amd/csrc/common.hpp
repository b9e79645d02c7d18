// Shared host/device definitions of libgmminterp: problem geometry, buffer
// layouts of the saved state and the workspace, and the per-image view every
// kernel body works on.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <type_traits>

#include "gmminterp.h"

namespace gmm {

constexpr int kBlockSide = 8;          // one wavefront owns an 8x8 pixel block
constexpr int kMaxChannels = 32;
constexpr float kMaxRadius = 12.0f;    // keeps exp2(-r^2/2 * log2(e)) a normal float
constexpr size_t kAlign = 256;
constexpr int kRadixItems = 4;         // keys per thread in a radix pass
constexpr int kRadixTile = 256 * kRadixItems;  // keys per workgroup in a radix pass
constexpr int kRadixMaxPasses = 4;     // bin keys of up to 32 bits
constexpr int kMaxDigits = 1024;       // digits of one radix pass (the single-call path sorts
                                       // keys of up to 10 bits in one pass)

inline size_t align_up(size_t x, size_t a = kAlign) { return (x + a - 1) / a * a; }

// Channel count the kernels are instantiated for: the smallest of
// {1,2,3,4,8,16,32} that is >= C (C + 1 for a normalised kernel, whose
// records carry the density factor in the last slot).  Extra channels are
// zero padding.
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

// Radix-sort plan for bin keys in [0, nb): number of passes and digit width.
inline void radix_plan(int nb, int* npass, int* dbits, int* kbits) {
  int bits = 0;
  while ((1LL << bits) < nb) ++bits;
  *kbits = bits;
  *npass = (bits + 7) / 8;
  *dbits = *npass ? (bits + *npass - 1) / *npass : 0;
}

// Forward work units (see forward_block_q): a unit is 2 x 2 blocks of 8x8
// pixels, evaluated by one 256-thread workgroup in one of three modes: the
// whole unit with one wavefront per block, or one half of it (blocks 0-1 or
// 2-3) with two wavefronts per block -- dense units are split in two so that
// no workgroup runs much longer than the rest.  The dispatcher hands
// consecutive workgroups to the 8 XCDs in turn, so when work items are
// launched in number order (the serving path) item i runs on XCD i % 8:
// units are numbered in groups of 8 that tile a 4 x 2 patch of units, and
// each XCD gets the same position in every patch -- a regular lattice over
// the image, so a dense region is shared by all XCDs instead of loading the
// few that own its columns.  (The single-call path launches the items in
// the order of a cost plan instead, heaviest first.)
constexpr int kPlanBuckets = 32;  // cost classes of the forward's work order
struct FwdUnits {
  int ux, uy, stx;  // units per row / column, 4x2 patches per row
  __host__ __device__ FwdUnits(int bx_blocks, int by_blocks)
      : ux((bx_blocks + 1) / 2), uy((by_blocks + 1) / 2), stx((ux + 3) / 4) {}
  __host__ __device__ int count() const { return stx * ((uy + 1) / 2) * 8; }
  // unit number -> unit coordinates; false for the padding units of the patches
  __host__ __device__ bool coords(int unit, int* cx, int* cy) const {
    const int st = unit >> 3, x = unit & 7;
    const int sy = st / stx;
    *cx = 4 * (st - sy * stx) + (x & 3);
    *cy = 2 * sy + (x >> 2);
    return *cx < ux && *cy < uy;
  }
};

struct Geometry {
  int B, N, C, H, W, T;
  int nbx, nby, nb;
  int CT, CS, CP;
  float radius;
  int per_point;
  int kern;                            // INTERP_KERNEL_* flags
  int nsig;                            // sigma values per point: 1 isotropic, 2 diagonal
  int st;                              // INTERP_STORAGE_* of the value arrays
  int vbytes;                          // bytes per stored value (4 or 2)
  int bx_blocks, by_blocks;            // 8x8 pixel blocks per image row / column
  int npass, dbits, kbits;             // radix sort of the bin keys
  int ntiles;                          // radix tiles per image
  int units256;                        // ceil(N / 256)
  int fwd_units;                       // forward work units per image (up to 4 channels)
};

// Byte offsets of every array inside the saved buffer and the workspace.
struct Layout {
  // saved
  size_t Z, reach, offset, perm, geo, col, saved_bytes;
  // workspace
  size_t binof, keysF, kA, vA, kB, vB, geoA, colA, geoB, colB, hist, dtot, rpart, prec, gpart, fplan,
      fwd_work_bytes, work_bytes;
};

// Digits a radix pass of this geometry may have: 2^kbits for keys of up to
// 10 bits (one pass on the single-call path), else 256.
inline int max_digits(const Geometry& g) { return g.kbits <= 10 ? 1 << g.kbits : 256; }

inline Layout make_layout(const Geometry& g) {
  Layout L{};
  size_t o = 0;
  const size_t B = g.B, N = g.N, HW = size_t(g.H) * g.W;
  L.Z = o;      o = align_up(o + B * HW * 4);
  L.reach = o;  o = align_up(o + B * 4);
  L.offset = o; o = align_up(o + B * (size_t(g.nb) + 1) * 4);
  L.perm = o;   o = align_up(o + B * N * 4);
  L.geo = o;    o = align_up(o + B * N * 16);
  L.col = o;    o = align_up(o + B * N * size_t(g.CS) * g.vbytes);
  L.saved_bytes = o;
  o = 0;
  L.binof = o;  o = align_up(o + B * N * 4);
  L.keysF = o;  o = align_up(o + B * N * 4);
  L.kA = o;     o = align_up(o + B * N * 4);
  L.vA = o;     o = align_up(o + B * N * 4);
  L.kB = o;     o = align_up(o + B * N * 4);
  L.vB = o;     o = align_up(o + B * N * 4);
  // narrow point records (CS = 4) between radix passes (the second set only
  // with 3+ passes); wide records are read from the inputs by the last pass
  const size_t NA = g.CS == 4 && g.npass >= 2 ? N : 0, NB = g.CS == 4 && g.npass >= 3 ? N : 0;
  L.geoA = o;   o = align_up(o + B * NA * 16);
  L.colA = o;   o = align_up(o + B * NA * 16);
  L.geoB = o;   o = align_up(o + B * NB * 16);
  L.colB = o;   o = align_up(o + B * NB * 16);
  L.hist = o;   o = align_up(o + B * size_t(max_digits(g)) * g.ntiles * 4);
  L.dtot = o;   o = align_up(o + B * size_t(max_digits(g)) * 4);
  L.rpart = o;  o = align_up(o + B * size_t(g.units256) * 4 + 4);
  // forward work order: 64 counters (list sizes), then kPlanBuckets lists of
  // up to 2 * B * fwd_units work items
  L.fplan = o;  o = align_up(o + (64 + size_t(kPlanBuckets) * 2 * B * g.fwd_units) * 4);
  // everything above is all the forward uses; the rest is the backward's
  L.fwd_work_bytes = o;
  L.prec = o;   o = align_up(o + B * HW * size_t(g.CP) * 4);
  L.gpart = o;  o = align_up(o + B * size_t(g.units256) * 2 * 4 + 8);
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
  if (p->kernel < 0 || p->kernel > (INTERP_KERNEL_NORMALIZED | INTERP_KERNEL_DIAGONAL))
    return "kernel must be a combination of INTERP_KERNEL_NORMALIZED and INTERP_KERNEL_DIAGONAL";
  if (p->storage < INTERP_STORAGE_F32 || p->storage > INTERP_STORAGE_F16)
    return "storage must be INTERP_STORAGE_F32, _BF16 or _F16";
  if (p->storage != INTERP_STORAGE_F32 && p->kernel != 0)
    return "bfloat16 and half storage take the default kernel";
  const int T = p->tile == 0 ? 8 : p->tile;
  if (T != 4 && T != 8 && T != 16 && T != 32 && T != 64) return "tile must be 0, 4, 8, 16, 32 or 64";
  const long long BN = (long long)p->B * p->N;
  const long long BHW = (long long)p->B * p->H * p->W;
  if (BN >= (1LL << 31)) return "B*N must be below 2^31";
  if (BHW >= (1LL << 31)) return "B*H*W must be below 2^31";
  if (BN * channel_template(p->C) >= (1LL << 31)) return "B*N*C must be below 2^31";
  if (BHW * pix_stride(p->C) >= (1LL << 31)) return "B*H*W*(C+1) must be below 2^31";
  g->B = p->B; g->N = p->N; g->C = p->C; g->H = p->H; g->W = p->W; g->T = T;
  g->nbx = (p->W + T - 1) / T;
  g->nby = (p->H + T - 1) / T;
  g->nb = g->nbx * g->nby;
  g->CT = channel_template(p->C);
  g->CS = col_stride(p->C);
  // pixel records: a gradient slot per channel, then beta
  g->CP = (g->CT + 1 + 3) / 4 * 4;
  g->radius = p->radius;
  g->per_point = p->sigma_per_point;
  g->kern = p->kernel;
  g->nsig = (p->kernel & INTERP_KERNEL_DIAGONAL) ? 2 : 1;
  g->st = p->storage;
  g->vbytes = p->storage == INTERP_STORAGE_F32 ? 4 : 2;
  g->bx_blocks = (p->W + kBlockSide - 1) / kBlockSide;
  g->by_blocks = (p->H + kBlockSide - 1) / kBlockSide;
  radix_plan(g->nb, &g->npass, &g->dbits, &g->kbits);
  g->ntiles = (p->N + kRadixTile - 1) / kRadixTile;
  g->units256 = (p->N + 255) / 256;
  g->fwd_units = FwdUnits(g->bx_blocks, g->by_blocks).count();
  if ((long long)g->fwd_units * g->B * kPlanBuckets * 2 >= (1LL << 31)) return "image too large";
  return "";
}

// Everything the kernel bodies need about ONE image of one problem: its
// shape, its inputs/outputs and its slices of the saved state and workspace.
// The view of image 0 plus image_of() gives every image of a batch.
struct ImageView {
  int N, C, H, W, T, nbx, nby, nb, CS, CP, per_point;
  int kern, nsig;           // kernel flags; sigma values per point (1 or 2)
  int st;                   // INTERP_STORAGE_* of values, out, grad_out, grad_values, col
  int values_vec4;          // C % 4 == 0 and values aligned to four elements: vector loads
  float r2;                 // f32(radius * radius): the diagonal kernel's test
  int npass, dbits, kbits, ntiles, units256;
  int bx_blocks, by_blocks;
  float radius, inv_tile;
  // inputs / outputs
  const float2* pos;        // [N]
  const float* sigma;       // per point: [N, nsig]; shared: the image's nsig values
  // values, out, grad_out, grad_values and col hold elements of the storage
  // type (st); the kernels read and write them through Val<ST>
  const float* values;      // [N, C]
  float* out;               // [C, H, W]
  const float* grad_out;    // [C, H, W]
  float* grad_pos;          // [N, 2] or null
  float* grad_sigma;        // like sigma, or null
  float* grad_values;       // [N, C] or null
  // saved state
  float* Z;                 // [H, W]
  float* reach;             // [1]
  int* offset;              // [nb + 1]
  int* perm;                // [N]
  float4* geo;              // [N]
  float* col;               // [N, CS] (storage type)
  // workspace
  int* binof;               // [N] bin key of each point (point order)
  int* keysF;               // [N] bin keys in sorted order
  int* kA; int* vA; int* kB; int* vB;   // radix ping-pong buffers: keys, point indices
  float4* geoA; float4* colA;           // and narrow point records (as geo, col)
  float4* geoB; float4* colB;
  int* hist;                // [hdig * ntiles] per (digit, tile) counts, then offsets
  int* dtot;                // [hdig] per-digit totals of the current radix pass
  int hdig;                 // digits per pass the hist and dtot arrays hold (max_digits)
  float* rpart;             // [units256] partial maxima of radius*sigma
  float* prec;              // [H, W, CP] backward pixel records
  float* gpart;             // [units256, 2] partial sums of dL/dsigma (shared sigma)
};

template <typename T>
__host__ __device__ inline T* shift(T* p, size_t n) { return p ? p + n : p; }
// p advanced by n elements of ebytes bytes each
template <typename T>
__host__ __device__ inline T* bshift(T* p, size_t n, size_t ebytes) {
  using Byte = typename std::conditional<std::is_const<T>::value, const char, char>::type;
  return p ? reinterpret_cast<T*>(reinterpret_cast<Byte*>(p) + n * ebytes) : p;
}

// The view of image b, given the view of image 0 of the same problem.
__host__ __device__ inline ImageView image_of(const ImageView& v0, int b) {
  if (b == 0) return v0;
  ImageView v = v0;
  const size_t bb = b, N = v0.N, HW = size_t(v0.H) * v0.W;
  v.pos = shift(v0.pos, bb * N);
  v.sigma = shift(v0.sigma, (v0.per_point ? bb * N : bb) * v0.nsig);
  // value arrays step in elements of the storage type
  const size_t vs = v0.st == INTERP_STORAGE_F32 ? 4 : 2;
  v.values = bshift(v0.values, bb * N * v0.C, vs);
  v.out = bshift(v0.out, bb * v0.C * HW, vs);
  v.grad_out = bshift(v0.grad_out, bb * v0.C * HW, vs);
  v.grad_pos = shift(v0.grad_pos, bb * N * 2);
  v.grad_sigma = shift(v0.grad_sigma, (v0.per_point ? bb * N : bb) * v0.nsig);
  v.grad_values = bshift(v0.grad_values, bb * N * v0.C, vs);
  v.Z = shift(v0.Z, bb * HW);
  v.reach = shift(v0.reach, bb);
  v.offset = shift(v0.offset, bb * (size_t(v0.nb) + 1));
  v.perm = shift(v0.perm, bb * N);
  v.geo = shift(v0.geo, bb * N);
  v.col = bshift(v0.col, bb * N * v0.CS, vs);
  v.binof = shift(v0.binof, bb * N);
  v.keysF = shift(v0.keysF, bb * N);
  v.kA = shift(v0.kA, bb * N);
  v.vA = shift(v0.vA, bb * N);
  v.kB = shift(v0.kB, bb * N);
  v.vB = shift(v0.vB, bb * N);
  v.geoA = shift(v0.geoA, bb * N);
  v.colA = shift(v0.colA, bb * N);
  v.geoB = shift(v0.geoB, bb * N);
  v.colB = shift(v0.colB, bb * N);
  v.hist = shift(v0.hist, bb * size_t(v0.hdig) * v0.ntiles);
  v.dtot = shift(v0.dtot, bb * size_t(v0.hdig));
  v.rpart = shift(v0.rpart, bb * v0.units256);
  v.prec = shift(v0.prec, bb * HW * v0.CP);
  v.gpart = shift(v0.gpart, bb * v0.units256 * 2);
  return v;
}

// The view of image 0 of a validated problem.
inline ImageView make_view(const Geometry& g, const Layout& L, void* saved, void* work,
                           const float* pos, const float* sigma, const float* values, float* out,
                           const float* grad_out, float* grad_pos, float* grad_sigma,
                           float* grad_values) {
  char* s = static_cast<char*>(saved);
  char* w = static_cast<char*>(work);
  ImageView v;
  v.N = g.N; v.C = g.C; v.H = g.H; v.W = g.W; v.T = g.T; v.nbx = g.nbx; v.nby = g.nby; v.nb = g.nb;
  v.CS = g.CS; v.CP = g.CP; v.per_point = g.per_point;
  v.kern = g.kern; v.nsig = g.nsig; v.st = g.st;
  v.values_vec4 = g.C % 4 == 0 && reinterpret_cast<uintptr_t>(values) % (4 * g.vbytes) == 0;
  v.r2 = g.radius * g.radius;  // one rounded float multiply, as the test specifies
  v.npass = g.npass; v.dbits = g.dbits; v.kbits = g.kbits; v.ntiles = g.ntiles;
  v.hdig = max_digits(g);
  v.units256 = g.units256;
  v.bx_blocks = g.bx_blocks; v.by_blocks = g.by_blocks;
  v.radius = g.radius;
  v.inv_tile = 1.0f / (float)g.T;
  v.pos = reinterpret_cast<const float2*>(pos);
  v.sigma = sigma;
  v.values = values;
  v.out = out;
  v.grad_out = grad_out;
  v.grad_pos = grad_pos;
  v.grad_sigma = grad_sigma;
  v.grad_values = grad_values;
  v.Z = s ? reinterpret_cast<float*>(s + L.Z) : nullptr;
  v.reach = s ? reinterpret_cast<float*>(s + L.reach) : nullptr;
  v.offset = s ? reinterpret_cast<int*>(s + L.offset) : nullptr;
  v.perm = s ? reinterpret_cast<int*>(s + L.perm) : nullptr;
  v.geo = s ? reinterpret_cast<float4*>(s + L.geo) : nullptr;
  v.col = s ? reinterpret_cast<float*>(s + L.col) : nullptr;
  v.binof = w ? reinterpret_cast<int*>(w + L.binof) : nullptr;
  v.keysF = w ? reinterpret_cast<int*>(w + L.keysF) : nullptr;
  v.kA = w ? reinterpret_cast<int*>(w + L.kA) : nullptr;
  v.vA = w ? reinterpret_cast<int*>(w + L.vA) : nullptr;
  v.kB = w ? reinterpret_cast<int*>(w + L.kB) : nullptr;
  v.vB = w ? reinterpret_cast<int*>(w + L.vB) : nullptr;
  v.geoA = w ? reinterpret_cast<float4*>(w + L.geoA) : nullptr;
  v.colA = w ? reinterpret_cast<float4*>(w + L.colA) : nullptr;
  v.geoB = w ? reinterpret_cast<float4*>(w + L.geoB) : nullptr;
  v.colB = w ? reinterpret_cast<float4*>(w + L.colB) : nullptr;
  v.hist = w ? reinterpret_cast<int*>(w + L.hist) : nullptr;
  v.dtot = w ? reinterpret_cast<int*>(w + L.dtot) : nullptr;
  v.rpart = w ? reinterpret_cast<float*>(w + L.rpart) : nullptr;
  v.prec = w ? reinterpret_cast<float*>(w + L.prec) : nullptr;
  v.gpart = w ? reinterpret_cast<float*>(w + L.gpart) : nullptr;
  return v;
}

// Optional per-kernel event timing (enabled by interp_profile_enable): the
// constructor records a start event on `st`, the destructor a stop event.
struct ProfRange {
  ProfRange(const char* name, hipStream_t st);
  ~ProfRange();
  int token;
  hipStream_t st;
};

// Host launchers of the single-call path (single.hip).
hipError_t launch_forward_all(const Geometry& g, const ImageView& v0, int* fplan, hipStream_t st);
hipError_t launch_backward_all(const Geometry& g, const ImageView& v0, hipStream_t st);
hipError_t launch_debug_count(const Geometry& g, const ImageView& v0, int* count, hipStream_t st);

}  // namespace gmm
