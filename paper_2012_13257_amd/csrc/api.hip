// extern "C" entry points of libgmminterp.so (declared in include/gmminterp.h):
// argument validation, buffer carving and kernel dispatch on the caller's
// stream.  No host synchronisation and no device allocation happen here.
#include <atomic>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"

namespace gmm {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int fail_hip(hipError_t e, const char* where) {
  g_last_error = std::string(where) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
  return INTERP_EHIP;
}

// ---------------------------------------------------------------------------
// Per-kernel event timing
// ---------------------------------------------------------------------------
namespace {
struct ProfRecord {
  std::string name;
  hipEvent_t start, stop;
};
std::mutex g_prof_mu;
std::vector<ProfRecord> g_prof;
std::atomic<int> g_prof_on{0};
// set while a call that must not create events (interp_forward_noalloc) launches
thread_local bool g_prof_suppress = false;

void prof_clear_locked() {
  for (auto& r : g_prof) {
    hipEventDestroy(r.start);
    hipEventDestroy(r.stop);
  }
  g_prof.clear();
}
}  // namespace

ProfRange::ProfRange(const char* name, hipStream_t s) : token(-1), st(s) {
  if (g_prof_suppress || !g_prof_on.load(std::memory_order_relaxed)) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
  ProfRecord r{name, nullptr, nullptr};
  if (hipEventCreate(&r.start) != hipSuccess) return;
  if (hipEventCreate(&r.stop) != hipSuccess) { hipEventDestroy(r.start); return; }
  hipEventRecord(r.start, st);
  std::lock_guard<std::mutex> g(g_prof_mu);
  token = (int)g_prof.size();
  g_prof.push_back(r);
}

ProfRange::~ProfRange() {
  if (token < 0) return;
  hipEvent_t stop;
  {
    std::lock_guard<std::mutex> g(g_prof_mu);
    if (token >= (int)g_prof.size()) return;
    stop = g_prof[token].stop;
  }
  hipEventRecord(stop, st);
}

// ---------------------------------------------------------------------------
// Static scratch of interp_forward_noalloc
// ---------------------------------------------------------------------------
// The forward's workspace for callers that cannot allocate: a file-scope
// device array, one copy per GPU the library runs on, held until the process
// ends.  Host code never passes the array's name to a kernel (on the host it
// is only a stand-in for the symbol): the device address of each GPU's copy
// is looked up once per device with hipGetSymbolAddress and used instead.
constexpr size_t kStaticScratchBytes = INTERP_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch`, per device
}  // namespace

// The current device's copy of the scratch array (looked up on the first call
// on that device, with that device current).
static int static_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(INTERP_EINVAL, "device ordinal out of range");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return fail_hip(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(INTERP_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return INTERP_OK;
}

static bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// Common validation of forward/backward inputs.  Returns INTERP_OK or an error.
static int check_io(const interp_problem* prob, Geometry* g, Layout* L, const float* pos,
                    const float* sigma, const float* values, const void* saved, size_t saved_size,
                    const void* work, size_t work_size) {
  std::string m = make_geometry(prob, g);
  if (!m.empty()) return fail(INTERP_EINVAL, m);
  *L = make_layout(*g);
  if (g->N > 0) {
    if (!pos || !sigma || !values) return fail(INTERP_EINVAL, "pos, sigma and values must not be NULL when N > 0");
    if (!aligned(pos, 8)) return fail(INTERP_EINVAL, "pos must be 8-byte aligned");
    if (!aligned(sigma, 4) || !aligned(values, 4)) return fail(INTERP_EINVAL, "sigma and values must be 4-byte aligned");
  }
  if (!saved) return fail(INTERP_EINVAL, "saved must not be NULL");
  if (!work) return fail(INTERP_EINVAL, "workspace must not be NULL");
  if (!aligned(saved, kAlign) || !aligned(work, kAlign))
    return fail(INTERP_EINVAL, "saved and workspace must be 256-byte aligned");
  if (saved_size < L->saved_bytes)
    return fail(INTERP_EINVAL, "saved buffer too small: need " + std::to_string(L->saved_bytes) +
                                   " bytes, got " + std::to_string(saved_size));
  if (work_size < L->work_bytes)
    return fail(INTERP_EINVAL, "workspace too small: need " + std::to_string(L->work_bytes) +
                                   " bytes, got " + std::to_string(work_size));
  return INTERP_OK;
}

}  // namespace gmm

using namespace gmm;

extern "C" {

size_t interp_workspace_bytes(const interp_problem* prob) {
  Geometry g;
  std::string m = make_geometry(prob, &g);
  if (!m.empty()) { fail(INTERP_EINVAL, m); return 0; }
  return make_layout(g).work_bytes;
}

size_t interp_saved_bytes(const interp_problem* prob) {
  Geometry g;
  std::string m = make_geometry(prob, &g);
  if (!m.empty()) { fail(INTERP_EINVAL, m); return 0; }
  return make_layout(g).saved_bytes;
}

int interp_forward(const interp_problem* prob, const float* pos, const float* sigma,
                   const float* values, float* out, void* saved, size_t saved_size,
                   void* workspace, size_t workspace_size, void* stream) {
  Geometry g;
  Layout L;
  int rc = check_io(prob, &g, &L, pos, sigma, values, saved, saved_size, workspace, workspace_size);
  if (rc != INTERP_OK) return rc;
  if (!out || !aligned(out, 4)) return fail(INTERP_EINVAL, "out must be a non-NULL 4-byte aligned pointer");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const ImageView v0 = make_view(g, L, saved, workspace, pos, sigma, values, out, nullptr, nullptr,
                                 nullptr, nullptr);
  int* fplan = reinterpret_cast<int*>(static_cast<char*>(workspace) + L.fplan);
  hipError_t e = launch_forward_all(g, v0, fplan, st);
  if (e != hipSuccess) return fail_hip(e, "forward kernels");
  g_last_error.clear();
  return INTERP_OK;
}

int interp_forward_noalloc(const interp_problem* prob, const float* pos, const float* sigma,
                           const float* values, float* out, void* saved, size_t saved_size,
                           void* stream) {
  Geometry g;
  std::string m = make_geometry(prob, &g);
  if (!m.empty()) return fail(INTERP_EINVAL, m);
  const Layout L = make_layout(g);
  if (L.fwd_work_bytes > kStaticScratchBytes)
    return fail(INTERP_EINVAL, "problem needs " + std::to_string(L.fwd_work_bytes) +
                                   " bytes of forward workspace; the static scratch of "
                                   "interp_forward_noalloc holds " +
                                   std::to_string(kStaticScratchBytes) +
                                   " (use interp_forward with a caller workspace)");
  void* work = nullptr;
  int rc = static_scratch(&work);
  if (rc != INTERP_OK) return rc;
  Geometry g2;
  Layout L2;
  rc = check_io(prob, &g2, &L2, pos, sigma, values, saved, saved_size, work, L.work_bytes);
  if (rc != INTERP_OK) return rc;
  if (!out || !aligned(out, 4)) return fail(INTERP_EINVAL, "out must be a non-NULL 4-byte aligned pointer");
  hipStream_t st = static_cast<hipStream_t>(stream);
  ImageView v0 = make_view(g, L, saved, work, pos, sigma, values, out, nullptr, nullptr, nullptr,
                           nullptr);
  v0.prec = nullptr;  // backward-only parts of the layout lie beyond the scratch
  v0.gpart = nullptr;
  int* fplan = reinterpret_cast<int*>(static_cast<char*>(work) + L.fplan);
  g_prof_suppress = true;
  hipError_t e = launch_forward_all(g, v0, fplan, st);
  g_prof_suppress = false;
  if (e != hipSuccess) return fail_hip(e, "forward kernels");
  g_last_error.clear();
  return INTERP_OK;
}

int interp_backward(const interp_problem* prob, const float* pos, const float* sigma,
                    const float* values, const float* out, const void* saved, size_t saved_size,
                    const float* grad_out, float* grad_pos, float* grad_sigma, float* grad_values,
                    void* workspace, size_t workspace_size, void* stream) {
  Geometry g;
  Layout L;
  int rc = check_io(prob, &g, &L, pos, sigma, values, saved, saved_size, workspace, workspace_size);
  if (rc != INTERP_OK) return rc;
  if (!out || !grad_out) return fail(INTERP_EINVAL, "out and grad_out must not be NULL");
  if (!aligned(grad_out, 4) || !aligned(out, 4)) return fail(INTERP_EINVAL, "out and grad_out must be 4-byte aligned");
  if (grad_pos && !aligned(grad_pos, 8)) return fail(INTERP_EINVAL, "grad_pos must be 8-byte aligned");
  if (grad_sigma && g.nsig == 2 && !aligned(grad_sigma, 8))
    return fail(INTERP_EINVAL, "grad_sigma of a diagonal kernel must be 8-byte aligned");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const ImageView v0 = make_view(g, L, const_cast<void*>(saved), workspace, pos, sigma, values,
                                 const_cast<float*>(out), grad_out, grad_pos, grad_sigma, grad_values);
  hipError_t e = launch_backward_all(g, v0, st);
  if (e != hipSuccess) return fail_hip(e, "backward kernels");
  g_last_error.clear();
  return INTERP_OK;
}

int interp_debug_bins(const interp_problem* prob, const void* saved, size_t saved_size,
                      const void* workspace, size_t workspace_size, int32_t* bin_of, int32_t* count,
                      int32_t* offset, int32_t* perm, void* stream) {
  Geometry g;
  std::string m = make_geometry(prob, &g);
  if (!m.empty()) return fail(INTERP_EINVAL, m);
  Layout L = make_layout(g);
  if (!saved || !workspace || saved_size < L.saved_bytes || workspace_size < L.work_bytes)
    return fail(INTERP_EINVAL, "saved/workspace missing or too small");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const char* s = static_cast<const char*>(saved);
  const char* w = static_cast<const char*>(workspace);
  const size_t BN = size_t(g.B) * g.N * 4;
  struct Cp { void* dst; const void* src; size_t n; } cps[3] = {
      {bin_of, w + L.binof, BN},
      {offset, s + L.offset, size_t(g.B) * (g.nb + 1) * 4},
      {perm, s + L.perm, BN}};
  for (auto& c : cps) {
    if (!c.dst || c.n == 0) continue;
    hipError_t e = hipMemcpyAsync(c.dst, c.src, c.n, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return fail_hip(e, "interp_debug_bins copy");
  }
  if (count) {
    const ImageView v0 = make_view(g, L, const_cast<void*>(saved), const_cast<void*>(workspace),
                                   nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                   nullptr);
    hipError_t e = launch_debug_count(g, v0, count, st);
    if (e != hipSuccess) return fail_hip(e, "interp_debug_bins count");
  }
  g_last_error.clear();
  return INTERP_OK;
}

const char* interp_last_error(void) { return g_last_error.c_str(); }

int interp_profile_enable(int on) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  if (on) prof_clear_locked();
  g_prof_on.store(on ? 1 : 0);
  return INTERP_OK;
}

int interp_profile_read(const char* prefix, double* total_ms, int64_t* launches) {
  if (!prefix || !total_ms || !launches) return fail(INTERP_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> g(g_prof_mu);
  const size_t np = std::strlen(prefix);
  double tot = 0.0;
  int64_t n = 0;
  for (auto& r : g_prof) {
    if (r.name.compare(0, np, prefix) != 0) continue;
    hipError_t e = hipEventSynchronize(r.stop);
    if (e != hipSuccess) return fail_hip(e, "interp_profile_read");
    float ms = 0.0f;
    e = hipEventElapsedTime(&ms, r.start, r.stop);
    if (e != hipSuccess) return fail_hip(e, "interp_profile_read");
    tot += ms;
    ++n;
  }
  *total_ms = tot;
  *launches = n;
  return INTERP_OK;
}

}  // extern "C"
