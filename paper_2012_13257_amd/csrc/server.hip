// Serving loop: continuous batching of independent interpolation requests.
//
// Device side: a job table (one ImageView per admitted request plus, per
// phase, the prefix sums of each job's work units) and one persistent
// "job-table" kernel per phase.  Each kernel runs a fixed grid that strides
// over the flattened work units of all jobs of the batch, finds the job of a
// unit by binary search and calls the same device function as the
// single-call path, so every request computes exactly the bits it would
// compute alone.  The phase sequences (binning with 1-3 radix passes, forward,
// with or without the backward) are captured once per batch context into HIP
// graphs; a batch is one table upload plus one replay, on the context's
// stream, of the graph that covers its jobs.  Per-job state lives in one
// device arena allocated at creation (the HBM budget).
//
// Host side: the Scheduler (scheduler.hpp) admits requests by free slots and
// arena space and launches batches on free contexts, so batches of requests
// that arrive while others run execute concurrently on the device.
#include <algorithm>
#include <cstring>
#include <string>

#include "kernels.hpp"
#include "scheduler.hpp"

namespace gmm {

int fail(int code, const std::string& msg);
int fail_hip(hipError_t e, const char* where);

namespace serve {

constexpr int kMaxJobs = 256;      // jobs per batch (table capacity)
constexpr int kContexts = 4;       // concurrent batches
constexpr int kServeMaxC = 4;      // channels per request on the serving path
constexpr int kServePasses = 3;    // radix passes the captured graphs cover

enum Phase {
  PH_KEYS = 0,
  PH_HIST0, PH_HIST1, PH_HIST2,
  PH_SCAN0, PH_SCAN1, PH_SCAN2,
  PH_SCAT0, PH_SCAT1, PH_SCAT2,
  PH_FINISH, PH_FWD, PH_BPIX, PH_BPOINT, PH_BSIG,
  PH_COUNT
};

// Workgroups per compute unit of each job-table kernel: as many as its LDS
// lets one compute unit hold (forward lists 32 KB: 5; adjoint window 37 KB:
// 4; the others 8), so a phase fills the chip once and then strides.
template <int PH>
constexpr int phase_wgs_per_cu() {
  return PH == PH_FWD ? 5 : PH == PH_BPOINT ? 4 : 8;
}

struct JobTable {
  int njobs;
  int pad[3];
  int units[PH_COUNT][kMaxJobs + 1];  // per phase: prefix sums of work units
  int ct[kMaxJobs];                   // channel template of each job
  ImageView view[kMaxJobs];           // last: only njobs entries are uploaded
};

// ---------------------------------------------------------------------------
// Job-table kernels
// ---------------------------------------------------------------------------

// LDS of each phase kernel: only what its phase uses
template <int PH>
struct PhaseLds {
  static constexpr int ints = (PH >= PH_SCAT0 && PH <= PH_SCAT2) ? dev::radix_scatter_lds_ints<256>()
                              : (PH == PH_BPOINT)                 ? 256 + 64
                              : PH == PH_KEYS                     ? kMaxDigits
                              : (PH >= PH_HIST0 && PH <= PH_HIST2) ? 256
                                                                  : 4;
  static constexpr int f4 = PH == PH_FWD ? dev::fwd_quarter_lds_f4<4>()
                            : PH == PH_BPOINT ? dev::kBwdStageF4
                                              : 1;
};

template <int PH>
__global__ __launch_bounds__(256) void kj_phase(const JobTable* __restrict__ T) {
  __shared__ float red4[4];
  __shared__ int lds_i[PhaseLds<PH>::ints];
  __shared__ float4 s_rec[PhaseLds<PH>::f4];
  const int nj = T->njobs;
  const int* U = T->units[PH];
  const int total = U[nj];
  // Radix tiles are dealt XCD by XCD (workgroup i runs on XCD i % 8): each
  // XCD takes one contiguous eighth of them, so the cache lines neighbouring
  // tiles share in the histograms and in the scatter's output are merged in
  // one L2.  The other phases keep the round-robin order, which balances
  // units of uneven cost (dense regions, large requests) over the XCDs.
  const bool banded = PH == PH_KEYS || (PH >= PH_HIST0 && PH <= PH_HIST2) ||
                      (PH >= PH_SCAT0 && PH <= PH_SCAT2);
  const int per8 = (total + 7) / 8;
  const int x = blockIdx.x & 7, nw = (int)(gridDim.x >> 3);
  const int u0 = banded ? x * per8 + (int)(blockIdx.x >> 3) : (int)blockIdx.x;
  const int ustep = banded ? nw : (int)gridDim.x;
  const int uend = banded ? min(total, (x + 1) * per8) : total;
  for (int u = u0; u < uend; u += ustep) {
    int lo = 0, hi = nj - 1;  // last job whose first unit is <= u
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (U[mid] <= u) lo = mid; else hi = mid - 1;
    }
    const int local = u - U[lo];
    const ImageView& v = T->view[lo];
    if constexpr (PH == PH_KEYS) {
      dev::bin_keys(v, local, red4, lds_i);
    } else if constexpr (PH >= PH_HIST0 && PH <= PH_HIST2) {
      dev::radix_hist(v, PH - PH_HIST0, local, lds_i);
    } else if constexpr (PH >= PH_SCAN0 && PH <= PH_SCAN2) {
      dev::radix_scan_digit(v, PH - PH_SCAN0, local, lds_i);
    } else if constexpr (PH >= PH_SCAT0 && PH <= PH_SCAT2) {
      dev::radix_scatter(v, PH - PH_SCAT0, local, lds_i);
    } else if constexpr (PH == PH_FINISH) {
      dev::bin_finish(v, local, red4);
    } else if constexpr (PH == PH_FWD) {
      // one item per unit, evaluated as the single-call path does: a heavy
      // unit as its two halves (one after the other), any other whole
      int c[4];
      dev::unit_candidates(v, local, c);
      const bool heavy = dev::unit_is_heavy(c);
      for (int h = 0; h < (heavy ? 2 : 1); ++h) {
        const int mode = heavy ? 1 + h : 0;
        if (h) __syncthreads();  // the lists of the first half are free again
        switch (T->ct[lo]) {
          case 1: dev::forward_block_q<1>(v, local, mode, s_rec); break;
          case 2: dev::forward_block_q<2>(v, local, mode, s_rec); break;
          case 3: dev::forward_block_q<3>(v, local, mode, s_rec); break;
          default: dev::forward_block_q<4>(v, local, mode, s_rec); break;
        }
      }
    } else if constexpr (PH == PH_BPIX) {
      switch (T->ct[lo]) {
        case 1: dev::bwd_pixel<1>(v, local); break;
        case 2: dev::bwd_pixel<2>(v, local); break;
        case 3: dev::bwd_pixel<3>(v, local); break;
        default: dev::bwd_pixel<4>(v, local); break;
      }
    } else if constexpr (PH == PH_BPOINT) {
      switch (T->ct[lo]) {
        case 1: dev::bwd_point<1>(v, local, red4, lds_i, s_rec); break;
        case 2: dev::bwd_point<2>(v, local, red4, lds_i, s_rec); break;
        case 3: dev::bwd_point<3>(v, local, red4, lds_i, s_rec); break;
        default: dev::bwd_point<4>(v, local, red4, lds_i, s_rec); break;
      }
    } else if constexpr (PH == PH_BSIG) {
      dev::bwd_sigma_sum(v, red4);
    }
    __syncthreads();
  }
}

// Grid sizes of the job-table kernels.  A full grid holds as many
// workgroups as fit the chip at once; a batch whose every phase has at most
// kSmallUnits units replays graphs of kSmallGrid-workgroup kernels instead,
// which the dispatcher starts and drains far sooner (a small request then
// does not pay for thousands of workgroups with no work, per phase).  A
// unit's result does not depend on the grid that computes it.
constexpr int kSmallGrid = 64;
constexpr int kSmallUnits = 2 * kSmallGrid;

// cus: compute units of the device; the grid is a multiple of 8 (the
// radix phases deal their tiles to the eight XCDs)
template <int PH>
void enqueue_phase(const JobTable* dtab, hipStream_t st, int cus, bool small) {
  const int full = (phase_wgs_per_cu<PH>() * cus + 7) / 8 * 8;
  const int grid = small ? std::min(full, kSmallGrid) : full;
  hipLaunchKernelGGL(kj_phase<PH>, dim3(grid), dim3(256), 0, st, dtab);
}

// The phase sequence of a batch whose jobs need at most np radix passes
// (1..3; a job with none is covered too) and, if bwd, a backward.  The first
// pass's histogram comes from the key phase, so there is no PH_HIST0.
void enqueue_phases(const JobTable* dtab, hipStream_t st, int cus, int np, bool bwd, bool small) {
  enqueue_phase<PH_KEYS>(dtab, st, cus, small);
  enqueue_phase<PH_SCAN0>(dtab, st, cus, small);
  enqueue_phase<PH_SCAT0>(dtab, st, cus, small);
  if (np >= 2) {
    enqueue_phase<PH_HIST1>(dtab, st, cus, small);
    enqueue_phase<PH_SCAN1>(dtab, st, cus, small);
    enqueue_phase<PH_SCAT1>(dtab, st, cus, small);
  }
  if (np >= 3) {
    enqueue_phase<PH_HIST2>(dtab, st, cus, small);
    enqueue_phase<PH_SCAN2>(dtab, st, cus, small);
    enqueue_phase<PH_SCAT2>(dtab, st, cus, small);
  }
  enqueue_phase<PH_FINISH>(dtab, st, cus, small);
  enqueue_phase<PH_FWD>(dtab, st, cus, small);
  if (bwd) {
    enqueue_phase<PH_BPIX>(dtab, st, cus, small);
    enqueue_phase<PH_BPOINT>(dtab, st, cus, small);
    enqueue_phase<PH_BSIG>(dtab, st, cus, small);
  }
}

// ---------------------------------------------------------------------------
// GPU executor
// ---------------------------------------------------------------------------

struct Request {
  interp_request r;
  Geometry g;
  Layout L;
};

class GpuExecutor {
 public:
  int contexts() const { return kContexts; }
  int max_batch() const { return kMaxJobs; }

  int init(int device, uint64_t budget) {
    device_ = device;
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return fail_hip(e, "hipSetDevice");
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess || cus <= 0) return fail_hip(e, "hipDeviceGetAttribute(compute units)");
    if (budget) {
      e = hipMalloc(&arena_, budget);
      if (e != hipSuccess) return fail_hip(e, "hipMalloc(arena)");
      // touch every page of the arena once now: the first use of fresh device
      // memory is slow, and no request should pay for it
      e = hipMemset(arena_, 0, budget);
      if (e != hipSuccess) return fail_hip(e, "hipMemset(arena)");
    }
    for (int c = 0; c < kContexts; ++c) {
      Ctx& x = ctx_[c];
      if ((e = hipMalloc(&x.dtab, sizeof(JobTable))) != hipSuccess) return fail_hip(e, "hipMalloc(table)");
      if ((e = hipHostMalloc(&x.htab, sizeof(JobTable))) != hipSuccess) return fail_hip(e, "hipHostMalloc(table)");
      std::memset(x.htab, 0, sizeof(JobTable));
      if ((e = hipStreamCreateWithFlags(&x.stream, hipStreamNonBlocking)) != hipSuccess)
        return fail_hip(e, "hipStreamCreate");
      if ((e = hipEventCreateWithFlags(&x.done, hipEventDisableTiming)) != hipSuccess)
        return fail_hip(e, "hipEventCreate");
      // an empty table so that the capture below reads defined memory
      if ((e = hipMemcpy(x.dtab, x.htab, sizeof(JobTable), hipMemcpyHostToDevice)) != hipSuccess)
        return fail_hip(e, "hipMemcpy(table)");
      // one graph per (grid size, radix passes, backward) combination,
      // captured once; a batch replays the one that covers the most passes
      // and the backward of its jobs, so it does not launch phases that have
      // no work, with small grids when all its phases have few units
      for (int gs = 0; gs < 2; ++gs)
      for (int np = 1; np <= kServePasses; ++np) {
        for (int bwd = 0; bwd < 2; ++bwd) {
          if ((e = hipStreamBeginCapture(x.stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
            return fail_hip(e, "hipStreamBeginCapture");
          enqueue_phases(x.dtab, x.stream, cus, np, bwd != 0, gs == 1);
          hipGraph_t graph = nullptr;
          e = hipStreamEndCapture(x.stream, &graph);
          if (e != hipSuccess) return fail_hip(e, "hipStreamEndCapture");
          hipGraphExec_t& ge = x.exec[gs][np - 1][bwd];
          e = hipGraphInstantiate(&ge, graph, nullptr, nullptr, 0);
          hipGraphDestroy(graph);
          if (e != hipSuccess) return fail_hip(e, "hipGraphInstantiate");
          // one replay over the empty table (every phase has zero units), so
          // the first batch that uses the graph does not pay its first-launch cost
          if ((e = hipGraphLaunch(ge, x.stream)) != hipSuccess) return fail_hip(e, "hipGraphLaunch");
          if ((e = hipStreamSynchronize(x.stream)) != hipSuccess) return fail_hip(e, "warm-up replay");
        }
      }
    }
    return INTERP_OK;
  }

  void release() {
    hipSetDevice(device_);
    for (int c = 0; c < kContexts; ++c) {
      Ctx& x = ctx_[c];
      if (x.stream) hipStreamSynchronize(x.stream);
      for (auto& grid : x.exec)
        for (auto& row : grid)
          for (hipGraphExec_t ge : row)
            if (ge) hipGraphExecDestroy(ge);
      if (x.done) hipEventDestroy(x.done);
      if (x.stream) hipStreamDestroy(x.stream);
      if (x.htab) hipHostFree(x.htab);
      if (x.dtab) hipFree(x.dtab);
      x = Ctx{};
    }
    if (arena_) hipFree(arena_);
    arena_ = nullptr;
  }

  void thread_init() { hipSetDevice(device_); }

  // Also called on a submitting thread (an idle server launches at once):
  // the server's device is made current for the call and the caller's
  // restored afterwards.
  int launch(int c, std::vector<Job<Request>*>& jobs) {
    int prev = device_;
    if (hipGetDevice(&prev) != hipSuccess) prev = device_;
    if (prev != device_) hipSetDevice(device_);
    const int rc = launch_on_device(c, jobs);
    if (prev != device_) hipSetDevice(prev);
    return rc;
  }

 private:
  int launch_on_device(int c, std::vector<Job<Request>*>& jobs) {
    Ctx& x = ctx_[c];
    JobTable* T = x.htab;
    const int nj = (int)jobs.size();
    T->njobs = nj;
    int need_passes = 1;
    bool need_bwd = false;
    for (int ph = 0; ph < PH_COUNT; ++ph) T->units[ph][0] = 0;
    for (int i = 0; i < nj; ++i) {
      const Request& rq = jobs[i]->req;
      const Geometry& g = rq.g;
      char* base = static_cast<char*>(arena_) + jobs[i]->arena_off;
      const interp_request& r = rq.r;
      T->view[i] = make_view(g, rq.L, base, base + rq.L.saved_bytes, r.pos, r.sigma, r.values, r.out,
                             r.grad_out, r.grad_out ? r.grad_pos : nullptr,
                             r.grad_out ? r.grad_sigma : nullptr,
                             r.grad_out ? r.grad_values : nullptr);
      T->ct[i] = g.CT;
      const bool bwd = r.grad_out != nullptr;
      need_bwd = need_bwd || bwd;
      need_passes = std::max(need_passes, g.N > 0 ? g.npass : 0);
      int u[PH_COUNT] = {};
      u[PH_KEYS] = g.N > 0 ? g.ntiles : 0;
      for (int p = 0; p < kServePasses; ++p) {
        const bool on = p < g.npass && g.N > 0;
        const int width = on ? std::min(g.dbits, g.kbits - p * g.dbits) : 0;
        u[PH_HIST0 + p] = on && p > 0 ? g.ntiles : 0;  // bin_keys counts the first pass
        u[PH_SCAN0 + p] = on ? 1 << width : 0;
        u[PH_SCAT0 + p] = on ? g.ntiles : 0;
      }
      u[PH_FINISH] = dev::finish_units(g.N);
      u[PH_FWD] = dev::fwd_units(g.bx_blocks, g.by_blocks);
      u[PH_BPIX] = bwd ? (g.H * g.W + 255) / 256 : 0;
      u[PH_BPOINT] = bwd && g.N > 0 ? g.units256 : 0;
      u[PH_BSIG] = bwd && !g.per_point && r.grad_sigma ? 1 : 0;
      for (int ph = 0; ph < PH_COUNT; ++ph) T->units[ph][i + 1] = T->units[ph][i] + u[ph];
    }
    // the batch starts after every event its requests were submitted with;
    // an event that has already completed needs no device-side wait (a wait
    // on another stream's event costs the batch far more than the query)
    hipError_t e;
    for (int i = 0; i < nj; ++i) {
      if (!jobs[i]->req.r.ready) continue;
      hipEvent_t ev = static_cast<hipEvent_t>(jobs[i]->req.r.ready);
      e = hipEventQuery(ev);
      if (e == hipSuccess) continue;
      if (e != hipErrorNotReady) return fail_hip(e, "hipEventQuery(ready)");
      e = hipStreamWaitEvent(x.stream, ev, 0);
      if (e != hipSuccess) return fail_hip(e, "hipStreamWaitEvent(ready)");
    }
    if (nj == 1) {
      // A batch of one request runs the single-call kernels on the context's
      // stream: the same results bit for bit, without the table upload and
      // the graph launch (which cost a lone small request a good part of
      // its latency).
      const Request& rq = jobs[0]->req;
      char* base = static_cast<char*>(arena_) + jobs[0]->arena_off;
      char* work = base + rq.L.saved_bytes;
      const ImageView& v0 = T->view[0];
      e = launch_forward_all(rq.g, v0, reinterpret_cast<int*>(work + rq.L.fplan), x.stream);
      if (e != hipSuccess) return fail_hip(e, "forward kernels");
      if (need_bwd) {
        e = launch_backward_all(rq.g, v0, x.stream);
        if (e != hipSuccess) return fail_hip(e, "backward kernels");
      }
      e = hipEventRecord(x.done, x.stream);
      if (e != hipSuccess) return fail_hip(e, "hipEventRecord");
      return INTERP_OK;
    }
    const size_t bytes = offsetof(JobTable, view) + sizeof(ImageView) * (size_t)nj;
    e = hipMemcpyAsync(x.dtab, T, bytes, hipMemcpyHostToDevice, x.stream);
    if (e != hipSuccess) return fail_hip(e, "hipMemcpyAsync(table)");
    int most = 0;
    for (int ph = 0; ph < PH_COUNT; ++ph) most = std::max(most, T->units[ph][nj]);
    const int gs = most <= kSmallUnits ? 1 : 0;
    e = hipGraphLaunch(x.exec[gs][need_passes - 1][need_bwd ? 1 : 0], x.stream);
    if (e != hipSuccess) return fail_hip(e, "hipGraphLaunch");
    e = hipEventRecord(x.done, x.stream);
    if (e != hipSuccess) return fail_hip(e, "hipEventRecord");
    return INTERP_OK;
  }

 public:
  int query(int c) {
    const hipError_t e = hipEventQuery(ctx_[c].done);
    if (e == hipSuccess) return 1;
    if (e == hipErrorNotReady) return 0;
    fail_hip(e, "batch");
    return INTERP_EHIP;
  }

  void wait(int c) { hipEventSynchronize(ctx_[c].done); }

 private:
  struct Ctx {
    JobTable* dtab = nullptr;
    JobTable* htab = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    hipGraphExec_t exec[2][kServePasses][2] = {};  // [small grids][radix passes - 1][backward]
  };
  int device_ = 0;
  void* arena_ = nullptr;
  Ctx ctx_[kContexts];
};

}  // namespace serve
}  // namespace gmm

struct interp_server {
  gmm::serve::GpuExecutor exec;
  std::unique_ptr<gmm::serve::Scheduler<gmm::serve::Request, gmm::serve::GpuExecutor>> sched;
};

using namespace gmm;

namespace {
// A request checked and sized for the server; "" or the reason it is invalid.
std::string make_request(const interp_request* req, serve::Request* rq, uint64_t* bytes) {
  rq->r = *req;
  std::string m = make_geometry(&req->prob, &rq->g);
  if (!m.empty()) return m;
  if (rq->g.B != 1) return "a serving request has B = 1";
  if (rq->g.C > serve::kServeMaxC) return "the serving path takes C <= 4";
  if (rq->g.kern != 0) return "the serving path takes the default kernel only";
  if (rq->g.st != INTERP_STORAGE_F32) return "the serving path takes float32 storage only";
  if (rq->g.npass > serve::kServePasses) return "too many bins for the serving path";
  if (rq->g.N > 0 && (!req->pos || !req->sigma || !req->values))
    return "pos, sigma and values must not be NULL when N > 0";
  if (!req->sigma && !rq->g.per_point && rq->g.N > 0) return "sigma must not be NULL";
  if (!req->out) return "out must not be NULL";
  if ((req->pos && (uintptr_t)req->pos % 8) || (req->grad_pos && (uintptr_t)req->grad_pos % 8))
    return "pos and grad_pos must be 8-byte aligned";
  rq->L = make_layout(rq->g);
  *bytes = serve::Arena::round(rq->L.saved_bytes) + serve::Arena::round(rq->L.work_bytes);
  rq->L.saved_bytes = serve::Arena::round(rq->L.saved_bytes);  // workspace starts at the next grain
  return "";
}

int queue_result(int rc) {
  if (rc == INTERP_ENOMEM) return fail(rc, "request can never fit the server's memory budget");
  if (rc == INTERP_EAGAIN) return fail(rc, "server queue is full");
  return rc;
}
}  // namespace

extern "C" {

int interp_server_create(const interp_server_config* cfg, interp_server** out) {
  if (!cfg || !out) return fail(INTERP_EINVAL, "NULL argument");
  if (cfg->max_slots < 1 || cfg->max_slots > 1024) return fail(INTERP_EINVAL, "max_slots must be in [1, 1024]");
  if (cfg->max_queue < 1) return fail(INTERP_EINVAL, "max_queue must be >= 1");
  if (cfg->hbm_budget_bytes == 0) return fail(INTERP_EINVAL, "hbm_budget_bytes must be > 0");
  auto* s = new interp_server();
  int rc = s->exec.init(cfg->device, cfg->hbm_budget_bytes);
  if (rc != INTERP_OK) {
    s->exec.release();
    delete s;
    return rc;
  }
  s->sched.reset(new serve::Scheduler<serve::Request, serve::GpuExecutor>(
      &s->exec, cfg->hbm_budget_bytes, cfg->max_slots, cfg->max_queue));
  *out = s;
  return INTERP_OK;
}

int interp_submit(interp_server* s, const interp_request* req, uint64_t* ticket) {
  if (!s || !req || !ticket) return fail(INTERP_EINVAL, "NULL argument");
  serve::Request rq;
  uint64_t bytes = 0;
  const std::string m = make_request(req, &rq, &bytes);
  if (!m.empty()) return fail(INTERP_EINVAL, m);
  return queue_result(s->sched->submit(rq, bytes, ticket));
}

int interp_submit_many(interp_server* s, const interp_request* reqs, int32_t n, uint64_t* tickets,
                       int32_t* n_queued) {
  if (!s || !n_queued || (n > 0 && (!reqs || !tickets))) return fail(INTERP_EINVAL, "NULL argument");
  *n_queued = 0;
  if (n < 0) return fail(INTERP_EINVAL, "n must be >= 0");
  std::vector<serve::Request> rq(n);
  std::vector<uint64_t> bytes(n);
  for (int i = 0; i < n; ++i) {
    const std::string m = make_request(&reqs[i], &rq[i], &bytes[i]);
    if (!m.empty()) return fail(INTERP_EINVAL, "request " + std::to_string(i) + ": " + m);
  }
  if (n == 0) return INTERP_OK;
  int queued = 0;
  const int rc = s->sched->submit_many(rq.data(), bytes.data(), n, tickets, &queued);
  *n_queued = queued;
  return queue_result(rc);
}

int interp_poll(interp_server* s, uint64_t ticket, interp_status* status) {
  if (!s || !status) return fail(INTERP_EINVAL, "NULL argument");
  const int rc = s->sched->poll(ticket, status);
  if (rc == INTERP_ENOTFOUND) return fail(rc, "unknown ticket");
  return rc;
}

int interp_server_drain(interp_server* s, int64_t timeout_ms) {
  if (!s) return fail(INTERP_EINVAL, "NULL argument");
  return s->sched->drain(timeout_ms);
}

int interp_server_destroy(interp_server* s) {
  if (!s) return fail(INTERP_EINVAL, "NULL argument");
  s->sched->shutdown();
  s->sched.reset();
  s->exec.release();
  delete s;
  return INTERP_OK;
}

}  // extern "C"
