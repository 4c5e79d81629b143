// Serving loop for many pseudo-experiment fits of one model (the coverage
// studies that motivate fast fitting, Sec. 1; the toy study loop of the
// benchmark protocol, Sec. 3.1).
//
// One worker thread owns the device.  Requests are converted and validated
// on the submitting thread and queued.  The worker admits them while a slot
// is free and their event storage and workspaces fit the device arena (the
// memory budget), starts each fit (start metric from the analytic Hessian),
// and advances every active fit with one ragged launch per iteration: the
// event kernel over all active fits' tiles, each fit's last workgroup taking
// its BFGS step.  Consecutive iterations with an unchanged active set are
// replayed from a captured HIP graph.  Finished fits are retired between
// replays (final Hessian for the covariance), freeing their slot and memory
// for new requests.  A fit's arithmetic does not depend on what else shares
// the launch, so its result is bitwise the same as a lone uml_fit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstddef>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "host.h"
#include "host_pool.h"
#include "scatter.h"

namespace uml {

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over one device allocation (256-byte granules).
class Arena {
 public:
  void init(char* base, size_t cap) {
    base_ = base;
    cap_ = cap;
    free_.clear();
    if (cap) free_[0] = cap;
  }
  bool alloc(size_t size, size_t* off) {
    size = (size + 255) / 256 * 256;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < size) continue;
      *off = it->first;
      const size_t rest = it->second - size, at = it->first + size;
      free_.erase(it);
      if (rest) free_[at] = rest;
      used_ += size;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t size) {
    size = (size + 255) / 256 * 256;
    used_ -= size;
    auto it = free_.emplace(off, size).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  char* at(size_t off) const { return base_ + off; }
  size_t used() const { return used_; }
  size_t cap() const { return cap_; }

 private:
  char* base_ = nullptr;
  size_t cap_ = 0, used_ = 0;
  std::map<size_t, size_t> free_;
};

struct Request {
  uint64_t ticket = 0;
  int64_t n = 0;
  bool weighted = false;
  bool generate = false;      // events drawn on the device (seed, gen_theta)
  uint64_t seed = 0;
  std::vector<double> gen_theta;
  std::vector<char> host;     // converted event storage (kernel order)
  std::vector<double> start;  // all parameters
  size_t bytes = 0;           // arena footprint
  double t_submit = 0.0;
};

struct Slot {
  bool used = false;
  Request req;
  uml_data data;
  size_t off = 0;
  DataLayout layout{};
  size_t o_work = 0, o_hess = 0;
};

// Pinned host staging of one slot: the start point (and the point events are
// drawn at) going up, the fit state coming down.  Pinned, so that the copies
// of a whole batch of slots are queued together and waited for once.
struct SlotHost {
  FitState fs;
  double theta[UML_MAX_PARAMS];
  double gen_theta[UML_MAX_PARAMS];
};

size_t round256(size_t x) { return (x + 255) / 256 * 256; }

// Packed uploads (scatter.h): pieces staged in one pinned buffer, sent with
// one copy per flush and placed by one kernel.  A flushed range stays in use
// until the stream has passed it, so the buffer starts over only after a
// synchronisation (reset).
struct Packer {
  char* h = nullptr;  // pinned
  char* d = nullptr;  // device
  size_t cap = 0, start = 0, used = 0;
  std::vector<PackRec> recs;
  bool unsynced = false;

  static size_t up8(size_t x) { return (x + 7) & ~size_t(7); }
  static size_t up16(size_t x) { return (x + 15) & ~size_t(15); }
  bool room(size_t payload) const {
    return up16(used + payload) + (recs.size() + 1) * sizeof(PackRec) <= cap;
  }
  // nbytes: a multiple of 8 (every piece here is made of 8-byte words)
  bool put(void* dst, const void* src, size_t nbytes) {
    if (nbytes % 8 || !room(nbytes)) return false;
    std::memcpy(h + used, src, nbytes);
    recs.push_back(PackRec{dst, int64_t(used - start), int64_t(nbytes)});
    used += nbytes;
    return true;
  }
  bool zero(void* dst, size_t nbytes) {
    if (nbytes % 8 || !room(0)) return false;
    recs.push_back(PackRec{dst, -1, int64_t(nbytes)});
    return true;
  }
  hipError_t flush(hipStream_t s) {
    if (recs.empty()) return hipSuccess;
    const size_t ro = up16(used);
    std::memcpy(h + ro, recs.data(), recs.size() * sizeof(PackRec));
    const size_t end = ro + recs.size() * sizeof(PackRec);
    hipError_t e = hipMemcpyAsync(d + start, h + start, end - start, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
      launch_scatter(reinterpret_cast<const PackRec*>(d + ro), int(recs.size()), d + start, s);
      e = hipGetLastError();
    }
    start = used = up16(end);
    recs.clear();
    unsynced = true;
    return e;
  }
  hipError_t reset(hipStream_t s) {
    const hipError_t e = unsynced ? hipStreamSynchronize(s) : hipSuccess;
    start = used = 0;
    recs.clear();
    unsynced = false;
    return e;
  }
};

// Grid sizes the batched iteration is captured for: the active fits' tiles,
// rounded up to the next size of a geometric ladder (ratio about 1.19), so a
// changing active set reuses a few captured graphs; the padding tiles exit
// at once.
int grid_bucket(int grid) {
  int b = 64;
  while (b < grid) b = std::max(b + 64, int(double(b) * 1.1892));
  return b;
}

struct CapturedGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

}  // namespace

}  // namespace uml

using namespace uml;

struct uml_server {
  const uml_model* m = nullptr;
  uml_server_options opt{};
  std::mutex mu;
  std::condition_variable cv_work, cv_result;
  std::deque<Request> pending;
  std::deque<uml_fit_result> results;
  uint64_t next_ticket = 1;
  int64_t submitted = 0, admitted = 0, finished = 0, iterations = 0;
  int64_t resident = 0, peak_resident = 0, budget_waits = 0;  // arena bytes in use
  double t_admit = 0.0, t_iterate = 0.0, t_retire = 0.0;     // worker phase times
  int active = 0;
  bool stop = false;
  int worker_error = 0;
  std::string worker_msg;
  std::thread worker;
  // device state
  hipStream_t stream = nullptr;
  void* arena_mem = nullptr;
  void* state_mem = nullptr;
  Arena arena;
  FitState* d_fs = nullptr;
  Job* d_jobs = nullptr;
  int2* d_map = nullptr;
  int map_cap = 0;
  SlotHost* h_slots = nullptr;  // pinned, one per slot
  int* h_done = nullptr;        // pinned, one per slot
  int* h_done_dev = nullptr;    // its device address (written by a kernel)
  // batched Hessian passes: job tables, tile map, sums (pinned and device)
  HessJob* h_hjobs = nullptr;
  HessJob* d_hjobs = nullptr;
  int2* h_hmap = nullptr;
  int2* d_hmap = nullptr;
  int hmap_cap = 0;
  int gmap_cap = 0;  // generation map entries
  double* h_hsums = nullptr;
  double* d_hsums = nullptr;
  unsigned int* d_genbad = nullptr;  // per slot: events that failed to draw
  unsigned int* h_genbad = nullptr;
  // batched generation: job table and block map (pinned and device)
  GenJob* h_genjobs = nullptr;
  GenJob* d_genjobs = nullptr;
  int2* h_genmap = nullptr;
  int2* d_genmap = nullptr;
  // packed uploads of admission, and the packed fit states of retirement
  Packer up;
  PackRec* h_grecs = nullptr;
  PackRec* d_grecs = nullptr;
  char* h_gst = nullptr;
  char* d_gst = nullptr;
  std::vector<Slot> slots;
  std::vector<Job> jobs;
  std::map<int, CapturedGraph> graphs;  // by grid bucket
  std::unique_ptr<HostPool> pool;       // per-fit host arithmetic of a batch
  std::vector<int> batch_rc;            // per fit of a batch: its return code
  std::vector<std::string> batch_err;   // and its message, if it failed
  std::vector<uml_fit_result> batch_res;  // per fit of a batch: its result
};

namespace uml {
namespace {

constexpr int kItersPerReplay = 4;

size_t request_bytes(const uml_model* m, int64_t n, bool weighted) {
  const DataLayout L = data_layout(m->plan, n, weighted);
  int ht = 0;
  return round256(L.bytes_events) + round256(L.bytes_work) + round256(hess_work_bytes(m, n, &ht));
}

int fail_worker(uml_server* S, int code, const std::string& msg) {
  std::lock_guard<std::mutex> lk(S->mu);
  S->worker_error = code;
  S->worker_msg = msg;
  S->stop = true;
  S->cv_result.notify_all();
  return code;
}

void push_result(uml_server* S, uml_fit_result& r, const Request& q) {
  r.ticket = q.ticket;
  r.latency_s = now_s() - q.t_submit;
  std::lock_guard<std::mutex> lk(S->mu);
  S->results.push_back(r);
  S->finished++;
  S->cv_result.notify_all();
}

void release_slot(uml_server* S, Slot& sl) {
  S->arena.release(sl.off, sl.req.bytes);
  sl.used = false;
  std::lock_guard<std::mutex> lk(S->mu);
  S->resident -= int64_t(sl.req.bytes);
}

struct Intake {
  int slot;
  size_t off;
  Request req;
};

// Admits a batch of requests: places each in its slot's arena memory,
// uploads its events, queues the Hessian pass at its start point (the start
// metric), waits once for the whole batch, then writes the fit states.  A
// request whose start point has P <= 0 somewhere is answered at once.
// The packed form of data_init_work plus the start point: the job, the
// cleared constant cache, counters and outputs, and theta (padded with zeros).
bool pack_init(Packer& up, const uml_data& d, const DataLayout& L, const double* theta_padded) {
  char* w = static_cast<char*>(d.d_work);
  return up.put(w + L.o_job, &d.job, sizeof(Job)) && up.zero(w + L.o_cst, L.o_theta - L.o_cst) &&
         up.put(w + L.o_theta, theta_padded, sizeof(double) * UML_MAX_PARAMS) &&
         up.zero(w + L.o_out, L.o_part - L.o_out);
}

// The parts of a new fit state the device reads: all but the rows of V and
// V0 past the free parameters (the device reads both only at rows and
// columns below nf).  Less than half of the state's bytes at nf = 17.
bool pack_fit_state(Packer& up, FitState* d, const FitState& h, int nf) {
  const size_t o_V = offsetof(FitState, V), o_V0 = offsetof(FitState, V0), o_f = offsetof(FitState, f);
  const size_t rows = sizeof(double) * UML_MAX_PARAMS * size_t(nf);
  char* dd = reinterpret_cast<char*>(d);
  const char* hh = reinterpret_cast<const char*>(&h);
  if (!up.put(dd, hh, o_V) || !up.put(dd + o_f, hh + o_f, sizeof(FitState) - o_f)) return false;
  return rows == 0 || (up.put(dd + o_V, hh + o_V, rows) && up.put(dd + o_V0, hh + o_V0, rows));
}

// What retirement reads of a finished fit state: theta, and the scalars
// from f on (counts and status).
constexpr size_t kRetTheta = sizeof(double) * UML_MAX_PARAMS;
constexpr size_t kRetTail = sizeof(FitState) - offsetof(FitState, f);
constexpr size_t kRetBytes = kRetTheta + kRetTail;

int admit_batch(uml_server* S, std::vector<Intake>& in) {
  const uml_model* m = S->m;
  const int ns = int(S->slots.size());
  UML_HIP_CHECK(S->up.reset(S->stream));
  int n_gen = 0, n_gmap = 0;  // requests drawn on the device, in one batched launch
  int64_t gen_total = 0;
  for (const auto& it : in)
    if (it.req.generate) gen_total += it.req.n;
  const int64_t gblock = gen_block_events(gen_total);
  for (auto& it : in) {
    Slot& sl = S->slots[it.slot];
    sl.off = it.off;
    sl.used = true;
    sl.req = std::move(it.req);
    sl.layout = data_layout(m->plan, sl.req.n, sl.req.weighted);
    sl.o_work = round256(sl.layout.bytes_events);
    sl.o_hess = sl.o_work + round256(sl.layout.bytes_work);
    sl.data = uml_data();
    data_bind(&sl.data, m, sl.req.n, sl.req.weighted, sl.layout, S->arena.at(sl.off),
              S->arena.at(sl.off + sl.o_work));
    sl.data.d_hwork = S->arena.at(sl.off + sl.o_hess);
    hess_work_bytes(m, sl.req.n, &sl.data.hess_tiles);
    sl.data.h_stage = S->h_slots[it.slot].theta;
    sl.data.owns_memory = 0;
    SlotHost& H = S->h_slots[it.slot];
    hipError_t e = hipSuccess;
    if (sl.req.generate) {  // drawn below; until then the output area holds the point
      std::memset(H.gen_theta, 0, sizeof(H.gen_theta));
      std::memcpy(H.gen_theta, sl.req.gen_theta.data(), sizeof(double) * m->plan.npar);
      if (!S->up.put(sl.data.d_out, H.gen_theta, sizeof(double) * UML_MAX_PARAMS))
        return set_error(UML_E_INVALID, "server: upload staging full");
      S->h_genjobs[n_gen] = GenJob{gen_out(&sl.data, S->d_genbad + it.slot), sl.data.d_out, sl.req.seed};
      for (int64_t b = 0; b * gblock < sl.req.n; ++b) {
        if (n_gmap >= S->gmap_cap) return set_error(UML_E_INVALID, "server: generation map full");
        S->h_genmap[n_gmap++] = make_int2(n_gen, int(b));
      }
      ++n_gen;
    } else {
      e = hipMemcpyAsync(sl.data.d_events, sl.req.host.data(), sl.req.host.size(), hipMemcpyHostToDevice,
                         S->stream);
    }
    if (e != hipSuccess) return set_error(UML_E_HIP, std::string("server upload: ") + hipGetErrorString(e));
  }
  if (n_gen) {  // one launch draws every generated request (their points placed first)
    // the failure counters cleared by the same packed upload
    if (!S->up.zero(S->d_genbad, (sizeof(unsigned int) * ns + 7) / 8 * 8))
      return set_error(UML_E_INVALID, "server: upload staging full");
    UML_HIP_CHECK(S->up.flush(S->stream));
    UML_HIP_CHECK(hipMemcpyAsync(S->d_genjobs, S->h_genjobs, sizeof(GenJob) * n_gen, hipMemcpyHostToDevice,
                                 S->stream));
    UML_HIP_CHECK(hipMemcpyAsync(S->d_genmap, S->h_genmap, sizeof(int2) * n_gmap, hipMemcpyHostToDevice,
                                 S->stream));
    launch_generate_batch(m->d_gplan, S->d_genjobs, S->d_genmap, n_gmap, gblock, m->plan.precision, S->stream);
    UML_HIP_CHECK(hipGetLastError());
  }
  // every work area initialised, start points included, in one packed upload
  for (auto& it : in) {
    Slot& sl = S->slots[it.slot];
    SlotHost& H = S->h_slots[it.slot];
    UML_HIP_CHECK(data_precompute(&sl.data, S->stream));
    std::memset(H.theta, 0, sizeof(H.theta));
    std::memcpy(H.theta, sl.req.start.data(), sizeof(double) * m->plan.npar);
    if (!pack_init(S->up, sl.data, sl.layout, H.theta))
      return set_error(UML_E_INVALID, "server: upload staging full");
  }
  UML_HIP_CHECK(S->up.flush(S->stream));
  const int nb = int(in.size()), M = hess_sums(m);
  std::vector<uml_data*> ds(nb);
  std::vector<const double*> th(nb);
  for (int j = 0; j < nb; ++j) {
    ds[j] = &S->slots[in[j].slot].data;
    th[j] = ds[j]->d_theta;
  }
  int rc = hessian_queue_batch(m, ds.data(), th.data(), nb, S->d_hsums, S->h_hjobs, S->d_hjobs, S->h_hmap,
                               S->d_hmap, S->hmap_cap, S->stream, "server");
  if (rc != UML_OK) return rc;
  UML_HIP_CHECK(hipMemcpyAsync(S->h_hsums, S->d_hsums, sizeof(double) * nb * M, hipMemcpyDeviceToHost,
                               S->stream));
  if (n_gen)
    UML_HIP_CHECK(hipMemcpyAsync(S->h_genbad, S->d_genbad, sizeof(unsigned int) * ns, hipMemcpyDeviceToHost,
                                 S->stream));
  UML_HIP_CHECK(hipStreamSynchronize(S->stream));
  // the start metrics, fit by fit on the host threads
  S->pool->run(nb, [&](int j) {
    const int i = in[j].slot;
    const Slot& sl = S->slots[i];
    SlotHost& H = S->h_slots[i];
    S->batch_rc[j] = UML_OK;
    if (sl.req.generate && S->h_genbad[i]) return;
    fit_state_begin(m, sl.req.start.data(), S->opt.fit, H.fs);
    S->batch_rc[j] = fit_state_metric(m, S->h_hsums + size_t(j) * M, H.fs, "server");
    if (S->batch_rc[j] != UML_OK) S->batch_err[j] = uml_last_error();  // this thread's message
  });
  int started = 0;  // fits that begin iterating
  for (int j = 0; j < nb; ++j) {
    const int i = in[j].slot;
    Slot& sl = S->slots[i];
    SlotHost& H = S->h_slots[i];
    std::vector<char>().swap(sl.req.host);  // uploaded
    if (sl.req.generate && S->h_genbad[i]) {  // some events could not be drawn
      uml_fit_result r;
      std::memset(&r, 0, sizeof(r));
      r.n_free = m->plan.nfree;
      r.status = UML_FIT_GENERATION_FAILED;
      r.nll = INFINITY;
      for (int k = 0; k < m->plan.npar; ++k) r.params[k] = sl.req.start[k];
      release_slot(S, sl);
      push_result(S, r, sl.req);
      continue;
    }
    if (S->batch_rc[j] != UML_OK) return set_error(S->batch_rc[j], S->batch_err[j]);
    if (H.fs.done) {  // P <= 0 at the start point
      uml_fit_result r;
      std::memset(&r, 0, sizeof(r));
      r.n_free = m->plan.nfree;
      r.status = H.fs.status;
      r.nll = INFINITY;
      for (int k = 0; k < m->plan.npar; ++k) r.params[k] = sl.req.start[k];
      rc = fill_bad_count(m, &sl.data, &r, S->stream, "server");
      if (rc != UML_OK) return rc;
      release_slot(S, sl);
      push_result(S, r, sl.req);
      continue;
    }
    Job J = sl.data.job;
    J.fit = S->d_fs + i;
    J.theta = S->d_fs[i].theta;
    J.out = S->d_fs[i].out;
    S->jobs[i] = J;
    if (!pack_fit_state(S->up, S->d_fs + i, H.fs, m->plan.nfree) ||
        !S->up.put(S->d_jobs + i, &S->jobs[i], sizeof(Job)))
      return set_error(UML_E_INVALID, "server: upload staging full");
    ++started;
  }
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->active += started;
  }
  UML_HIP_CHECK(S->up.flush(S->stream));  // the fit states and jobs of the admitted fits
  return UML_OK;
}

// Retires a batch of finished fits: queues, for each, the copy of its fit
// state and the Hessian pass at its final point (read on the device), waits
// once, then forms the results (covariance from the inverse Hessian) and
// frees the slots.  Newton polishing, when asked for, runs fit by fit.
int retire_batch(uml_server* S, const std::vector<int>& fin) {
  const uml_model* m = S->m;
  const Plan& P = m->plan;
  const bool polish = S->opt.fit.polish > 0;
  const int nb = int(fin.size()), M = hess_sums(m);
  // what is read of the finished fit states, collected by one kernel and
  // one copy
  for (int j = 0; j < nb; ++j) {
    char* f = reinterpret_cast<char*>(S->d_fs + fin[j]);
    const int64_t o = int64_t(kRetBytes) * j;
    S->h_grecs[2 * j] = PackRec{f, o, int64_t(kRetTheta)};
    S->h_grecs[2 * j + 1] = PackRec{f + offsetof(FitState, f), o + int64_t(kRetTheta), int64_t(kRetTail)};
  }
  UML_HIP_CHECK(
      hipMemcpyAsync(S->d_grecs, S->h_grecs, sizeof(PackRec) * 2 * nb, hipMemcpyHostToDevice, S->stream));
  launch_gather(S->d_grecs, 2 * nb, S->d_gst, S->stream);
  UML_HIP_CHECK(hipGetLastError());
  UML_HIP_CHECK(hipMemcpyAsync(S->h_gst, S->d_gst, kRetBytes * nb, hipMemcpyDeviceToHost, S->stream));
  if (!polish) {  // the Hessian pass at each final point, read on the device
    std::vector<uml_data*> ds(nb);
    std::vector<const double*> th(nb);
    for (int j = 0; j < nb; ++j) {
      ds[j] = &S->slots[fin[j]].data;
      th[j] = S->d_fs[fin[j]].theta;
    }
    int rc = hessian_queue_batch(m, ds.data(), th.data(), nb, S->d_hsums, S->h_hjobs, S->d_hjobs,
                                 S->h_hmap, S->d_hmap, S->hmap_cap, S->stream, "server");
    if (rc != UML_OK) return rc;
    UML_HIP_CHECK(hipMemcpyAsync(S->h_hsums, S->d_hsums, sizeof(double) * nb * M, hipMemcpyDeviceToHost,
                                 S->stream));
  }
  UML_HIP_CHECK(hipStreamSynchronize(S->stream));
  // the results, fit by fit on the host threads (the device work of
  // polishing and of counting bad events comes after, in order)
  S->pool->run(nb, [&](int j) {
    FitState& F = S->h_slots[fin[j]].fs;  // theta and the scalars (the rest is not read)
    std::memcpy(F.theta, S->h_gst + kRetBytes * j, kRetTheta);
    std::memcpy(&F.f, S->h_gst + kRetBytes * j + kRetTheta, kRetTail);
    uml_fit_result& r = S->batch_res[j];
    std::memset(&r, 0, sizeof(r));
    r.n_free = P.nfree;
    r.n_iter = F.n_iter;
    r.n_eval = F.n_eval;
    r.status = F.status;
    if (r.status == UML_FIT_PDF_NONPOSITIVE) {
      for (int k = 0; k < P.npar; ++k) r.params[k] = F.theta[k];
      r.nll = INFINITY;
    } else if (!polish) {
      finish_from_sums(m, S->h_hsums + size_t(j) * M, F.theta, S->opt.fit, &r, "server");
    }
  });
  int64_t freed = 0;  // arena bytes of the retired fits
  for (int j = 0; j < nb; ++j) {
    const int i = fin[j];
    Slot& sl = S->slots[i];
    const FitState& F = S->h_slots[i].fs;
    uml_fit_result& r = S->batch_res[j];
    if (r.status != UML_FIT_PDF_NONPOSITIVE && polish) {
      std::vector<double> theta(F.theta, F.theta + P.npar);
      int rc = finish_fit(m, &sl.data, theta, S->opt.fit, &r, S->stream, "server");
      if (rc != UML_OK) return rc;
    }
    int rc = fill_bad_count(m, &sl.data, &r, S->stream, "server");
    if (rc != UML_OK) return rc;
    S->arena.release(sl.off, sl.req.bytes);
    sl.used = false;
    freed += int64_t(sl.req.bytes);
    r.ticket = sl.req.ticket;
    r.latency_s = now_s() - sl.req.t_submit;
  }
  {  // the batch's results, under one lock and one notification
    std::lock_guard<std::mutex> lk(S->mu);
    for (int j = 0; j < nb; ++j) S->results.push_back(S->batch_res[j]);
    S->finished += nb;
    S->active -= nb;
    S->resident -= freed;
  }
  S->cv_result.notify_all();
  return UML_OK;
}

// The captured batched iteration for a grid bucket (captured on first use).
int graph_for(uml_server* S, int bucket, hipGraphExec_t* exec) {
  auto it = S->graphs.find(bucket);
  if (it != S->graphs.end()) {
    *exec = it->second.exec;
    return UML_OK;
  }
  const uml_model* m = S->m;
  LaunchArgs a{};
  a.job0 = S->jobs[0];
  a.jobs = S->d_jobs;
  a.tmap = S->d_map;
  a.grid = bucket;
  a.precision = m->plan.precision;
  a.stream = S->stream;
  CapturedGraph g;
  hipError_t e = hipStreamBeginCapture(S->stream, hipStreamCaptureModeThreadLocal);
  for (int k = 0; k < kItersPerReplay && e == hipSuccess; ++k) m->family->eval(a);
  if (e == hipSuccess) e = hipStreamEndCapture(S->stream, &g.graph);
  if (e == hipSuccess) e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    if (g.graph) (void)hipGraphDestroy(g.graph);
    return set_error(UML_E_HIP, std::string("server graph: ") + hipGetErrorString(e));
  }
  S->graphs[bucket] = g;
  *exec = g.exec;
  return UML_OK;
}

// Device and pinned memory and the stream of a server (what was allocated).
void free_server_memory(uml_server* S) {
  if (S->arena_mem) (void)hipFree(S->arena_mem);
  if (S->state_mem) (void)hipFree(S->state_mem);
  for (void* p : {static_cast<void*>(S->h_slots), static_cast<void*>(S->h_done),
                  static_cast<void*>(S->h_hjobs), static_cast<void*>(S->h_hmap),
                  static_cast<void*>(S->h_hsums), static_cast<void*>(S->h_genbad),
                  static_cast<void*>(S->h_genjobs), static_cast<void*>(S->h_genmap),
                  static_cast<void*>(S->up.h), static_cast<void*>(S->h_grecs), static_cast<void*>(S->h_gst)})
    if (p) (void)hipHostFree(p);
  for (void* p : {static_cast<void*>(S->up.d), static_cast<void*>(S->d_grecs), static_cast<void*>(S->d_gst)})
    if (p) (void)hipFree(p);
  if (S->stream) (void)hipStreamDestroy(S->stream);
}

void worker_main(uml_server* S) {
  (void)hipSetDevice(S->m->device);
  const int ns = int(S->slots.size());
  std::vector<int2> map;
  std::vector<int> fin;
  bool dirty = true;
  int bucket = 0;
  while (true) {
    std::vector<Intake> intake;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      if (S->stop && S->pending.empty() && S->active == 0) break;
      // admission, in arrival order: a free slot and room in the arena (the
      // memory budget); the arena belongs to this thread
      for (int i = 0; i < ns && !S->pending.empty(); ++i) {
        if (S->slots[i].used) continue;
        size_t off = 0;
        if (!S->arena.alloc(S->pending.front().bytes, &off)) {
          S->budget_waits++;
          break;
        }
        S->resident += int64_t(S->pending.front().bytes);
        S->peak_resident = std::max(S->peak_resident, S->resident);
        intake.push_back({i, off, std::move(S->pending.front())});
        S->pending.pop_front();
      }
      if (intake.empty() && S->active == 0) {
        S->cv_work.wait_for(lk, std::chrono::milliseconds(2));
        continue;
      }
      S->admitted += int64_t(intake.size());
    }
    if (!intake.empty()) {
      const double t0 = now_s();
      int rc = admit_batch(S, intake);
      {
        std::lock_guard<std::mutex> lk(S->mu);
        S->t_admit += now_s() - t0;
      }
      if (rc != UML_OK) {
        fail_worker(S, rc, uml_last_error());
        return;
      }
      dirty = true;
    }
    if (S->active == 0) continue;
    if (dirty) {  // ragged tile map over the active fits, padded to its grid bucket
      map.clear();
      for (int i = 0; i < ns; ++i)
        if (S->slots[i].used)
          for (int t = 0; t < S->slots[i].data.n_tiles; ++t) map.push_back(make_int2(i, t));
      bucket = grid_bucket(int(map.size()));
      if (bucket > S->map_cap) {
        fail_worker(S, UML_E_INVALID, "server: tile map capacity exceeded");
        return;
      }
      map.resize(bucket, make_int2(-1, -1));
      hipError_t e = hipMemcpyAsync(S->d_map, map.data(), sizeof(int2) * map.size(),
                                    hipMemcpyHostToDevice, S->stream);
      if (e != hipSuccess) {
        fail_worker(S, UML_E_HIP, hipGetErrorString(e));
        return;
      }
      dirty = false;
    }
    const double t_it = now_s();
    hipGraphExec_t exec = nullptr;
    int rc = graph_for(S, bucket, &exec);
    if (rc != UML_OK) {
      fail_worker(S, rc, uml_last_error());
      return;
    }
    hipError_t e = hipGraphLaunch(exec, S->stream);
    if (e == hipSuccess) {  // every fit's done flag, written by a kernel straight into pinned memory
      launch_collect_ints(&S->d_fs[0].done, int64_t(sizeof(FitState)), ns, S->h_done_dev, S->stream);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(S->stream);
    if (e != hipSuccess) {
      fail_worker(S, UML_E_HIP, std::string("server iteration: ") + hipGetErrorString(e));
      return;
    }
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->iterations += kItersPerReplay;
      S->t_iterate += now_s() - t_it;
    }
    fin.clear();
    for (int i = 0; i < ns; ++i)
      if (S->slots[i].used && S->h_done[i]) fin.push_back(i);
    if (!fin.empty()) {
      const double t0 = now_s();
      rc = retire_batch(S, fin);
      {
        std::lock_guard<std::mutex> lk(S->mu);
        S->t_retire += now_s() - t0;
      }
      if (rc != UML_OK) {
        fail_worker(S, rc, uml_last_error());
        return;
      }
      dirty = true;
    }
  }
}

}  // namespace
}  // namespace uml

extern "C" {

void uml_server_options_default(uml_server_options* o) {
  if (!o) return;
  o->max_slots = 256;
  o->hbm_budget = int64_t(4) << 30;
  o->max_pending = 1 << 20;
  uml_fit_options_default(&o->fit);
}

int uml_server_create(const uml_model* m, const uml_server_options* opts, uml_server** out) {
  if (!out || !m) return set_error(UML_E_INVALID, "uml_server_create: null argument");
  *out = nullptr;
  uml_server* S = new (std::nothrow) uml_server();
  if (!S) return set_error(UML_E_NOMEM, "uml_server_create: out of host memory");
  S->m = m;
  uml_server_options_default(&S->opt);
  if (opts) S->opt = *opts;
  if (S->opt.max_slots <= 0) S->opt.max_slots = 256;
  if (S->opt.hbm_budget <= 0) S->opt.hbm_budget = int64_t(4) << 30;
  if (S->opt.max_pending <= 0) S->opt.max_pending = 1 << 20;
  if (int rc = check_fit_options(S->opt.fit, "uml_server_create")) {
    delete S;
    return rc;
  }
  if (S->opt.fit.method != UML_METHOD_BFGS) {
    delete S;
    return set_error(UML_E_UNSUPPORTED, "uml_server_create: the server runs device BFGS fits only");
  }
  const int ns = S->opt.max_slots;
  S->slots.resize(ns);
  S->jobs.resize(ns);
  S->batch_rc.resize(ns);
  S->batch_err.resize(ns);
  S->batch_res.resize(ns);
  // helpers for the per-fit host arithmetic: up to three, leaving cores to
  // the caller
  const int hw = int(std::thread::hardware_concurrency());
  S->pool = std::make_unique<HostPool>(std::max(0, std::min(3, hw / 2 - 1)));
  // tile map capacity: the arena holds at most budget / (bytes of one tile)
  const DataLayout one = data_layout(m->plan, 1, false);
  const int64_t tile_bytes = int64_t(one.E) * kBlock * (m->plan.precision == UML_MIXED ? 4 : 8);
  S->map_cap = grid_bucket(
      int(std::min<int64_t>(S->opt.hbm_budget / std::max<int64_t>(tile_bytes, 1) + ns, 1 << 22)));
  // Hessian tile map capacity: a request has at most n / 256 + 1 Hessian
  // tiles, and the arena holds at most budget / (bytes per event) events
  const int64_t ev_bytes = int64_t(m->plan.ndim) * (m->plan.precision == UML_MIXED ? 4 : 8);
  S->hmap_cap = int(std::min<int64_t>(S->opt.hbm_budget / (256 * ev_bytes) + ns, 1 << 22));
  // generation map capacity: a batch of T events in blocks of
  // gen_block_events(T) has at most kGenTargetWaves blocks, or T / 512 if
  // its blocks are the largest, plus one partial block per request
  S->gmap_cap = int(std::min<int64_t>(kGenTargetWaves + S->opt.hbm_budget / (512 * ev_bytes) + ns, 1 << 22));
  const int M = hess_sums(m);
  auto fail = [&](hipError_t e, const char* what) {
    free_server_memory(S);
    delete S;
    return set_error(e == hipErrorOutOfMemory ? UML_E_NOMEM : UML_E_HIP,
                     std::string("uml_server_create: ") + what + ": " + hipGetErrorString(e));
  };
  hipError_t e = hipSetDevice(m->device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking);
  if (e != hipSuccess) return fail(e, "stream");
  e = hipMalloc(&S->arena_mem, size_t(S->opt.hbm_budget));
  if (e != hipSuccess) return fail(e, "arena");
  const size_t o_jobs = round256(sizeof(FitState) * ns), o_map = o_jobs + round256(sizeof(Job) * ns);
  const size_t o_hjobs = o_map + round256(sizeof(int2) * size_t(S->map_cap));
  const size_t o_hmap = o_hjobs + round256(sizeof(HessJob) * ns);
  const size_t o_hsums = o_hmap + round256(sizeof(int2) * size_t(S->hmap_cap));
  const size_t o_genbad = o_hsums + round256(sizeof(double) * size_t(ns) * M);
  const size_t o_genjobs = o_genbad + round256(sizeof(unsigned int) * ns);
  const size_t o_genmap = o_genjobs + round256(sizeof(GenJob) * ns);
  e = hipMalloc(&S->state_mem, o_genmap + sizeof(int2) * size_t(S->gmap_cap));
  if (e != hipSuccess) return fail(e, "fit states");
  e = hipMemset(S->state_mem, 0, o_map);
  if (e != hipSuccess) return fail(e, "fit states");
  e = hipHostMalloc(reinterpret_cast<void**>(&S->h_slots), sizeof(SlotHost) * ns, hipHostMallocDefault);
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void**>(&S->h_done), sizeof(int) * ns, hipHostMallocMapped);
  if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void**>(&S->h_done_dev), S->h_done, 0);
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void**>(&S->h_hjobs), sizeof(HessJob) * ns, hipHostMallocDefault);
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void**>(&S->h_hmap), sizeof(int2) * size_t(S->hmap_cap),
                      hipHostMallocDefault);
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void**>(&S->h_hsums), sizeof(double) * size_t(ns) * M,
                      hipHostMallocDefault);
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void**>(&S->h_genbad), sizeof(unsigned int) * ns,
                      hipHostMallocDefault);
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void**>(&S->h_genjobs), sizeof(GenJob) * ns, hipHostMallocDefault);
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void**>(&S->h_genmap), sizeof(int2) * size_t(S->gmap_cap),
                      hipHostMallocDefault);
  // packed transfers: every piece one admission batch uploads (fit state,
  // two jobs, two parameter vectors per request, their records and padding),
  // and the fit states one retirement batch collects
  S->up.cap = size_t(ns) * (sizeof(FitState) + 2 * sizeof(Job) + 2 * sizeof(double) * UML_MAX_PARAMS +
                            8 * sizeof(PackRec)) + (64 << 10);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&S->up.h), S->up.cap, hipHostMallocDefault);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&S->up.d), S->up.cap);
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void**>(&S->h_grecs), sizeof(PackRec) * 2 * ns, hipHostMallocDefault);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&S->d_grecs), sizeof(PackRec) * 2 * ns);
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void**>(&S->h_gst), kRetBytes * ns, hipHostMallocDefault);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&S->d_gst), kRetBytes * ns);
  if (e != hipSuccess) return fail(e, "pinned staging");
  S->arena.init(static_cast<char*>(S->arena_mem), size_t(S->opt.hbm_budget));
  S->d_fs = reinterpret_cast<FitState*>(S->state_mem);
  S->d_jobs = reinterpret_cast<Job*>(static_cast<char*>(S->state_mem) + o_jobs);
  S->d_map = reinterpret_cast<int2*>(static_cast<char*>(S->state_mem) + o_map);
  S->d_hjobs = reinterpret_cast<HessJob*>(static_cast<char*>(S->state_mem) + o_hjobs);
  S->d_hmap = reinterpret_cast<int2*>(static_cast<char*>(S->state_mem) + o_hmap);
  S->d_hsums = reinterpret_cast<double*>(static_cast<char*>(S->state_mem) + o_hsums);
  S->d_genbad = reinterpret_cast<unsigned int*>(static_cast<char*>(S->state_mem) + o_genbad);
  S->d_genjobs = reinterpret_cast<GenJob*>(static_cast<char*>(S->state_mem) + o_genjobs);
  S->d_genmap = reinterpret_cast<int2*>(static_cast<char*>(S->state_mem) + o_genmap);
  // idle slots read as finished so that their (never mapped) tiles do nothing
  std::vector<FitState> idle(ns);
  for (auto& F : idle) {
    std::memset(&F, 0, sizeof(F));
    F.done = 1;
  }
  e = hipMemcpy(S->d_fs, idle.data(), sizeof(FitState) * ns, hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail(e, "fit states");
  for (auto& J : S->jobs) std::memset(&J, 0, sizeof(J));
  S->worker = std::thread(worker_main, S);
  *out = S;
  return UML_OK;
}

int uml_server_submit(uml_server* S, const uml_request* q, uint64_t* ticket) {
  if (!S || !q || !ticket) return set_error(UML_E_INVALID, "uml_server_submit: null argument");
  const Plan& P = S->m->plan;
  Request r;
  r.n = q->n_events;
  if (q->generate) {
    if (q->n_events < 0) return set_error(UML_E_INVALID, "uml_server_submit: negative event count");
    const double* gt = q->gen_theta ? q->gen_theta : S->m->theta0.data();
    int rc = check_generation_theta(S->m, gt, "uml_server_submit");
    if (rc != UML_OK) return rc;
    r.generate = true;
    r.seed = q->seed;
    r.gen_theta.assign(gt, gt + P.npar);
  } else {
    r.weighted = q->w != nullptr;
    int rc = convert_events(P, q->n_events, q->cols, q->dtype, q->w, r.host, "uml_server_submit");
    if (rc != UML_OK) return rc;
  }
  r.start.resize(P.npar);
  for (int k = 0; k < P.npar; ++k) r.start[k] = q->start ? q->start[k] : S->m->theta0[k];
  r.bytes = request_bytes(S->m, r.n, r.weighted);
  if (int64_t(r.bytes) > S->opt.hbm_budget)
    return set_error(UML_E_BUDGET, "uml_server_submit: the request needs " +
                                       std::to_string(r.bytes) + " bytes, more than the budget");
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->worker_error) return set_error(S->worker_error, "uml_server_submit: " + S->worker_msg);
  if (int64_t(S->pending.size()) >= S->opt.max_pending)
    return set_error(UML_E_QUEUE_FULL, "uml_server_submit: too many pending requests");
  r.ticket = S->next_ticket++;
  r.t_submit = now_s();
  *ticket = r.ticket;
  S->pending.push_back(std::move(r));
  S->submitted++;
  S->cv_work.notify_one();
  return UML_OK;
}

int uml_server_poll(uml_server* S, uml_fit_result* out, int32_t max, int32_t* n_out, int32_t timeout_us) {
  if (!S || !n_out || (max > 0 && !out)) return set_error(UML_E_INVALID, "uml_server_poll: bad argument");
  *n_out = 0;
  std::unique_lock<std::mutex> lk(S->mu);
  auto ready = [&] {
    return !S->results.empty() || S->worker_error ||
           (timeout_us < 0 && S->finished >= S->submitted);
  };
  if (timeout_us > 0)
    S->cv_result.wait_for(lk, std::chrono::microseconds(timeout_us), ready);
  else if (timeout_us < 0)
    S->cv_result.wait(lk, ready);
  while (*n_out < max && !S->results.empty()) {
    out[(*n_out)++] = S->results.front();
    S->results.pop_front();
  }
  if (S->worker_error) return set_error(S->worker_error, "uml_server_poll: " + S->worker_msg);
  if (*n_out == 0 && timeout_us != 0) return set_error(UML_E_TIMEOUT, "uml_server_poll: no result");
  return UML_OK;
}

int uml_server_stats_get(uml_server* S, uml_server_stats* st) {
  if (!S || !st) return set_error(UML_E_INVALID, "uml_server_stats_get: null argument");
  std::lock_guard<std::mutex> lk(S->mu);
  st->submitted = S->submitted;
  st->admitted = S->admitted;
  st->finished = S->finished;
  st->pending = int64_t(S->pending.size());
  st->active = S->active;
  st->iterations = S->iterations;
  st->resident_bytes = S->resident;
  st->peak_resident_bytes = S->peak_resident;
  st->budget_waits = S->budget_waits;
  st->t_admit_s = S->t_admit;
  st->t_iterate_s = S->t_iterate;
  st->t_retire_s = S->t_retire;
  return UML_OK;
}

int uml_server_drain(uml_server* S) {
  if (!S) return set_error(UML_E_INVALID, "uml_server_drain: null argument");
  std::unique_lock<std::mutex> lk(S->mu);
  S->cv_result.wait(lk, [&] { return S->finished >= S->submitted || S->worker_error; });
  if (S->worker_error) return set_error(S->worker_error, "uml_server_drain: " + S->worker_msg);
  return UML_OK;
}

void uml_server_destroy(uml_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    S->pending.clear();
    S->cv_work.notify_all();
  }
  if (S->worker.joinable()) S->worker.join();
  if (S->stream) (void)hipStreamSynchronize(S->stream);
  for (auto& kv : S->graphs) {
    (void)hipGraphExecDestroy(kv.second.exec);
    (void)hipGraphDestroy(kv.second.graph);
  }
  free_server_memory(S);
  delete S;
}

}  // extern "C"
