// Serving runtime of the library (the ks_server_* calls of include/ks.h).
//
// Independent minimisation requests (each one run of Alg. 3 on its own system) arrive at
// any time.  The server owns no device memory: it sub-allocates the caller's workspace,
// first fit, by each request's HBM footprint (the system workspace plus its orbital
// block).  n_slots worker threads each take the oldest queued request once a slot and a
// region are free, run it to its stopping rule on a stream of their own and release the
// region, so a request that arrives while others run starts as soon as memory frees up
// and its kernels overlap with theirs on the device.  Admission is strictly in arrival
// order: a request that does not fit yet holds back the ones behind it, which keeps
// large requests from starving.  Every request runs the same kernels with the same
// reduction order as a lone ks_minimize call, so its result does not depend on what else
// is resident.
//
// In batched mode (ks_server_create_batched) one engine thread does continuous batching:
// between trial steps it admits queued requests while regions and batch places are free,
// advances every resident request by one trial with one launch per kernel for all of
// them, and retires the ones that stopped.  Requests the lockstep runner cannot take run
// alone on the engine thread.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include <hip/hip_runtime.h>

#include "ks_common.h"

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Job {
  ks_request rq{};
  std::vector<double> R, Z, vext;
  std::vector<unsigned char> X0;
  size_t ws_bytes = 0;  // system workspace
  size_t x_bytes = 0;   // orbital block (n x p)
  double t_submit = 0.0;
};

struct Region {
  size_t off, size;
};

}  // namespace

struct ks_server {
  char* base = nullptr;
  size_t bytes = 0;
  int device = 0;
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_work, cv_idle;
  std::deque<Job*> queue;
  std::vector<Region> free_list;  // sorted by offset, coalesced
  std::vector<ks_completion> done;
  std::vector<std::thread> workers;
  int running = 0;
  bool stop = false;
  int max_batch = 0;  // > 0: batched mode

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }

  // First fit; returns false when no free region is large enough.
  bool take(size_t need, size_t* off) {
    for (size_t i = 0; i < free_list.size(); ++i) {
      Region& r = free_list[i];
      if (r.size >= need) {
        *off = r.off;
        r.off += need;
        r.size -= need;
        if (r.size == 0) free_list.erase(free_list.begin() + i);
        return true;
      }
    }
    return false;
  }

  void give(size_t off, size_t size) {
    auto it = std::lower_bound(free_list.begin(), free_list.end(), off,
                               [](const Region& r, size_t o) { return r.off < o; });
    it = free_list.insert(it, Region{off, size});
    // merge with the right neighbour, then the left one
    auto nx = it + 1;
    if (nx != free_list.end() && it->off + it->size == nx->off) {
      it->size += nx->size;
      free_list.erase(nx);
    }
    if (it != free_list.begin()) {
      auto pv = it - 1;
      if (pv->off + pv->size == it->off) {
        pv->size += it->size;
        free_list.erase(it);
      }
    }
  }
};

namespace {

// Runs one admitted request in the region at base + off on stream st.
void run_job(ks_server* sv, Job* jb, size_t off, hipStream_t st, ks_completion* c) {
  const ks_system_desc& d = jb->rq.desc;  // ld was reset to p at submit
  char* ws = sv->base + off;
  char* X = ws + align_up(jb->ws_bytes);
  c->status = KS_OK;
  hipError_t e = hipMemcpyAsync(X, jb->X0.data(), jb->x_bytes, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) {
    c->status = KS_E_HIP;
    return;
  }
  ks_system* sys = nullptr;
  int rc = ks_create_system(&d, ws, jb->ws_bytes, st, &sys);
  // replayed trial graphs cut the launch overhead that dominates small systems
  if (rc == KS_OK) (void)ks_enable_graphs(sys, 1);
  if (rc == KS_OK) rc = ks_minimize(sys, X, &jb->rq.params, &c->result);
  // a run stopped by the iteration cap still returns its last iterate
  if ((rc == KS_OK || rc == KS_E_NOT_CONVERGED) && jb->rq.X_out) {
    e = hipMemcpyAsync(jb->rq.X_out, X, jb->x_bytes, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) rc = KS_E_HIP;
  }
  ks_destroy_system(sys);
  if (hipStreamSynchronize(st) != hipSuccess && rc == KS_OK) rc = KS_E_HIP;
  c->status = rc;
}

void worker(ks_server* sv) {
  hipStream_t st = nullptr;
  const bool ok = hipSetDevice(sv->device) == hipSuccess &&
                  hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
  for (;;) {
    Job* jb = nullptr;
    size_t off = 0;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      sv->cv_work.wait(lk, [&] {
        if (sv->stop) return true;
        if (sv->queue.empty()) return false;
        Job* h = sv->queue.front();
        return sv->take(align_up(h->ws_bytes) + align_up(h->x_bytes), &off);
      });
      if (sv->stop) break;
      jb = sv->queue.front();
      sv->queue.pop_front();
      ++sv->running;
    }
    // the next queued request may fit as well
    sv->cv_work.notify_all();
    ks_completion c{};
    c.id = jb->rq.id;
    c.t_submit = jb->t_submit;
    c.t_admit = sv->now();
    c.bytes = align_up(jb->ws_bytes) + align_up(jb->x_bytes);
    if (ok) run_job(sv, jb, off, st, &c);
    else c.status = KS_E_HIP;
    c.t_done = sv->now();
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      sv->give(off, c.bytes);
      sv->done.push_back(c);
      --sv->running;
    }
    delete jb;
    sv->cv_work.notify_all();
    sv->cv_idle.notify_all();
  }
  if (st) (void)hipStreamDestroy(st);
}

// Whether the lockstep runner takes the request (its limits are in include/ks.h).
bool batch_ok(const ks_request& rq) {
  const ks_system_desc& d = rq.desc;
  return d.disc == KS_DISC_FD7 && d.hartree_solver == KS_HARTREE_PCG_FD &&
         (d.terms & KS_TERM_HARTREE) && d.p <= 32 && rq.params.retraction == KS_QR &&
         (d.precision == KS_PREC_FP64 || d.precision == KS_PREC_FP32);
}

struct Resident {
  Job* jb;
  size_t off;
  ks_system* sys;
  char* X;
  ks_completion c;
};

void finish_resident(ks_server* sv, Resident* rs, int code, const ks_result& r,
                     hipStream_t st) {
  rs->c.status = code;
  rs->c.result = r;
  if ((code == KS_OK || code == KS_E_NOT_CONVERGED) && rs->jb->rq.X_out) {
    hipError_t e = hipMemcpyAsync(rs->jb->rq.X_out, rs->X, rs->jb->x_bytes,
                                  hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) rs->c.status = KS_E_HIP;
  }
  ks_destroy_system(rs->sys);
  rs->c.t_done = sv->now();
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->give(rs->off, rs->c.bytes);
    sv->done.push_back(rs->c);
    --sv->running;
  }
  delete rs->jb;
  delete rs;
  sv->cv_idle.notify_all();
}

void batch_worker(ks_server* sv) {
  hipStream_t st = nullptr;
  const bool ok = hipSetDevice(sv->device) == hipSuccess &&
                  hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
  ks::BatchEngine* eng = ok ? ks::batch_create(st) : nullptr;
  for (;;) {
    std::vector<std::pair<Job*, size_t>> admit;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      auto fill = [&] {
        size_t off = 0;
        while (!sv->queue.empty() &&
               (eng ? ks::batch_size(eng) : 0) + (int)admit.size() < sv->max_batch) {
          Job* h = sv->queue.front();
          if (!sv->take(align_up(h->ws_bytes) + align_up(h->x_bytes), &off)) break;
          sv->queue.pop_front();
          ++sv->running;
          admit.emplace_back(h, off);
        }
      };
      fill();
      if (admit.empty() && (!eng || ks::batch_size(eng) == 0)) {
        sv->cv_work.wait(lk, [&] {
          if (sv->stop) return true;
          fill();
          return !admit.empty();
        });
        if (sv->stop && admit.empty()) break;
      }
    }
    for (auto& a : admit) {
      Resident* rs = new Resident{a.first, a.second, nullptr, nullptr, ks_completion{}};
      Job* jb = a.first;
      rs->c.id = jb->rq.id;
      rs->c.t_submit = jb->t_submit;
      rs->c.t_admit = sv->now();
      rs->c.bytes = align_up(jb->ws_bytes) + align_up(jb->x_bytes);
      char* ws = sv->base + a.second;
      rs->X = ws + align_up(jb->ws_bytes);
      ks_result r{};
      int rc = ok ? KS_OK : KS_E_HIP;
      if (rc == KS_OK &&
          hipMemcpyAsync(rs->X, jb->X0.data(), jb->x_bytes, hipMemcpyHostToDevice, st) !=
              hipSuccess)
        rc = KS_E_HIP;
      if (rc == KS_OK) rc = ks_create_system(&jb->rq.desc, ws, jb->ws_bytes, st, &rs->sys);
      if (rc == KS_OK && batch_ok(jb->rq)) {
        ks::batch_add(eng, rs->sys, rs->X, &jb->rq.params, rs);
        continue;  // batch_add parks failures and instant stops in the finished list
      }
      // not for the lockstep runner: run it alone here
      if (rc == KS_OK) rc = ks_minimize(rs->sys, rs->X, &jb->rq.params, &r);
      finish_resident(sv, rs, rc, r, st);
    }
    if (eng && ks::batch_size(eng) > 0) ks::batch_tick(eng);
    void* tag = nullptr;
    ks_result r{};
    int code = KS_OK;
    while (eng && ks::batch_take(eng, &tag, &r, &code))
      finish_resident(sv, static_cast<Resident*>(tag), code, r, st);
    sv->cv_work.notify_all();
  }
  // stop: finish what is resident so every admitted request completes
  while (eng && ks::batch_size(eng) > 0) {
    ks::batch_tick(eng);
    void* tag = nullptr;
    ks_result r{};
    int code = KS_OK;
    while (ks::batch_take(eng, &tag, &r, &code))
      finish_resident(sv, static_cast<Resident*>(tag), code, r, st);
  }
  ks::batch_destroy(eng);
  if (st) (void)hipStreamDestroy(st);
}

}  // namespace

extern "C" {

int ks_server_create(void* dev_workspace, size_t ws_bytes, int n_slots, ks_server** out) {
  if (!out) return KS_E_INVAL;
  *out = nullptr;
  if (!dev_workspace || ws_bytes == 0 || n_slots < 1 || n_slots > 64) return KS_E_INVAL;
  if (reinterpret_cast<uintptr_t>(dev_workspace) % kAlign != 0) return KS_E_INVAL;
  if (!ks::device_range(dev_workspace, ws_bytes)) return KS_E_INVAL;
  ks_server* sv = new ks_server();
  if (hipGetDevice(&sv->device) != hipSuccess) {
    delete sv;
    return KS_E_HIP;
  }
  sv->base = static_cast<char*>(dev_workspace);
  sv->bytes = ws_bytes / kAlign * kAlign;
  sv->free_list.push_back(Region{0, sv->bytes});
  sv->t0 = std::chrono::steady_clock::now();
  for (int i = 0; i < n_slots; ++i) sv->workers.emplace_back(worker, sv);
  *out = sv;
  return KS_OK;
}

int ks_server_create_batched(void* dev_workspace, size_t ws_bytes, int max_batch,
                             ks_server** out) {
  if (!out) return KS_E_INVAL;
  *out = nullptr;
  if (!dev_workspace || ws_bytes == 0 || max_batch < 1 || max_batch > ks::kMaxBatch)
    return KS_E_INVAL;
  if (reinterpret_cast<uintptr_t>(dev_workspace) % kAlign != 0) return KS_E_INVAL;
  if (!ks::device_range(dev_workspace, ws_bytes)) return KS_E_INVAL;
  ks_server* sv = new ks_server();
  if (hipGetDevice(&sv->device) != hipSuccess) {
    delete sv;
    return KS_E_HIP;
  }
  sv->base = static_cast<char*>(dev_workspace);
  sv->bytes = ws_bytes / kAlign * kAlign;
  sv->free_list.push_back(Region{0, sv->bytes});
  sv->t0 = std::chrono::steady_clock::now();
  sv->max_batch = max_batch;
  sv->workers.emplace_back(batch_worker, sv);
  *out = sv;
  return KS_OK;
}

int ks_server_submit(ks_server* sv, const ks_request* rq) {
  if (!sv || !rq || !rq->X0) return KS_E_INVAL;
  // orbital blocks of a request are dense (ld = p) on the host and on the device
  ks_system_desc d = rq->desc;
  d.ld = 0;
  const size_t ws = ks_workspace_bytes(&d);
  if (ws == 0) return KS_E_INVAL;  // the descriptor failed validation
  Job* jb = new Job();
  jb->rq = *rq;
  jb->rq.desc.ld = 0;
  const size_t n = (size_t)d.nx * d.ny * d.nz;
  const size_t es = d.precision == KS_PREC_FP32 ? 4 : 8;
  jb->ws_bytes = ws;
  jb->x_bytes = n * (size_t)d.p * es;
  jb->X0.assign(static_cast<const unsigned char*>(rq->X0),
                static_cast<const unsigned char*>(rq->X0) + n * (size_t)d.p * es);
  jb->rq.X0 = nullptr;
  if (d.n_nuclei > 0) {
    jb->R.assign(d.R, d.R + 3 * (size_t)d.n_nuclei);
    jb->Z.assign(d.Z, d.Z + d.n_nuclei);
    jb->rq.desc.R = jb->R.data();
    jb->rq.desc.Z = jb->Z.data();
  }
  if (d.v_ext_override) {
    jb->vext.assign(d.v_ext_override, d.v_ext_override + n);
    jb->rq.desc.v_ext_override = jb->vext.data();
  }
  std::lock_guard<std::mutex> lk(sv->mu);
  jb->t_submit = sv->now();
  if (align_up(jb->ws_bytes) + align_up(jb->x_bytes) > sv->bytes) {
    ks_completion c{};
    c.id = rq->id;
    c.status = KS_E_NOMEM;
    c.t_submit = c.t_admit = c.t_done = jb->t_submit;
    c.bytes = align_up(jb->ws_bytes) + align_up(jb->x_bytes);
    sv->done.push_back(c);
    delete jb;
    sv->cv_idle.notify_all();
    return KS_OK;
  }
  sv->queue.push_back(jb);
  sv->cv_work.notify_all();
  return KS_OK;
}

int ks_server_poll(ks_server* sv, ks_completion* out, int max, int* n_out) {
  if (!sv || !n_out || max < 0 || (max > 0 && !out)) return KS_E_INVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  const int k = std::min<int>(max, (int)sv->done.size());
  std::copy(sv->done.begin(), sv->done.begin() + k, out);
  sv->done.erase(sv->done.begin(), sv->done.begin() + k);
  *n_out = k;
  return KS_OK;
}

int ks_server_wait_idle(ks_server* sv) {
  if (!sv) return KS_E_INVAL;
  std::unique_lock<std::mutex> lk(sv->mu);
  sv->cv_idle.wait(lk, [&] { return sv->queue.empty() && sv->running == 0; });
  return KS_OK;
}

int ks_server_pending(ks_server* sv) {
  if (!sv) return 0;
  std::lock_guard<std::mutex> lk(sv->mu);
  return (int)sv->queue.size() + sv->running;
}

void ks_server_destroy(ks_server* sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
    for (Job* j : sv->queue) delete j;
    sv->queue.clear();
  }
  sv->cv_work.notify_all();
  for (auto& t : sv->workers) t.join();
  delete sv;
}

}  // extern "C"
