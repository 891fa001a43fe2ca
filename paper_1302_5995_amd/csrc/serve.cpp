// Serving layer of the DtN library: resident operators, continuous batching of
// applies per operator (the solve stage of Section 1.1 run as a service), builds
// interleaved on their own thread and stream, and admission by HBM footprint.
//
// Threads of one server:
//   scheduler - forms batches (oldest pending request first, then every pending
//               request of the same operator in arrival order up to max_cols
//               columns) into a free pipeline slot, stages their columns into the
//               slot's pinned buffer and enqueues copy-in, split-K apply and
//               copy-out on the slot's stream;
//   completer - waits for the slots in launch order, copies each batch's columns
//               out to the requests and completes them;
//   builder   - runs queued builds when their footprint fits the budget;
//   copy pool - a few helper threads that split each batch's host copies (pageable
//               request memory <-> pinned staging) into pieces, so that staging
//               keeps up with the device: one core copies far slower than the
//               device applies.
// kSlots slots on kSlots streams let the staging of one batch, the device work of
// the batches after it and the completion of the ones before it all overlap.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <atomic>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <set>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/dtn.h"
#include "kernels.h"
#include "runtime.h"

using namespace dtn;

namespace {

long long clock_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Req {
  long long ticket = 0, seq = 0;
  int kind = 0;                      // 0: apply, 1: build
  int op_id = -1;
  int k = 0;
  const double* G = nullptr;
  double* Y = nullptr;
  dtn_build_desc desc{};
  int status = DTN_OK;
  bool done = false;
  int batch_cols = 0;
  long long t_arrival = 0, t_start = 0, t_done = 0;
};

struct OpEntry {
  dtn_op* op = nullptr;
  bool owned = false;                // built by the server (freed on removal)
  bool live = false;
  size_t charge = 0;                 // bytes charged for the operator itself
  std::deque<Req*> pending;
  int inflight = 0;                  // requests of this operator inside a running batch
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  double* hG = nullptr;              // pinned host staging
  double* hY = nullptr;
  double* dG = nullptr;              // device staging
  double* dY = nullptr;
  double* part = nullptr;            // split-K partial sums
  int cap_nb = 0;                    // staging sized for nb <= cap_nb and max_cols columns
  std::vector<Req*> reqs;
  int op_id = -1, nb = 0, cols = 0;
  bool busy = false;                 // taken by the scheduler until the completer releases it
  int err = DTN_OK;
};

constexpr int kSlots = 4;
constexpr size_t kPieceBytes = 256 << 10;   // unit of work of the copy pool
constexpr int kMaxCopyThreads = 6;

struct Piece {
  void* dst;
  const void* src;
  size_t bytes;
};

// One set of host copies: the caller and the pool's helpers claim pieces from `next`.
struct CopyJob {
  std::vector<Piece> pieces;
  std::atomic<size_t> next{0};
  std::atomic<size_t> left{0};
  int users = 0;                     // helpers inside work_on (guarded by the pool's mutex)
  void add(void* dst, const void* src, size_t bytes) {
    for (size_t o = 0; o < bytes; o += kPieceBytes)
      pieces.push_back({(char*)dst + o, (const char*)src + o, std::min(kPieceBytes, bytes - o)});
  }
};

class CopyPool {
 public:
  void start() {
    const unsigned hc = std::thread::hardware_concurrency();
    const int n = std::min<int>(kMaxCopyThreads, hc > 2 ? (int)hc - 2 : 0);
    for (int t = 0; t < n; ++t) th_.emplace_back([this] { worker(); });
  }
  void stop() {
    {
      std::lock_guard<std::mutex> g(mu_);
      quit_ = true;
    }
    cv_job_.notify_all();
    for (std::thread& t : th_) t.join();
    th_.clear();
  }
  // Runs every piece of j; returns when all are copied and no helper touches j any more.
  void run(CopyJob& j) {
    j.next.store(0);
    j.left.store(j.pieces.size());
    j.users = 0;
    if (th_.empty() || j.pieces.size() < 2) {
      for (const Piece& p : j.pieces) std::memcpy(p.dst, p.src, p.bytes);
      return;
    }
    {
      std::lock_guard<std::mutex> g(mu_);
      jobs_.push_back(&j);
    }
    cv_job_.notify_all();
    work_on(j);
    std::unique_lock<std::mutex> lk(mu_);
    cv_done_.wait(lk, [&] { return j.left.load() == 0; });
    auto it = std::find(jobs_.begin(), jobs_.end(), &j);
    if (it != jobs_.end()) jobs_.erase(it);
    cv_done_.wait(lk, [&] { return j.users == 0; });
  }

 private:
  void work_on(CopyJob& j) {
    for (;;) {
      const size_t i = j.next.fetch_add(1);
      if (i >= j.pieces.size()) return;
      std::memcpy(j.pieces[i].dst, j.pieces[i].src, j.pieces[i].bytes);
      if (j.left.fetch_sub(1) == 1) {
        std::lock_guard<std::mutex> g(mu_);
        cv_done_.notify_all();
      }
    }
  }
  void worker() {
    for (;;) {
      CopyJob* j = nullptr;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_job_.wait(lk, [&] { return quit_ || !jobs_.empty(); });
        if (jobs_.empty()) return;   // quit_ and nothing left
        j = jobs_.front();
        if (j->next.load() >= j->pieces.size()) {   // every piece claimed: retire it from the queue
          jobs_.pop_front();
          continue;
        }
        j->users++;
      }
      work_on(*j);
      {
        std::lock_guard<std::mutex> g(mu_);
        j->users--;
      }
      cv_done_.notify_all();
    }
  }
  std::mutex mu_;
  std::condition_variable cv_job_, cv_done_;
  std::deque<CopyJob*> jobs_;
  std::vector<std::thread> th_;
  bool quit_ = false;
};

}  // namespace

struct dtn_srv {
  int device = 0;
  size_t budget = 0;
  int max_cols = 0;
  std::mutex mu;
  std::condition_variable cv_work;   // scheduler and builder
  std::condition_variable cv_done;   // waiters
  long long next_ticket = 0, next_seq = 0;
  std::map<long long, Req*> tickets;
  std::vector<OpEntry> ops;
  std::deque<Req*> builds;
  size_t charged = 0;                // operators + plan workspaces + staging
  size_t plans_charge = 0;           // build plans' workspaces (cached for the process lifetime)
  size_t staging_charge = 0;
  int staging_nb = 0;                // staging charged for operators up to this nb
  std::set<std::string> plans_charged;   // plan-cache keys whose workspaces are charged
  long long pending_applies = 0;
  bool stop = false;
  Slot slots[kSlots];
  std::deque<int> launched;          // slots in launch order, waiting for the completer
  bool sched_done = false;
  std::condition_variable cv_launched;
  hipStream_t build_stream = nullptr;
  std::thread sched, completer, builder;
  CopyPool pool;
  // statistics of completed applies since the last reset
  std::vector<double> lat_ms;
  std::vector<double> build_lat_ms;    // arrival to resident, completed builds
  long long applies_done = 0, builds_done = 0, solves = 0, batches = 0, refused = 0;
  double batch_cols_sum = 0.0;
  long long first_arrival = LLONG_MAX, last_done = 0;
};

namespace {

// Device bytes the pipeline slots need for operators with nb rows.
size_t staging_bytes(int nb, int max_cols) {
  return kSlots * (2 * (size_t)nb * max_cols * sizeof(double) + apply_splitk_workspace(nb, max_cols));
}

// Charge needed to make an operator of size nb resident (operator + staging growth).
size_t op_need(const dtn_srv* S, int nb, size_t op_bytes, size_t* new_staging) {
  const size_t st = std::max(S->staging_charge, staging_bytes(nb, S->max_cols));
  if (new_staging) *new_staging = st;
  return op_bytes + (st - S->staging_charge);
}

void slot_free(int dev, Slot& sl) {
  if (sl.hG) (void)hipHostFree(sl.hG);
  if (sl.hY) (void)hipHostFree(sl.hY);
  dev_release(dev, sl.dG);
  dev_release(dev, sl.dY);
  dev_release(dev, sl.part);
  sl.hG = sl.hY = sl.dG = sl.dY = sl.part = nullptr;
  sl.cap_nb = 0;
}

int slot_reserve(int dev, Slot& sl, int nb, int max_cols) {
  if (nb <= sl.cap_nb) return DTN_OK;
  slot_free(dev, sl);
  const size_t bytes = (size_t)nb * max_cols * sizeof(double);
  if (hipHostMalloc((void**)&sl.hG, bytes, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&sl.hY, bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    slot_free(dev, sl);
    return DTN_ENOMEM;
  }
  sl.dG = (double*)dev_alloc(dev, bytes);
  sl.dY = (double*)dev_alloc(dev, bytes);
  sl.part = (double*)dev_alloc(dev, apply_splitk_workspace(nb, max_cols));
  if (!sl.dG || !sl.dY || !sl.part) {
    slot_free(dev, sl);
    return DTN_ENOMEM;
  }
  sl.cap_nb = nb;
  return DTN_OK;
}

void finish_locked(dtn_srv* S, Req* r, int status) {
  r->status = status;
  r->done = true;
  r->t_done = clock_ns();
}

// Stage one batch into its slot and enqueue its device work (no lock held; the slot's
// requests are owned by it).
int slot_launch(dtn_srv* S, Slot& sl, const dtn_op* op, int cap_nb) {
  int rc = slot_reserve(S->device, sl, std::max(op->nb, cap_nb), S->max_cols);
  if (rc != DTN_OK) return rc;
  const int nb = op->nb;
  CopyJob job;
  size_t off = 0;
  for (Req* r : sl.reqs) {
    job.add(sl.hG + off, r->G, (size_t)nb * r->k * sizeof(double));
    off += (size_t)nb * r->k;
  }
  S->pool.run(job);
  const size_t bytes = off * sizeof(double);
  if (hipMemcpyAsync(sl.dG, sl.hG, bytes, hipMemcpyHostToDevice, sl.stream) != hipSuccess) return DTN_EDEVICE;
  if (op->T) {
    if (launch_apply_splitk(op->T, nb, sl.dG, nb, sl.cols, sl.dY, nb, sl.part, sl.stream, S->max_cols) != hipSuccess)
      return DTN_EDEVICE;
  } else {
    // an operator kept as HBS factors only: the telescoping apply (handle workspace, ordered across slots)
    const int rc2 = hbs_apply_handle(const_cast<dtn_op*>(op), sl.dG, nb, sl.cols, sl.dY, nb, sl.stream);
    if (rc2 != DTN_OK) return rc2;
  }
  if (hipMemcpyAsync(sl.hY, sl.dY, bytes, hipMemcpyDeviceToHost, sl.stream) != hipSuccess) return DTN_EDEVICE;
  if (hipEventRecord(sl.ev, sl.stream) != hipSuccess) return DTN_EDEVICE;
  return DTN_OK;
}

// Wait for a slot's batch, copy its columns out and complete its requests.
void slot_complete(dtn_srv* S, Slot& sl) {
  int rc = sl.err;
  if (rc == DTN_OK && hipEventSynchronize(sl.ev) != hipSuccess) rc = DTN_EDEVICE;
  if (rc == DTN_OK) {
    CopyJob job;
    size_t off = 0;
    for (Req* r : sl.reqs) {
      job.add(r->Y, sl.hY + off, (size_t)sl.nb * r->k * sizeof(double));
      off += (size_t)sl.nb * r->k;
    }
    S->pool.run(job);
  }
  {
    std::lock_guard<std::mutex> g(S->mu);
    for (Req* r : sl.reqs) {
      finish_locked(S, r, rc);
      if (rc == DTN_OK) {
        S->lat_ms.push_back((r->t_done - r->t_arrival) * 1e-6);
        S->applies_done++;
        S->solves += r->k;
        S->first_arrival = std::min(S->first_arrival, r->t_arrival);
        S->last_done = std::max(S->last_done, r->t_done);
      }
    }
    if (rc == DTN_OK) {
      S->batches++;
      S->batch_cols_sum += sl.cols;
    }
    S->ops[sl.op_id].inflight -= (int)sl.reqs.size();
    sl.reqs.clear();
    sl.busy = false;
    sl.err = DTN_OK;
  }
  S->cv_done.notify_all();
  S->cv_work.notify_all();
}

int free_slot_locked(const dtn_srv* S) {
  for (int q = 0; q < kSlots; ++q)
    if (!S->slots[q].busy) return q;
  return -1;
}

void scheduler_main(dtn_srv* S) {
  (void)hipSetDevice(S->device);
  for (;;) {
    const dtn_op* op = nullptr;
    int cap_nb = 0, si = -1;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&] {
        return (S->pending_applies > 0 && free_slot_locked(S) >= 0) || (S->stop && S->pending_applies == 0);
      });
      if (S->pending_applies == 0) break;   // stop requested and every apply handed out
      si = free_slot_locked(S);
      Slot& sl = S->slots[si];
      // operator of the oldest pending request
      int best = -1;
      long long best_seq = LLONG_MAX;
      for (size_t q = 0; q < S->ops.size(); ++q) {
        const OpEntry& E = S->ops[q];
        if (E.live && !E.pending.empty() && E.pending.front()->seq < best_seq) {
          best_seq = E.pending.front()->seq;
          best = (int)q;
        }
      }
      OpEntry& E = S->ops[best];
      int cols = 0;
      const long long t_start = clock_ns();
      while (!E.pending.empty() && cols + E.pending.front()->k <= S->max_cols) {
        Req* r = E.pending.front();
        E.pending.pop_front();
        r->t_start = t_start;
        cols += r->k;
        sl.reqs.push_back(r);
      }
      for (Req* r : sl.reqs) r->batch_cols = cols;
      S->pending_applies -= (long long)sl.reqs.size();
      E.inflight += (int)sl.reqs.size();
      sl.op_id = best;
      sl.nb = E.op->nb;
      sl.cols = cols;
      sl.busy = true;
      op = E.op;
      cap_nb = S->staging_nb;
    }
    Slot& sl = S->slots[si];
    sl.err = slot_launch(S, sl, op, cap_nb);
    {
      std::lock_guard<std::mutex> g(S->mu);
      S->launched.push_back(si);
    }
    S->cv_launched.notify_one();
  }
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->sched_done = true;
  }
  S->cv_launched.notify_one();
}

void completer_main(dtn_srv* S) {
  (void)hipSetDevice(S->device);
  for (;;) {
    int si = -1;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_launched.wait(lk, [&] { return !S->launched.empty() || S->sched_done; });
      if (S->launched.empty()) return;
      si = S->launched.front();
      S->launched.pop_front();
    }
    slot_complete(S, S->slots[si]);
  }
}

void builder_main(dtn_srv* S) {
  (void)hipSetDevice(S->device);
  for (;;) {
    Req* r = nullptr;
    size_t need = 0, t_bytes = 0, new_staging = 0, plan_bytes = 0;
    bool plan_new = false;
    std::string key;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      for (;;) {
        if (!S->builds.empty()) {
          Req* h = S->builds.front();
          const int nb = 4 * (h->desc.n - 1);
          t_bytes = (size_t)nb * nb * sizeof(double);
          dtn_build_desc hd = h->desc;
          hd.device = S->device;
          key = plan_cache_key(S->device, hd);
          plan_new = !S->plans_charged.count(key);
          if (plan_new && plan_footprint(S->device, hd, plan_bytes) != DTN_OK) {
            S->builds.pop_front();
            finish_locked(S, h, DTN_EINVAL);
            S->refused++;
            S->cv_done.notify_all();
            continue;
          }
          need = op_need(S, nb, t_bytes, &new_staging) + (plan_new ? plan_bytes : 0);
          if (S->charged + need <= S->budget) {
            r = h;
            S->builds.pop_front();
            S->charged += need;
            S->staging_charge = new_staging;
            S->staging_nb = std::max(S->staging_nb, nb);
            if (plan_new) {
              S->plans_charged.insert(key);
              S->plans_charge += plan_bytes;
            }
            break;
          }
          if (S->stop) {   // cannot fit and nothing will be released any more
            S->builds.pop_front();
            finish_locked(S, h, DTN_EBUSY);
            S->refused++;
            S->cv_done.notify_all();
            continue;
          }
        } else if (S->stop) {
          return;
        }
        S->cv_work.wait(lk);
      }
      r->t_start = clock_ns();
    }
    dtn_build_desc D = r->desc;
    D.device = S->device;
    D.stream = S->build_stream;
    dtn_op* op = dtn_build_ex(&D);
    int rc = DTN_OK;
    if (!op) {
      const std::string& e = last_err();
      rc = e.find("singular") != std::string::npos     ? DTN_ESINGULAR
           : e.find("allocation") != std::string::npos ? DTN_ENOMEM
           : e.find("failed") != std::string::npos     ? DTN_EDEVICE
                                                       : DTN_EINVAL;
    }
    {
      std::lock_guard<std::mutex> g(S->mu);
      if (op) {
        OpEntry E;
        E.op = op;
        E.owned = true;
        E.live = true;
        E.charge = t_bytes;
        S->ops.push_back(E);
        r->op_id = (int)S->ops.size() - 1;
        S->builds_done++;
        S->build_lat_ms.push_back((clock_ns() - r->t_arrival) * 1e-6);
      } else {
        S->charged -= t_bytes;   // the plan stays cached (and charged)
      }
      finish_locked(S, r, rc);
    }
    S->cv_done.notify_all();
    S->cv_work.notify_all();
  }
}

long long submit_apply_at(dtn_srv* S, int op_id, const double* G, int k, double* Y, long long t_arrival) {
  if (!S || !G || !Y) { set_err("NULL argument"); return DTN_EINVAL; }
  if (k < 1 || k > S->max_cols) { set_err("k must be in [1, max_batch_cols]"); return DTN_EINVAL; }
  if (G == Y) { set_err("G and Y alias"); return DTN_EINVAL; }
  Req* r = new Req();
  r->kind = 0;
  r->op_id = op_id;
  r->k = k;
  r->G = G;
  r->Y = Y;
  r->t_arrival = t_arrival;
  {
    std::lock_guard<std::mutex> g(S->mu);
    if (S->stop) { delete r; set_err("server is shutting down"); return DTN_EBUSY; }
    if (op_id < 0 || op_id >= (int)S->ops.size() || !S->ops[op_id].live) {
      delete r;
      set_err("unknown operator id");
      return DTN_EINVAL;
    }
    r->ticket = S->next_ticket++;
    r->seq = S->next_seq++;
    S->tickets[r->ticket] = r;
    S->ops[op_id].pending.push_back(r);
    S->pending_applies++;
  }
  S->cv_work.notify_all();
  return r->ticket;
}

}  // namespace

extern "C" {

long long dtn_srv_now_ns(void) { return clock_ns(); }

dtn_srv* dtn_srv_create(size_t budget_bytes, int device, int max_batch_cols) {
  if (max_batch_cols < 1 || max_batch_cols > 4096) { set_err("max_batch_cols must be in [1, 4096]"); return nullptr; }
  if (device_ready(device) != DTN_OK) return nullptr;
  if (hipSetDevice(device) != hipSuccess) { set_err("hipSetDevice failed"); return nullptr; }
  dtn_srv* S = new dtn_srv();
  S->device = device;
  S->budget = budget_bytes;
  S->max_cols = max_batch_cols;
  bool ok = hipStreamCreateWithFlags(&S->build_stream, hipStreamNonBlocking) == hipSuccess;
  for (Slot& sl : S->slots) {
    ok = ok && hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) == hipSuccess;
  }
  if (!ok) {
    set_err("stream/event creation failed");
    for (Slot& sl : S->slots) {
      if (sl.stream) (void)hipStreamDestroy(sl.stream);
      if (sl.ev) (void)hipEventDestroy(sl.ev);
    }
    if (S->build_stream) (void)hipStreamDestroy(S->build_stream);
    delete S;
    return nullptr;
  }
  S->pool.start();
  S->sched = std::thread(scheduler_main, S);
  S->completer = std::thread(completer_main, S);
  S->builder = std::thread(builder_main, S);
  return S;
}

int dtn_srv_add_op(dtn_srv* S, dtn_op* op) {
  if (!S || !op) { set_err("NULL argument"); return DTN_EINVAL; }
  if (op->device != S->device) { set_err("operator lives on another device"); return DTN_EINVAL; }
  std::lock_guard<std::mutex> g(S->mu);
  // the handle's device memory: dense T and / or HBS factors (plus the HBS apply's workspace)
  const size_t t_bytes = (op->T ? (size_t)op->nb * op->nb * sizeof(double) : 0) + hbs_bytes(op) +
                         (op->T ? 0 : hbs_work_bytes(op->hbs, std::max(S->max_cols, 64)));
  size_t new_staging = 0;
  const size_t need = op_need(S, op->nb, t_bytes, &new_staging);
  if (S->charged + need > S->budget) {
    S->refused++;
    set_err("operator does not fit the remaining HBM budget");
    return DTN_EBUSY;
  }
  S->charged += need;
  S->staging_charge = new_staging;
  S->staging_nb = std::max(S->staging_nb, op->nb);
  OpEntry E;
  E.op = op;
  E.owned = false;
  E.live = true;
  E.charge = t_bytes;
  S->ops.push_back(E);
  return (int)S->ops.size() - 1;
}

int dtn_srv_remove_op(dtn_srv* S, int op_id) {
  if (!S) { set_err("NULL server"); return DTN_EINVAL; }
  dtn_op* to_free = nullptr;
  {
    std::lock_guard<std::mutex> g(S->mu);
    if (op_id < 0 || op_id >= (int)S->ops.size() || !S->ops[op_id].live) { set_err("unknown operator id"); return DTN_EINVAL; }
    OpEntry& E = S->ops[op_id];
    if (!E.pending.empty() || E.inflight > 0) { set_err("requests on this operator are pending"); return DTN_EBUSY; }
    E.live = false;
    S->charged -= E.charge;
    if (E.owned) to_free = E.op;
    E.op = nullptr;
  }
  if (to_free) dtn_free(to_free);
  S->cv_work.notify_all();
  return DTN_OK;
}

int dtn_srv_op_nb(dtn_srv* S, int op_id) {
  if (!S) { set_err("NULL server"); return DTN_EINVAL; }
  std::lock_guard<std::mutex> g(S->mu);
  if (op_id < 0 || op_id >= (int)S->ops.size() || !S->ops[op_id].live) { set_err("unknown operator id"); return DTN_EINVAL; }
  return S->ops[op_id].op->nb;
}

long long dtn_srv_submit_apply(dtn_srv* S, int op_id, const double* G, int k, double* Y) {
  return submit_apply_at(S, op_id, G, k, Y, clock_ns());
}

static long long submit_build_at(dtn_srv* S, const dtn_build_desc* desc, long long t_arrival);

long long dtn_srv_submit_build(dtn_srv* S, const dtn_build_desc* desc) {
  return submit_build_at(S, desc, clock_ns());
}

static long long submit_build_at(dtn_srv* S, const dtn_build_desc* desc, long long t_arrival) {
  if (!S || !desc) { set_err("NULL argument"); return DTN_EINVAL; }
  const dtn_build_desc& D = *desc;
  if (D.n < 3 || D.n > 65536 || D.leaf < 4) { set_err("bad n or leaf"); return DTN_EINVAL; }
  const int nb = 4 * (D.n - 1);
  size_t plan_bytes = 0;
  std::string key;
  dtn_build_desc Dd = D;
  Dd.device = S->device;
  key = plan_cache_key(S->device, Dd);
  if (plan_footprint(S->device, Dd, plan_bytes) != DTN_OK) return DTN_EINVAL;
  Req* r = new Req();
  r->kind = 1;
  r->desc = D;
  r->t_arrival = t_arrival;
  {
    std::lock_guard<std::mutex> g(S->mu);
    if (S->stop) { delete r; set_err("server is shutting down"); return DTN_EBUSY; }
    // never fits: even with every resident operator removed (plans and staging stay charged)
    const bool plan_new = !S->plans_charged.count(key);
    const size_t fixed = std::max(S->staging_charge, staging_bytes(nb, S->max_cols)) + S->plans_charge;
    const size_t need = (size_t)nb * nb * sizeof(double) + (plan_new ? plan_bytes : 0);
    if (fixed + need > S->budget) {
      delete r;
      S->refused++;
      set_err("build footprint exceeds the HBM budget");
      return DTN_EBUSY;
    }
    r->ticket = S->next_ticket++;
    r->seq = S->next_seq++;
    S->tickets[r->ticket] = r;
    S->builds.push_back(r);
  }
  S->cv_work.notify_all();
  return r->ticket;
}

int dtn_srv_poll(dtn_srv* S, long long ticket) {
  if (!S) { set_err("NULL server"); return DTN_EINVAL; }
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->tickets.find(ticket);
  if (it == S->tickets.end()) { set_err("unknown ticket"); return DTN_EINVAL; }
  return it->second->done ? 1 : 0;
}

int dtn_srv_wait(dtn_srv* S, long long ticket, dtn_srv_result* out) {
  if (!S) { set_err("NULL server"); return DTN_EINVAL; }
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->tickets.find(ticket);
  if (it == S->tickets.end()) { set_err("unknown ticket"); return DTN_EINVAL; }
  Req* r = it->second;
  S->cv_done.wait(lk, [&] { return r->done; });
  if (out) {
    out->status = r->status;
    out->op_id = r->op_id;
    out->k = r->k;
    out->batch_cols = r->batch_cols;
    out->t_arrival_ns = r->t_arrival;
    out->t_start_ns = r->t_start;
    out->t_done_ns = r->t_done;
  }
  const int st = r->status;
  S->tickets.erase(it);
  delete r;
  return st;
}

int dtn_srv_replay(dtn_srv* S, int count, const dtn_srv_request* reqs, long long* tickets) {
  if (!S || count < 0 || (count > 0 && (!reqs || !tickets))) { set_err("bad arguments"); return DTN_EINVAL; }
  const long long t0 = clock_ns();
  for (int q = 0; q < count; ++q) {
    const long long target = t0 + reqs[q].t_offset_ns;
    for (;;) {
      const long long now = clock_ns();
      if (now >= target) break;
      if (target - now > 200000) std::this_thread::sleep_for(std::chrono::nanoseconds(target - now - 100000));
    }
    const long long t = reqs[q].build ? submit_build_at(S, reqs[q].build, target)
                                      : submit_apply_at(S, reqs[q].op_id, reqs[q].G, reqs[q].k, reqs[q].Y, target);
    tickets[q] = t;
    if (t < 0) {
      for (int r = q + 1; r < count; ++r) tickets[r] = DTN_EINVAL;
      return (int)t;
    }
  }
  return DTN_OK;
}

int dtn_srv_stats_get(dtn_srv* S, dtn_srv_stats* out) {
  if (!S || !out) { set_err("NULL argument"); return DTN_EINVAL; }
  std::lock_guard<std::mutex> g(S->mu);
  std::memset(out, 0, sizeof(*out));
  out->applies_done = S->applies_done;
  out->builds_done = S->builds_done;
  out->solves_done = S->solves;
  out->batches = S->batches;
  out->refused = S->refused;
  out->budget_bytes = S->budget;
  out->resident_bytes = S->charged;
  for (const OpEntry& E : S->ops) out->resident_ops += E.live ? 1 : 0;
  if (!S->lat_ms.empty()) {
    std::vector<double> v = S->lat_ms;
    std::sort(v.begin(), v.end());
    const size_t m = v.size();
    out->p50_ms = v[(m - 1) / 2];
    out->p99_ms = v[std::min(m - 1, (size_t)std::ceil(0.99 * m) - 1)];
    double sum = 0.0;
    for (double x : v) sum += x;
    out->mean_ms = sum / m;
  }
  out->mean_batch_cols = S->batches ? S->batch_cols_sum / S->batches : 0.0;
  if (!S->build_lat_ms.empty()) {
    std::vector<double> v = S->build_lat_ms;
    std::sort(v.begin(), v.end());
    const size_t m = v.size();
    out->build_p50_ms = v[(m - 1) / 2];
    out->build_p99_ms = v[std::min(m - 1, (size_t)std::ceil(0.99 * m) - 1)];
  }
  if (S->applies_done > 0 && S->last_done > S->first_arrival) {
    out->span_s = (S->last_done - S->first_arrival) * 1e-9;
    out->solves_per_s = S->solves / out->span_s;
  }
  return DTN_OK;
}

int dtn_srv_stats_reset(dtn_srv* S) {
  if (!S) { set_err("NULL server"); return DTN_EINVAL; }
  std::lock_guard<std::mutex> g(S->mu);
  S->lat_ms.clear();
  S->build_lat_ms.clear();
  S->applies_done = S->builds_done = S->solves = S->batches = S->refused = 0;
  S->batch_cols_sum = 0.0;
  S->first_arrival = LLONG_MAX;
  S->last_done = 0;
  return DTN_OK;
}

void dtn_srv_destroy(dtn_srv* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  if (S->sched.joinable()) S->sched.join();
  if (S->completer.joinable()) S->completer.join();
  if (S->builder.joinable()) S->builder.join();
  S->pool.stop();
  (void)hipSetDevice(S->device);
  for (Slot& sl : S->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    slot_free(S->device, sl);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.ev) (void)hipEventDestroy(sl.ev);
  }
  if (S->build_stream) (void)hipStreamDestroy(S->build_stream);
  for (OpEntry& E : S->ops)
    if (E.live && E.owned) dtn_free(E.op);
  for (auto& kv : S->tickets) delete kv.second;
  delete S;
}

}  // extern "C"
