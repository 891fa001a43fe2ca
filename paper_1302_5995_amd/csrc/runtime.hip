// Runtime and C ABI of the DtN library: device contexts, a caching device
// allocator, the plan cache, execution of a plan (the build of Section 3.3)
// and the apply stage (Section 1.1, step 2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <tuple>
#include <vector>
#include <thread>
#include <unordered_map>

#include "../../include/dtn.h"
#include "kernels.h"
#include "plan.h"
#include "runtime.h"

namespace dtn {

static thread_local std::string g_err;
static thread_local int g_err_code = 0;   // code of the last failed build on this thread
void set_err(const std::string& s) { g_err = s; }
const std::string& last_err() { return g_err; }

#define HIPCHK(expr, code)                                                                  \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) {                                                                 \
      set_err(std::string(#expr) + " failed: " + hipGetErrorString(e_));                   \
      return code;                                                                          \
    }                                                                                       \
  } while (0)

// ---------------------------------------------------------------------------
// Caching device allocator: freed blocks are kept per exact (rounded) size and
// reused; on allocation failure the cache is released and the request retried.
// ---------------------------------------------------------------------------
class Pool {
 public:
  void* alloc(size_t bytes) {
    const size_t sz = round(bytes);
    std::lock_guard<std::mutex> g(mu_);
    auto it = free_.find(sz);
    if (it != free_.end()) {
      void* p = it->second;
      free_.erase(it);
      cached_ -= sz;
      used_[p] = sz;
      in_use_ += sz;
      return p;
    }
    void* p = nullptr;
    if (hipMalloc(&p, sz) != hipSuccess) {
      (void)hipGetLastError();
      release_cache_locked();
      if (hipMalloc(&p, sz) != hipSuccess) { (void)hipGetLastError(); return nullptr; }
    }
    used_[p] = sz;
    in_use_ += sz;
    return p;
  }
  void release(void* p) {
    if (!p) return;
    std::lock_guard<std::mutex> g(mu_);
    auto it = used_.find(p);
    if (it == used_.end()) return;
    free_.emplace(it->second, p);
    cached_ += it->second;
    in_use_ -= it->second;
    used_.erase(it);
  }
  size_t in_use() const { return in_use_; }

 private:
  static size_t round(size_t b) {
    const size_t g = b >= (1u << 20) ? (size_t)2 << 20 : 256;
    return (b + g - 1) / g * g;
  }
  void release_cache_locked() {
    for (auto& kv : free_) (void)hipFree(kv.second);
    free_.clear();
    cached_ = 0;
  }
  std::mutex mu_;
  std::multimap<size_t, void*> free_;
  std::map<void*, size_t> used_;
  size_t in_use_ = 0, cached_ = 0;
};

constexpr int kSideStreams = 4;   // streams of the concurrent structured merges of a phase

constexpr size_t kPinBytes = 32u << 20;   // pinned staging buffer of the host-buffer copies, per device

struct Device {
  bool ready = false;
  hipStream_t stream = nullptr;
  hipStream_t side[kSideStreams] = {};
  double* pin = nullptr;              // kPinBytes of pinned host memory (hipHostMalloc), on first use
  std::mutex pin_mu;
  double* noalloc_part = nullptr;   // this device's address of the allocation-free apply's partials
  Pool pool;
  std::mutex mu;
};

static Device g_dev[64];

int device_ready(int dev) {
  if (dev < 0 || dev >= 64) { set_err("device ordinal out of range"); return DTN_EINVAL; }
  Device& D = g_dev[dev];
  std::lock_guard<std::mutex> g(D.mu);
  if (D.ready) return DTN_OK;
  int count = 0;
  HIPCHK(hipGetDeviceCount(&count), DTN_EDEVICE);
  if (dev >= count) { set_err("no such HIP device"); return DTN_EDEVICE; }
  HIPCHK(hipSetDevice(dev), DTN_EDEVICE);
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, dev), DTN_EDEVICE);
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    set_err(std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950");
    return DTN_EDEVICE;
  }
  HIPCHK(kernels_init(), DTN_EDEVICE);
  if (const char* cache = std::getenv("DTN_TUNE_CACHE")) {
    // autotuned tiles of earlier runs on this architecture (a missing file is not an error)
    std::ifstream in(cache);
    if (in) {
      std::stringstream ss;
      ss << in.rdbuf();
      std::string err;
      if (!tune_load_json(ss.str(), "gfx950", err)) { set_err(err); return DTN_EINVAL; }
    }
  }
  HIPCHK(noalloc_scratch_address(&D.noalloc_part), DTN_EDEVICE);
  if (!D.noalloc_part) { set_err("no device address for the apply scratch array"); return DTN_EDEVICE; }
  HIPCHK(hipStreamCreateWithFlags(&D.stream, hipStreamNonBlocking), DTN_EDEVICE);
  for (hipStream_t& q : D.side) HIPCHK(hipStreamCreateWithFlags(&q, hipStreamNonBlocking), DTN_EDEVICE);
  D.ready = true;
  return DTN_OK;
}

// ---------------------------------------------------------------------------
// Kernel profiler: HIP events around every launch, accumulated per family.
// ---------------------------------------------------------------------------
struct ProfFamily {
  long long launches = 0;
  double ms = 0, flops = 0, bytes = 0;
};
static std::mutex g_prof_mu;
static bool g_prof_on = false;
static std::map<std::string, ProfFamily> g_prof;
static std::set<std::string> g_prof_only;   // families to record; empty: all
static std::vector<hipEvent_t> g_event_pool;

static hipEvent_t event_get() {
  {
    std::lock_guard<std::mutex> g(g_prof_mu);
    if (!g_event_pool.empty()) {
      hipEvent_t e = g_event_pool.back();
      g_event_pool.pop_back();
      return e;
    }
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

class Prof {
 public:
  struct Rec { hipEvent_t a, b; const char* fam; double flops, bytes; };
  Prof() {
    std::lock_guard<std::mutex> g(g_prof_mu);
    only_ = g_prof_only;
  }
  // Tuning runs: every launch recorded, times summed per family name into `sink` (not the global table).
  explicit Prof(std::map<std::string, double>* sink) : tune_sink(sink) {}
  std::map<std::string, double>* tune_sink = nullptr;
  // Launches of families outside the selection get an empty record (no events), which keeps
  // begin/end paired.
  void begin(const char* fam, double flops, double bytes, hipStream_t s) {
    const bool rec = only_.empty() || only_.count(fam) > 0;
    Rec r{rec ? event_get() : nullptr, rec ? event_get() : nullptr, fam, flops, bytes};
    if (r.a) (void)hipEventRecord(r.a, s);
    cur_.push_back(r);
  }
  void end(hipStream_t s) {
    if (!cur_.empty() && cur_.back().b) (void)hipEventRecord(cur_.back().b, s);
  }
  // Call after the stream has been synchronised.
  void collect() {
    std::lock_guard<std::mutex> g(g_prof_mu);
    for (auto& r : cur_) {
      float ms = 0.0f;
      if (r.a && r.b && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess && tune_sink) {
        (*tune_sink)[r.fam] += ms;
      } else if (r.a && r.b && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
        ProfFamily& f = g_prof[r.fam];
        f.launches++;
        f.ms += ms;
        f.flops += r.flops;
        f.bytes += r.bytes;
      }
      if (r.a) g_event_pool.push_back(r.a);
      if (r.b) g_event_pool.push_back(r.b);
    }
    cur_.clear();
  }
 private:
  std::vector<Rec> cur_;
  std::set<std::string> only_;
};

static bool prof_enabled() {
  std::lock_guard<std::mutex> g(g_prof_mu);
  return g_prof_on;
}

// Profiler family of a GEMM launch: the product's role plus the kernel instantiation that runs it
// (no suffix: 64 x 64 FP64 tiles; _t32: 32 x 32 FP64 tiles; _t128: 128 x 128 FP64 tiles; _f32: FP32
// MFMA of mixed-precision plans), so that each family maps to one kernel.
const char* gemm_family(const char* role, int cfg, int prec) {
  static std::mutex mu;
  static std::set<std::string> names;   // node-based: c_str() stays valid
  const char* suffix = prec == 1 ? "_f32" : cfg == 3 ? "_t32" : cfg == 4 ? "_t32k64" : cfg == 1 || cfg == 2 ? "_t128" : "";
  std::lock_guard<std::mutex> g(mu);
  return names.insert(std::string(role) + suffix).first->c_str();
}

// A stable C string for a name (kept for the process lifetime).
static const char* intern_name(const std::string& s) {
  static std::mutex mu;
  static std::set<std::string> names;
  std::lock_guard<std::mutex> g(mu);
  return names.insert(s).first->c_str();
}

#define PROF_BEGIN(pr, fam, fl, by, s) do { if (pr) (pr)->begin(fam, fl, by, s); } while (0)
#define PROF_END(pr, s) do { if (pr) (pr)->end(s); } while (0)

// ---------------------------------------------------------------------------
// Plans resident on a device.
// ---------------------------------------------------------------------------
struct DevPlan {
  Plan plan;
  int device = 0;
  SchurTask* d_tasks = nullptr;
  LargeMerge* d_large = nullptr;
  GemmDesc* d_gemms = nullptr;
  BaseBlock* d_bases = nullptr;
  CoupleDesc* d_couples = nullptr;
  PcholDesc* d_pchols = nullptr;
  int* d_ip = nullptr;
  double* aux = nullptr;
  double* ws = nullptr;
  double* lva = nullptr;
  double* lvb = nullptr;
  double* half = nullptr;
  double* coef = nullptr;
  DevStatus* status = nullptr;
  size_t bytes = 0;
  std::mutex run_mu;   // builds sharing this plan's workspace run one at a time
  ~DevPlan() {
    Pool& P = g_dev[device].pool;
    for (void* p : {(void*)d_tasks, (void*)d_large, (void*)d_gemms, (void*)d_bases, (void*)d_couples, (void*)d_pchols, (void*)d_ip,
                    (void*)aux, (void*)ws, (void*)lva, (void*)lvb, (void*)half, (void*)coef, (void*)status})
      P.release(p);
  }
};

static std::mutex g_plan_mu;
static std::map<std::string, std::shared_ptr<DevPlan>> g_plans;

static std::string plan_key(int dev, const std::vector<ProbSpec>& specs, bool fast, bool mixed = false,
                            double tol = 0.0, int hbs_level = -1, int tune_force = -1) {
  char tb[96];
  std::snprintf(tb, sizeof(tb), "T%.17g,%d,G%d,F%d", tol, hbs_level, tune_generation(), tune_force);
  std::string k = std::to_string(dev) + (fast ? "F" : "P") + (mixed ? "M" : "D") + tb;
  for (const ProbSpec& sp : specs)
    k += ":" + std::to_string(sp.n) + "," + std::to_string(sp.leaf) + "," + std::to_string(sp.conv) +
         (sp.sym ? (sp.definite ? "s+" : "s") : "") + (sp.net ? "n" : "");
  return k;
}

template <class T>
static int upload(Pool& P, T*& dst, const std::vector<T>& src, size_t& bytes) {
  const size_t b = std::max<size_t>(1, src.size()) * sizeof(T);
  dst = (T*)P.alloc(b);
  if (!dst) { set_err("device allocation failed (plan tables)"); return DTN_ENOMEM; }
  bytes += b;
  if (!src.empty()) HIPCHK(hipMemcpy(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice), DTN_EDEVICE);
  return DTN_OK;
}

static int get_plan(int dev, const std::vector<ProbSpec>& specs, bool fast, bool mixed, double tol, int hbs_level,
                    std::shared_ptr<DevPlan>& out, int tune_force = -1) {
  std::lock_guard<std::mutex> g(g_plan_mu);
  const std::string key = plan_key(dev, specs, fast, mixed, tol, hbs_level, tune_force);
  auto it = g_plans.find(key);
  if (it != g_plans.end()) { out = it->second; return DTN_OK; }
  auto dp = std::make_shared<DevPlan>();
  dp->device = dev;
  std::string err;
  if (!plan_make_many(specs, fast, dp->plan, err, mixed, tol, hbs_level, tune_force)) {
    set_err("plan: " + err);
    return DTN_EINVAL;
  }
  Plan& P = dp->plan;
  Pool& pool = g_dev[dev].pool;
  int rc;
  std::vector<int> ip = P.ipool;
  ip.resize(P.ipool.size() + P.int_ws + 1, 0);
  if ((rc = upload(pool, dp->d_tasks, P.tasks, dp->bytes)) != DTN_OK) return rc;
  if ((rc = upload(pool, dp->d_large, P.large, dp->bytes)) != DTN_OK) return rc;
  if ((rc = upload(pool, dp->d_gemms, P.gemms, dp->bytes)) != DTN_OK) return rc;
  if ((rc = upload(pool, dp->d_bases, P.bases, dp->bytes)) != DTN_OK) return rc;
  if ((rc = upload(pool, dp->d_couples, P.couples, dp->bytes)) != DTN_OK) return rc;
  if ((rc = upload(pool, dp->d_pchols, P.pchols, dp->bytes)) != DTN_OK) return rc;
  if ((rc = upload(pool, dp->d_ip, ip, dp->bytes)) != DTN_OK) return rc;
  if ((rc = upload(pool, dp->aux, P.aux, dp->bytes)) != DTN_OK) return rc;
  auto dalloc = [&](double*& p, size_t cnt) {
    p = (double*)pool.alloc(std::max<size_t>(cnt, 1) * 8);
    dp->bytes += cnt * 8;
    return p != nullptr;
  };
  if (!dalloc(dp->ws, P.ws_doubles) || !dalloc(dp->lva, P.lva_doubles) || !dalloc(dp->lvb, P.lvb_doubles) ||
      !dalloc(dp->half, P.half_doubles) || !dalloc(dp->coef, P.coef_doubles)) {
    set_err("device allocation failed (plan workspace)");
    return DTN_ENOMEM;
  }
  dp->status = (DevStatus*)pool.alloc(sizeof(DevStatus));
  if (!dp->status) { set_err("device allocation failed (status)"); return DTN_ENOMEM; }
  g_plans[key] = dp;
  out = dp;
  return DTN_OK;
}

void* dev_alloc(int dev, size_t bytes) { return g_dev[dev].pool.alloc(bytes); }

// Copies between caller host buffers and device memory go through the device's pinned staging buffer,
// a column chunk at a time (column-major rows x cols, leading dimensions in elements): the runtime never
// has to pin or stage pageable memory itself.  Synchronous on s.
static int host_copy(int dev, bool to_host, double* h, size_t ldh, double* d, size_t ldd, size_t rows, size_t cols,
                     hipStream_t s) {
  if (rows == 0 || cols == 0) return DTN_OK;
  Device& D = g_dev[dev];
  std::lock_guard<std::mutex> g(D.pin_mu);
  if (!D.pin) {
    if (hipHostMalloc((void**)&D.pin, kPinBytes, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      D.pin = nullptr;
      set_err("pinned staging allocation failed");
      return DTN_ENOMEM;
    }
  }
  const size_t per = std::max<size_t>(1, kPinBytes / (rows * sizeof(double)));
  if (rows * sizeof(double) > kPinBytes) { set_err("a column exceeds the staging buffer"); return DTN_EINVAL; }
  for (size_t c0 = 0; c0 < cols; c0 += per) {
    const size_t kc = std::min(per, cols - c0);
    if (to_host) {
      HIPCHK(hipMemcpy2DAsync(D.pin, rows * sizeof(double), d + c0 * ldd, ldd * sizeof(double), rows * sizeof(double), kc,
                              hipMemcpyDeviceToHost, s), DTN_EDEVICE);
      HIPCHK(hipStreamSynchronize(s), DTN_EDEVICE);
      for (size_t c = 0; c < kc; ++c) std::memcpy(h + (c0 + c) * ldh, D.pin + c * rows, rows * sizeof(double));
    } else {
      for (size_t c = 0; c < kc; ++c) std::memcpy(D.pin + c * rows, h + (c0 + c) * ldh, rows * sizeof(double));
      HIPCHK(hipMemcpy2DAsync(d + c0 * ldd, ldd * sizeof(double), D.pin, rows * sizeof(double), rows * sizeof(double), kc,
                              hipMemcpyHostToDevice, s), DTN_EDEVICE);
      HIPCHK(hipStreamSynchronize(s), DTN_EDEVICE);
    }
  }
  return DTN_OK;
}

void dev_release(int dev, void* p) { g_dev[dev].pool.release(p); }

// Device bytes get_plan allocates for plan P (tables, workspaces, status word).
static size_t plan_device_bytes(const Plan& P) {
  auto tab = [](size_t cnt, size_t sz) { return std::max<size_t>(1, cnt) * sz; };
  return tab(P.tasks.size(), sizeof(SchurTask)) + tab(P.large.size(), sizeof(LargeMerge)) +
         tab(P.gemms.size(), sizeof(GemmDesc)) + tab(P.bases.size(), sizeof(BaseBlock)) +
         tab(P.couples.size(), sizeof(CoupleDesc)) + tab(P.pchols.size(), sizeof(PcholDesc)) +
         tab(P.ipool.size() + P.int_ws + 1, sizeof(int)) + tab(P.aux.size(), sizeof(double)) +
         8 * (std::max<size_t>(P.ws_doubles, 1) + std::max<size_t>(P.lva_doubles, 1) +
              std::max<size_t>(P.lvb_doubles, 1) + std::max<size_t>(P.half_doubles, 1) +
              std::max<size_t>(P.coef_doubles, 1)) +
         sizeof(DevStatus);
}

static ProbSpec spec_of(const dtn_build_desc& D) {
  ProbSpec sp;
  sp.n = D.n; sp.leaf = D.leaf; sp.conv = D.conv;
  sp.net = D.coef_form == DTN_COEF_NETWORK;
  // symmetric operator: no convection, or a network (each link's conductance enters both its rows)
  sp.sym = (D.b == nullptr && D.c == nullptr) || sp.net;
  // nonneg: d >= 0 at every interior node (known on the host only; device fields count as unknown)
  sp.nonneg = 0;
  if (!D.d) {
    sp.nonneg = 1;
  } else if (D.coeff_mem == DTN_MEM_HOST) {
    bool ok = true;
    for (int j = 1; j + 1 < D.n && ok; ++j)
      for (int i = 1; i + 1 < D.n; ++i)
        if (!(D.d[i + (size_t)D.n * j] >= 0.0)) { ok = false; break; }
    sp.nonneg = ok ? 1 : 0;
  }
  sp.definite = sp.sym && sp.nonneg;
  return sp;
}

// DTN_MIXED runs FP32 products only on problems with d >= 0 everywhere: where d < 0 (Helmholtz) the
// interface blocks can be near-singular and the FP32 rounding of any level's products is amplified far
// beyond 1e-6 (on the 20-wavelength n = 1024 benchmark even the lowest large merges alone give 3e-5),
// so such builds run in FP64 and report it.
static bool mixed_effective(const dtn_build_desc* D, int count) {
  if (D[0].precision != DTN_MIXED) return false;
  for (int p = 0; p < count; ++p)
    if (!spec_of(D[p]).nonneg) return false;
  return true;
}

std::string plan_cache_key(int dev, const dtn_build_desc& D) {
  return plan_key(dev, {spec_of(D)}, D.pivoting == DTN_PIVOT_AUTO, mixed_effective(&D, 1), D.tol,
                  D.hbs_min_level);
}

int plan_footprint(int dev, const dtn_build_desc& D, size_t& bytes) {
  const ProbSpec sp = spec_of(D);
  const bool mixed = mixed_effective(&D, 1);
  const bool fast = D.pivoting == DTN_PIVOT_AUTO;
  bytes = 0;
  std::vector<bool> kinds{fast};
  if (fast) kinds.push_back(false);    // the partial-pivoting plan an unpivoted build falls back to
  for (const bool f : kinds) {
    {
      std::lock_guard<std::mutex> g(g_plan_mu);
      if (g_plans.count(plan_key(dev, {sp}, f, mixed, D.tol, D.hbs_min_level))) continue;
    }
    Plan P;
    std::string err;
    if (!plan_make_many({sp}, f, P, err, mixed, D.tol, D.hbs_min_level)) { set_err("plan: " + err); return DTN_EINVAL; }
    bytes += plan_device_bytes(P);
  }
  return DTN_OK;
}

// Enqueue the whole build of one plan on stream s.  fused: every launch covers all boxes of a
// phase (the batched form); plain: the same kernels with one box, merge or product per launch
// (the comparator form: no fusion across boxes).
// A captured level: after phase `phase`, `count` doubles from level buffer `buf` at `off` go to dst.
struct CapCopy {
  int phase, buf;
  long long off, count;
  double* dst;
};

// Interface order of a merge's K_ii for its HBS form: each P3 node (the first child's interface, in its
// ring order along the shared edge) followed by its five-point neighbour in P4.  In the plain order
// [P3; P4] the block coupling the two halves is a full-rank anti-diagonal, so no tree over that order
// has low-rank off-diagonal blocks; in the pair order every off-diagonal block is a block of S33 or S44
// between disjoint stretches of the edge plus at most one coupling entry.  False if some node of P3 or
// P4 has no partner (then the merge keeps the dense inverse).
static bool pair_order(const Plan& P, const SchurTask& t, std::vector<int>& src) {
  const int e = t.e, i = t.i, i1 = t.i1, i2 = i - i1;
  if (i1 != i2 || i1 <= 0) return false;
  const int* node = P.ipool.data() + t.idx + e + i;   // node codes (j << 16) | i of the local order
  std::unordered_map<int, int> at4;
  for (int c = 0; c < i2; ++c) at4[node[e + i1 + c]] = c;
  std::vector<char> used(i2, 0);
  src.clear();
  for (int r = 0; r < i1; ++r) {
    const int p = node[e + r], pi = p & 0xFFFF, pj = p >> 16;
    const int nb[4][2] = {{pi - 1, pj}, {pi + 1, pj}, {pi, pj - 1}, {pi, pj + 1}};
    int hit = -1;
    for (const auto& d : nb) {
      if (d[0] < 0 || d[1] < 0) continue;
      const auto it = at4.find((d[1] << 16) | d[0]);
      if (it != at4.end() && !used[it->second]) { hit = it->second; break; }
    }
    if (hit < 0) return false;
    used[hit] = 1;
    src.push_back(r);
    src.push_back(i1 + hit);
  }
  return true;
}

// Section 6, Step 1 for one dense merge: K_ii (gathered at m.inv) in the pair order, in equal-rank HBS
// form at local tolerance tol, inverted by Algorithm 1, and X = K_ii^{-1} diag(S31, S42) formed by
// Algorithm 2 into m.x (the dense path's X), in place of the recursive block inverse and the X products.
constexpr int kStructuredLeaf = 64;   // HBS leaf size of an interface block

static int structured_x(const DevPlan& dp, const LargeMerge& m, double tol, hipStream_t s) {
  const SchurTask& t = m.t;
  std::vector<int> src;
  if (!pair_order(dp.plan, t, src)) { set_err("structured merge: interface nodes do not pair up"); return DTN_EINVAL; }
  return hbs_perm_solve(dp.device, dp.ws + m.inv, t.i, src, dp.ws + m.b31, t.i1, t.e1, dp.ws + m.b42, t.e - t.e1,
                        tol, kStructuredLeaf, dp.ws + m.x, t.i, s);
}

// The interface solves of a structured phase: the merges are independent, so they run concurrently,
// one host thread and one side stream each (at most kSideStreams at once), after the work already on s
// (the gathers of K_ii, S31, S42); each solve ends synchronised, so s continues once all have returned.
static int structured_phase_x(const DevPlan& dp, const Phase& ph, double kii_tol, hipStream_t s) {
  Device& D = g_dev[dp.device];
  const int nlm = ph.large_count, nt = std::min(nlm, kSideStreams);
  HIPCHK(hipStreamSynchronize(s), DTN_EDEVICE);
  std::vector<int> rcs(nlm, DTN_OK);
  std::vector<std::string> errs(nlm);
  auto work = [&](int w) {
    if (hipSetDevice(dp.device) != hipSuccess) {
      rcs[w] = DTN_EDEVICE;
      errs[w] = "hipSetDevice failed (structured merge)";
      return;
    }
    for (int q = w; q < nlm; q += nt) {
      rcs[q] = structured_x(dp, dp.plan.large[ph.large_first + q], kii_tol, D.side[w]);
      if (rcs[q] != DTN_OK) { errs[q] = last_err(); return; }
    }
  };
  std::vector<std::thread> pool;
  for (int w = 1; w < nt; ++w) pool.emplace_back(work, w);
  work(0);
  for (auto& th : pool) th.join();
  for (int q = 0; q < nlm; ++q)
    if (rcs[q] != DTN_OK) {
      set_err(errs[q]);
      return rcs[q];
    }
  return DTN_OK;
}

// Merges of a fast, dense phase whose K_ii is inverted in HBS form (kii_tol > 0): those the
// compression rule selects (hbs_min_level >= 0: levels <= it; else both children's rings >= 1000),
// when every merge of the phase has a paired interface.
static bool structured_phase(const Plan& P, const Phase& ph, double kii_tol, int kii_level) {
  if (!(kii_tol > 0.0) || !P.fast || P.mixed || ph.compressed || ph.large_count == 0) return false;
  std::vector<int> src;
  for (int q = 0; q < ph.large_count; ++q) {
    const SchurTask& t = P.large[ph.large_first + q].t;
    if (kii_level < 0 && std::min(t.m1, t.m2) < kCompMinChild) return false;
    if (!pair_order(P, t, src)) return false;
  }
  return kii_level < 0 || ph.min_level <= kii_level;
}

// Body loads of one build (Section 7.3): the right-hand-side updates planned for the plan the build runs
// on, and their device buffers (released with the object, after the build's stream has drained).
struct BodyDev {
  int dev = 0;
  BodyPlan plan;
  double* buf = nullptr;       // BUF_BODY: every box's condensed right-hand sides
  double* scr = nullptr;       // BUF_BSCR: one phase's scratch
  BodyJob* d_jobs = nullptr;
  HbsGj* d_gjs = nullptr;
  GemmDesc* d_gemms = nullptr;
  int* d_nodes = nullptr;      // sorted node codes, then the caller's index of each
  double h2 = 0.0;
  ~BodyDev() {
    for (void* p : {(void*)buf, (void*)scr, (void*)d_jobs, (void*)d_gjs, (void*)d_gemms, (void*)d_nodes})
      if (p) dev_release(dev, p);
  }
};

static int body_setup(int dev, const Plan& P, const dtn_build_desc& D, hipStream_t s, std::unique_ptr<BodyDev>& out) {
  auto B = std::make_unique<BodyDev>();
  B->dev = dev;
  std::vector<int> codes(D.n_body);
  for (int q = 0; q < D.n_body; ++q) {
    const int k = D.body_nodes[q];
    if (k < 0 || k >= D.n * D.n) { set_err("body loads: node index out of the grid"); return DTN_EINVAL; }
    codes[q] = ((k / D.n) << 16) | (k % D.n);
  }
  std::string err;
  if (!body_plan_make(P, codes, gj_block_class, B->plan, err) || !body_plan_check(P, B->plan, err)) {
    set_err(err);
    return DTN_EINVAL;
  }
  const BodyPlan& bp = B->plan;
  auto get = [&](size_t bytes) { return dev_alloc(dev, std::max<size_t>(bytes, 256)); };
  B->buf = (double*)get(bp.body_doubles * sizeof(double));
  B->scr = (double*)get(std::max<size_t>(bp.scr_doubles, 1) * sizeof(double));
  B->d_jobs = (BodyJob*)get(std::max<size_t>(bp.jobs.size(), 1) * sizeof(BodyJob));
  B->d_gjs = (HbsGj*)get(std::max<size_t>(bp.gjs.size(), 1) * sizeof(HbsGj));
  B->d_gemms = (GemmDesc*)get(std::max<size_t>(bp.gemms.size(), 1) * sizeof(GemmDesc));
  B->d_nodes = (int*)get(2 * (size_t)std::max(bp.count, 1) * sizeof(int));
  if (!B->buf || !B->scr || !B->d_jobs || !B->d_gjs || !B->d_gemms || !B->d_nodes) {
    set_err("device allocation failed (body loads)");
    return DTN_ENOMEM;
  }
  std::vector<int> ints(bp.nodes);
  ints.insert(ints.end(), bp.user.begin(), bp.user.end());
  auto up = [&](void* d, const void* h, size_t bytes) {
    return bytes == 0 || hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, s) == hipSuccess;
  };
  if (!up(B->d_jobs, bp.jobs.data(), bp.jobs.size() * sizeof(BodyJob)) ||
      !up(B->d_gjs, bp.gjs.data(), bp.gjs.size() * sizeof(HbsGj)) ||
      !up(B->d_gemms, bp.gemms.data(), bp.gemms.size() * sizeof(GemmDesc)) ||
      !up(B->d_nodes, ints.data(), ints.size() * sizeof(int)) || hipStreamSynchronize(s) != hipSuccess) {
    set_err("body loads: upload failed");
    return DTN_EDEVICE;
  }
  const double h = 1.0 / (D.n - 1);
  B->h2 = h * h;
  out = std::move(B);
  return DTN_OK;
}

// The right-hand-side updates of phase q (after the phase's own merges, while its children's S and its
// interface inverses are still in place).
static int body_phase(const DevPlan& dp, const BodyDev& bd, size_t q, const DevBufs& B, hipStream_t s) {
  const BodyPhase& ph = bd.plan.phases[q];
  if (ph.job_count <= 0) return DTN_OK;
  const int chunks = (int)std::min<long long>(256, std::max<long long>(1, ph.elems_max / 4096));
  HIPCHK(launch_body_gather(bd.d_jobs + ph.job_first, ph.job_count, chunks, dp.d_ip, bd.d_nodes, B, bd.h2, s),
         DTN_EDEVICE);
  for (size_t g = 0; g < ph.gj_first.size(); ++g)
    HIPCHK(launch_gj_blocks(bd.d_gjs + ph.gj_first[g], ph.gj_count[g], ph.gj_cls[g], bd.scr, dp.status, s), DTN_EDEVICE);
  if (ph.zg_count > 0)
    HIPCHK(launch_gemm_batched(bd.d_gemms + ph.zg_first, ph.zg_count, ph.zg_tiles, 0, B, dp.d_ip, s, 0, 0, ph.zg_mode),
           DTN_EDEVICE);
  if (ph.ug_count > 0)
    HIPCHK(launch_gemm_batched(bd.d_gemms + ph.ug_first, ph.ug_count, ph.ug_tiles, 0, B, dp.d_ip, s, 0, 0, 0),
           DTN_EDEVICE);
  return DTN_OK;
}

static int run_plan(DevPlan& dp, double* const* T, hipStream_t s, std::vector<hipEvent_t>* marks, Prof* pr,
                    bool plain, const int* ring_rows, const std::vector<CapCopy>* caps = nullptr,
                    double kii_tol = 0.0, int kii_level = -1, int* structured = nullptr,
                    const BodyDev* body = nullptr) {
  const Plan& P = dp.plan;
  DevBufs B{};
  if (body) {
    B.p[BUF_BODY] = body->buf;
    B.p[BUF_BSCR] = body->scr;
  }
  B.p[BUF_WS] = dp.ws;
  B.p[BUF_LVA] = dp.lva;
  B.p[BUF_LVB] = dp.lvb;
  B.p[BUF_HALF] = dp.half;
  B.p[BUF_OUT] = T[0];
  B.p[BUF_COEF] = dp.coef;
  B.p[BUF_AUX] = dp.aux;
  auto gemm = [&](const char* role, const LaunchGemm& G) -> int {
    if (G.count <= 0) return DTN_OK;
    const char* fam = !pr ? role
                      : pr->tune_sink ? intern_name("T|" + G.sig + "|" + std::to_string(G.cfg))
                                      : gemm_family(role, G.cfg, G.prec);
    if (!plain) {
      PROF_BEGIN(pr, fam, G.flops, G.bytes, s);
      HIPCHK(launch_gemm_batched(dp.d_gemms + G.first, G.count, G.tiles, G.cfg, B, dp.d_ip, s, 0, G.prec, G.mode,
                                 dp.d_large),
             DTN_EDEVICE);
      PROF_END(pr, s);
      return DTN_OK;
    }
    for (int k = 0; k < G.count; ++k) {
      const GemmDesc& g = P.gemms[G.first + k];
      const double M = g.M, N = g.N, K = g.K;
      PROF_BEGIN(pr, fam, 2.0 * M * N * K, 8.0 * (M * K + K * N + (g.beta != 0.0 ? 2.0 : 1.0) * M * N), s);
      const int dt = g.tri ? g.tiles_m * (g.tiles_m + 1) / 2 : g.tiles_m * g.tiles_n;
      HIPCHK(launch_gemm_batched(dp.d_gemms + G.first, G.count, dt * std::max(1, g.ksplit), G.cfg,
                                 B, dp.d_ip, s, g.tile_start, G.prec, G.mode, dp.d_large),
             DTN_EDEVICE);
      PROF_END(pr, s);
    }
    return DTN_OK;
  };
  HIPCHK(launch_reset(nullptr, 0, B, dp.status, s), DTN_EDEVICE);
  for (size_t q = 0; q < P.phases.size(); ++q) {
    const Phase& ph = P.phases[q];
    if (ph.small_count > 0) {
      const int nl = plain ? ph.small_count : 1;
      for (int u = 0; u < nl; ++u) {
        const SchurTask* tk = dp.d_tasks + ph.small_first + (plain ? u : 0);
        const int cnt = plain ? 1 : ph.small_count;
        int imax = ph.small_imax, cols = ph.small_threads;
        size_t lds = ph.small_lds;
        double fl = ph.small_flops, by = ph.small_bytes;
        if (plain) {
          const SchurTask& t = P.tasks[ph.small_first + u];
          const double e = t.e, i = t.i;
          imax = t.i;
          cols = t.i + t.e;
          lds = P.fast ? ((size_t)t.i * t.e + 64) * 8 : (size_t)t.i * (t.i + t.e) * 8;
          fl = t.kind == 1 ? 2.0 / 3.0 * i * i * i + 2.0 * i * i * e + e * e * i : 0.0;
          by = 8.0 * ((i + e) * (i + e) + e * e);
        }
        PROF_BEGIN(pr, "small_schur", fl, by, s);
        if (P.fast)
          HIPCHK(launch_small_fast(tk, cnt, ph.kind == PH_BASE, imax, cols, lds, dp.d_ip, B, dp.status, s),
                 DTN_EDEVICE);
        else
          HIPCHK(launch_small(tk, cnt, lds, dp.d_ip, B, dp.status, s), DTN_EDEVICE);
        PROF_END(pr, s);
      }
    }
    if (ph.large_count > 0) {
      const int nlm_all = ph.large_count;
      const long long elems = (long long)ph.imax * ph.imax + 2LL * ph.imax * ph.emax + (long long)ph.emax * ph.emax;
      const int bper = (int)std::min<long long>(1024, std::max<long long>(1, elems / 4096));
      for (int u = 0; u < (plain ? nlm_all : 1); ++u) {
        const LargeMerge* lm = dp.d_large + ph.large_first + (plain ? u : 0);
        const int nlm = plain ? 1 : nlm_all;
        HIPCHK(launch_reset(lm, nlm, B, nullptr, s), DTN_EDEVICE);
        PROF_BEGIN(pr, "large_gather", 0.0, ph.gather_bytes / (plain ? nlm_all : 1), s);
        HIPCHK(launch_large_gather(lm, nlm, bper, dp.d_ip, B, s), DTN_EDEVICE);
        PROF_END(pr, s);
      }
      const bool sx = structured_phase(P, ph, kii_tol, kii_level);
      for (const InvOp& op : ph.inv_ops) {
        if (sx) break;   // K_ii inverted in HBS form below
        if (op.base_first >= 0) {
          for (int u = 0; u < (plain ? op.base_count : 1); ++u) {
            const int cnt = plain ? 1 : op.base_count;
            // algorithmic work of a diagonal block: its LU factorisation, 2/3 bs^3 flops (the merge
            // model's cost of eliminating it; the explicit inverse formed here does three times that),
            // the block read once and written once
            double bytes = 0.0, flops = 0.0;
            for (int q = 0; q < cnt; ++q) {
              const double b = P.bases[op.base_first + (plain ? u : 0) + q].bs;
              bytes += 16.0 * b * b;
              flops += 2.0 / 3.0 * b * b * b;
            }
            PROF_BEGIN(pr, "base_inv", flops, bytes, s);
            HIPCHK(launch_base_inv(dp.d_bases + op.base_first + (plain ? u : 0), cnt, B, dp.status, s), DTN_EDEVICE);
            PROF_END(pr, s);
          }
        } else if (op.couple_first >= 0) {
          for (int u = 0; u < (plain ? op.couple_count : 1); ++u) {
            const int cnt = plain ? 1 : op.couple_count, c0 = op.couple_first + (plain ? u : 0);
            long long most = 0;
            double bytes = 0.0, flops = 0.0;
            for (int q = 0; q < cnt; ++q) {
              const CoupleDesc& c = P.couples[c0 + q];
              const double h1 = c.h1, h2 = c.h2;
              most = std::max(most, 2LL * c.h1 * c.h2 + (long long)c.h2 * c.h2);
              bytes += 8.0 * (4.0 * h1 * h2 + 3.0 * h2 * h2);   // X11 columns and rows read, Wb, Wc written, A22 updated
              flops += 2.0 * h1 * h2 + 3.0 * h2 * h2;
            }
            const int bper = (int)std::min<long long>(1024, std::max<long long>(1, most / 2048));
            PROF_BEGIN(pr, "couple", flops, bytes, s);
            HIPCHK(launch_couple(dp.d_couples + c0, cnt, bper, dp.d_ip, B, s), DTN_EDEVICE);
            PROF_END(pr, s);
          }
        } else {
          int rc = gemm("gemm_inv", op.gemm);
          if (rc != DTN_OK) return rc;
        }
      }
      const double W = ph.gje_w;
      for (size_t k = 0; k < ph.gje_update.size(); ++k) {
        const int c0 = (int)k * ph.gje_w;
        for (int u = 0; u < (plain ? nlm_all : 1); ++u) {
          const LargeMerge* lm = dp.d_large + ph.large_first + (plain ? u : 0);
          const int nlm = plain ? 1 : nlm_all;
          PROF_BEGIN(pr, "gje_panel", 2.0 * nlm * ph.imax * W * W, 16.0 * nlm * ph.imax * W, s);
          HIPCHK(launch_gje_panel(ph.gje_nt, ph.gje_r, ph.gje_w, lm, nlm, c0, dp.d_ip, B, dp.status, s), DTN_EDEVICE);
          PROF_END(pr, s);
          PROF_BEGIN(pr, "gje_swap", 0.0, 24.0 * nlm * ph.imax * W, s);
          HIPCHK(launch_gje_swap(lm, nlm, ph.imax, c0, dp.d_ip, B, s), DTN_EDEVICE);
          PROF_END(pr, s);
        }
        int rc = gemm("gemm_update", ph.gje_update[k]);
        if (rc != DTN_OK) return rc;
      }
      if (!P.fast) {
        for (int u = 0; u < (plain ? nlm_all : 1); ++u)
          HIPCHK(launch_gje_kmap(dp.d_large + ph.large_first + (plain ? u : 0), plain ? 1 : nlm_all, ph.imax, dp.d_ip, s),
                 DTN_EDEVICE);
      }
      for (const CompOp& op : ph.comp_ops) {
        if (op.pchol_first >= 0) {
          PROF_BEGIN(pr, "pchol", 0.0, 0.0, s);
          HIPCHK(launch_pchol(dp.d_pchols + op.pchol_first, op.pchol_count, B, dp.d_ip, dp.status, s), DTN_EDEVICE);
          PROF_END(pr, s);
        } else {
          int rc = gemm("gemm_comp", op.gemm);
          if (rc != DTN_OK) return rc;
        }
      }
      int rc = DTN_OK;
      if (sx) {
        PROF_BEGIN(pr, "hbs_kii", 0.0, 0.0, s);
        rc = structured_phase_x(dp, ph, kii_tol, s);
        if (rc != DTN_OK) return rc;
        PROF_END(pr, s);
        if (structured) *structured += ph.large_count;
      } else {
        rc = gemm("gemm_x", ph.xgemm);
        if (rc != DTN_OK) return rc;
      }
      rc = gemm("gemm_schur", ph.sgemm);
      if (rc != DTN_OK) return rc;
      rc = gemm("gemm_schur", ph.sgemm_tri);
      if (rc != DTN_OK) return rc;
    }
    if (body) {
      PROF_BEGIN(pr, "body", 0.0, 0.0, s);
      const int rcb = body_phase(dp, *body, q, B, s);
      if (rcb != DTN_OK) return rcb;
      PROF_END(pr, s);
    }
    if (caps)
      for (const CapCopy& c : *caps)
        if (c.phase == (int)q)
          HIPCHK(hipMemcpyAsync(c.dst, (c.buf == BUF_LVA ? dp.lva : dp.lvb) + c.off, (size_t)c.count * sizeof(double),
                                hipMemcpyDeviceToDevice, s), DTN_EDEVICE);
    if (marks) HIPCHK(hipEventRecord((*marks)[q], s), DTN_EDEVICE);
  }
  for (size_t p = 0; p < P.probs.size(); ++p) {
    const ProbPlan& pp = P.probs[p];
    const double* root = (pp.root_buf == BUF_LVA ? dp.lva : dp.lvb) + pp.root_off;
    PROF_BEGIN(pr, "scale_copy", 0.0, 16.0 * pp.nb * (double)pp.nb, s);
    const int rr = ring_rows ? ring_rows[p] : DTN_RING_R1;
    if (rr == DTN_RING_R1) {
      HIPCHK(launch_scale_copy(root, T[p], (long long)pp.nb * pp.nb, (double)(pp.n - 1), s), DTN_EDEVICE);
    } else {
      const double h = 1.0 / (pp.n - 1);
      HIPCHK(launch_root_rows(root, T[p], pp.n, rr, dp.coef + pp.coef_off, h * h, pp.conv == DTN_CONV_PAPER ? h : 0.5 * h,
                              s), DTN_EDEVICE);
    }
    PROF_END(pr, s);
  }
  return DTN_OK;
}

int hbs_apply_handle(dtn_op* op, const double* X, int ldx, int k, double* Y, int ldy, hipStream_t s, bool inverse) {
  const HbsRep* H = inverse ? op->hbsi : op->hbs;
  if (!H) {
    set_err(inverse ? "the handle has no inverse HBS factors (dtn_hbs_invert)" : "the handle has no HBS factors");
    return DTN_EINVAL;
  }
  std::lock_guard<std::mutex> g(op->part_mu);
  Device& dev = g_dev[op->device];
  if (!op->hbs_ev) HIPCHK(hipEventCreateWithFlags(&op->hbs_ev, hipEventDisableTiming), DTN_EDEVICE);
  if (op->hbs_ev_recorded) HIPCHK(hipStreamWaitEvent(s, op->hbs_ev, 0), DTN_EDEVICE);
  if (hbs_work_bytes(H, k) > op->hbs_work_cap) {
    // grow the workspace once earlier applies using it have finished
    if (op->hbs_ev_recorded) HIPCHK(hipEventSynchronize(op->hbs_ev), DTN_EDEVICE);
    if (op->hbs_work) dev.pool.release(op->hbs_work);
    const size_t bytes = hbs_work_bytes(H, std::max(k, 64));
    op->hbs_work = (double*)dev.pool.alloc(bytes);
    op->hbs_work_cap = op->hbs_work ? bytes : 0;
    if (!op->hbs_work) { set_err("device allocation failed (HBS apply workspace)"); return DTN_ENOMEM; }
  }
  HIPCHK(hbs_apply(H, X, ldx, k, Y, ldy, op->hbs_work, s), DTN_EDEVICE);
  HIPCHK(hipEventRecord(op->hbs_ev, s), DTN_EDEVICE);
  op->hbs_ev_recorded = true;
  return DTN_OK;
}

}  // namespace dtn

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
using namespace dtn;


extern "C" {

const char* dtn_version(void) { return "dtn-gfx950 0.1"; }

const char* dtn_last_error(void) { return g_err.c_str(); }

void dtn_build_desc_init(dtn_build_desc* d) {
  if (!d) return;
  std::memset(d, 0, sizeof(*d));
  d->n = 0;
  d->coeff_mem = DTN_MEM_HOST;
  d->leaf = 32;
  d->tol = 0.0;
  d->hbs_min_level = -1;
  d->precision = DTN_FP64;
  d->batching = DTN_FUSED;
  d->conv = DTN_CONV_CENTRAL;
  d->device = 0;
  d->stream = nullptr;
  d->pivoting = DTN_PIVOT_AUTO;
  d->ring_rows = DTN_RING_R1;
  d->coef_form = DTN_COEF_PDE;
  d->capture_level = -1;
  d->budget_bytes = 0;
}

static bool finite_host(const double* x, size_t cnt) {
  for (size_t q = 0; q < cnt; ++q)
    if (!std::isfinite(x[q])) return false;
  return true;
}

// One execution of a plan over `count` problems: coefficients in, operators T[p] out, device
// status read back.  All descriptors share the device, stream, batching and precision of D[0].
// Level capture of problem p of plan P into op (capture_level >= 0): the box layout and, once, the
// device buffer; the copy to issue after the phase that completes the level.
static int setup_capture(const Plan& P, int p, int level, dtn_op* op, std::vector<CapCopy>& caps) {
  const ProbPlan& pp = P.probs[p];
  if (level > pp.Lr) {
    set_err("capture_level " + std::to_string(level) + " is deeper than the dissection (" + std::to_string(pp.Lr) + ")");
    return DTN_EINVAL;
  }
  std::vector<std::vector<Rect>> boxes;
  quadtree_levels(pp.n, pp.Lr, boxes);
  op->cap_rects.clear();
  op->cap_offs.clear();
  long long total = 0;
  for (const Rect& b : boxes[level]) {
    op->cap_rects.insert(op->cap_rects.end(), {b.x0, b.x1, b.y0, b.y1});
    op->cap_offs.push_back(total);
    total += (long long)b.ring() * b.ring();
  }
  if (!op->cap) {
    op->cap = (double*)g_dev[op->device].pool.alloc(std::max<long long>(total, 1) * sizeof(double));
    if (!op->cap) { set_err("device allocation failed (captured level)"); return DTN_ENOMEM; }
  }
  const bool even = level % 2 == 0;
  caps.push_back({level == pp.Lr ? 0 : 2 * (pp.Lr - level), even ? BUF_LVA : BUF_LVB,
                  even ? pp.lva_base : pp.lvb_base, total, op->cap});
  return DTN_OK;
}

static long long capture_doubles(int n, int leaf, int level) {
  const int Lr = std::max(user_depth(n, leaf), user_depth(n, kBaseSide));
  if (level < 0 || level > Lr) return 0;
  std::vector<std::vector<Rect>> boxes;
  quadtree_levels(n, Lr, boxes);
  long long total = 0;
  for (const Rect& b : boxes[level]) total += (long long)b.ring() * b.ring();
  return total;
}

static int build_into(const dtn_build_desc* D, int count, bool fast, double* const* T, DevStatus& hs,
                      dtn_stats* st, int tune_force = -1, Prof* tune_prof = nullptr, dtn_op* const* ops = nullptr) {
  std::vector<ProbSpec> specs(count);
  for (int p = 0; p < count; ++p) {
    specs[p] = spec_of(D[p]);
  }
  std::shared_ptr<DevPlan> dp;
  const bool mixed = mixed_effective(D, count);
  int rc = get_plan(D[0].device, specs, fast, mixed, D[0].tol, D[0].hbs_min_level, dp, tune_force);
  if (rc != DTN_OK) return rc;
  Device& dev = g_dev[D[0].device];
  hipStream_t s = D[0].stream ? (hipStream_t)D[0].stream : dev.stream;
  std::lock_guard<std::mutex> g(dp->run_mu);
  const Plan& P = dp->plan;
  for (int p = 0; p < count; ++p) {
    const size_t nn = (size_t)D[p].n * D[p].n;
    const hipMemcpyKind kind = D[p].coeff_mem == DTN_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    const double* fields[3] = {D[p].b, D[p].c, D[p].d};
    for (int f = 0; f < 3; ++f) {
      double* dst = dp->coef + P.probs[p].coef_off + f * nn;
      if (fields[f]) HIPCHK(hipMemcpyAsync(dst, fields[f], nn * sizeof(double), kind, s), DTN_EDEVICE);
      else HIPCHK(hipMemsetAsync(dst, 0, nn * sizeof(double), s), DTN_EDEVICE);
    }
  }
  std::vector<hipEvent_t> marks(P.phases.size() + 1, nullptr);
  struct EvGuard {
    std::vector<hipEvent_t>& v;
    ~EvGuard() { for (auto& e : v) if (e) (void)hipEventDestroy(e); }
  } guard{marks};
  for (auto& e : marks) HIPCHK(hipEventCreate(&e), DTN_EDEVICE);
  HIPCHK(hipEventRecord(marks.back(), s), DTN_EDEVICE);
  const auto t0 = std::chrono::steady_clock::now();
  std::unique_ptr<Prof> own(prof_enabled() && !tune_prof ? new Prof() : nullptr);
  Prof* prof_p = tune_prof ? tune_prof : own.get();
  std::vector<int> rows(count);
  for (int p = 0; p < count; ++p) rows[p] = D[p].ring_rows;
  std::vector<CapCopy> caps;
  if (ops)
    for (int p = 0; p < count; ++p)
      if (D[p].capture_level >= 0 && ops[p]) {
        rc = setup_capture(P, p, D[p].capture_level, ops[p], caps);
        if (rc != DTN_OK) return rc;
      }
  std::unique_ptr<BodyDev> body;
  if (ops && ops[0] && D[0].n_body > 0) {
    rc = body_setup(D[0].device, P, D[0], s, body);
    if (rc != DTN_OK) return rc;
    if (!ops[0]->body) {
      ops[0]->body = (double*)dev.pool.alloc((size_t)P.probs[0].nb * D[0].n_body * sizeof(double));
      if (!ops[0]->body) { set_err("device allocation failed (body operator)"); return DTN_ENOMEM; }
    }
    ops[0]->body_count = D[0].n_body;
  }
  int structured = 0;
  rc = run_plan(*dp, T, s, &marks, prof_p, D[0].batching == DTN_PLAIN, rows.data(), caps.empty() ? nullptr : &caps,
                D[0].kii_tol, D[0].hbs_min_level, &structured, body.get());
  if (rc == DTN_OK && body) {
    const int nb = P.probs[0].nb;
    rc = launch_body_out(body->buf + body->plan.root_off, nb, body->plan.count, body->d_nodes + body->plan.count,
                         -(double)(D[0].n - 1), ops[0]->body, nb, s) == hipSuccess ? DTN_OK : DTN_EDEVICE;
    if (rc != DTN_OK) set_err("body loads: output failed");
  }
  if (rc != DTN_OK) {
    (void)hipStreamSynchronize(s);
    if (prof_p) prof_p->collect();
    return rc;
  }
  HIPCHK(hipMemcpyAsync(&hs, dp->status, sizeof(hs), hipMemcpyDeviceToHost, s), DTN_EDEVICE);
  HIPCHK(hipStreamSynchronize(s), DTN_EDEVICE);
  const auto t1 = std::chrono::steady_clock::now();
  // ranks of the compressed blocks (first + residual pass), largest per level
  std::vector<int> level_rank(32, 0);
  if (!P.rank_slots.empty()) {
    std::vector<int> iw(P.int_ws + 1);
    HIPCHK(hipMemcpy(iw.data(), dp->d_ip + P.ipool.size(), iw.size() * sizeof(int), hipMemcpyDeviceToHost),
           DTN_EDEVICE);
    const int ib = (int)P.ipool.size();
    for (const RankSlot& r : P.rank_slots)
      if (r.level >= 0 && r.level < 32)
        level_rank[r.level] = std::max(level_rank[r.level], iw[r.first - ib] + iw[r.second - ib]);
  }
  if (prof_p) prof_p->collect();
  double ratio, growth;
  std::memcpy(&ratio, &hs.min_ratio_bits, sizeof(double));
  std::memcpy(&growth, &hs.max_growth_bits, sizeof(double));
  const double build_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  for (int p = 0; p < count; ++p) {
    const ProbPlan& pp = P.probs[p];
    dtn_stats& o = st[p];
    o = dtn_stats{};
    o.n = pp.n;
    o.nb = pp.nb;
    o.leaf = pp.leaf;
    o.levels = pp.L;
    o.precision = mixed ? DTN_MIXED : DTN_FP64;   // the precision that ran
    o.batching = D[p].batching;
    o.build_ms = build_ms;           // of the whole (possibly multi-problem) build
    o.flops = pp.model_flops;
    for (int l = 0; l <= pp.L && l < 32; ++l) o.level_flops[l] = pp.level_model_flops[l];
    for (int l = 0; l < 32; ++l) o.max_rank[l] = count == 1 ? level_rank[l] : 0;
    if (count == 1) {
      float prev_ms = 0.0f;
      for (size_t q = 0; q < P.phases.size(); ++q) {
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, marks.back(), marks[q]);
        const int lvl = std::min(P.phases[q].level, pp.L);
        if (lvl >= 0 && lvl < 32) o.level_ms[lvl] += ms - prev_ms;
        prev_ms = ms;
      }
    }
    o.min_pivot_ratio = ratio;
    o.max_growth = growth;
    o.pivoting_used = fast ? DTN_PIVOT_AUTO : DTN_PIVOT_PARTIAL;
    o.peak_workspace_bytes = dp->bytes;
    o.structured_merges = structured;
  }
  return DTN_OK;
}

static bool validate_desc(const dtn_build_desc& D) {
  if (D.n < 3 || D.n > 65536) { set_err("n must be in [3, 65536]"); return false; }
  if (D.leaf < 4) { set_err("leaf must be >= 4"); return false; }
  if (!(D.tol >= 0.0) || !std::isfinite(D.tol)) { set_err("tol must be finite and >= 0"); return false; }
  if (D.conv != DTN_CONV_CENTRAL && D.conv != DTN_CONV_PAPER) { set_err("bad conv"); return false; }
  if (D.coeff_mem != DTN_MEM_HOST && D.coeff_mem != DTN_MEM_DEVICE) { set_err("bad coeff_mem"); return false; }
  if (D.precision != DTN_FP64 && D.precision != DTN_MIXED) { set_err("bad precision"); return false; }
  if (D.batching != DTN_FUSED && D.batching != DTN_PLAIN) { set_err("bad batching"); return false; }
  if (D.pivoting != DTN_PIVOT_AUTO && D.pivoting != DTN_PIVOT_PARTIAL) { set_err("bad pivoting"); return false; }
  if (D.ring_rows != DTN_RING_R1 && D.ring_rows != DTN_RING_R2 && D.ring_rows != DTN_RING_R3) {
    set_err("bad ring_rows");
    return false;
  }
  if (D.coef_form != DTN_COEF_PDE && D.coef_form != DTN_COEF_NETWORK) { set_err("bad coef_form"); return false; }
  if (D.capture_level < -1) { set_err("capture_level must be -1 or a quadtree level >= 0"); return false; }
  if (!(D.kii_tol >= 0.0) || !std::isfinite(D.kii_tol)) { set_err("kii_tol must be finite and >= 0"); return false; }
  if (D.n_body < 0 || (D.n_body > 0 && !D.body_nodes)) { set_err("n_body must be >= 0, with body_nodes"); return false; }
  if (D.n_body > 0 && (D.tol > 0.0 || D.kii_tol > 0.0 || D.ring_rows != DTN_RING_R1)) {
    set_err("body loads need tol = 0, kii_tol = 0 and the R1 ring rows");
    return false;
  }
  if (D.kii_tol > 0.0 && (D.tol > 0.0 || D.precision != DTN_FP64)) {
    set_err("kii_tol (HBS inverse of K_ii) runs on dense FP64 merges only: tol must be 0 and precision DTN_FP64");
    return false;
  }
  if (D.coef_form == DTN_COEF_NETWORK) {
    if (!D.b || !D.c) { set_err("the network form needs both conductance fields (b: east links, c: north links)"); return false; }
    if (D.ring_rows == DTN_RING_R2) { set_err("DTN_RING_R2 is defined for the PDE form only"); return false; }
  }
  const size_t nn = (size_t)D.n * D.n;
  if (D.coeff_mem == DTN_MEM_HOST) {
    for (const double* f : {D.b, D.c, D.d})
      if (f && !finite_host(f, nn)) { set_err("coefficient array holds NaN or Inf"); return false; }
  }
  return true;
}

// Build `count` problems in one plan (shared launches); out[p] receives the handles.
static int build_group(const dtn_build_desc* descs, int count, dtn_op** out) {
  for (int p = 0; p < count; ++p) out[p] = nullptr;
  const int device = descs[0].device;
  if (device_ready(device) != DTN_OK) return DTN_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) { set_err("hipSetDevice failed"); return DTN_EDEVICE; }
  Device& dev = g_dev[device];
  std::vector<std::unique_ptr<dtn_op>> ops(count);
  std::vector<double*> T(count, nullptr);
  auto release_all = [&]() {
    for (int p = 0; p < count; ++p) {
      if (ops[p] && ops[p]->T) { dev.pool.release(ops[p]->T); ops[p]->T = nullptr; }
      if (ops[p] && ops[p]->cap) { dev.pool.release(ops[p]->cap); ops[p]->cap = nullptr; }
      if (ops[p] && ops[p]->body) { dev.pool.release(ops[p]->body); ops[p]->body = nullptr; }
    }
  };
  if (descs[0].budget_bytes > 0) {
    // everything the build may allocate, before allocating any of it
    size_t need = 0;
    for (int p = 0; p < count; ++p) {
      size_t pb = 0;
      const int rc = plan_footprint(device, descs[p], pb);
      if (rc != DTN_OK) return rc;
      const size_t nb = 4 * (size_t)(descs[p].n - 1);
      need += pb + nb * nb * sizeof(double) +
              (size_t)capture_doubles(descs[p].n, descs[p].leaf, descs[p].capture_level) * sizeof(double);
    }
    if (need > descs[0].budget_bytes) {
      set_err("the build needs " + std::to_string(need) + " device bytes, over its budget of " +
              std::to_string(descs[0].budget_bytes));
      return DTN_ENOMEM;
    }
  }
  for (int p = 0; p < count; ++p) {
    ops[p] = std::make_unique<dtn_op>();
    ops[p]->device = device;
    ops[p]->n = descs[p].n;
    ops[p]->nb = 4 * (descs[p].n - 1);
    ops[p]->leaf = descs[p].leaf;
    const size_t tbytes = (size_t)ops[p]->nb * ops[p]->nb * sizeof(double);
    ops[p]->T = (double*)dev.pool.alloc(tbytes);
    if (!ops[p]->T) { release_all(); set_err("device allocation failed (operator)"); return DTN_ENOMEM; }
    T[p] = ops[p]->T;
  }
  std::vector<dtn_stats> st(count);
  DevStatus hs{};
  const bool fast = descs[0].pivoting == DTN_PIVOT_AUTO;
  std::vector<dtn_op*> raw(count);
  for (int p = 0; p < count; ++p) raw[p] = ops[p].get();
  int rc = build_into(descs, count, fast, T.data(), hs, st.data(), -1, nullptr, raw.data());
  double growth = 0.0;
  std::memcpy(&growth, &hs.max_growth_bits, sizeof(double));
  if (rc == DTN_OK && fast && (hs.weak || hs.nonfinite || growth > kGrowthLimit)) {
    // a pivot of the unpivoted path was too small, or its block recursion grew the entries: redo the
    // build with partial pivoting
    hs = DevStatus{};
    rc = build_into(descs, count, false, T.data(), hs, st.data(), -1, nullptr, raw.data());
  }
  if (rc == DTN_OK && hs.nonfinite) { set_err("non-finite pivot during the build"); rc = DTN_ESINGULAR; }
  if (rc == DTN_OK && hs.singular) {
    set_err("singular interior block (pivot below DTN_PIVOT_RTOL of the block scale)");
    rc = DTN_ESINGULAR;
  }
  if (rc == DTN_OK && hs.rank_capped) {
    set_err("a compressed block reached the rank cap (96 columns) at this tol: raise tol or lower hbs_min_level");
    rc = DTN_ERANK;
  }
  if (rc != DTN_OK) { release_all(); return rc; }
  for (int p = 0; p < count; ++p) {
    ops[p]->stats = st[p];
    ops[p]->stats.op_bytes = (size_t)ops[p]->nb * ops[p]->nb * sizeof(double) +
                             (size_t)ops[p]->nb * ops[p]->body_count * sizeof(double) +
                             (ops[p]->cap_offs.empty() ? 0 : (size_t)capture_doubles(descs[p].n, descs[p].leaf,
                                                                                      descs[p].capture_level) * 8);
    out[p] = ops[p].release();
  }
  return DTN_OK;
}

dtn_op* dtn_build_ex(const dtn_build_desc* desc) {
  g_err.clear();
  g_err_code = DTN_OK;
  if (!desc) { set_err("NULL descriptor"); g_err_code = DTN_EINVAL; return nullptr; }
  if (!validate_desc(*desc)) { g_err_code = DTN_EINVAL; return nullptr; }
  dtn_op* op = nullptr;
  g_err_code = build_group(desc, 1, &op);
  return g_err_code == DTN_OK ? op : nullptr;
}

int dtn_last_build_code(void) { return g_err_code; }

dtn_op* dtn_build(int n, const double* b, const double* c, const double* d, int leaf, double tol) {
  dtn_build_desc D;
  dtn_build_desc_init(&D);
  D.n = n; D.b = b; D.c = c; D.d = d; D.leaf = leaf; D.tol = tol;
  return dtn_build_ex(&D);
}

int dtn_build_many(int count, const dtn_build_desc* descs, dtn_op** out) {
  g_err.clear();
  if (count < 0 || (count > 0 && (!descs || !out))) { set_err("bad arguments"); return DTN_EINVAL; }
  if (count == 0) return DTN_OK;
  for (int q = 0; q < count; ++q) out[q] = nullptr;
  for (int q = 0; q < count; ++q)
    if (!validate_desc(descs[q])) return DTN_EINVAL;
  for (int q = 1; q < count; ++q) {
    if (descs[q].device != descs[0].device || descs[q].stream != descs[0].stream ||
        descs[q].batching != descs[0].batching || descs[q].precision != descs[0].precision ||
        descs[q].pivoting != descs[0].pivoting || descs[q].tol != descs[0].tol ||
        descs[q].hbs_min_level != descs[0].hbs_min_level || descs[q].kii_tol != descs[0].kii_tol ||
        descs[q].n_body != 0 || descs[0].n_body != 0) {
      set_err("dtn_build_many: every descriptor must name the same device, stream, batching, precision, pivoting, "
              "tol, hbs_min_level and kii_tol, and carry no body loads");
      return DTN_EINVAL;
    }
  }
  return build_group(descs, count, out);
}

int dtn_nb(const dtn_op* op) {
  if (!op) { set_err("NULL handle"); return DTN_EINVAL; }
  return op->nb;
}

int dtn_level_count(const dtn_op* op) {
  if (!op) { set_err("NULL handle"); return DTN_EINVAL; }
  if (!op->cap) { set_err("the build captured no level (capture_level)"); return DTN_EINVAL; }
  return (int)op->cap_offs.size();
}

int dtn_level_box(const dtn_op* op, int q, int rect[4], double* S, int lds) {
  g_err.clear();
  if (!op || !rect) { set_err("NULL argument"); return DTN_EINVAL; }
  if (!op->cap) { set_err("the build captured no level (capture_level)"); return DTN_EINVAL; }
  if (q < 0 || q >= (int)op->cap_offs.size()) { set_err("box index out of range"); return DTN_EINVAL; }
  for (int k = 0; k < 4; ++k) rect[k] = op->cap_rects[4 * q + k];
  if (!S) return DTN_OK;
  const int m = 2 * (rect[1] - rect[0] - 1) + 2 * (rect[3] - rect[2] - 1);
  if (lds < m) { set_err("lds smaller than the box's ring"); return DTN_EINVAL; }
  HIPCHK(hipSetDevice(op->device), DTN_EDEVICE);
  HIPCHK(hipDeviceSynchronize(), DTN_EDEVICE);
  return host_copy(op->device, true, S, lds, op->cap + op->cap_offs[q], m, m, m, g_dev[op->device].stream);
}

const double* dtn_device_ptr(const dtn_op* op) { return op ? op->T : nullptr; }

// Y = T G on the 128 x 128 (or 64 x 64) MFMA GEMM: no workspace.
static hipError_t apply_gemm(const dtn_op* op, const double* dG, int ldg, int k, double* dY, int ldy, hipStream_t s) {
  DevBufs B{};
  B.p[BUF_OUT] = op->T;
  B.p[BUF_G] = const_cast<double*>(dG);
  B.p[BUF_Y] = dY;
  GemmDesc g{};
  g.M = op->nb; g.N = k; g.K = op->nb;
  g.bufA = BUF_OUT; g.bufB = BUF_G; g.bufC = BUF_Y;
  g.lda = op->nb; g.ldb = ldg; g.ldc = ldy;
  g.rmapC = g.cmapC = g.kmapA = -1;
  g.alpha = 1.0; g.beta = 0.0;
  // 128 x 128 tiles with eight waves (1.43x over 64 x 64 on nb = 4092, k = 1024) once both sides
  // fill them; 64 x 64 below
  const int cfg = (g.M >= 128 && g.N >= 128) ? 2 : 0;
  return launch_gemm_single(g, cfg, B, s);
}

int dtn_apply_device_noalloc(dtn_op* op, const double* dG, int ldg, int k, double* dY, int ldy, void* stream) {
  g_err.clear();
  if (!op || !dG || !dY) { set_err("NULL argument"); return DTN_EINVAL; }
  if (k < 1 || ldg < op->nb || ldy < op->nb) { set_err("bad k or leading dimension"); return DTN_EINVAL; }
  if (dG == dY) { set_err("G and Y alias"); return DTN_EINVAL; }
  if (!op->T) { set_err("dtn_apply_device_noalloc: the handle holds HBS factors only"); return DTN_EINVAL; }
  if (op->nb > kNoAllocMaxNb) {
    set_err("dtn_apply_device_noalloc: nb = " + std::to_string(op->nb) + " exceeds its scratch limit of " +
            std::to_string(kNoAllocMaxNb) + " ring rows (n <= 2048); use dtn_apply_device");
    return DTN_EINVAL;
  }
  Device& dev = g_dev[op->device];
  if (!dev.ready || !dev.noalloc_part) { set_err("device not initialised"); return DTN_EDEVICE; }
  if (apply_splitk_workspace(op->nb, kNoAllocCols) > noalloc_scratch_bytes()) {
    set_err("dtn_apply_device_noalloc: workspace exceeds the scratch array");
    return DTN_EINVAL;
  }
  HIPCHK(hipSetDevice(op->device), DTN_EDEVICE);
  hipStream_t s = stream ? (hipStream_t)stream : dev.stream;
  if (k <= kApplySplitkMaxK)
    HIPCHK(launch_apply_splitk(op->T, op->nb, dG, ldg, k, dY, ldy, dev.noalloc_part, s, kNoAllocCols), DTN_EDEVICE);
  else
    HIPCHK(apply_gemm(op, dG, ldg, k, dY, ldy, s), DTN_EDEVICE);
  return DTN_OK;
}

int dtn_apply_device(dtn_op* op, const double* dG, int ldg, int k, double* dY, int ldy, void* stream) {
  g_err.clear();
  if (!op || !dG || !dY) { set_err("NULL argument"); return DTN_EINVAL; }
  if (k < 1 || ldg < op->nb || ldy < op->nb) { set_err("bad k or leading dimension"); return DTN_EINVAL; }
  if (dG == dY) { set_err("G and Y alias"); return DTN_EINVAL; }
  HIPCHK(hipSetDevice(op->device), DTN_EDEVICE);
  hipStream_t s = stream ? (hipStream_t)stream : g_dev[op->device].stream;
  if (!op->T) return hbs_apply_handle(op, dG, ldg, k, dY, ldy, s);
  const double nbd = op->nb;
  const bool narrow = k <= kApplySplitkMaxK;
  std::unique_ptr<Prof> pr(prof_enabled() ? new Prof() : nullptr);
  if (narrow) {
    // split-K streaming kernel: T read once, partial sums in the handle's buffer
    std::lock_guard<std::mutex> g(op->part_mu);
    if (!op->part) {
      op->part = (double*)g_dev[op->device].pool.alloc(apply_splitk_workspace(op->nb, kApplySplitkMaxK));
      if (!op->part) { set_err("device allocation failed (apply workspace)"); return DTN_ENOMEM; }
      HIPCHK(hipEventCreateWithFlags(&op->part_ev, hipEventDisableTiming), DTN_EDEVICE);
    }
    if (op->part_ev_recorded) HIPCHK(hipStreamWaitEvent(s, op->part_ev, 0), DTN_EDEVICE);
    PROF_BEGIN(pr.get(), "apply_splitk", 2.0 * nbd * nbd * k, 8.0 * (nbd * nbd + 2.0 * nbd * k), s);
    HIPCHK(launch_apply_splitk(op->T, op->nb, dG, ldg, k, dY, ldy, op->part, s), DTN_EDEVICE);
    PROF_END(pr.get(), s);
    HIPCHK(hipEventRecord(op->part_ev, s), DTN_EDEVICE);
    op->part_ev_recorded = true;
  } else {
    PROF_BEGIN(pr.get(), "apply_gemm", 2.0 * nbd * nbd * k, 8.0 * (nbd * nbd + 2.0 * nbd * k), s);
    HIPCHK(apply_gemm(op, dG, ldg, k, dY, ldy, s), DTN_EDEVICE);
    PROF_END(pr.get(), s);
  }
  if (pr) {
    HIPCHK(hipStreamSynchronize(s), DTN_EDEVICE);
    pr->collect();
  }
  return DTN_OK;
}

int dtn_apply(dtn_op* op, const double* G, int k, double* Y) {
  g_err.clear();
  if (!op || !G || !Y) { set_err("NULL argument"); return DTN_EINVAL; }
  if (k < 1) { set_err("k must be >= 1"); return DTN_EINVAL; }
  if (G == Y) { set_err("G and Y alias"); return DTN_EINVAL; }
  HIPCHK(hipSetDevice(op->device), DTN_EDEVICE);
  Device& dev = g_dev[op->device];
  const size_t bytes = (size_t)op->nb * k * sizeof(double);
  double* dG = (double*)dev.pool.alloc(bytes);
  double* dY = (double*)dev.pool.alloc(bytes);
  if (!dG || !dY) { dev.pool.release(dG); dev.pool.release(dY); set_err("device allocation failed"); return DTN_ENOMEM; }
  int rc = DTN_OK;
  hipStream_t s = dev.stream;
  rc = host_copy(op->device, false, const_cast<double*>(G), op->nb, dG, op->nb, op->nb, k, s);
  if (rc == DTN_OK) rc = dtn_apply_device(op, dG, op->nb, k, dY, op->nb, s);
  if (rc == DTN_OK) rc = host_copy(op->device, true, Y, op->nb, dY, op->nb, op->nb, k, s);
  dev.pool.release(dG);
  dev.pool.release(dY);
  return rc;
}

int dtn_export_dense(const dtn_op* op, double* T, int ldt) {
  g_err.clear();
  if (!op || !T) { set_err("NULL argument"); return DTN_EINVAL; }
  if (ldt < op->nb) { set_err("ldt < nb"); return DTN_EINVAL; }
  HIPCHK(hipSetDevice(op->device), DTN_EDEVICE);
  HIPCHK(hipDeviceSynchronize(), DTN_EDEVICE);
  if (!op->T) {
    // HBS only: the matrix the factors stand for, applied to the identity in column chunks
    const int nb = op->nb, chunk = 256;
    Device& dev = g_dev[op->device];
    std::vector<double> eye((size_t)nb * chunk);
    double* dI = (double*)dev.pool.alloc((size_t)nb * chunk * sizeof(double));
    double* dY = (double*)dev.pool.alloc((size_t)nb * chunk * sizeof(double));
    int rc = (dI && dY) ? DTN_OK : DTN_ENOMEM;
    if (rc != DTN_OK) set_err("device allocation failed (export)");
    for (int c0 = 0; c0 < nb && rc == DTN_OK; c0 += chunk) {
      const int kc = std::min(chunk, nb - c0);
      std::fill(eye.begin(), eye.end(), 0.0);
      for (int c = 0; c < kc; ++c) eye[(c0 + c) + (size_t)c * nb] = 1.0;
      rc = host_copy(op->device, false, eye.data(), nb, dI, nb, nb, kc, dev.stream);
      if (rc == DTN_OK) rc = hbs_apply_handle(const_cast<dtn_op*>(op), dI, nb, kc, dY, nb, dev.stream);
      if (rc == DTN_OK) rc = host_copy(op->device, true, T + (size_t)c0 * ldt, ldt, dY, nb, nb, kc, dev.stream);
    }
    dev.pool.release(dI);
    dev.pool.release(dY);
    return rc;
  }
  return host_copy(op->device, true, T, ldt, op->T, op->nb, op->nb, op->nb, g_dev[op->device].stream);
}

int dtn_hbs_compress(dtn_op* op, double tol, int leaf, int drop_dense) {
  g_err.clear();
  if (!op) { set_err("NULL handle"); return DTN_EINVAL; }
  HIPCHK(hipSetDevice(op->device), DTN_EDEVICE);
  Device& dev = g_dev[op->device];
  HIPCHK(hipDeviceSynchronize(), DTN_EDEVICE);   // builds and applies of T on other streams
  const int rc = hbs_compress(op, tol, leaf, dev.stream);
  if (rc != DTN_OK) return rc;
  if (drop_dense) {
    dev.pool.release(op->T);
    op->T = nullptr;
    if (op->part) { dev.pool.release(op->part); op->part = nullptr; }
  }
  op->stats.op_bytes = (op->T ? (size_t)op->nb * op->nb * sizeof(double) : 0) + hbs_bytes(op);
  return DTN_OK;
}

int dtn_hbs_get(const dtn_op* op, dtn_hbs_info* out) {
  if (!op || !out) { set_err("NULL argument"); return DTN_EINVAL; }
  hbs_info(op->hbs, out);
  return op->hbs ? DTN_OK : DTN_EINVAL;
}

int dtn_hbs_invert(dtn_op* op, double tol, int leaf) {
  g_err.clear();
  if (!op) { set_err("NULL handle"); return DTN_EINVAL; }
  HIPCHK(hipSetDevice(op->device), DTN_EDEVICE);
  Device& dev = g_dev[op->device];
  HIPCHK(hipDeviceSynchronize(), DTN_EDEVICE);   // builds and applies of T on other streams
  const int rc = hbs_invert(op, tol, leaf, dev.stream);
  if (rc != DTN_OK) return rc;
  op->stats.op_bytes = (op->T ? (size_t)op->nb * op->nb * sizeof(double) : 0) + hbs_bytes(op);
  return DTN_OK;
}

int dtn_hbs_inverse_get(const dtn_op* op, dtn_hbs_info* out) {
  if (!op || !out) { set_err("NULL argument"); return DTN_EINVAL; }
  hbs_info(op->hbsi, out);
  return op->hbsi ? DTN_OK : DTN_EINVAL;
}

int dtn_apply_hbs_inverse_device(dtn_op* op, const double* dX, int ldx, int k, double* dY, int ldy, void* stream) {
  g_err.clear();
  if (!op || !dX || !dY) { set_err("NULL argument"); return DTN_EINVAL; }
  if (k < 1 || ldx < op->nb || ldy < op->nb) { set_err("bad k or leading dimension"); return DTN_EINVAL; }
  if (dX == dY) { set_err("X and Y alias"); return DTN_EINVAL; }
  HIPCHK(hipSetDevice(op->device), DTN_EDEVICE);
  hipStream_t s = stream ? (hipStream_t)stream : g_dev[op->device].stream;
  return hbs_apply_handle(op, dX, ldx, k, dY, ldy, s, true);
}

int dtn_apply_hbs_device(dtn_op* op, const double* dG, int ldg, int k, double* dY, int ldy, void* stream) {
  g_err.clear();
  if (!op || !dG || !dY) { set_err("NULL argument"); return DTN_EINVAL; }
  if (k < 1 || ldg < op->nb || ldy < op->nb) { set_err("bad k or leading dimension"); return DTN_EINVAL; }
  if (dG == dY) { set_err("G and Y alias"); return DTN_EINVAL; }
  HIPCHK(hipSetDevice(op->device), DTN_EDEVICE);
  hipStream_t s = stream ? (hipStream_t)stream : g_dev[op->device].stream;
  return hbs_apply_handle(op, dG, ldg, k, dY, ldy, s);
}

int dtn_stats_get(const dtn_op* op, dtn_stats* out) {
  if (!op || !out) { set_err("NULL argument"); return DTN_EINVAL; }
  *out = op->stats;
  return DTN_OK;
}

int dtn_profile_enable(int on) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  g_prof_on = on != 0;
  return DTN_OK;
}

int dtn_plan_check(int n, int leaf, double tol, int mixed, int fast, int sym) {
  if (n < 3 || leaf < 4 || !(tol >= 0.0)) { set_err("plan_check: n >= 3, leaf >= 4 and tol >= 0 required"); return DTN_EINVAL; }
  ProbSpec sp;
  sp.n = n; sp.leaf = leaf; sp.conv = 0; sp.sym = sym != 0; sp.definite = sym == 1;
  Plan P;
  std::string err;
  if (!plan_make_many({sp}, fast != 0, P, err, mixed != 0, tol, -1)) { set_err("plan: " + err); return DTN_EINVAL; }
  if (!plan_check(P, err)) { set_err("plan_check: " + err); return DTN_EINVAL; }
  return DTN_OK;
}

int dtn_body_plan_check(int n, int leaf, int fast, int sym, int n_body, const int* nodes) {
  if (n < 3 || leaf < 4 || n_body < 1 || !nodes) { set_err("body_plan_check: bad arguments"); return DTN_EINVAL; }
  ProbSpec sp;
  sp.n = n; sp.leaf = leaf; sp.conv = 0; sp.sym = sym != 0; sp.definite = sym == 1;
  Plan P;
  std::string err;
  if (!plan_make_many({sp}, fast != 0, P, err, false, 0.0, -1)) { set_err("plan: " + err); return DTN_EINVAL; }
  std::vector<int> codes(n_body);
  for (int q = 0; q < n_body; ++q) {
    if (nodes[q] < 0 || nodes[q] >= n * n) { set_err("body_plan_check: node index out of the grid"); return DTN_EINVAL; }
    codes[q] = ((nodes[q] / n) << 16) | (nodes[q] % n);
  }
  BodyPlan B;
  if (!body_plan_make(P, codes, gj_block_class, B, err) || !body_plan_check(P, B, err)) {
    set_err(err);
    return DTN_EINVAL;
  }
  return DTN_OK;
}

int dtn_plan_footprint(const dtn_build_desc* desc, size_t* bytes, char* key, int keylen) {
  if (!desc || !bytes) { set_err("plan_footprint: NULL argument"); return DTN_EINVAL; }
  if (desc->n < 3 || desc->leaf < 4 || !(desc->tol >= 0.0)) {
    set_err("plan_footprint: n >= 3, leaf >= 4 and tol >= 0 required");
    return DTN_EINVAL;
  }
  size_t b = 0;
  const int rc = plan_footprint(desc->device, *desc, b);
  if (rc != DTN_OK) return rc;
  *bytes = b;
  if (key && keylen > 0) {
    const std::string k = plan_cache_key(desc->device, *desc);
    const size_t m = std::min<size_t>(k.size(), (size_t)keylen - 1);
    std::memcpy(key, k.data(), m);
    key[m] = '\0';
  }
  return DTN_OK;
}

int dtn_plan_check_tiles(int n, int leaf, double tol, int mixed, int fast, int sym, int tile) {
  if (n < 3 || leaf < 4 || !(tol >= 0.0)) { set_err("plan_check: n >= 3, leaf >= 4 and tol >= 0 required"); return DTN_EINVAL; }
  if (tile != -1 && tile != 0 && tile != 2 && tile != 3 && tile != 4) { set_err("plan_check: tile must be -1, 0, 2, 3 or 4"); return DTN_EINVAL; }
  ProbSpec sp;
  sp.n = n; sp.leaf = leaf; sp.conv = 0; sp.sym = sym != 0; sp.definite = sym == 1;
  Plan P;
  std::string err;
  if (!plan_make_many({sp}, fast != 0, P, err, mixed != 0, tol, -1, tile)) { set_err("plan: " + err); return DTN_EINVAL; }
  if (!plan_check(P, err)) { set_err("plan_check: " + err); return DTN_EINVAL; }
  return DTN_OK;
}

int dtn_tune(const dtn_build_desc* desc, int reps, char* report, int len) {
  g_err.clear();
  if (!desc || reps < 1) { set_err("dtn_tune: NULL descriptor or reps < 1"); return DTN_EINVAL; }
  if (!validate_desc(*desc)) return DTN_EINVAL;
  if (desc->batching != DTN_FUSED) { set_err("dtn_tune: tunes the fused build only"); return DTN_EINVAL; }
  if (device_ready(desc->device) != DTN_OK) return DTN_EDEVICE;
  HIPCHK(hipSetDevice(desc->device), DTN_EDEVICE);
  Device& dev = g_dev[desc->device];
  const int nb = 4 * (desc->n - 1);
  double* T = (double*)dev.pool.alloc((size_t)nb * nb * sizeof(double));
  if (!T) { set_err("device allocation failed (tuning output)"); return DTN_ENOMEM; }
  const bool fast = desc->pivoting == DTN_PIVOT_AUTO;
  std::map<std::string, std::map<int, double>> ms;   // signature -> tile -> summed ms per build
  std::map<std::string, std::map<int, int>> runs;    // builds that timed (signature, tile)
  std::map<std::string, int> deflt;                  // signature -> the fixed thresholds' tile
  int rc = DTN_OK;
  for (const int cand : {-1, 0, 2, 3, 4}) {           // -1: the planner's fixed thresholds
    for (int r = 0; r <= reps && rc == DTN_OK; ++r) {
      std::map<std::string, double> sink;
      Prof pr(&sink);
      DevStatus hs{};
      dtn_stats st{};
      rc = build_into(desc, 1, fast, &T, hs, &st, cand, &pr);
      if (r == 0) continue;                          // warm-up (plan creation, first touches)
      for (const auto& kv : sink) {
        if (kv.first.rfind("T|", 0) != 0) continue;    // product launches only: "T|<sig>|<tile>"
        const std::string name = kv.first.substr(2);
        const size_t bar = name.rfind('|');
        const int tile = std::atoi(name.c_str() + bar + 1);
        ms[name.substr(0, bar)][tile] += kv.second;
        runs[name.substr(0, bar)][tile] += 1;   // the thresholds' own tile is also timed by its forced run
        if (cand < 0) deflt[name.substr(0, bar)] = tile;
      }
    }
  }
  dev.pool.release(T);
  {
    std::lock_guard<std::mutex> g(g_plan_mu);
    g_plans.clear();                                 // tuning plans and plans of the old table
  }
  if (rc != DTN_OK) return rc;
  std::ostringstream o;
  o << "{";
  bool first = true;
  for (const auto& kv : ms) {
    int best = -1;
    double bt = 0.0;
    for (const auto& c : kv.second) {
      const double avg = c.second / runs[kv.first][c.first];
      if (best < 0 || avg < bt) { best = c.first; bt = avg; }
    }
    // keep the thresholds' tile unless another is faster by more than the timing noise (3 %)
    if (deflt.count(kv.first) && kv.second.count(deflt[kv.first])) {
      const int d0 = deflt[kv.first];
      if (kv.second.at(d0) / runs[kv.first][d0] <= 1.03 * bt) best = d0;
    }
    tune_put(kv.first, best);
    o << (first ? "" : ", ") << "\"" << kv.first << "\": {\"tile\": " << best << ", \"default\": "
      << (deflt.count(kv.first) ? deflt[kv.first] : -1) << ", \"ms\": {";
    bool f2 = true;
    for (const auto& c : kv.second) {
      o << (f2 ? "" : ", ") << "\"" << c.first << "\": " << c.second / runs[kv.first][c.first];
      f2 = false;
    }
    o << "}}";
    first = false;
  }
  o << "}";
  if (report && len > 0) {
    const std::string r = o.str();
    const size_t m = std::min<size_t>(r.size(), (size_t)len - 1);
    std::memcpy(report, r.data(), m);
    report[m] = '\0';
  }
  if (const char* cache = std::getenv("DTN_TUNE_CACHE")) {
    std::ofstream out(cache);
    if (out) out << tune_json("gfx950");
  }
  return (int)ms.size();
}

int dtn_tune_enable(int on) {
  tune_enable(on != 0);
  return DTN_OK;
}

int dtn_tune_clear(void) {
  tune_clear();
  return DTN_OK;
}

int dtn_tune_save(const char* path) {
  if (!path) { set_err("dtn_tune_save: NULL path"); return DTN_EINVAL; }
  std::ofstream out(path);
  if (!out) { set_err(std::string("cannot write ") + path); return DTN_EINVAL; }
  out << tune_json("gfx950");
  return out ? DTN_OK : DTN_EINVAL;
}

int dtn_tune_load(const char* path) {
  if (!path) { set_err("dtn_tune_load: NULL path"); return DTN_EINVAL; }
  std::ifstream in(path);
  if (!in) { set_err(std::string("cannot read ") + path); return DTN_EINVAL; }
  std::stringstream ss;
  ss << in.rdbuf();
  std::string err;
  if (!tune_load_json(ss.str(), "gfx950", err)) { set_err(err); return DTN_EINVAL; }
  return DTN_OK;
}

int dtn_tune_size(void) { return (int)tune_size(); }

int dtn_profile_select(const char* families) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  g_prof_only.clear();
  if (!families) return DTN_OK;
  std::string cur;
  for (const char* p = families;; ++p) {
    if (*p == ',' || *p == '\0') {
      if (!cur.empty()) g_prof_only.insert(cur);
      cur.clear();
      if (*p == '\0') break;
    } else if (*p != ' ') {
      cur.push_back(*p);
    }
  }
  return DTN_OK;
}

int dtn_profile_reset(void) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  g_prof.clear();
  return DTN_OK;
}

int dtn_profile_read(dtn_prof_entry* out, int max) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  if (max < 0 || (max > 0 && !out)) { set_err("bad arguments"); return DTN_EINVAL; }
  int q = 0;
  for (auto& kv : g_prof) {
    if (q >= max) break;
    std::memset(&out[q], 0, sizeof(dtn_prof_entry));
    std::strncpy(out[q].name, kv.first.c_str(), sizeof(out[q].name) - 1);
    out[q].launches = kv.second.launches;
    out[q].total_ms = kv.second.ms;
    out[q].flops = kv.second.flops;
    out[q].bytes = kv.second.bytes;
    ++q;
  }
  return max == 0 ? (int)g_prof.size() : q;
}

dtn_op* dtn_import_dense(int nb, const double* T, int ldt, int device) {
  g_err.clear();
  if (nb < 1 || !T || ldt < nb) { set_err("import: need nb >= 1, T non-NULL and ldt >= nb"); return nullptr; }
  if (device_ready(device) != DTN_OK) return nullptr;
  if (hipSetDevice(device) != hipSuccess) { (void)hipGetLastError(); set_err("import: hipSetDevice failed"); return nullptr; }
  Device& dev = g_dev[device];
  auto op = std::make_unique<dtn_op>();
  op->device = device;
  op->nb = nb;
  op->n = nb % 4 == 0 ? nb / 4 + 1 : 0;
  op->T = (double*)dev.pool.alloc((size_t)nb * nb * sizeof(double));
  if (!op->T) { set_err("device allocation failed (imported operator)"); return nullptr; }
  if (host_copy(device, false, const_cast<double*>(T), ldt, op->T, nb, nb, nb, dev.stream) != DTN_OK) {
    dev.pool.release(op->T);
    return nullptr;
  }
  op->stats.n = op->n;
  op->stats.nb = nb;
  return op.release();
}

int dtn_body_count(const dtn_op* op) {
  if (!op) { set_err("NULL handle"); return DTN_EINVAL; }
  return op->body_count;
}

int dtn_body_get(const dtn_op* op, double* F, int ldf) {
  g_err.clear();
  if (!op || !F) { set_err("NULL argument"); return DTN_EINVAL; }
  if (!op->body) { set_err("the handle was built without body loads"); return DTN_EINVAL; }
  if (ldf < op->nb) { set_err("ldf < nb"); return DTN_EINVAL; }
  HIPCHK(hipSetDevice(op->device), DTN_EDEVICE);
  HIPCHK(hipDeviceSynchronize(), DTN_EDEVICE);
  return host_copy(op->device, true, F, ldf, op->body, op->nb, op->nb, op->body_count, g_dev[op->device].stream);
}

const double* dtn_body_ptr(const dtn_op* op) { return op ? op->body : nullptr; }

int dtn_apply_body_device(dtn_op* op, const double* dG, int ldg, const double* dQ, int ldq, int k, double* dY,
                          int ldy, void* stream) {
  g_err.clear();
  if (!op || !dG || !dQ || !dY) { set_err("NULL argument"); return DTN_EINVAL; }
  if (!op->body) { set_err("the handle was built without body loads"); return DTN_EINVAL; }
  if (k < 1 || ldq < op->body_count || ldg < op->nb || ldy < op->nb) { set_err("bad k or leading dimension"); return DTN_EINVAL; }
  int rc = dtn_apply_device(op, dG, ldg, k, dY, ldy, stream);
  if (rc != DTN_OK) return rc;
  hipStream_t s = stream ? (hipStream_t)stream : g_dev[op->device].stream;
  DevBufs B{};
  B.p[BUF_OUT] = op->body;
  B.p[BUF_G] = const_cast<double*>(dQ);
  B.p[BUF_Y] = dY;
  GemmDesc g{};
  g.M = op->nb; g.N = k; g.K = op->body_count;
  g.bufA = BUF_OUT; g.bufB = BUF_G; g.bufC = BUF_Y;
  g.lda = op->nb; g.ldb = ldq; g.ldc = ldy;
  g.rmapC = g.cmapC = g.kmapA = -1;
  g.kcnt = -1;
  g.tiles_m = (g.M + gemm_tile_m(0) - 1) / gemm_tile_m(0);
  g.tiles_n = (g.N + gemm_tile_n(0) - 1) / gemm_tile_n(0);
  g.alpha = 1.0; g.beta = 1.0;
  HIPCHK(launch_gemm_single(g, 0, B, s), DTN_EDEVICE);
  return DTN_OK;
}

void dtn_free(dtn_op* op) {
  if (!op) return;
  // applies may still be reading T on any stream: wait before its memory is reused
  if ((op->T || op->hbs || op->hbsi) && hipSetDevice(op->device) == hipSuccess) (void)hipDeviceSynchronize();
  if (op->T) g_dev[op->device].pool.release(op->T);
  hbs_release(op);
  if (op->hbs_work) g_dev[op->device].pool.release(op->hbs_work);
  if (op->hbs_ev) (void)hipEventDestroy(op->hbs_ev);
  if (op->part) g_dev[op->device].pool.release(op->part);
  if (op->part_ev) (void)hipEventDestroy(op->part_ev);
  if (op->cap) g_dev[op->device].pool.release(op->cap);
  if (op->body) g_dev[op->device].pool.release(op->body);
  delete op;
}

}  // extern "C"
