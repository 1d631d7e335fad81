// libqoc serving engine: continuous batching of GRAPE forward + gradient
// requests of mixed d and N on one GPU.
//
// Requests wait in a FIFO queue and are admitted in order while their device
// footprint (inputs, outputs and the per-problem workspace, about
// 4 N D^2 c bytes of per-slice arrays at D >= 32) fits the engine's device arena and
// a descriptor slot is free.  Admitted requests are grouped by padded
// dimension D; each D bucket owns a stream and a hipGraph of the eight
// persistent stage kernels, captured once, whose item counts, prefix sums
// and descriptor slots are read from a small device table.  A tick of a
// bucket uploads that table for every request admitted to the bucket since
// its last tick, replays the graph, and queues the copies of F and the
// gradient back to pinned host memory; requests arriving meanwhile are
// admitted as memory and slots free up and join the bucket's next tick.
// Buckets tick independently, so the work of small and large problems
// overlaps on the device.  The fixed graph with item tables padded to the
// bucket's capacity is the pad-and-mask technique of App. A.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "qoc.h"
#include "qoc_internal.hpp"

using namespace qoc;

namespace {

int efail(int code, const char* msg) {
  set_last_error(msg);
  return code;
}

// First-fit allocator over [0, size) with 256-byte granularity.
class FirstFit {
 public:
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
    used_ = 0;
  }
  bool alloc(size_t n, size_t& off) {
    n = align_up(n);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        off = it->first;
        size_t rest = it->second - n;
        free_.erase(it);
        if (rest) free_[off + n] = rest;
        used_ += n;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = align_up(n);
    used_ -= n;
    auto it = free_.emplace(off, n).first;
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
  size_t used() const { return used_; }

 private:
  std::map<size_t, size_t> free_;
  size_t used_ = 0;
};

enum ReqState { QUEUED, ADMITTED, RUNNING, DONE };

// Device (and pinned host) image of one request:
//   H0 | Hc | u | V | F | grad | workspace   (FP64 inputs and outputs)
struct Req {
  int64_t id;
  int d, m, N, D;
  double dt;
  ReqState state = QUEUED;
  size_t dev_off = 0, dev_bytes = 0;
  size_t host_off = 0, host_bytes = 0;
  size_t in_bytes = 0;           // H0 | Hc | u | V
  size_t F_off = 0, grad_off = 0, ws_off = 0;
  int slot = -1;
  Layout lo;
};

constexpr int kDims[4] = {16, 32, 64, 128};
constexpr int kStages = ST_COUNT;

int bucket_of(int D) {
  for (int i = 0; i < 4; ++i)
    if (kDims[i] == D) return i;
  return -1;
}

int persistent_grid(int D) {
  switch (D) {
    case 16: return 2048;
    case 32: return 1024;
    case 64: return 512;
    default: return kScratchSlots;
  }
}

struct Bucket {
  int D = 0;
  hipStream_t stream = nullptr;
  hipGraphExec_t exec = nullptr;
  int* tab_dev = nullptr;   // kStages tables of table_ints ints
  int* tab_host = nullptr;  // pinned
  hipEvent_t done = nullptr;
  bool busy = false;
  std::vector<int64_t> pending, running;
};

}  // namespace

struct qoc_engine {
  int precision = 1;
  int max_active = 0;
  int table_ints = 0;
  uint64_t pool_bytes = 0;
  char* pool = nullptr;
  FirstFit dev;
  uint64_t host_bytes = 0;
  char* hpool = nullptr;  // pinned
  FirstFit host;
  ProbDesc* descs_dev = nullptr;
  ProbDesc* descs_host = nullptr;  // pinned staging, one per slot
  void* scratch128 = nullptr;
  std::vector<int> free_slots;
  std::deque<int64_t> queue;
  std::unordered_map<int64_t, Req> reqs;
  Bucket buckets[4];
  std::vector<int64_t> finished;
  int64_t next_id = 0;
  std::mutex mu;
};

namespace {

size_t input_bytes(int d, int m, int N) { return (size_t)d * d * 16 * (m + 2) + (size_t)m * N * 8; }

// Device bytes of one request: inputs, F and gradient, and its workspace.
Layout request_layout(int precision, int d, int m, int N) {
  // one problem, no descriptor table; D = 128 scratch is held by the engine;
  // the latency chunk length
  Layout lo = make_layout(1, d, m, N, precision, engine_chunk(N), 0);
  return lo;
}

size_t request_device_bytes(const Layout& lo, int d, int m, int N) {
  return align_up(input_bytes(d, m, N)) + align_up(8 + (size_t)m * N * 8) + lo.per_prob;
}

size_t request_host_bytes(int d, int m, int N) { return align_up(input_bytes(d, m, N)) + align_up(8 + (size_t)m * N * 8); }

void free_request(qoc_engine* E, Req& r) {
  if (r.dev_bytes) E->dev.release(r.dev_off, r.dev_bytes);
  r.dev_bytes = 0;
  if (r.slot >= 0) E->free_slots.push_back(r.slot);
  r.slot = -1;
}

hipError_t capture(qoc_engine* E, Bucket& b) {
  Launch L;
  memset(&L, 0, sizeof L);
  L.descs = E->descs_dev;
  L.flags = RUN_FID | RUN_BWD | RUN_GRAD;
  L.stream = b.stream;
  L.scratch = b.D == 128 ? E->scratch128 : nullptr;
  L.dyn_grid = persistent_grid(b.D);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(b.stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  const Range none = {0, 0, 0, 0, 0};
  for (int s = 0; s < kStages && e == hipSuccess; ++s) {
    L.dyn = b.tab_dev + (size_t)s * E->table_ints;
    e = launch_stage(E->precision, b.D, s, L, none);
  }
  hipError_t e2 = hipStreamEndCapture(b.stream, &g);
  if (e == hipSuccess) e = e2;
  if (e == hipSuccess) e = hipGraphInstantiate(&b.exec, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  return e;
}

// Item tables of one tick: per stage nprob, total, prefix sums, slots.
void build_tables(qoc_engine* E, Bucket& b) {
  const int n = (int)b.pending.size();
  for (int s = 0; s < kStages; ++s) {
    int* t = b.tab_host + (size_t)s * E->table_ints;
    t[0] = n;
    int* start = t + 2;
    int* slot = t + 3 + n;
    int acc = 0;
    for (int i = 0; i < n; ++i) {
      const Req& r = E->reqs[b.pending[i]];
      start[i] = acc;
      slot[i] = r.slot;
      int items = 0;
      switch (s) {
        case ST_PREP: items = r.m + 2; break;
        case ST_PLAN: case ST_EXPM: case ST_ADJ: items = r.N; break;
        case ST_SCAN: case ST_MC: case ST_BSCAN: items = r.lo.P; break;
        case ST_CARRY: items = r.lo.PG; break;  // carry groups
      }
      acc += items;
    }
    start[n] = acc;
    t[1] = acc;
  }
}

hipError_t launch_tick(qoc_engine* E, Bucket& b) {
  hipError_t e = hipSuccess;
  if (!b.exec) {
    e = capture(E, b);
    if (e != hipSuccess) return e;
  }
  for (int64_t id : b.pending) {
    Req& r = E->reqs[id];
    char* dbase = E->pool + r.dev_off;
    char* hbase = E->hpool + r.host_off;
    ProbDesc& P = E->descs_host[r.slot];
    const double* H0 = reinterpret_cast<const double*>(dbase);
    const double* Hc = H0 + 2 * (size_t)r.d * r.d;
    const double* u = Hc + 2 * (size_t)r.d * r.d * r.m;
    const double* V = u + (size_t)r.m * r.N;
    // the API's default: a Newton-Schulz step on every chunk product
    const double tol = E->precision == QOC_FP64 ? -1.0 : 0.0;
    fill_desc(P, r.lo, dbase + r.ws_off, r.d, r.m, r.N, r.dt, RUN_FID | RUN_BWD | RUN_GRAD, H0, Hc, u, V,
              reinterpret_cast<double*>(dbase + r.F_off), reinterpret_cast<double*>(dbase + r.grad_off), nullptr, tol);
    if (e == hipSuccess) e = hipMemcpyAsync(dbase, hbase, r.in_bytes, hipMemcpyHostToDevice, b.stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(E->descs_dev + r.slot, &P, sizeof(ProbDesc), hipMemcpyHostToDevice, b.stream);
  }
  build_tables(E, b);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b.tab_dev, b.tab_host, (size_t)kStages * E->table_ints * sizeof(int), hipMemcpyHostToDevice,
                       b.stream);
  if (e == hipSuccess) e = hipGraphLaunch(b.exec, b.stream);
  for (int64_t id : b.pending) {
    Req& r = E->reqs[id];
    char* dbase = E->pool + r.dev_off;
    char* hbase = E->hpool + r.host_off + align_up(r.in_bytes);
    // F then the gradient, contiguous on both sides
    if (e == hipSuccess)
      e = hipMemcpyAsync(hbase, dbase + r.F_off, 8 + (size_t)r.m * r.N * 8, hipMemcpyDeviceToHost, b.stream);
    r.state = RUNNING;
  }
  if (e == hipSuccess) e = hipEventRecord(b.done, b.stream);
  b.running.swap(b.pending);
  b.pending.clear();
  b.busy = true;
  return e;
}

void harvest(qoc_engine* E, Bucket& b, bool wait) {
  if (!b.busy) return;
  hipError_t q = wait ? hipEventSynchronize(b.done) : hipEventQuery(b.done);
  if (q != hipSuccess) return;
  for (int64_t id : b.running) {
    Req& r = E->reqs[id];
    r.state = DONE;
    free_request(E, r);
    E->finished.push_back(id);
  }
  b.running.clear();
  b.busy = false;
}

void admit(qoc_engine* E) {
  while (!E->queue.empty() && !E->free_slots.empty()) {
    Req& r = E->reqs[E->queue.front()];
    size_t off;
    if (!E->dev.alloc(r.dev_bytes, off)) break;  // FIFO: wait until memory frees up
    r.dev_off = off;
    r.slot = E->free_slots.back();
    E->free_slots.pop_back();
    r.state = ADMITTED;
    E->buckets[bucket_of(r.D)].pending.push_back(r.id);
    E->queue.pop_front();
  }
}

}  // namespace

extern "C" {

uint64_t qoc_engine_footprint(int precision, int d, int m, int N) {
  if (d < 1 || d > 128 || m < 1 || N < 1) return 0;
  return request_device_bytes(request_layout(precision, d, m, N), d, m, N);
}

int qoc_engine_create(int precision, uint64_t pool_bytes, uint64_t host_bytes, int max_active, qoc_engine** out) {
  if (!out) return efail(QOC_ERR_ARG, "out must be non-null");
  *out = nullptr;
  if (precision != QOC_FP64 && precision != QOC_FP32 && precision != QOC_BF16X3)
    return efail(QOC_ERR_UNSUPPORTED, "unknown precision");
  if (max_active < 1 || pool_bytes == 0 || host_bytes == 0) return efail(QOC_ERR_ARG, "bad engine sizes");
  qoc_engine* E = new qoc_engine;
  E->precision = precision;
  E->max_active = max_active;
  E->table_ints = (int)align_up((3 + 2 * (size_t)max_active) * sizeof(int)) / (int)sizeof(int);
  E->pool_bytes = pool_bytes;
  E->host_bytes = host_bytes;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&E->pool), pool_bytes);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&E->hpool), host_bytes, hipHostMallocDefault);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&E->descs_dev), sizeof(ProbDesc) * max_active);
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void**>(&E->descs_host), sizeof(ProbDesc) * max_active, hipHostMallocDefault);
  if (e == hipSuccess && precision != QOC_BF16X3)
    e = hipMalloc(&E->scratch128, (size_t)kScratchSlots * kScratchMats * 2 * 128 * 128 * (precision == QOC_FP64 ? 8 : 4));
  for (int i = 0; i < 4 && e == hipSuccess; ++i) {
    Bucket& b = E->buckets[i];
    b.D = kDims[i];
    e = hipStreamCreateWithFlags(&b.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&b.tab_dev), sizeof(int) * kStages * E->table_ints);
    if (e == hipSuccess)
      e = hipHostMalloc(reinterpret_cast<void**>(&b.tab_host), sizeof(int) * kStages * E->table_ints,
                        hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b.done, hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    set_last_error((std::string("engine allocation: ") + hipGetErrorString(e)).c_str());
    qoc_engine_destroy(E);
    return QOC_ERR_OOM;
  }
  E->dev.reset(pool_bytes);
  E->host.reset(host_bytes);
  for (int i = max_active - 1; i >= 0; --i) E->free_slots.push_back(i);
  *out = E;
  return QOC_OK;
}

int qoc_engine_destroy(qoc_engine* E) {
  if (!E) return QOC_OK;
  for (auto& b : E->buckets) {
    if (b.stream) (void)hipStreamSynchronize(b.stream);
    if (b.exec) (void)hipGraphExecDestroy(b.exec);
    if (b.done) (void)hipEventDestroy(b.done);
    if (b.tab_dev) (void)hipFree(b.tab_dev);
    if (b.tab_host) (void)hipHostFree(b.tab_host);
    if (b.stream) (void)hipStreamDestroy(b.stream);
  }
  if (E->scratch128) (void)hipFree(E->scratch128);
  if (E->descs_dev) (void)hipFree(E->descs_dev);
  if (E->descs_host) (void)hipHostFree(E->descs_host);
  if (E->hpool) (void)hipHostFree(E->hpool);
  if (E->pool) (void)hipFree(E->pool);
  delete E;
  return QOC_OK;
}

int qoc_engine_submit(qoc_engine* E, int d, int m, int N, const qoc_z* H0, const qoc_z* Hc, const double* u,
                      double dt, const qoc_z* V, int64_t* id) {
  if (!E || !H0 || !Hc || !u || !V || !id) return efail(QOC_ERR_ARG, "null argument");
  if (d < 1 || m < 1 || N < 1) return efail(QOC_ERR_ARG, "need d, m, N >= 1");
  if (d > 128) return efail(QOC_ERR_UNSUPPORTED, "d exceeds 128");
  if (!(dt > 0) || !std::isfinite(dt)) return efail(QOC_ERR_ARG, "dt must be finite and > 0");
  const int D = padded_dim(d);
  if (E->precision == QOC_BF16X3 && (D < 32 || D > 64))
    return efail(QOC_ERR_UNSUPPORTED, "split-BF16 engines serve 17 <= d <= 64");
  std::lock_guard<std::mutex> lk(E->mu);
  Req r;
  r.id = E->next_id++;
  r.d = d;
  r.m = m;
  r.N = N;
  r.D = D;
  r.dt = dt;
  r.lo = request_layout(E->precision, d, m, N);
  r.in_bytes = input_bytes(d, m, N);
  r.F_off = align_up(r.in_bytes);
  r.grad_off = r.F_off + 8;
  r.ws_off = r.F_off + align_up(8 + (size_t)m * N * 8);
  r.dev_bytes = request_device_bytes(r.lo, d, m, N);
  r.host_bytes = request_host_bytes(d, m, N);
  if (r.dev_bytes > E->pool_bytes) return efail(QOC_ERR_OOM, "request exceeds the engine's device pool");
  size_t hoff;
  if (!E->host.alloc(r.host_bytes, hoff)) return efail(QOC_ERR_OOM, "engine host staging is full");
  r.host_off = hoff;
  char* h = E->hpool + hoff;
  const size_t dd = (size_t)d * d * 16;
  memcpy(h, H0, dd);
  memcpy(h + dd, Hc, dd * m);
  memcpy(h + dd * (m + 1), u, (size_t)m * N * 8);
  memcpy(h + dd * (m + 1) + (size_t)m * N * 8, V, dd);
  E->reqs.emplace(r.id, r);
  E->queue.push_back(r.id);
  *id = r.id;
  return QOC_OK;
}

int qoc_engine_step(qoc_engine* E, int wait) {
  if (!E) return efail(QOC_ERR_ARG, "null engine");
  std::lock_guard<std::mutex> lk(E->mu);
  for (auto& b : E->buckets) harvest(E, b, false);
  admit(E);
  for (auto& b : E->buckets) {
    if (b.busy || b.pending.empty()) continue;
    hipError_t e = launch_tick(E, b);
    if (e != hipSuccess) {
      set_last_error((std::string("engine tick: ") + hipGetErrorString(e)).c_str());
      return QOC_ERR_DEVICE;
    }
  }
  if (wait) {
    bool any = false;
    for (auto& b : E->buckets) any = any || b.busy;
    if (any && E->finished.empty()) {
      // block on the earliest busy bucket
      for (auto& b : E->buckets)
        if (b.busy) {
          harvest(E, b, true);
          break;
        }
    }
  }
  return QOC_OK;
}

int qoc_engine_poll(qoc_engine* E, int max, int64_t* ids, double* F, int* n) {
  if (!E || !n || (max > 0 && (!ids || !F))) return efail(QOC_ERR_ARG, "null argument");
  std::lock_guard<std::mutex> lk(E->mu);
  int k = 0;
  while (k < max && !E->finished.empty()) {
    const int64_t id = E->finished.front();
    E->finished.erase(E->finished.begin());
    const Req& r = E->reqs[id];
    ids[k] = id;
    memcpy(&F[k], E->hpool + r.host_off + align_up(r.in_bytes), 8);
    ++k;
  }
  *n = k;
  return QOC_OK;
}

int qoc_engine_fetch(qoc_engine* E, int64_t id, double* grad) {
  if (!E) return efail(QOC_ERR_ARG, "null engine");
  std::lock_guard<std::mutex> lk(E->mu);
  auto it = E->reqs.find(id);
  if (it == E->reqs.end() || it->second.state != DONE) return efail(QOC_ERR_ARG, "unknown or unfinished request");
  Req& r = it->second;
  if (grad) memcpy(grad, E->hpool + r.host_off + align_up(r.in_bytes) + 8, (size_t)r.m * r.N * 8);
  E->host.release(r.host_off, r.host_bytes);
  E->reqs.erase(it);
  return QOC_OK;
}

int qoc_engine_stats(qoc_engine* E, int64_t* queued, int64_t* active, uint64_t* pool_used) {
  if (!E) return efail(QOC_ERR_ARG, "null engine");
  std::lock_guard<std::mutex> lk(E->mu);
  int64_t a = 0;
  for (auto& b : E->buckets) a += (int64_t)(b.pending.size() + b.running.size());
  if (queued) *queued = (int64_t)E->queue.size();
  if (active) *active = a;
  if (pool_used) *pool_used = E->dev.used();
  return QOC_OK;
}

}  // extern "C"
