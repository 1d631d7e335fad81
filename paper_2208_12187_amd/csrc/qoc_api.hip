// libqoc C ABI: argument checks, workspace layout, descriptor upload and the
// launch sequence of the GRAPE hot path (see include/qoc.h for the contract).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "qoc.h"
#include "qoc_internal.hpp"
#include "qoc_plan.hpp"

using qoc::Launch;
using qoc::Layout;
using qoc::ProbDesc;
using qoc::align_up;
using qoc::kAlign;
using qoc::make_layout;
using qoc::padded_dim;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int check_dims(int B, int d, int m, int N, int precision) {
  if (B < 1) return fail(QOC_ERR_ARG, "batch size B = %d must be >= 1", B);
  if (d < 1 || m < 1 || N < 1) return fail(QOC_ERR_ARG, "need d, m, N >= 1 (got d=%d m=%d N=%d)", d, m, N);
  if (d > 128) return fail(QOC_ERR_UNSUPPORTED, "d = %d exceeds the supported maximum 128", d);
  if (precision != QOC_FP64 && precision != QOC_FP32 && precision != QOC_BF16X3)
    return fail(QOC_ERR_UNSUPPORTED, "precision %d is not available", precision);
  if (precision == QOC_BF16X3 && (padded_dim(d) < 32 || padded_dim(d) > 64))
    return fail(QOC_ERR_UNSUPPORTED, "split-BF16 products are built for 17 <= d <= 64 (got d = %d)", d);
  return QOC_OK;
}

bool finite_all(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

// |H - H^dag|_max <= 1e-12 max(1, |H|_max)
bool hermitian(const qoc_z* H, int d) {
  double hmax = 0, dmax = 0;
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) {
      const qoc_z x = H[a * d + b], y = H[b * d + a];
      hmax = std::max(hmax, std::max(fabs(x.re), fabs(x.im)));
      dmax = std::max(dmax, std::max(fabs(x.re - y.re), fabs(x.im + y.im)));
    }
  return dmax <= 1e-12 * std::max(1.0, hmax);
}

// |V^dag V - I|_max <= 1e-8: the fidelity |Tr(V^dag X_N)|^2 / d^2 is bounded
// by 1 only for a unitary target.
bool unitary(const qoc_z* V, int d) {
  double worst = 0;
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) {
      double re = a == b ? -1.0 : 0.0, im = 0.0;
      for (int c = 0; c < d; ++c) {  // (V^dag V)_ab = sum_c conj(V_ca) V_cb
        const qoc_z x = V[c * d + a], y = V[c * d + b];
        re += x.re * y.re + x.im * y.im;
        im += x.re * y.im - x.im * y.re;
      }
      worst = std::max(worst, std::max(fabs(re), fabs(im)));
    }
  return worst <= 1e-8;
}

int validate_host(int d, int m, int N, const qoc_z* H0, const qoc_z* Hc, const double* u, const qoc_z* V,
                  bool generators) {
  const size_t dd = (size_t)d * d;
  if (!finite_all(&H0->re, 2 * dd) || !finite_all(&Hc->re, 2 * dd * m) || !finite_all(u, (size_t)m * N) ||
      (V && !finite_all(&V->re, 2 * dd)))
    return fail(QOC_ERR_NONFINITE, "an input holds NaN or Inf");
  if (generators) return QOC_OK;  // general generators and targets: no symmetry to check
  if (!hermitian(H0, d)) return fail(QOC_ERR_NOT_HERMITIAN, "H0 is not Hermitian");
  for (int j = 0; j < m; ++j)
    if (!hermitian(Hc + (size_t)j * dd, d)) return fail(QOC_ERR_NOT_HERMITIAN, "Hc[%d] is not Hermitian", j);
  if (V && !unitary(V, d)) return fail(QOC_ERR_NOT_UNITARY, "V is not unitary (|V^dag V - I|_max > 1e-8)");
  return QOC_OK;
}

qoc_options defaults() {
  qoc_options o;
  qoc_default_options(&o);
  return o;
}

// Stage sequence of the path.  Without checkpointing: prep, plan, expm, the
// forward scans, carry, then for the gradient mc, the backward scans (which
// start every chunk from its mc) and the adjoint.  With checkpointing the
// per-slice arrays hold one segment at a time: a first sweep over segments
// (expm, forward scans) yields every chunk total, the carry and mc run once,
// and a second sweep recomputes each segment's propagators and local products
// (forward and backward passes in one launch) before its adjoint pass.  The
// recomputation is bitwise identical.
hipError_t enqueue(int precision, const Layout& Lo, const Launch& L, int N, int flags) {
  using namespace qoc;
  const int D = Lo.D;
  const Range all = {0, N, 0, Lo.P, 0};
  hipError_t e = hipSuccess;
  auto run = [&](int st, const Range& rg) {
    if (e == hipSuccess) e = launch_stage(precision, D, st, L, rg);
  };
  run(ST_PREP, all);
  run(ST_PLAN, all);
  const bool grad = (flags & RUN_GRAD) != 0;
  if (Lo.G >= Lo.P) {
    run(ST_EXPM, all);
    run(ST_SCAN, all);
    run(ST_CARRY, all);
    if (grad) {
      run(ST_MC, all);
      run(ST_BSCAN, all);
      run(ST_ADJ, all);
    }
    return e;
  }
  auto segment = [&](int c_lo) {
    const int c_n = std::min(Lo.G, Lo.P - c_lo);
    const int s_lo = c_lo * Lo.L;
    const int s_hi = std::min(N, (c_lo + c_n) * Lo.L);
    return Range{s_lo, s_hi - s_lo, c_lo, c_n, s_lo, 0};
  };
  for (int c = 0; c < Lo.P; c += Lo.G) {
    const Range rg = segment(c);
    run(ST_EXPM, rg);
    run(ST_SCAN, rg);
  }
  run(ST_CARRY, all);
  if (grad) {
    run(ST_MC, all);
    for (int c = 0; c < Lo.P; c += Lo.G) {
      Range rg = segment(c);
      rg.recompute = 1;
      run(ST_EXPM, rg);
      run(ST_SCAN, rg);  // the forward and backward passes of the segment together
      run(ST_ADJ, rg);
    }
  }
  return e;
}

// Re-unitarisation threshold of a call: off in FP64.
// By default every chunk product gets the Newton-Schulz step (threshold 0):
// the chunk residuals are at the rounding level, 0.6-1.0 u sqrt(d L) with
// u = 2^-24 for d = 8 ... 128 and L = 8 ... 128, yet removing that
// non-unitary part of the rounding error makes Tr(V^dag X_N) about ten times
// more accurate, which the gradient of a problem with a small |g| needs
// (dF/du is proportional to conj(g), so an absolute error in g is relative
// to |g| there).  The residual is still measured and reported.
double reun_tol(const qoc_options& o) {
  if (o.precision == QOC_FP64 || o.reunitarise_tol < 0 || o.generators) return -1.0;
  return o.reunitarise_tol;
}

// Enqueue the path for a uniform batch whose inputs and outputs are in
// device memory.  flags: qoc::RUN_* bits.
int run_dev(int B, int d, int m, int N, const void* H0, const void* Hc, const void* u, double dt, const void* V,
            void* F, void* grad, void* XN, void* ws, size_t ws_bytes, const qoc_options* opt_in, int flags,
            void* g_out = nullptr) {
  const qoc_options opt = opt_in ? *opt_in : defaults();
  int rc = check_dims(B, d, m, N, opt.precision);
  if (rc) return rc;
  if (!(dt > 0) || !std::isfinite(dt)) return fail(QOC_ERR_ARG, "dt must be finite and > 0");
  if (!H0 || !Hc || !u) return fail(QOC_ERR_ARG, "H0, Hc and u must be non-null");
  if ((flags & qoc::RUN_FID) && (!V || (!F && !g_out))) return fail(QOC_ERR_ARG, "V and F must be non-null");
  if ((flags & qoc::RUN_GRAD) && !grad) return fail(QOC_ERR_ARG, "grad must be non-null");
  if (!ws) return fail(QOC_ERR_ARG, "workspace must be non-null");
  if (((uintptr_t)ws) % kAlign) return fail(QOC_ERR_ARG, "workspace must be 256-byte aligned");
  const Layout Lo = make_layout(B, d, m, N, opt.precision, opt.chunk, opt.hbm_budget);
  if (ws_bytes < Lo.total)
    return fail(QOC_ERR_ARG, "workspace holds %zu bytes, %zu needed", ws_bytes, Lo.total);

  char* base = static_cast<char*>(ws);
  std::vector<ProbDesc> descs(B);
  const size_t dd = (size_t)d * d;
  const double tol = reun_tol(opt);
  for (int b = 0; b < B; ++b) {
    char* pb = base + Lo.desc_bytes + (size_t)b * Lo.per_prob;
    fill_desc(descs[b], Lo, pb, d, m, N, dt,
              flags | (opt.dense_controls ? qoc::CTRL_DENSE : 0) | (opt.generators ? qoc::RUN_GENERAL : 0),
              static_cast<const double*>(H0) + 2 * dd * b,
              static_cast<const double*>(Hc) + 2 * dd * m * b, static_cast<const double*>(u) + (size_t)m * N * b,
              V ? static_cast<const double*>(V) + 2 * dd * b : nullptr, F ? static_cast<double*>(F) + b : nullptr,
              // the complex dg of the trace gradient takes two doubles per entry
              grad ? static_cast<double*>(grad) + (size_t)m * N * b * ((flags & qoc::RUN_RAWDG) ? 2 : 1) : nullptr,
              XN ? static_cast<double*>(XN) + 2 * dd * b : nullptr, tol,
              opt.diagnostics ? opt.diagnostics + 4 * b : nullptr);
    if (g_out) descs[b].g = static_cast<double*>(g_out) + 2 * b;
  }
  hipStream_t st = static_cast<hipStream_t>(opt.stream);
  hipError_t e = hipMemcpyAsync(base, descs.data(), (size_t)B * sizeof(ProbDesc), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return fail(QOC_ERR_DEVICE, "descriptor upload: %s", hipGetErrorString(e));

  Launch L;
  L.descs = reinterpret_cast<const ProbDesc*>(base);
  L.nprob = B;
  L.uniformN = N;
  L.uniformP = Lo.P;
  L.slice_start = nullptr;
  L.chunk_start = nullptr;
  L.total_slices = B * N;
  L.total_chunks = B * Lo.P;
  L.max_m = m;
  L.flags = flags;
  L.stream = st;
  L.scratch = Lo.scratch_bytes ? base + Lo.scratch : nullptr;
  L.dyn = nullptr;
  L.dyn_grid = 0;
  e = enqueue(opt.precision, Lo, L, N, flags);
  if (e != hipSuccess) return fail(QOC_ERR_DEVICE, "kernel launch: %s", hipGetErrorString(e));
  return QOC_OK;
}

// ---------------------------------------------------------------- static scratch

// Workspace of qoc_gradient_dev_noalloc: a file-scope device array, one copy
// per GPU, held until the process ends.  In host code its name is only a
// host-side stand-in: kernels get the device address that
// hipGetSymbolAddress returns for the current device, looked up once per
// device and kept in scratch_ptr.
static __device__ __align__(256) unsigned char scratch[QOC_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of scratch, or null (error set).
void* scratch_ptr() {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    fail(QOC_ERR_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    return nullptr;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    fail(QOC_ERR_DEVICE, "device index %d beyond the %d the static scratch supports", dev, kMaxDevices);
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      fail(QOC_ERR_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
      return nullptr;
    }
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

// Device buffers of a host call, freed on scope exit.
struct DevBufs {
  std::vector<void*> ptrs;
  ~DevBufs() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  void* alloc(size_t n) {
    void* p = nullptr;
    if (hipMalloc(&p, n ? n : 1) != hipSuccess) return nullptr;
    ptrs.push_back(p);
    return p;
  }
};

int run_host(int d, int m, int N, const qoc_z* H0, const qoc_z* Hc, const double* u, double dt, const qoc_z* V,
             double* F, double* grad, qoc_z* XN, const qoc_options* opt_in, int flags) {
  const qoc_options opt = opt_in ? *opt_in : defaults();
  int rc = check_dims(1, d, m, N, opt.precision);
  if (rc) return rc;
  if (!H0 || !Hc || !u) return fail(QOC_ERR_ARG, "H0, Hc and u must be non-null");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(QOC_ERR_ARG, "dt must be finite and > 0");
  if ((flags & qoc::RUN_FID) && (!V || !F)) return fail(QOC_ERR_ARG, "V and F must be non-null");
  if ((flags & qoc::RUN_GRAD) && !grad) return fail(QOC_ERR_ARG, "grad must be non-null");
  if (!(flags & qoc::RUN_FID) && !XN) return fail(QOC_ERR_ARG, "U_total must be non-null");
  if (opt.validate) {
    rc = validate_host(d, m, N, H0, Hc, u, V, opt.generators != 0);
    if (rc) return rc;
  }
  const size_t dd = (size_t)d * d;
  const size_t ws_bytes = make_layout(1, d, m, N, opt.precision, opt.chunk, opt.hbm_budget).total;
  DevBufs bufs;
  void* dH0 = bufs.alloc(dd * 16);
  void* dHc = bufs.alloc(dd * 16 * m);
  void* du = bufs.alloc((size_t)m * N * 8);
  void* dV = V ? bufs.alloc(dd * 16) : nullptr;
  void* dF = bufs.alloc(8);
  void* dgrad = grad ? bufs.alloc((size_t)m * N * 8) : nullptr;
  void* dXN = XN ? bufs.alloc(dd * 16) : nullptr;
  void* dws = bufs.alloc(ws_bytes);
  void* ddiag = opt.diagnostics ? bufs.alloc(4 * sizeof(double)) : nullptr;
  if (!dH0 || !dHc || !du || (V && !dV) || !dF || (grad && !dgrad) || (XN && !dXN) || !dws)
    return fail(QOC_ERR_OOM, "device allocation of %zu workspace bytes failed", ws_bytes);
  hipStream_t st = static_cast<hipStream_t>(opt.stream);
  hipError_t e = hipSuccess;
  e = e ? e : hipMemcpyAsync(dH0, H0, dd * 16, hipMemcpyHostToDevice, st);
  e = e ? e : hipMemcpyAsync(dHc, Hc, dd * 16 * m, hipMemcpyHostToDevice, st);
  e = e ? e : hipMemcpyAsync(du, u, (size_t)m * N * 8, hipMemcpyHostToDevice, st);
  if (V) e = e ? e : hipMemcpyAsync(dV, V, dd * 16, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return fail(QOC_ERR_DEVICE, "upload: %s", hipGetErrorString(e));
  qoc_options o2 = opt;
  o2.diagnostics = static_cast<double*>(ddiag);
  rc = run_dev(1, d, m, N, dH0, dHc, du, dt, dV, dF, dgrad, dXN, dws, ws_bytes, &o2, flags);
  if (rc) return rc;
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(QOC_ERR_DEVICE, "execution: %s", hipGetErrorString(e));
  if (F) e = e ? e : hipMemcpy(F, dF, 8, hipMemcpyDeviceToHost);
  if (grad) e = e ? e : hipMemcpy(grad, dgrad, (size_t)m * N * 8, hipMemcpyDeviceToHost);
  if (XN) e = e ? e : hipMemcpy(XN, dXN, dd * 16, hipMemcpyDeviceToHost);
  if (ddiag) e = e ? e : hipMemcpy(opt.diagnostics, ddiag, 4 * sizeof(double), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(QOC_ERR_DEVICE, "download: %s", hipGetErrorString(e));
  return QOC_OK;
}

// ---------------------------------------------------------------- stage timing

struct StageTimer {
  std::mutex mu;
  bool on = false;
  struct Rec {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  hipEvent_t open[qoc::ST_ALL] = {};
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};

StageTimer& timer() {
  static StageTimer t;
  return t;
}

}  // namespace

namespace qoc {
void set_last_error(const char* msg) { g_err = msg; }

void stage_mark(int stage, bool begin, hipStream_t st) {
  StageTimer& T = timer();
  if (!T.on) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
  std::lock_guard<std::mutex> lk(T.mu);
  hipEvent_t e = T.get();
  if (!e) return;
  if (hipEventRecord(e, st) != hipSuccess) {
    T.pool.push_back(e);
    return;
  }
  if (begin) {
    if (T.open[stage]) T.pool.push_back(T.open[stage]);
    T.open[stage] = e;
  } else if (T.open[stage]) {
    T.recs.push_back({stage, T.open[stage], e});
    T.open[stage] = nullptr;
  } else {
    T.pool.push_back(e);
  }
}
}  // namespace qoc

extern "C" {

int qoc_stage_timing(int enable) {
  timer().on = enable != 0;
  return QOC_OK;
}

int qoc_stage_times(int n, double* ms, int64_t* launches) {
  StageTimer& T = timer();
  std::lock_guard<std::mutex> lk(T.mu);
  for (int i = 0; i < n; ++i) {
    if (ms) ms[i] = 0;
    if (launches) launches[i] = 0;
  }
  int rc = QOC_OK;
  for (auto& r : T.recs) {
    float t = 0;
    hipError_t e = hipEventSynchronize(r.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&t, r.a, r.b);
    if (e != hipSuccess) rc = fail(QOC_ERR_DEVICE, "stage timing: %s", hipGetErrorString(e));
    if (r.stage < n) {
      if (ms) ms[r.stage] += t;
      if (launches) launches[r.stage] += 1;
    }
    T.pool.push_back(r.a);
    T.pool.push_back(r.b);
  }
  T.recs.clear();
  return rc;
}

const char* qoc_stage_name(int stage) {
  static const char* names[] = {"prep", "plan", "expm", "scan", "carry", "mc", "bscan", "adjoint",
                                "state_chain", "state_grad"};
  return (stage >= 0 && stage < qoc::ST_ALL) ? names[stage] : "";
}


void qoc_default_options(qoc_options* opt) {
  if (!opt) return;
  memset(opt, 0, sizeof *opt);
  opt->precision = QOC_FP64;
  opt->validate = 0;
  opt->hbm_budget = 0;
  opt->reunitarise_tol = 0.0;
  opt->diagnostics = nullptr;
  opt->stream = nullptr;
  opt->chunk = 0;
  opt->dense_controls = 0;
  opt->generators = 0;
}

int qoc_propagate(int d, int m, int N, const qoc_z* H0, const qoc_z* Hc, const double* u, double dt,
                  qoc_z* U_total, const qoc_options* opt) {
  return run_host(d, m, N, H0, Hc, u, dt, nullptr, nullptr, nullptr, U_total, opt, 0);
}

int qoc_fidelity(int d, int m, int N, const qoc_z* H0, const qoc_z* Hc, const double* u, double dt,
                 const qoc_z* V, double* F, const qoc_options* opt) {
  return run_host(d, m, N, H0, Hc, u, dt, V, F, nullptr, nullptr, opt, qoc::RUN_FID);
}

int qoc_gradient(int d, int m, int N, const qoc_z* H0, const qoc_z* Hc, const double* u, double dt,
                 const qoc_z* V, double* F, double* grad, const qoc_options* opt) {
  return run_host(d, m, N, H0, Hc, u, dt, V, F, grad, nullptr, opt,
                  qoc::RUN_FID | qoc::RUN_BWD | qoc::RUN_GRAD);
}

int qoc_engine_chunk(int d, int N) {
  if (d < 1 || d > 128 || N < 1) return 0;
  return qoc::engine_chunk(N);
}

int qoc_default_chunk(int d, int N) {
  if (d < 1 || d > 128 || N < 1) return 0;
  return qoc::default_chunk(qoc::padded_dim(d), N);
}

size_t qoc_workspace_size(int B, int d, int m, int N, int precision, int chunk, uint64_t hbm_budget) {
  if (check_dims(B, d, m, N, precision)) return 0;
  return make_layout(B, d, m, N, precision, chunk, hbm_budget).total;
}

int qoc_propagate_dev(int B, int d, int m, int N, const void* H0, const void* Hc, const void* u, double dt,
                      void* U_total, void* workspace, size_t ws_bytes, const qoc_options* opt) {
  if (!U_total) return fail(QOC_ERR_ARG, "U_total must be non-null");
  return run_dev(B, d, m, N, H0, Hc, u, dt, nullptr, nullptr, nullptr, U_total, workspace, ws_bytes, opt, 0);
}

int qoc_fidelity_dev(int B, int d, int m, int N, const void* H0, const void* Hc, const void* u, double dt,
                     const void* V, void* F, void* workspace, size_t ws_bytes, const qoc_options* opt) {
  return run_dev(B, d, m, N, H0, Hc, u, dt, V, F, nullptr, nullptr, workspace, ws_bytes, opt, qoc::RUN_FID);
}

int qoc_gradient_dev(int B, int d, int m, int N, const void* H0, const void* Hc, const void* u, double dt,
                     const void* V, void* F, void* grad, void* workspace, size_t ws_bytes,
                     const qoc_options* opt) {
  return run_dev(B, d, m, N, H0, Hc, u, dt, V, F, grad, nullptr, workspace, ws_bytes, opt,
                 qoc::RUN_FID | qoc::RUN_BWD | qoc::RUN_GRAD);
}

int qoc_trace_gradient_dev(int B, int d, int m, int N, const void* H0, const void* Hc, const void* u, double dt,
                           const void* V, void* g, void* dg, void* workspace, size_t ws_bytes,
                           const qoc_options* opt) {
  if (!g || !dg) return fail(QOC_ERR_ARG, "g and dg must be non-null");
  return run_dev(B, d, m, N, H0, Hc, u, dt, V, nullptr, dg, nullptr, workspace, ws_bytes, opt,
                 qoc::RUN_FID | qoc::RUN_BWD | qoc::RUN_GRAD | qoc::RUN_RAWDG, g);
}

int qoc_gradient_dev_noalloc(int B, int d, int m, int N, const void* H0, const void* Hc, const void* u, double dt,
                             const void* V, void* F, void* grad, const qoc_options* opt_in) {
  const qoc_options opt = opt_in ? *opt_in : defaults();
  int rc = check_dims(B, d, m, N, opt.precision);
  if (rc) return rc;
  const size_t need = make_layout(B, d, m, N, opt.precision, opt.chunk, opt.hbm_budget).total;
  if (need > QOC_NOALLOC_SCRATCH_BYTES)
    return fail(QOC_ERR_ARG,
                "the call needs %zu bytes of workspace; the static scratch holds %llu (pass a smaller batch or "
                "N, an hbm_budget, or use qoc_gradient_dev with a workspace)",
                need, (unsigned long long)QOC_NOALLOC_SCRATCH_BYTES);
  void* ws = scratch_ptr();
  if (!ws) return QOC_ERR_DEVICE;
  return run_dev(B, d, m, N, H0, Hc, u, dt, V, F, grad, nullptr, ws, QOC_NOALLOC_SCRATCH_BYTES, &opt,
                 qoc::RUN_FID | qoc::RUN_BWD | qoc::RUN_GRAD);
}

int qoc_slice_plan(int d, int m, int N, const qoc_z* H0, const qoc_z* Hc, const double* u, double dt,
                   int precision, int with_gradient, int32_t* plan) {
  if (d < 1 || m < 1 || N < 1 || !H0 || !Hc || !u || !plan || !(dt > 0))
    return fail(QOC_ERR_ARG, "invalid arguments to qoc_slice_plan");
  if (precision != QOC_FP64 && precision != QOC_FP32 && precision != QOC_BF16X3)
    return fail(QOC_ERR_UNSUPPORTED, "precision %d is not available", precision);
  const double ur = precision == QOC_FP64 ? 0x1p-53 : 0x1p-24;
  const bool ps_expm = precision == QOC_FP32 && qoc::padded_dim(d) == 128;  // as the kernels
  auto norm1 = [d](const qoc_z* H) {
    double best = 0;
    for (int b = 0; b < d; ++b) {
      double s = 0;
      for (int a = 0; a < d; ++a) s += sqrt(fma(H[a * d + b].re, H[a * d + b].re, H[a * d + b].im * H[a * d + b].im));
      best = std::max(best, s);
    }
    return best;
  };
  std::vector<double> nrm(m + 1);
  nrm[0] = norm1(H0);
  for (int j = 0; j < m; ++j) nrm[j + 1] = norm1(Hc + (size_t)j * d * d);
  for (int k = 0; k < N; ++k) {
    double th = nrm[0];
    for (int j = 0; j < m; ++j) th = fma(fabs(u[(size_t)j * N + k]), nrm[j + 1], th);
    th *= dt;
    qoc::SlicePlan p = qoc::choose_plan(th, ur, with_gradient != 0, ps_expm);
    plan[3 * k] = p.s;
    plan[3 * k + 1] = p.q;
    plan[3 * k + 2] = p.qb;
  }
  return QOC_OK;
}

const char* qoc_last_error(void) { return g_err.c_str(); }

const char* qoc_version(void) { return "libqoc 0.1.0 (gfx950)"; }

}  // extern "C"
