/*
 * libqoc: piecewise-constant quantum optimal control (GRAPE) on AMD MI355X.
 *
 * The problem (GRAPE, Khaneja et al., J. Magn. Reson. 172 (2005); hbar = 1):
 *
 *   H_k  = H0 + sum_{j<m} u[j*N + k] * Hc[j]         slice Hamiltonian, k = 0..N-1
 *   U_k  = exp(-i * dt * H_k)                          slice propagator
 *   X_N  = U_{N-1} ... U_1 U_0                         slice 0 acts first
 *   g    = Tr(V^dag X_N),   F = |g|^2 / d^2            phase-insensitive fidelity
 *   grad[j*N + k] = dF / du[j*N + k]                   exact derivative of the
 *                                                      piecewise-constant model
 *
 * Matrices are d x d, row-major, complex interleaved (re, im) in double
 * precision (qoc_z).  H0 and every Hc[j] must be Hermitian and V unitary.
 * u and grad are m x N row-major doubles.  Supported sizes: 1 <= d <= 128,
 * m >= 1, N >= 1.
 *
 * Ownership: the caller owns every buffer; the library keeps no pointer to
 * caller memory after a call returns.  Host entry points (no _dev suffix) take
 * host pointers, allocate and free their own device memory, and return when
 * the results are in the host buffers.  _dev entry points take device pointers
 * and a caller-provided device workspace, enqueue all work on opt->stream
 * (NULL: the default stream) and return without waiting; outputs are valid
 * once that stream has completed.
 *
 * Errors: every entry point returns QOC_OK (0) or a negative qoc_status.  On
 * error nothing has been launched and the outputs are untouched;
 * qoc_last_error() then returns a message for the calling thread.  No entry
 * point aborts or throws across this boundary.
 */
#ifndef QOC_H
#define QOC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  double re, im;
} qoc_z; /* complex128, interleaved */

typedef enum {
  QOC_OK = 0,
  QOC_ERR_ARG = -1,           /* bad size, NULL pointer, dt <= 0, workspace too small */
  QOC_ERR_NOT_HERMITIAN = -2, /* validate != 0 and H0 or some Hc[j] is not Hermitian */
  QOC_ERR_NONFINITE = -3,     /* validate != 0 and an input holds NaN or Inf */
  QOC_ERR_OOM = -4,           /* device allocation failed (host entry points) */
  QOC_ERR_DEVICE = -5,        /* a HIP runtime call or kernel launch failed */
  QOC_ERR_UNSUPPORTED = -6,   /* d > 128 or an unknown precision */
  QOC_ERR_NOT_UNITARY = -7    /* validate != 0 and |V^dag V - I|_max > 1e-8, or a state
                                 whose norm differs from 1 by more than 1e-8 */
} qoc_status;

typedef enum {
  QOC_FP64 = 0,  /* complex128 GEMMs on FP64 MFMA */
  QOC_FP32 = 1,  /* complex64 GEMMs on FP32 MFMA; norms, traces and inner products in FP64 */
  QOC_BF16X3 = 2 /* the adjoint's complex products (the Frechet series and its traces)
                    as three split-BF16 MFMA products (hi*hi + hi*lo + lo*hi) with FP32
                    accumulation; propagators, scans and carries as QOC_FP32; FP32
                    storage; FP64 norms, traces and inner products; 17 <= d <= 64 */
} qoc_precision;

typedef struct {
  int32_t precision;      /* qoc_precision; default QOC_FP64 */
  int32_t validate;       /* nonzero: host entry points (no _dev suffix) check that every
                             input is finite, that H0 and each Hc[j] are Hermitian
                             (|H - H^dag|_max <= 1e-12 max(1, |H|_max)) and that V is
                             unitary (|V^dag V - I|_max <= 1e-8), before any device
                             work.  The _dev entry points never read their inputs on
                             the host and ignore it: a non-Hermitian or non-finite
                             input gives unspecified results there, never an error. */
  uint64_t hbm_budget;    /* bytes for the per-slice and per-chunk arrays of a call
                             (stored propagators, and at d > 16 the slice
                             Hamiltonians and, in QOC_FP32, the squares
                             (A_k / 2^s)^2 kept for the adjoint); 0 = no limit.
                             When those arrays exceed it, slices are
                             processed in checkpoint segments and recomputed
                             for the gradient pass (same results, more work).
                             The floor is one chunk of slices per segment plus
                             the per-chunk arrays: a smaller budget is raised to
                             it (qoc_workspace_size reports the actual size). */
  double reunitarise_tol; /* reduced precision: every chunk product S of the
                             scans is checked in FP64, r = |S^dag S - I|_F, and gets one
                             Newton-Schulz step S (3I - S^dag S)/2 when r exceeds it.
                             0 = default: a step on every chunk product (removing the
                             non-unitary part of the rounding error keeps Tr(V^dag X_N)
                             about ten times more accurate); < 0 disables; never
                             applied in FP64. */
  void* stream;           /* hipStream_t for _dev calls; NULL = default stream */
  int32_t chunk;          /* slices per scan chunk; 0 = qoc_default_chunk(d, N) */
  int32_t dense_controls; /* 0 (default): when every control Hc[j] has at most one
                             nonzero per row (Pauli strings, for instance), the slice
                             Hamiltonians are assembled and (except FP64 at d > 64)
                             the gradient's inner products Tr(Z_k^dag Hc[j]) taken
                             entry by entry, O(d) per control instead of O(d^2),
                             with the same terms; nonzero: always the dense kernels */
  double* diagnostics;    /* optional, 4 doubles per problem (device memory for _dev calls,
                             host memory for host calls): [0] |X_N^dag X_N - I|_F,
                             [1] largest chunk residual r, [2] number of Newton-Schulz
                             steps (integer stored as uint64 bits), [3] unused */
  int32_t generators;     /* 0 (default): H0 and Hc[j] are Hermitian Hamiltonians and
                             U_k = exp(-i dt H_k).  Nonzero: they are general complex
                             generators G0, G[j] (no symmetry assumed) and the slice map is
                             S_k = exp(dt (G0 + sum_j u[j*N + k] G[j])); X_N, g, F and the
                             exact gradient are defined as above with U_k replaced by S_k.
                             Open-system (Lindblad) dynamics in Liouville space is this
                             case, with d the Liouville dimension.  The re-unitarisation
                             check is off, validate checks finiteness only, and the
                             unitary (qoc_propagate/fidelity/gradient[_dev], noalloc,
                             trace) entry points take it; the state and engine ones do not. */
} qoc_options; /* pass NULL for all defaults */

/* Fill *opt with the defaults listed above. */
void qoc_default_options(qoc_options* opt);

/*
 * Total propagator X_N = U_{N-1} ... U_0 (defined above).
 * H0: d*d, Hc: m*d*d (control j at Hc + j*d*d), u: m*N, U_total: d*d output.
 */
int qoc_propagate(int d, int m, int N, const qoc_z* H0, const qoc_z* Hc, const double* u,
                  double dt, qoc_z* U_total, const qoc_options* opt);

/* Fidelity F = |Tr(V^dag X_N)|^2 / d^2 against the d*d target V. */
int qoc_fidelity(int d, int m, int N, const qoc_z* H0, const qoc_z* Hc, const double* u,
                 double dt, const qoc_z* V, double* F, const qoc_options* opt);

/* F and its exact gradient grad[j*N + k] = dF/du[j*N + k] (m*N output). */
int qoc_gradient(int d, int m, int N, const qoc_z* H0, const qoc_z* Hc, const double* u,
                 double dt, const qoc_z* V, double* F, double* grad, const qoc_options* opt);

/*
 * Batched device entry points: B independent problems with the same d, m, N
 * and dt, stored back to back in device memory:
 *   H0 [B][d][d], Hc [B][m][d][d], u [B][m][N], V [B][d][d]  (qoc_z / double),
 *   F [B], grad [B][m][N], U_total [B][d][d].
 * workspace must hold qoc_workspace_size(B, d, m, N, opt->precision, opt->chunk,
 * opt->hbm_budget) bytes of device memory (0 for invalid sizes), 256-byte
 * aligned; its contents need no initialisation and are clobbered.  Calls that
 * share a workspace must be ordered on one stream.
 */
size_t qoc_workspace_size(int B, int d, int m, int N, int precision, int chunk, uint64_t hbm_budget);

/*
 * Default slices per scan chunk (opt->chunk = 0): ceil(sqrt(N / 2)) for
 * d <= 64, ceil(sqrt(N)) for 64 < d <= 128.  The carry over the chunk totals
 * runs in groups of ceil(sqrt(chunks)), so a problem's chain of dependent
 * products is about 2 chunk + 2 sqrt(chunks) long.  0 for d outside [1, 128]
 * or N < 1.
 */
int qoc_default_chunk(int d, int N);

/*
 * Slices per scan chunk that the serving engine uses for a request:
 * ceil(sqrt(N / 8)), shorter than the default because a tick holds few
 * problems and the chain of dependent products then bounds a request's
 * latency.  A host or device call with opt->chunk set to it returns the
 * engine's results bit for bit.  0 for d outside [1, 128] or N < 1.
 */
int qoc_engine_chunk(int d, int N);

int qoc_propagate_dev(int B, int d, int m, int N, const void* H0, const void* Hc,
                      const void* u, double dt, void* U_total, void* workspace,
                      size_t ws_bytes, const qoc_options* opt);

int qoc_fidelity_dev(int B, int d, int m, int N, const void* H0, const void* Hc,
                     const void* u, double dt, const void* V, void* F, void* workspace,
                     size_t ws_bytes, const qoc_options* opt);

int qoc_gradient_dev(int B, int d, int m, int N, const void* H0, const void* Hc,
                     const void* u, double dt, const void* V, void* F, void* grad,
                     void* workspace, size_t ws_bytes, const qoc_options* opt);

/*
 * The complex trace and its derivative instead of F and dF/du:
 *   g[b] = Tr(V_b^dag X_N)  (complex128),  dg[b][j][k] = d g[b] / d u[b][j][k]  (complex128),
 * exact for the piecewise-constant model.  V need not be unitary: with V the
 * residual R = X_N - e^{i phi} V0 of a least-squares fit, Re(dg) is J^T r for
 * the real residual vector r = (Re vec R, Im vec R) and its Jacobian J in u;
 * with V = e_a e_b^T it is the row d(X_N)_ab / du of that Jacobian.  Same
 * layouts, options, workspace (qoc_workspace_size) and errors as
 * qoc_gradient_dev; g and dg are device memory of 2 B and 2 B m N doubles.
 */
int qoc_trace_gradient_dev(int B, int d, int m, int N, const void* H0, const void* Hc,
                           const void* u, double dt, const void* V, void* g, void* dg,
                           void* workspace, size_t ws_bytes, const qoc_options* opt);

/*
 * qoc_gradient_dev without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same batch layout, outputs, options and
 * results as qoc_gradient_dev (the same kernels on the same workspace layout),
 * but the workspace is a static device array of QOC_NOALLOC_SCRATCH_BYTES
 * bytes inside libqoc: one copy per GPU, looked up on the first call on that
 * device and held until the process ends.  The call allocates no device
 * memory.  A call whose qoc_workspace_size(B, d, m, N, opt->precision,
 * opt->chunk, opt->hbm_budget) exceeds QOC_NOALLOC_SCRATCH_BYTES returns
 * QOC_ERR_ARG before touching the device (a smaller batch, a smaller N or an
 * hbm_budget can bring it under).  Every call on one GPU shares that GPU's
 * array and keeps the last call's contents; every part of it that a kernel
 * reads is written earlier in the same call, so nothing needs clearing
 * between calls.  Calls that overlap on one GPU (different streams, or host
 * threads without ordering) race on it and must not be issued.
 */
#define QOC_NOALLOC_SCRATCH_BYTES (64ull << 20)

int qoc_gradient_dev_noalloc(int B, int d, int m, int N, const void* H0, const void* Hc,
                             const void* u, double dt, const void* V, void* F, void* grad,
                             const qoc_options* opt);

/*
 * State-to-state transfer (the state form of GRAPE in Khaneja et al. 2005):
 * the same slices act on a state instead of the identity,
 *
 *   psi_{k+1} = U_k psi_k  (psi_0 given),   g = <chi|psi_N> = sum_a conj(chi[a]) psi_N[a],
 *   F = |g|^2,   grad[j*N + k] = dF/du[j*N + k]  (exact derivative of the piecewise-constant model),
 *
 * with psi_0 and the target chi unit vectors of d complex entries (qoc_z).
 * No d x d propagator is formed: each slice is applied to a vector (and to
 * the costate lam_k = U_k^dag lam_{k+1}, lam_N = chi) by a Taylor polynomial
 * of the slice's plan (qoc_slice_plan), and the derivative is the plan's
 * truncated Frechet series taken between the costate and the state.  FP64
 * and FP32 only (QOC_BF16X3 returns QOC_ERR_UNSUPPORTED); opt->validate also
 * checks |psi0| = |chi| = 1 within 1e-8 (QOC_ERR_NOT_UNITARY otherwise);
 * chunk, hbm_budget, reunitarise_tol and diagnostics are ignored.
 *
 * Batched device forms: psi0 [B][d], chi [B][d], psiN [B][d] (qoc_z), F [B],
 * grad [B][m][N], the other inputs as for qoc_gradient_dev; workspace of
 * qoc_state_workspace_size(B, d, m, N, precision) bytes (0 for invalid sizes),
 * 256-byte aligned, contents clobbered; calls sharing it must be ordered on
 * one stream.  Errors as for the other entry points.
 */
size_t qoc_state_workspace_size(int B, int d, int m, int N, int precision);

int qoc_state_propagate(int d, int m, int N, const qoc_z* H0, const qoc_z* Hc, const double* u,
                        double dt, const qoc_z* psi0, qoc_z* psiN, const qoc_options* opt);

int qoc_state_gradient(int d, int m, int N, const qoc_z* H0, const qoc_z* Hc, const double* u,
                       double dt, const qoc_z* psi0, const qoc_z* chi, double* F, double* grad,
                       const qoc_options* opt);

int qoc_state_propagate_dev(int B, int d, int m, int N, const void* H0, const void* Hc,
                            const void* u, double dt, const void* psi0, void* psiN,
                            void* workspace, size_t ws_bytes, const qoc_options* opt);

int qoc_state_gradient_dev(int B, int d, int m, int N, const void* H0, const void* Hc,
                           const void* u, double dt, const void* psi0, const void* chi, void* F,
                           void* grad, void* workspace, size_t ws_bytes, const qoc_options* opt);

/*
 * Scaling exponent and Taylor degrees the kernels use for each slice of one
 * problem (host pointers): plan[3*k + 0] = s, plan[3*k + 1] = q (degree of
 * the exp series), plan[3*k + 2] = qb (degree of the Frechet block series).
 * theta_k = dt (|H0|_1 + sum_j |u[j*N + k]| |Hc[j]|_1) bounds |dt H_k|_1;
 * q and qb are the least degrees whose Taylor remainder bounds at
 * r = theta_k / 2^s are at most the unit roundoff of the precision, and s
 * minimises the number of complex matrix products (with_gradient selects the
 * count of the gradient path).  Returns QOC_OK or QOC_ERR_ARG.
 */
int qoc_slice_plan(int d, int m, int N, const qoc_z* H0, const qoc_z* Hc, const double* u,
                   double dt, int precision, int with_gradient, int32_t* plan);

/*
 * Per-stage kernel timing (diagnostics).  While enabled, every launch records
 * a pair of hipEvents on its stream around each stage of the path.
 * qoc_stage_times(n, ms, launches) waits for the recorded events, writes for
 * stages 0..n-1 the summed milliseconds and the number of timed launches, and
 * clears the record.  Stages: 0 prep, 1 plan, 2 expm, 3 scan (forward),
 * 4 carry, 5 mc, 6 bscan (backward scan), 7 adjoint, and for the state path
 * 8 state_chain (state and costate propagation), 9 state_grad (see
 * qoc_stage_name).
 * Returns QOC_OK or QOC_ERR_DEVICE.
 */
int qoc_stage_timing(int enable);
int qoc_stage_times(int n, double* ms, int64_t* launches);
const char* qoc_stage_name(int stage);

/*
 * Serving engine: continuous batching of forward + gradient requests of
 * mixed d and N (one precision per engine).
 *
 * Requests are queued by qoc_engine_submit (host inputs are copied into the
 * engine's pinned staging before it returns) and admitted in FIFO order
 * while their device footprint (qoc_engine_footprint: inputs, outputs and
 * the per-slice arrays of the path, about 5 N D^2 c bytes at D >= 32 in
 * QOC_FP32, 4 N D^2 c in the other precisions and 3 N D^2 c at D = 16, with
 * c the bytes of one complex element) fits the
 * engine's device pool and one of max_active descriptor slots is free.
 * Admitted requests are grouped by padded dimension D (16, 32, 64, 128); each
 * group has its own stream and a captured graph of the path's kernels that a
 * tick replays for every request admitted to the group since its previous
 * tick.  qoc_engine_step harvests finished ticks, admits queued requests
 * and starts ticks on idle groups (wait != 0: if nothing has finished,
 * block until one tick does).  qoc_engine_poll returns up to max finished
 * request ids with their fidelities; qoc_engine_fetch copies a finished
 * request's gradient (m*N doubles, may be NULL) and releases its staging.
 * Submitting more than the staging holds returns QOC_ERR_OOM; a request
 * larger than the device pool is rejected with QOC_ERR_OOM at submit.
 * Engine calls are serialised by an internal lock.  Stage timing does not
 * cover engine launches.
 */
typedef struct qoc_engine qoc_engine;

uint64_t qoc_engine_footprint(int precision, int d, int m, int N);
int qoc_engine_create(int precision, uint64_t pool_bytes, uint64_t host_bytes, int max_active,
                      qoc_engine** engine);
int qoc_engine_destroy(qoc_engine* engine);
int qoc_engine_submit(qoc_engine* engine, int d, int m, int N, const qoc_z* H0, const qoc_z* Hc,
                      const double* u, double dt, const qoc_z* V, int64_t* id);
int qoc_engine_step(qoc_engine* engine, int wait);
int qoc_engine_poll(qoc_engine* engine, int max, int64_t* ids, double* F, int* n);
int qoc_engine_fetch(qoc_engine* engine, int64_t id, double* grad);
int qoc_engine_stats(qoc_engine* engine, int64_t* queued, int64_t* active, uint64_t* pool_used);

/* Message for the last non-OK status returned on the calling thread. */
const char* qoc_last_error(void);

/* Library version string. */
const char* qoc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* QOC_H */
