// Internal types shared by the libqoc host code and its kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>

namespace qoc {

// One GRAPE problem as the kernels see it.  Pointers marked (user) point into
// caller memory; the rest point into the workspace.  Matrices of the compute
// precision T live in one of two internal layouts: "planar" (row-major D x D
// real plane followed by the imaginary plane, zero-padded from d to D) or
// "PF" (the register order of a wavefront panel, see qoc_device.hpp).
struct ProbDesc {
  int d, D, m, N;  // true dimension, padded dimension, controls, slices
  int L, P;        // slices per scan chunk, number of chunks
  int CG, PG;      // chunks per carry group, number of carry groups
  int flags, pad_;
  double dt;
  const double* H0z;  // (user) d*d complex128, interleaved
  const double* Hcz;  // (user) m*d*d complex128
  const double* u;    // (user) m*N
  const double* Vz;   // (user) d*d complex128 target, or null
  double* F;          // (user or workspace) fidelity
  double* grad;       // (user) m*N gradient, or null
  double* XN;         // (user) d*d complex128 total propagator, or null
  void* Hint;         // (m+1) planar matrices: [0] = H0, [1 + j] = Hc[j]
  void* Vint;         // PF matrix: V
  double* norms;      // m+1 one-norms of H0, Hc[j] (FP64)
  int* mcol;          // m*D: column of the nonzero of row a of Hc[j] (a if the row is empty)
  void* mval;         // m*D complex values (re, im) of those entries, in precision T
  int* mok;           // m flags: bit 0, Hc[j] has at most one nonzero per row (dense kernels not
                      // forced); bit 1, also a bijection from rows to columns (a permutation
                      // with weights: Pauli strings)
  int* minv;          // m*D: row a with col_j(a) = b, valid where mok bit 1 is set (null where
                      // no layout holds it)
  int* sq;            // per slice: s | q << 8 | qb << 16
  void* delta;        // N PF matrices: U_k - I
  void* hk;           // N matrices kept by the expm pass for the adjoint (D >= 32): planar H_k
                      // at D <= 64, X = A_k / 2^s in PF layout at D = 128
  void* x2;           // N PF matrices kept by the expm pass for the adjoint (D >= 32, FP32): (A_k / 2^s)^2
  void* xprev;        // N PF matrices: U_{k-1} ... U_{k0}   (I at a chunk start)
  void* bloc;         // N PF matrices: U_{k+1}^dag ... U_{k1-1}^dag mc[c] (mc[c] at a chunk end)
  void* tf;           // P PF matrices: forward chunk totals (their conjugate transposes are the backward ones)
  void* cf;           // P PF matrices: forward carry into each chunk
  void* cb;           // P PF matrices: backward carry out of each chunk
  void* mc;           // P PF matrices: cb[c] cf[c]^dag
  void* grp;          // 4 x PG PF matrices: forward and backward group totals, then the
                      // forward and backward carries into each group
  double* g;          // complex128 Tr(V^dag X_N)
  double* diag;       // [0] ||X_N^dag X_N - I||_F; [1] largest chunk residual (FP64
                      // bits, atomic max); [2] re-unitarisation steps (uint64 count)
  double reun_tol;    // re-unitarisation threshold for chunk totals, < 0: off
  // state-to-state path (qoc_state_*): XN above receives psi_N (d complex128)
  const double* psi0z;  // (user) d complex128 initial state, or null
  const double* chiz;   // (user) d complex128 target state, or null
  void* psi;            // N + 1 vectors of D complex T: psi_0 .. psi_N
  void* lam;            // N + 1 vectors of D complex T: lam_0 .. lam_N
};

enum : int {
  RUN_BWD = 1,   // backward scans (needed for the gradient)
  RUN_GRAD = 2,  // adjoint pass and gradient
  RUN_FID = 4,   // fidelity against V
  CTRL_DENSE = 8,  // always the dense control kernels (qoc_options.dense_controls)
  RUN_RAWDG = 16,  // write dg/du[j][k] = d Tr(V^dag X_N) / du[j][k] (complex) instead of dF/du
  RUN_GENERAL = 32,  // H0, Hc are general generators G (stored as i G; see prep_one)
};

// A launch over many problems that share d (and hence D) and the precision.
// When every problem has the same N (and therefore the same chunk count),
// uniformN / uniformP are those values and the start arrays are unused;
// otherwise slice_start / chunk_start are exclusive prefix sums on the device.
struct Launch {
  const ProbDesc* descs;  // device array of nprob descriptors
  int nprob;
  int uniformN, uniformP;
  const int* slice_start;  // device, nprob + 1 entries (or null)
  const int* chunk_start;  // device, nprob + 1 entries (or null)
  int total_slices, total_chunks;
  int max_m;
  int flags;
  hipStream_t stream;
  void* scratch;  // D = 128 only: kScratchSlots per-workgroup regions of kScratchMats matrices
  // Engine launches: item counts and prefix sums in device memory (see Work)
  // and a fixed persistent grid size; null / 0 for API launches.
  const int* dyn;
  int dyn_grid;
};

// D = 128 kernels run persistent grids of at most kScratchSlots workgroups;
// each owns kScratchMats stored matrices of scratch in the workspace.
constexpr int kScratchSlots = 256;
constexpr int kScratchMats = 6;

// Stages of the path, for the optional per-stage event timing.
enum Stage : int { ST_PREP = 0, ST_PLAN, ST_EXPM, ST_SCAN, ST_CARRY, ST_MC, ST_BSCAN, ST_ADJ, ST_COUNT };
// Stages of the state-to-state path (timed only; not part of the engine's graph).
enum : int { ST_SCHAIN = ST_COUNT, ST_SGRAD, ST_ALL };
void stage_mark(int stage, bool begin, hipStream_t st);

// Sub-range of a uniform launch: slices [s_lo, s_lo + s_n) and chunks
// [c_lo, c_lo + c_n) of every problem (s_n / c_n = 0: all, from the start
// arrays); the per-slice arrays delta / xprev / bloc hold slices from kbase
// on (checkpointed segments keep only a window of them).  recompute marks
// the second sweep of a checkpointed call, whose forward scans only rebuild
// the local products: their chunk totals were checked, stored and consumed by
// the carry in the first sweep, so the re-unitarisation check is not repeated.
struct Range {
  int s_lo, s_n, c_lo, c_n, kbase;
  int recompute;
};

// Work items of one kernel launch.  API launches pass nprob / total / start
// by value (start = null with a uniform range); engine launches replayed from
// a captured graph read them from device memory instead:
// dyn[0] = nprob, dyn[1] = total items, dyn[2 .. 2 + nprob] = item prefix
// sums, dyn[3 + nprob .. 3 + 2 nprob) = index of each problem in descs.
struct Work {
  const ProbDesc* descs;
  int nprob, total;
  const int* start;
  Range rg;
  const int* dyn;
};

// Message returned by qoc_last_error() on the calling thread.
void set_last_error(const char* msg);

// Enqueue one stage of the path.  Returns a hipError_t.
hipError_t launch_stage(int precision, int D, int stage, const Launch& L, const Range& rg);

// ---------------------------------------------------------------- workspace layout

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

inline int padded_dim(int d) {
  if (d <= 16) return 16;
  if (d <= 32) return 32;
  if (d <= 64) return 64;
  return 128;
}

inline size_t elem_size(int precision) { return precision == 0 ? 8 : 4; }

// Default slices per scan chunk.  The scans' dependency depth is about
// 2 L + (carry depth), with the grouped carry 2 L + 2 sqrt(N / L).  For
// D <= 64, L = ceil(sqrt(N / 2)) keeps the batched throughput of
// L = ceil(sqrt(N)) while shortening a single problem's chain.  D = 128 keeps
// ceil(sqrt(N)): its scans run on at most 256 workgroups (one scratch slot
// each), and the extra chunks of a shorter L cost batches a second round.
inline int default_chunk(int D, int N) {
  return std::max(1, (int)ceil(sqrt(D == 128 ? (double)N : 0.5 * N)));
}

// Slices per scan chunk of a serving-engine request: ceil(sqrt(N / 8)).  A
// tick holds few problems, so the chain of a request bounds its latency
// (about 2 L + 2 sqrt(N / L) dependent products): shorter chunks than the
// batch default cut it (one problem, d = 64, N = 2000: 0.70 -> 0.61 ms;
// d = 128, N = 1000: 5.45 -> 4.42 ms), at a cost of about 2% in throughput
// at batch 32.
inline int engine_chunk(int N) { return std::max(1, (int)ceil(sqrt(N / 8.0))); }

// The carry over the P chunk totals runs in groups of CG =
// ceil(sqrt(P)) chunks: a serial chain inside every group, one over the PG
// group totals, then one combination per chunk, so that its depth is about
// 2 sqrt(P) + 3 products instead of P.
inline void carry_groups(int P, int& CG, int& PG) {
  CG = std::max(1, (int)ceil(sqrt((double)P)));
  PG = (P + CG - 1) / CG;
}

// Byte offsets of one problem's workspace regions, and the total size.
struct Layout {
  int D, L, P;
  int esize;  // bytes of one real element of the compute precision
  int CG, PG;  // carry groups (carry_groups)
  int G;  // chunks per checkpoint segment (G = P: everything stored, no recompute)
  int W;  // slices held by the per-slice arrays (N, or G * L when segmented)
  size_t desc_bytes;  // descriptor table at the start of the workspace
  size_t Hint, Vint, norms, mono, sq, delta, hk, x2, xprev, bloc, tf, cf, cb, mc, grp, small;
  int per_slice;  // per-slice arrays: delta, xprev, bloc, hk at D >= 32, x2 at D >= 32 in FP32
                  // (null in the descriptor where absent)
  size_t per_prob;
  size_t scratch, scratch_bytes;  // D = 128: per-workgroup scratch after the problems
  size_t total;
};

// hbm_budget (bytes, 0 = unlimited) bounds the stored propagators of the
// batch: the per-slice arrays (three stored propagators, and the slice
// Hamiltonians and, in FP32, the squares (A_k / 2^s)^2 at D >= 32) plus the four per-chunk and four per-group arrays.  When the
// full arrays do not fit, slices are processed in segments of G chunks whose
// per-slice arrays are recomputed for the adjoint pass (sqrt(N)
// checkpointing: with L of order sqrt(N) and G = 1 the storage is O(sqrt(N))).
inline Layout make_layout(int B, int d, int m, int N, int precision, int chunk, uint64_t hbm_budget) {
  Layout Lo;
  Lo.D = padded_dim(d);
  Lo.esize = (int)elem_size(precision);
  Lo.L = chunk > 0 ? std::min(chunk, N) : default_chunk(Lo.D, N);
  if (Lo.L < 1) Lo.L = 1;
  Lo.P = (N + Lo.L - 1) / Lo.L;
  carry_groups(Lo.P, Lo.CG, Lo.PG);
  const size_t mat = 2ull * Lo.D * Lo.D * elem_size(precision);
  Lo.G = Lo.P;
  // per-slice arrays: delta, xprev, bloc; hk at D >= 32; x2 at D >= 32 in FP32
  // (not for the split-BF16 adjoint, which the extra read does not speed up)
  Lo.per_slice = Lo.D >= 32 ? (precision == 1 /* QOC_FP32 */ ? 5 : 4) : 3;
  const double per_call = 4.0 * Lo.P + 4.0 * Lo.PG;  // per-chunk and per-group arrays, in matrices
  const double full = (double)B * ((double)Lo.per_slice * N + per_call) * (double)mat;
  if (hbm_budget > 0 && full > (double)hbm_budget) {
    const double avail = (double)hbm_budget / B - per_call * (double)mat;
    const double per_chunk = (double)Lo.per_slice * Lo.L * (double)mat;
    Lo.G = avail >= per_chunk ? (int)std::min<double>(Lo.P, floor(avail / per_chunk)) : 1;
  }
  Lo.W = Lo.G >= Lo.P ? N : std::min(N, Lo.G * Lo.L);
  size_t o = 0;
  Lo.Hint = o; o = align_up(o + (size_t)(m + 1) * mat);
  Lo.Vint = o; o = align_up(o + mat);
  Lo.norms = o; o = align_up(o + (size_t)(m + 1) * 8);
  Lo.mono = o; o = align_up(o + (size_t)m * Lo.D * (8 + 2 * elem_size(precision)) + (size_t)m * 4);
  Lo.sq = o; o = align_up(o + (size_t)N * 4);
  Lo.delta = o; o = align_up(o + (size_t)Lo.W * mat);
  Lo.hk = o; o = align_up(o + (Lo.per_slice >= 4 ? (size_t)Lo.W * mat : 0));
  Lo.x2 = o; o = align_up(o + (Lo.per_slice == 5 ? (size_t)Lo.W * mat : 0));
  Lo.xprev = o; o = align_up(o + (size_t)Lo.W * mat);
  Lo.bloc = o; o = align_up(o + (size_t)Lo.W * mat);
  Lo.tf = o; o = align_up(o + (size_t)Lo.P * mat);
  Lo.cf = o; o = align_up(o + (size_t)Lo.P * mat);
  Lo.cb = o; o = align_up(o + (size_t)Lo.P * mat);
  Lo.mc = o; o = align_up(o + (size_t)Lo.P * mat);
  Lo.grp = o; o = align_up(o + 4 * (size_t)Lo.PG * mat);
  Lo.small = o; o = align_up(o + 128);
  Lo.per_prob = o;
  Lo.desc_bytes = align_up((size_t)B * sizeof(ProbDesc));
  Lo.scratch = Lo.desc_bytes + (size_t)B * Lo.per_prob;
  Lo.scratch_bytes = Lo.D == 128 ? (size_t)qoc::kScratchSlots * qoc::kScratchMats * mat : 0;
  Lo.total = Lo.scratch + Lo.scratch_bytes;
  return Lo;
}


// Descriptor of one problem whose workspace region starts at pb (layout Lo).
// Input and output pointers may be null where the launch does not use them.
inline void fill_desc(ProbDesc& P, const Layout& Lo, char* pb, int d, int m, int N, double dt, int flags,
                      const double* H0, const double* Hc, const double* u, const double* V, double* F, double* grad,
                      double* XN, double reun_tol = -1.0, double* diag = nullptr) {
  memset(&P, 0, sizeof P);
  P.d = d;
  P.D = Lo.D;
  P.m = m;
  P.N = N;
  P.L = Lo.L;
  P.P = Lo.P;
  P.CG = Lo.CG;
  P.PG = Lo.PG;
  P.flags = flags;
  P.dt = dt;
  P.H0z = H0;
  P.Hcz = Hc;
  P.u = u;
  P.Vz = V;
  P.grad = grad;
  P.XN = XN;
  P.Hint = pb + Lo.Hint;
  P.Vint = V ? pb + Lo.Vint : nullptr;
  P.norms = reinterpret_cast<double*>(pb + Lo.norms);
  P.mval = pb + Lo.mono;
  P.mcol = reinterpret_cast<int*>(pb + Lo.mono + (size_t)m * Lo.D * 2 * Lo.esize);
  P.mok = P.mcol + (size_t)m * Lo.D;
  P.minv = P.mok + m;
  P.sq = reinterpret_cast<int*>(pb + Lo.sq);
  P.delta = pb + Lo.delta;
  P.hk = Lo.per_slice >= 4 ? pb + Lo.hk : nullptr;
  P.x2 = Lo.per_slice == 5 ? pb + Lo.x2 : nullptr;
  P.xprev = pb + Lo.xprev;
  P.bloc = pb + Lo.bloc;
  P.tf = pb + Lo.tf;
  P.cf = pb + Lo.cf;
  P.cb = pb + Lo.cb;
  P.mc = pb + Lo.mc;
  P.grp = pb + Lo.grp;
  double* small = reinterpret_cast<double*>(pb + Lo.small);
  P.g = small;                    // 2 doubles
  P.F = F ? F : small + 2;        // 1 double
  P.diag = diag ? diag : small + 4;  // 4 doubles
  P.reun_tol = reun_tol;
}

}  // namespace qoc
