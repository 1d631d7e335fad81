// Internal types shared by the libqoc host code and its kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace qoc {

// One GRAPE problem as the kernels see it.  Pointers marked (user) point into
// caller memory; the rest point into the workspace.  Matrices of the compute
// precision T live in one of two internal layouts: "planar" (row-major D x D
// real plane followed by the imaginary plane, zero-padded from d to D) or
// "PF" (the register order of a wavefront panel, see qoc_device.hpp).
struct ProbDesc {
  int d, D, m, N;  // true dimension, padded dimension, controls, slices
  int L, P;        // slices per scan chunk, number of chunks
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
  int* sq;            // per slice: s | q << 8 | qb << 16
  void* delta;        // N PF matrices: U_k - I
  void* xprev;        // N PF matrices: U_{k-1} ... U_{k0}   (I at a chunk start)
  void* bloc;         // N PF matrices: U_{k+1}^dag ... U_{k1-1}^dag (I at a chunk end)
  void* tf;           // P PF matrices: forward chunk totals
  void* tb;           // P PF matrices: backward chunk totals
  void* cf;           // P PF matrices: forward carry into each chunk
  void* cb;           // P PF matrices: backward carry out of each chunk
  void* mc;           // P PF matrices: cb[c] cf[c]^dag
  double* g;          // complex128 Tr(V^dag X_N)
  double* diag;       // [0] = ||X_N^dag X_N - I||_F
};

enum : int {
  RUN_BWD = 1,   // backward scans (needed for the gradient)
  RUN_GRAD = 2,  // adjoint pass and gradient
  RUN_FID = 4,   // fidelity against V
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
enum Stage : int { ST_PREP = 0, ST_PLAN, ST_EXPM, ST_SCAN, ST_CARRY, ST_MC, ST_ADJ, ST_COUNT };
void stage_mark(int stage, bool begin, hipStream_t st);

// Sub-range of a uniform launch: slices [s_lo, s_lo + s_n) and chunks
// [c_lo, c_lo + c_n) of every problem (s_n / c_n = 0: all, from the start
// arrays); the per-slice arrays delta / xprev / bloc hold slices from kbase
// on (checkpointed segments keep only a window of them).
struct Range {
  int s_lo, s_n, c_lo, c_n, kbase;
};

// Work items of one kernel launch.  API launches pass nprob / total / start
// by value (start = null with a uniform range); engine launches replayed from
// a captured graph read them from device memory instead:
// dyn[0] = nprob, dyn[1] = total items, dyn[2 .. 2 + nprob] = item prefix sums.
struct Work {
  const ProbDesc* descs;
  int nprob, total;
  const int* start;
  Range rg;
  const int* dyn;
};

// Enqueue one stage of the path.  Returns a hipError_t.
hipError_t launch_stage(int precision, int D, int stage, const Launch& L, const Range& rg);

}  // namespace qoc
