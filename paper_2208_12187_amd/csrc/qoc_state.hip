// State-to-state GRAPE on gfx950: the propagation of one state and one
// costate through the N slices and the exact gradient of F = |<chi|psi_N>|^2
// (GRAPE, Khaneja et al., J. Magn. Reson. 172 (2005), state transfer).
//
//   psi_{k+1} = U_k psi_k,       lam_N = chi,  lam_k = U_k^dag lam_{k+1}
//   g = <chi|psi_N>,  F = |g|^2,  dF/du[j][k] = 2 Re(conj(g) lam_{k+1}^dag L(A_k, E_j) psi_k)
//
// with A_k = -i dt H_k and E_j = -i dt Hc[j].  Nothing here forms a d x d
// propagator: every step is the action of a matrix on vectors.
//
//  * U_k psi is applied as T_q(A_k/R)^R psi, R = 2^s, with the (s, q, qb)
//    plan of the matrix path: Horner on the vector in delta form,
//    delta <- (A/R)(x + delta)/i for i = q..1, then x <- x + delta.
//  * The Frechet term.  Truncated at the plan's degree qb (the same
//    truncation as the block exponent [[A, E], [0, A]]),
//        lam^dag L(A, E) psi = sum_{i + l <= qb - 1} (A^dag^i lam)^dag E (A^l psi) / (i + l + 1)!
//    so with a_i = (A^dag)^i lam = (-A)^i lam and b_l = A^l psi it is a
//    double sum of bilinear forms a_i^dag Hc[j] b_l: 2 (qb - 1) matrix-vector
//    products per slice plus, for controls with one nonzero per row,
//    O(qb^2 d) per control.  With R > 1 the derivative of V^R, V = T_q(A/R),
//    is sum_r (V^dag^(R-1-r) lam)^dag L_V (V^r psi); the sub-step costates are
//    carried forward as V lam (V is unitary to the plan's unit roundoff).
//
// Thread layout: TPR threads per row, each holding CPT consecutive entries of
// its row of the slice Hamiltonian in registers (re and im planes); a
// matrix-vector product is CPT complex FMAs per thread against a vector in
// LDS and a reduction over the TPR lanes of the row.  Inner products and the
// overlap accumulate in FP64.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "qoc.h"
#include "qoc_device.hpp"
#include "qoc_internal.hpp"
#include "qoc_plan.hpp"

namespace qoc {

template <int D>
struct SV {
  static constexpr int TPR = D == 128 ? 8 : 4;  // threads per row
  static constexpr int CPT = D / TPR;           // row entries per thread
  static constexpr int NT = D * TPR;            // threads per workgroup
  static constexpr int NW = NT / 64;            // wavefronts
};

// Controls with at most one nonzero per row take the row-table path up to
// this many controls; beyond it (or with a dense control) the dense one.
constexpr int kStateMonoMax = 16;
// Taylor powers kept per vector: q <= 18 and qb <= 19 whenever r <= 1 in
// FP64 (1/19! < 2^-53), which the plan guarantees.
constexpr int kStateQMax = 19;
// Slices whose plans and amplitudes the chains stage in LDS at a time.
constexpr int kChainBlock = 64;
// Consecutive slices per gradient workgroup (H0 and the row tables are loaded
// once for them).
constexpr int kGradSlices = 8;

template <typename T>
struct cpx {
  T re, im;
};

// Global vectors of cpx<T>: element i, through address space 1.
template <typename T>
__device__ __forceinline__ void vec_put(cpx<T>* v, size_t i, T re, T im) {
  T* p = reinterpret_cast<T*>(v) + 2 * i;
  gp(p)[0] = re;
  gp(p)[1] = im;
}
template <typename T>
__device__ __forceinline__ void vec_get(const cpx<T>* v, size_t i, T& re, T& im) {
  const T* p = reinterpret_cast<const T*>(v) + 2 * i;
  re = gp(p)[0];
  im = gp(p)[1];
}

struct StateWork {
  const ProbDesc* descs;
  int nprob;
  int flags;
};

template <int D>
__device__ __forceinline__ bool state_mono(const ProbDesc& P) {
  if (P.m > kStateMonoMax) return false;
  for (int j = 0; j < P.m; ++j)
    if (!gp(P.mok)[j]) return false;
  return true;
}

// Row entries [c0, c0 + CPT) of a planar D x D matrix of precision T.
template <typename T, int D>
__device__ __forceinline__ void row_load(T (&re)[SV<D>::CPT], T (&im)[SV<D>::CPT], const T* M, int row, int c0) {
  constexpr int CPT = SV<D>::CPT;
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    re[c] = gp(M)[row * D + c0 + c];
    im[c] = gp(M)[D * D + row * D + c0 + c];
  }
}

// Registers of one thread: its entries of the slice Hamiltonian (row-table
// path: H0 only; the controls are added inside the products).
template <typename T, int D>
struct HRow {
  T re[SV<D>::CPT], im[SV<D>::CPT];
};

// Dense path: H_k = H0 + sum_j u[j][k] Hc[j], entries of this thread.
template <typename T, int D>
__device__ __forceinline__ void assemble_row(HRow<T, D>& H, const ProbDesc& P, int k, int row, int c0) {
  constexpr int CPT = SV<D>::CPT;
  const T* Hint = reinterpret_cast<const T*>(P.Hint);
  row_load<T, D>(H.re, H.im, Hint, row, c0);
  for (int j = 0; j < P.m; ++j) {
    const T uj = (T)gp(P.u)[(size_t)j * P.N + k];
    const T* Hj = Hint + (size_t)(j + 1) * 2 * D * D;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      H.re[c] += uj * gp(Hj)[row * D + c0 + c];
      H.im[c] += uj * gp(Hj)[D * D + row * D + c0 + c];
    }
  }
}

// LDS row tables of the controls: column and value of the nonzero of row a of
// Hc[j] (in precision T), read from the tables k_prep wrote.
template <typename T, int D>
struct CtlTab {
  int col[kStateMonoMax * D];
  cpx<T> val[kStateMonoMax * D];
};

template <typename T, int D>
__device__ __forceinline__ void ctl_load(CtlTab<T, D>& C, const ProbDesc& P) {
  const T* mv = reinterpret_cast<const T*>(P.mval);
  for (int e = threadIdx.x; e < P.m * D; e += SV<D>::NT) {
    C.col[e] = gp(P.mcol)[e];
    C.val[e].re = gp(mv)[2 * e];
    C.val[e].im = gp(mv)[2 * e + 1];
  }
}

// The row-table control terms of this thread's row, held in registers for a
// whole chain (the gradient kernel, whose register budget sets its
// occupancy, reads them from the LDS table instead): controls j = cg, cg + TPR, ... (at most KC), their
// columns col_j(row) and entries Hc[j][row][col_j], and the weighted entries
// u[j][k] Hc[j][row][col_j] of the current slice.  Absent controls get
// column `row` (in bounds) and weight 0.
template <typename T, int D>
struct CtlRegs {
  static constexpr int KC = (kStateMonoMax + SV<D>::TPR - 1) / SV<D>::TPR;
  int col[KC];
  T vr[KC], vi[KC];
  T wr[KC], wi[KC];
};

template <typename T, int D>
__device__ __forceinline__ void ctl_regs_load(CtlRegs<T, D>& R, const CtlTab<T, D>& C, int m, int row, int cg) {
#pragma unroll
  for (int t = 0; t < CtlRegs<T, D>::KC; ++t) {
    const int j = cg + SV<D>::TPR * t;
    const int e = j * D + row;
    R.col[t] = j < m ? C.col[e] : row;
    R.vr[t] = j < m ? C.val[e].re : (T)0;
    R.vi[t] = j < m ? C.val[e].im : (T)0;
    R.wr[t] = R.wi[t] = 0;
  }
}

// The slice's weights from its amplitudes us[j] (LDS).
template <typename T, int D>
__device__ __forceinline__ void ctl_regs_weigh(CtlRegs<T, D>& R, const T* us, int m, int cg) {
#pragma unroll
  for (int t = 0; t < CtlRegs<T, D>::KC; ++t) {
    const int j = cg + SV<D>::TPR * t;
    const T u = j < m ? us[j] : (T)0;
    R.wr[t] = u * R.vr[t];
    R.wi[t] = u * R.vi[t];
  }
}

// y = (H z)[row] for this thread's row, complete in every lane of the row
// group: H0 (or H_k) entries from registers, plus, on the row-table path
// (R not null), sum over this thread's controls of w_j z[col_j].  The
// control entries' vector reads are issued with the first group of columns.
template <typename T, int D>
__device__ __forceinline__ void row_apply_r(const HRow<T, D>& H, const cpx<T>* z, const CtlRegs<T, D>* R,
                                            int cg, T& yr, T& yi) {
  constexpr int CPT = SV<D>::CPT, TPR = SV<D>::TPR, KC = CtlRegs<T, D>::KC;
  const int c0 = cg * CPT;
  T ar = 0, ai = 0;
  if (R) {
    cpx<T> v[KC];
#pragma unroll
    for (int t = 0; t < KC; ++t) v[t] = z[R->col[t]];
#pragma unroll
    for (int t = 0; t < KC; ++t) {
      ar = fma(R->wr[t], v[t].re, ar);
      ar = fma(-R->wi[t], v[t].im, ar);
      ai = fma(R->wr[t], v[t].im, ai);
      ai = fma(R->wi[t], v[t].re, ai);
    }
  }
#pragma unroll
  for (int c4 = 0; c4 < CPT; c4 += 4) {
#pragma unroll
    for (int c = c4; c < c4 + 4; ++c) {
      const cpx<T> v = z[c0 + c];
      ar = fma(H.re[c], v.re, ar);
      ar = fma(-H.im[c], v.im, ar);
      ai = fma(H.re[c], v.im, ai);
      ai = fma(H.im[c], v.re, ai);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int o = 1; o < TPR; o <<= 1) {
    ar += __shfl_xor(ar, o, 64);
    ai += __shfl_xor(ai, o, 64);
  }
  yr = ar;
  yi = ai;
}

// y = (H z)[row] for this thread's row, complete in every lane of the row
// group: H0 (or H_k) entries from registers, plus, on the row-table path,
// sum over the controls j = cg, cg + TPR, ... of us[j] Hc[j][row][col_j] z[col_j].
template <typename T, int D>
__device__ __forceinline__ void row_apply(const HRow<T, D>& H, const cpx<T>* z, const CtlTab<T, D>* C,
                                          const T* us, int m, int row, int cg, T& yr, T& yi) {
  constexpr int CPT = SV<D>::CPT, TPR = SV<D>::TPR;
  const int c0 = cg * CPT;
  T ar = 0, ai = 0;
  // groups of four columns, so that at most four vector entries are in
  // flight from LDS (hoisting all CPT loads costs 4 CPT registers)
#pragma unroll
  for (int c4 = 0; c4 < CPT; c4 += 4) {
#pragma unroll
    for (int c = c4; c < c4 + 4; ++c) {
      const cpx<T> v = z[c0 + c];
      ar = fma(H.re[c], v.re, ar);
      ar = fma(-H.im[c], v.im, ar);
      ai = fma(H.re[c], v.im, ai);
      ai = fma(H.im[c], v.re, ai);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  if (C) {
    for (int j = cg; j < m; j += TPR) {
      const int e = j * D + row;
      const cpx<T> h = C->val[e];
      const cpx<T> v = z[C->col[e]];
      const T wr = us[j] * h.re, wi = us[j] * h.im;
      ar = fma(wr, v.re, ar);
      ar = fma(-wi, v.im, ar);
      ai = fma(wr, v.im, ai);
      ai = fma(wi, v.re, ai);
    }
  }
#pragma unroll
  for (int o = 1; o < TPR; o <<= 1) {
    ar += __shfl_xor(ar, o, 64);
    ai += __shfl_xor(ai, o, 64);
  }
  yr = ar;
  yi = ai;
}

// Sum of v over the rows of the workgroup: lanes of one row hold equal
// copies, so only the TPR-strided lanes are added.  Returns the total in
// every thread; red holds NW doubles.
template <int D>
__device__ __forceinline__ double rows_sum(double v, double* red) {
  constexpr int TPR = SV<D>::TPR, NW = SV<D>::NW;
#pragma unroll
  for (int o = TPR; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) t += red[w];
  return t;
}

// ---------------------------------------------------------------- chains

// One workgroup per (problem, direction).  Forward: psi_0 -> psi_N, storing
// every psi_k, then g, F (and psi_N when asked for).  Backward: chi -> lam_0,
// storing every lam_k.  Each slice is applied as T_q(+-A_k/R)^R.
// MONO: the row-table path (every control has at most one nonzero per row, at
// most kStateMonoMax controls) or the dense one; both are launched and each
// workgroup leaves at once when its problem takes the other.
template <typename T, int D, bool MONO>
__global__ __launch_bounds__(SV<D>::NT) void k_state_chain(StateWork W) {
  constexpr int TPR = SV<D>::TPR, CPT = SV<D>::CPT, NW = SV<D>::NW;
  __shared__ cpx<T> zb[2][D];
  __shared__ CtlTab<T, D> ctl;
  __shared__ T ub[kChainBlock][kStateMonoMax];  // row-table path: u[j][k] of the block's slices
  __shared__ int sqb[kChainBlock];              // the block's plans
  __shared__ double red[2 * NW];
  const int p = blockIdx.x, bwd = blockIdx.y;
  const ProbDesc P = W.descs[p];  // a copy: stores cannot alias it
  const int row = threadIdx.x / TPR, cg = threadIdx.x % TPR;
  const int d = P.d, m = P.m, N = P.N;
  if (state_mono<D>(P) != MONO) return;
  constexpr bool mono = MONO;
  HRow<T, D> H;
  CtlRegs<T, D> CR;
  if constexpr (MONO) {
    row_load<T, D>(H.re, H.im, reinterpret_cast<const T*>(P.Hint), row, cg * CPT);
    ctl_load<T, D>(ctl, P);
    __syncthreads();
    ctl_regs_load<T, D>(CR, ctl, m, row, cg);
  }
  // the chain's vector: x[row], held by every lane of the row group
  const double* src = bwd ? P.chiz : P.psi0z;
  T xr = 0, xi = 0;
  if (row < d) {
    xr = (T)src[2 * row];
    xi = (T)src[2 * row + 1];
  }
  cpx<T>* store = reinterpret_cast<cpx<T>*>(bwd ? P.lam : P.psi);
  if (cg == 0 && store) vec_put(store, (size_t)(bwd ? N : 0) * D + row, xr, xi);
  int buf = 0;
  for (int step = 0; step < N; ++step) {
    const int k = bwd ? N - 1 - step : step;
    const int bi = step % kChainBlock;  // position in the block of slices staged in LDS
    if (bi == 0) {
      // the plans (and, on the row-table path, the amplitudes) of the next
      // kChainBlock slices in chain order: one round trip per block
      __syncthreads();  // the previous block's entries have been read
      const int nb = min(kChainBlock, N - step);
      for (int e = threadIdx.x; e < nb; e += SV<D>::NT) sqb[e] = gp(P.sq)[bwd ? k - e : k + e];
      if constexpr (MONO)
        for (int e = threadIdx.x; e < m * nb; e += SV<D>::NT) {
          const int j = e / nb, t = e - j * nb;
          ub[t][j] = (T)gp(P.u)[(size_t)j * N + (bwd ? k - t : k + t)];
        }
      __syncthreads();
    }
    const int sq = sqb[bi];
    const int s = sq & 0xff, q = (sq >> 8) & 0xff;
    // A z = -i c (H z) forward; the adjoint step uses -A = +i c H.
    const double c = ldexp(P.dt, -s) * (bwd ? -1.0 : 1.0);
    if constexpr (MONO) ctl_regs_weigh<T, D>(CR, ub[bi], m, cg);  // the slice's amplitudes
    else assemble_row<T, D>(H, P, k, row, cg * CPT);
    for (int r = 0; r < (1 << s); ++r) {
      T dr = 0, di = 0;  // delta
      for (int i = q; i >= 1; --i) {
        if (cg == 0) zb[buf][row] = cpx<T>{xr + dr, xi + di};
        __syncthreads();
        T yr, yi;
        row_apply_r<T, D>(H, zb[buf], mono ? &CR : nullptr, cg, yr, yi);
        const T f = (T)(c / i);
        dr = f * yi;  // -i f (yr + i yi) = f yi - i f yr
        di = -f * yr;
        buf ^= 1;
      }
      xr += dr;
      xi += di;
    }
    if (cg == 0 && store) vec_put(store, (size_t)(bwd ? k : k + 1) * D + row, xr, xi);
  }
  if (!bwd) {
    // g = <chi|psi_N> in FP64
    double gr = 0, gi = 0;
    if (row < d) {
      const double cr = P.chiz ? P.chiz[2 * row] : 0.0, ci = P.chiz ? P.chiz[2 * row + 1] : 0.0;
      gr = cr * (double)xr + ci * (double)xi;
      gi = cr * (double)xi - ci * (double)xr;
    }
    gr = rows_sum<D>(gr, red);
    gi = rows_sum<D>(gi, red + NW);
    if (threadIdx.x == 0 && P.chiz) {
      P.g[0] = gr;
      P.g[1] = gi;
      P.F[0] = gr * gr + gi * gi;
    }
    if (P.XN && cg == 0 && row < d) {
      P.XN[2 * row] = (double)xr;
      P.XN[2 * row + 1] = (double)xi;
    }
  }
}

// ---------------------------------------------------------------- gradient

// One workgroup per kGradSlices consecutive slices of a problem; per slice k: the Taylor powers b_l = (A/R)^l psi
// and a_i = (-A/R)^i lam in LDS, then per control
// G_j = sum_{i + l <= qb - 1} a_i^dag Hc[j] b_l / (i + l + 1)!  (FP64), summed
// over the R sub-steps, and dF/du[j][k] = (2 dt / R) Im(conj(g) G_j).
template <typename T, int D, bool MONO>
__global__ __launch_bounds__(SV<D>::NT) void k_state_grad(StateWork W) {
  constexpr int TPR = SV<D>::TPR, CPT = SV<D>::CPT, NW = SV<D>::NW;
  constexpr int KM = (kStateMonoMax + TPR - 1) / TPR;  // row-table controls per thread
  __shared__ cpx<T> av[kStateQMax][D];
  __shared__ cpx<T> bv[kStateQMax][D];
  __shared__ CtlTab<T, D> ctl;
  __shared__ T us[kStateMonoMax];
  __shared__ double red[2 * NW];
  __shared__ double gacc[2 * kStateMonoMax * NW];
  const ProbDesc& P0 = W.descs[0];
  const int per = (P0.N + kGradSlices - 1) / kGradSlices;  // workgroups per problem (uniform N)
  const int pidx = blockIdx.x / per;
  const ProbDesc P = W.descs[pidx];
  const int row = threadIdx.x / TPR, cg = threadIdx.x % TPR, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int m = P.m, N = P.N;
  if (state_mono<D>(P) != MONO) return;
  constexpr bool mono = MONO;
  HRow<T, D> H;
  if constexpr (MONO) {  // H0 and the row tables serve every slice of the workgroup
    row_load<T, D>(H.re, H.im, reinterpret_cast<const T*>(P.Hint), row, cg * CPT);
    ctl_load<T, D>(ctl, P);
  }
  const int kb = (blockIdx.x - pidx * per) * kGradSlices;
  for (int k = kb; k < min(N, kb + kGradSlices); ++k) {
  const int sq = gp(P.sq)[k];
  const int s = sq & 0xff, q = (sq >> 8) & 0xff, qb = (sq >> 16) & 0xff;
  const int R = 1 << s;
  // powers 0..Qp (q <= 18 and qb <= 19 by the plan; the bound only guards LDS)
  const int Qp = min(max(q, qb - 1), kStateQMax - 1);
  const int qe = min(q, Qp), qbe = min(qb, Qp + 1);
  const double c = ldexp(P.dt, -s);
  __syncthreads();  // the previous slice is done with us[], the powers and gacc
  if constexpr (MONO) {
    if ((int)threadIdx.x < m) us[threadIdx.x] = (T)gp(P.u)[(size_t)threadIdx.x * N + k];
  } else {
    assemble_row<T, D>(H, P, k, row, cg * CPT);
  }
  const cpx<T>* psi = reinterpret_cast<const cpx<T>*>(P.psi) + (size_t)k * D;
  const cpx<T>* lam = reinterpret_cast<const cpx<T>*>(P.lam) + (size_t)(R == 1 ? k + 1 : k) * D;
  T pr, pi, lr, li;
  vec_get(psi, row, pr, pi);  // psi_r (row entry, every lane of the row)
  vec_get(lam, row, lr, li);  // lam_r
  __syncthreads();  // row tables and us[] visible
  // R > 1: lam_0 = V lam_k  (V^dag^(R-1) lam_{k+1} = V lam_k, V unitary)
  if (R > 1) {
    T dr = 0, di = 0;
    for (int i = q; i >= 1; --i) {
      if (cg == 0) bv[0][row] = cpx<T>{lr + dr, li + di};
      __syncthreads();
      T yr, yi;
      row_apply<T, D>(H, bv[0], mono ? &ctl : nullptr, us, m, row, cg, yr, yi);
      __syncthreads();
      const T f = (T)(c / i);
      dr = f * yi;
      di = -f * yr;
    }
    lr += dr;
    li += di;
  }
  double accr[KM], acci[KM];  // row-table path: this thread's controls
#pragma unroll
  for (int t = 0; t < KM; ++t) accr[t] = acci[t] = 0.0;
  for (int r = 0; r < R; ++r) {
    // powers: b_0 = psi_r, a_0 = lam_r, b_{l+1} = (A/R) b_l = -i c H b_l, a_{i+1} = +i c H a_i
    if (cg == 0) {
      bv[0][row] = cpx<T>{pr, pi};
      av[0][row] = cpx<T>{lr, li};
    }
    __syncthreads();
    for (int l = 1; l <= Qp; ++l) {
      T yr, yi, zr, zi;
      row_apply<T, D>(H, bv[l - 1], mono ? &ctl : nullptr, us, m, row, cg, yr, yi);
      row_apply<T, D>(H, av[l - 1], mono ? &ctl : nullptr, us, m, row, cg, zr, zi);
      if (cg == 0) {
        bv[l][row] = cpx<T>{(T)c * yi, -(T)c * yr};
        av[l][row] = cpx<T>{-(T)c * zi, (T)c * zr};
      }
      __syncthreads();
    }
    // bilinear forms a_i^dag Hc[j] b_l, weighted by 1 / (i + l + 1)!
    if constexpr (MONO) {
#pragma unroll
      for (int t = 0; t < KM; ++t) {
        const int j = cg + t * TPR;
        if (j < m) {
          const int e = j * D + row;
          const int col = ctl.col[e];
          const double hr = (double)ctl.val[e].re, hi = (double)ctl.val[e].im;
          double sr = 0, si = 0;
          double f0 = 1.0;  // 1 / (i + 1)!
          for (int i = 0; i < qbe; ++i) {
            f0 /= (double)(i + 1);
            // w = sum_{l <= qb - 1 - i} b_l[col] / (i + l + 1)!
            double wr = 0, wi = 0, f = f0;
            for (int l = 0; l + i < qbe; ++l) {
              wr += f * (double)bv[l][col].re;
              wi += f * (double)bv[l][col].im;
              f /= (double)(i + l + 2);
            }
            // conj(a_i[row]) * val * w
            const double ar = (double)av[i][row].re, ai = (double)av[i][row].im;
            const double vr = hr * wr - hi * wi, vi = hr * wi + hi * wr;
            sr += ar * vr + ai * vi;
            si += ar * vi - ai * vr;
          }
          accr[t] += sr;
          acci[t] += si;
        }
      }
    } else {
      // Hc[j] b_l by rows, one control at a time
      const T* Hint = reinterpret_cast<const T*>(P.Hint);
      for (int j = 0; j < m; ++j) {
        HRow<T, D> C;
        row_load<T, D>(C.re, C.im, Hint + (size_t)(j + 1) * 2 * D * D, row, cg * CPT);
        double sr = 0, si = 0;
        double f0 = 1.0;  // 1 / (l + 1)!
        for (int l = 0; l < qbe; ++l) {
          T hr, hi;
          row_apply<T, D>(C, bv[l], nullptr, us, 0, row, cg, hr, hi);
          f0 /= (double)(l + 1);
          // sum_{i <= qb - 1 - l} conj(a_i[row]) / (i + l + 1)!
          double f = f0;
          double wr = 0, wi = 0;
          for (int i = 0; i + l < qbe; ++i) {
            wr += f * (double)av[i][row].re;
            wi += f * (double)av[i][row].im;
            f /= (double)(i + l + 2);
          }
          sr += wr * (double)hr + wi * (double)hi;
          si += wr * (double)hi - wi * (double)hr;
        }
        // the TPR lanes of a row hold equal copies: rows_sum adds one per row
        sr = rows_sum<D>(sr, red);
        si = rows_sum<D>(si, red + NW);
        // the gradient is linear in G_j: add this sub-step's share
        if (threadIdx.x == 0) {
          const double v = 2.0 * c * (P.g[0] * si - P.g[1] * sr);
          double* out = P.grad + (size_t)j * N + k;
          *out = r == 0 ? v : *out + v;
        }
      }
    }
    if (r + 1 < R) {
      // psi_{r+1} = sum_l b_l / l!,  lam_{r+1} = V lam_r = sum_i (-1)^i a_i / i!
      T nr = 0, ni = 0, mr = 0, mi = 0;
      T f = 1;
      for (int l = 0; l <= qe; ++l) {
        nr += f * bv[l][row].re;
        ni += f * bv[l][row].im;
        const T sg = (l & 1) ? -f : f;
        mr += sg * av[l][row].re;
        mi += sg * av[l][row].im;
        f /= (T)(l + 1);
      }
      pr = nr;
      pi = ni;
      lr = mr;
      li = mi;
      __syncthreads();  // every lane has read the powers before they are overwritten
    }
  }
  // gradient: (2 dt / R) Im(conj(g) G_j) (the dense path has written it)
  const double g0 = P.g[0], g1 = P.g[1];
  const double scale = 2.0 * c;  // 2 dt / R
  if constexpr (MONO) {
    // rows -> wavefront: lanes with the same cg hold the same controls
#pragma unroll
    for (int t = 0; t < KM; ++t) {
#pragma unroll
      for (int o = TPR; o < 64; o <<= 1) {
        accr[t] += __shfl_xor(accr[t], o, 64);
        acci[t] += __shfl_xor(acci[t], o, 64);
      }
    }
    __syncthreads();
    if (lane < TPR) {
#pragma unroll
      for (int t = 0; t < KM; ++t) {
        const int j = lane + t * TPR;
        if (j < m) {
          gacc[2 * (j * NW + wv)] = accr[t];
          gacc[2 * (j * NW + wv) + 1] = acci[t];
        }
      }
    }
    __syncthreads();
    if ((int)threadIdx.x < m) {
      const int j = threadIdx.x;
      double sr = 0, si = 0;
      for (int w = 0; w < NW; ++w) {
        sr += gacc[2 * (j * NW + w)];
        si += gacc[2 * (j * NW + w) + 1];
      }
      P.grad[(size_t)j * N + k] = scale * (g0 * si - g1 * sr);
    }
  }
  }  // slices of the workgroup
}

template <typename T, int D>
static hipError_t launch_state(const StateWork& W, int B, int N, int grad, hipStream_t st) {
  const dim3 cg(B, grad ? 2 : 1), gg(B * ((N + kGradSlices - 1) / kGradSlices)), nt(SV<D>::NT);
  stage_mark(ST_SCHAIN, true, st);
  hipLaunchKernelGGL((k_state_chain<T, D, true>), cg, nt, 0, st, W);
  hipLaunchKernelGGL((k_state_chain<T, D, false>), cg, nt, 0, st, W);
  stage_mark(ST_SCHAIN, false, st);
  if (grad) {
    stage_mark(ST_SGRAD, true, st);
    hipLaunchKernelGGL((k_state_grad<T, D, true>), gg, nt, 0, st, W);
    hipLaunchKernelGGL((k_state_grad<T, D, false>), gg, nt, 0, st, W);
    stage_mark(ST_SGRAD, false, st);
  }
  return hipGetLastError();
}

static hipError_t launch_state_path(int precision, int D, const StateWork& W, int B, int N, int grad,
                                    hipStream_t st) {
  if (precision == 0) {
    switch (D) {
      case 16: return launch_state<double, 16>(W, B, N, grad, st);
      case 32: return launch_state<double, 32>(W, B, N, grad, st);
      case 64: return launch_state<double, 64>(W, B, N, grad, st);
      case 128: return launch_state<double, 128>(W, B, N, grad, st);
    }
  } else if (precision == 1) {
    switch (D) {
      case 16: return launch_state<float, 16>(W, B, N, grad, st);
      case 32: return launch_state<float, 32>(W, B, N, grad, st);
      case 64: return launch_state<float, 64>(W, B, N, grad, st);
      case 128: return launch_state<float, 128>(W, B, N, grad, st);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace qoc

// ---------------------------------------------------------------- host side

namespace {

using qoc::ProbDesc;

int sfail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  qoc::set_last_error(buf);
  return code;
}

struct StateLayout {
  int D;
  size_t esize, desc_bytes, Hint, norms, mono, sq, psi, lam, small, per_prob, total;
};

StateLayout make_state_layout(int B, int d, int m, int N, int precision) {
  using qoc::align_up;
  StateLayout Lo;
  Lo.D = qoc::padded_dim(d);
  Lo.esize = qoc::elem_size(precision);
  const size_t mat = 2ull * Lo.D * Lo.D * Lo.esize, vec = 2ull * Lo.D * Lo.esize;
  size_t o = 0;
  Lo.Hint = o; o = align_up(o + (size_t)(m + 1) * mat);
  Lo.norms = o; o = align_up(o + (size_t)(m + 1) * 8);
  Lo.mono = o; o = align_up(o + (size_t)m * Lo.D * (4 + 2 * Lo.esize) + (size_t)m * 4);
  Lo.sq = o; o = align_up(o + (size_t)N * 4);
  Lo.psi = o; o = align_up(o + (size_t)(N + 1) * vec);
  Lo.lam = o; o = align_up(o + (size_t)(N + 1) * vec);
  Lo.small = o; o = align_up(o + 128);
  Lo.per_prob = o;
  Lo.desc_bytes = align_up((size_t)B * sizeof(ProbDesc));
  Lo.total = Lo.desc_bytes + (size_t)B * Lo.per_prob;
  return Lo;
}

int check_state_dims(int B, int d, int m, int N, int precision) {
  if (B < 1) return sfail(QOC_ERR_ARG, "batch size B = %d must be >= 1", B);
  if (d < 1 || m < 1 || N < 1) return sfail(QOC_ERR_ARG, "need d, m, N >= 1 (got d=%d m=%d N=%d)", d, m, N);
  if (d > 128) return sfail(QOC_ERR_UNSUPPORTED, "d = %d exceeds the supported maximum 128", d);
  if (precision != QOC_FP64 && precision != QOC_FP32)
    return sfail(QOC_ERR_UNSUPPORTED, "the state-to-state path runs in FP64 or FP32 (precision %d)", precision);
  return QOC_OK;
}

qoc_options state_defaults() {
  qoc_options o;
  qoc_default_options(&o);
  return o;
}

int run_state_dev(int B, int d, int m, int N, const void* H0, const void* Hc, const void* u, double dt,
                  const void* psi0, const void* chi, void* F, void* grad, void* psiN, void* ws, size_t ws_bytes,
                  const qoc_options* opt_in, bool with_grad) {
  const qoc_options opt = opt_in ? *opt_in : state_defaults();
  int rc = check_state_dims(B, d, m, N, opt.precision);
  if (rc) return rc;
  if (opt.generators) return sfail(QOC_ERR_UNSUPPORTED, "the state-to-state path takes Hermitian Hamiltonians only");
  if (!(dt > 0) || !std::isfinite(dt)) return sfail(QOC_ERR_ARG, "dt must be finite and > 0");
  if (!H0 || !Hc || !u || !psi0) return sfail(QOC_ERR_ARG, "H0, Hc, u and psi0 must be non-null");
  if (with_grad && (!chi || !F || !grad)) return sfail(QOC_ERR_ARG, "chi, F and grad must be non-null");
  if (!with_grad && !psiN) return sfail(QOC_ERR_ARG, "psiN must be non-null");
  if (!ws) return sfail(QOC_ERR_ARG, "workspace must be non-null");
  if (((uintptr_t)ws) % qoc::kAlign) return sfail(QOC_ERR_ARG, "workspace must be 256-byte aligned");
  const StateLayout Lo = make_state_layout(B, d, m, N, opt.precision);
  if (ws_bytes < Lo.total) return sfail(QOC_ERR_ARG, "workspace holds %zu bytes, %zu needed", ws_bytes, Lo.total);

  char* base = static_cast<char*>(ws);
  std::vector<ProbDesc> descs(B);
  const size_t dd = (size_t)d * d;
  const int flags = (with_grad ? (qoc::RUN_GRAD | qoc::RUN_BWD | qoc::RUN_FID) : 0) |
                    (opt.dense_controls ? qoc::CTRL_DENSE : 0);
  for (int b = 0; b < B; ++b) {
    char* pb = base + Lo.desc_bytes + (size_t)b * Lo.per_prob;
    ProbDesc& P = descs[b];
    memset(&P, 0, sizeof P);
    P.d = d;
    P.D = Lo.D;
    P.m = m;
    P.N = N;
    P.L = N;
    P.P = 1;
    P.CG = P.PG = 1;
    P.flags = flags;
    P.dt = dt;
    P.H0z = static_cast<const double*>(H0) + 2 * dd * b;
    P.Hcz = static_cast<const double*>(Hc) + 2 * dd * m * b;
    P.u = static_cast<const double*>(u) + (size_t)m * N * b;
    P.Hint = pb + Lo.Hint;
    P.norms = reinterpret_cast<double*>(pb + Lo.norms);
    P.mval = pb + Lo.mono;
    P.mcol = reinterpret_cast<int*>(pb + Lo.mono + (size_t)m * Lo.D * 2 * Lo.esize);
    P.mok = P.mcol + (size_t)m * Lo.D;
    P.sq = reinterpret_cast<int*>(pb + Lo.sq);
    double* small = reinterpret_cast<double*>(pb + Lo.small);
    P.g = small;
    P.F = F ? static_cast<double*>(F) + b : small + 2;
    P.diag = small + 4;
    P.reun_tol = -1.0;
    P.grad = grad ? static_cast<double*>(grad) + (size_t)m * N * b : nullptr;
    P.XN = psiN ? static_cast<double*>(psiN) + 2 * (size_t)d * b : nullptr;
    P.psi0z = static_cast<const double*>(psi0) + 2 * (size_t)d * b;
    P.chiz = chi ? static_cast<const double*>(chi) + 2 * (size_t)d * b : nullptr;
    P.psi = with_grad ? pb + Lo.psi : nullptr;
    P.lam = with_grad ? pb + Lo.lam : nullptr;
  }
  hipStream_t st = static_cast<hipStream_t>(opt.stream);
  hipError_t e = hipMemcpyAsync(base, descs.data(), (size_t)B * sizeof(ProbDesc), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return sfail(QOC_ERR_DEVICE, "descriptor upload: %s", hipGetErrorString(e));

  qoc::Launch L;
  memset(&L, 0, sizeof L);
  L.descs = reinterpret_cast<const ProbDesc*>(base);
  L.nprob = B;
  L.uniformN = N;
  L.uniformP = 1;
  L.total_slices = B * N;
  L.total_chunks = B;
  L.max_m = m;
  L.flags = flags;
  L.stream = st;
  const qoc::Range all = {0, N, 0, 1, 0, 0};
  e = qoc::launch_stage(opt.precision, Lo.D, qoc::ST_PREP, L, all);
  if (e == hipSuccess) e = qoc::launch_stage(opt.precision, Lo.D, qoc::ST_PLAN, L, all);
  if (e == hipSuccess) {
    const qoc::StateWork W = {L.descs, B, flags};
    e = qoc::launch_state_path(opt.precision, Lo.D, W, B, N, with_grad ? 1 : 0, st);
  }
  if (e != hipSuccess) return sfail(QOC_ERR_DEVICE, "kernel launch: %s", hipGetErrorString(e));
  return QOC_OK;
}

bool finite_vals(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

bool hermitian_mat(const qoc_z* H, int d) {
  double hmax = 0, dmax = 0;
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) {
      const qoc_z x = H[a * d + b], y = H[b * d + a];
      hmax = std::max(hmax, std::max(fabs(x.re), fabs(x.im)));
      dmax = std::max(dmax, std::max(fabs(x.re - y.re), fabs(x.im + y.im)));
    }
  return dmax <= 1e-12 * std::max(1.0, hmax);
}

bool unit_norm(const qoc_z* v, int d) {
  double s = 0;
  for (int a = 0; a < d; ++a) s += v[a].re * v[a].re + v[a].im * v[a].im;
  return fabs(sqrt(s) - 1.0) <= 1e-8;
}

struct SBufs {
  std::vector<void*> ptrs;
  ~SBufs() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  void* alloc(size_t n) {
    void* p = nullptr;
    if (hipMalloc(&p, n ? n : 1) != hipSuccess) return nullptr;
    ptrs.push_back(p);
    return p;
  }
};

int run_state_host(int d, int m, int N, const qoc_z* H0, const qoc_z* Hc, const double* u, double dt,
                   const qoc_z* psi0, const qoc_z* chi, double* F, double* grad, qoc_z* psiN,
                   const qoc_options* opt_in, bool with_grad) {
  const qoc_options opt = opt_in ? *opt_in : state_defaults();
  int rc = check_state_dims(1, d, m, N, opt.precision);
  if (rc) return rc;
  if (!H0 || !Hc || !u || !psi0) return sfail(QOC_ERR_ARG, "H0, Hc, u and psi0 must be non-null");
  if (!(dt > 0) || !std::isfinite(dt)) return sfail(QOC_ERR_ARG, "dt must be finite and > 0");
  if (with_grad && (!chi || !F || !grad)) return sfail(QOC_ERR_ARG, "chi, F and grad must be non-null");
  if (!with_grad && !psiN) return sfail(QOC_ERR_ARG, "psiN must be non-null");
  const size_t dd = (size_t)d * d;
  if (opt.validate) {
    if (!finite_vals(&H0->re, 2 * dd) || !finite_vals(&Hc->re, 2 * dd * m) || !finite_vals(u, (size_t)m * N) ||
        !finite_vals(&psi0->re, 2 * (size_t)d) || (chi && !finite_vals(&chi->re, 2 * (size_t)d)))
      return sfail(QOC_ERR_NONFINITE, "an input holds NaN or Inf");
    if (!hermitian_mat(H0, d)) return sfail(QOC_ERR_NOT_HERMITIAN, "H0 is not Hermitian");
    for (int j = 0; j < m; ++j)
      if (!hermitian_mat(Hc + (size_t)j * dd, d)) return sfail(QOC_ERR_NOT_HERMITIAN, "Hc[%d] is not Hermitian", j);
    if (!unit_norm(psi0, d) || (chi && !unit_norm(chi, d)))
      return sfail(QOC_ERR_NOT_UNITARY, "psi0 and chi must have unit norm (within 1e-8)");
  }
  const size_t ws_bytes = make_state_layout(1, d, m, N, opt.precision).total;
  SBufs bufs;
  void* dH0 = bufs.alloc(dd * 16);
  void* dHc = bufs.alloc(dd * 16 * m);
  void* du = bufs.alloc((size_t)m * N * 8);
  void* dpsi0 = bufs.alloc((size_t)d * 16);
  void* dchi = chi ? bufs.alloc((size_t)d * 16) : nullptr;
  void* dF = bufs.alloc(8);
  void* dgrad = grad ? bufs.alloc((size_t)m * N * 8) : nullptr;
  void* dpsiN = psiN ? bufs.alloc((size_t)d * 16) : nullptr;
  void* dws = bufs.alloc(ws_bytes);
  if (!dH0 || !dHc || !du || !dpsi0 || (chi && !dchi) || !dF || (grad && !dgrad) || (psiN && !dpsiN) || !dws)
    return sfail(QOC_ERR_OOM, "device allocation of %zu workspace bytes failed", ws_bytes);
  hipStream_t st = static_cast<hipStream_t>(opt.stream);
  hipError_t e = hipSuccess;
  e = e ? e : hipMemcpyAsync(dH0, H0, dd * 16, hipMemcpyHostToDevice, st);
  e = e ? e : hipMemcpyAsync(dHc, Hc, dd * 16 * m, hipMemcpyHostToDevice, st);
  e = e ? e : hipMemcpyAsync(du, u, (size_t)m * N * 8, hipMemcpyHostToDevice, st);
  e = e ? e : hipMemcpyAsync(dpsi0, psi0, (size_t)d * 16, hipMemcpyHostToDevice, st);
  if (chi) e = e ? e : hipMemcpyAsync(dchi, chi, (size_t)d * 16, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return sfail(QOC_ERR_DEVICE, "upload: %s", hipGetErrorString(e));
  rc = run_state_dev(1, d, m, N, dH0, dHc, du, dt, dpsi0, dchi, with_grad ? dF : nullptr, dgrad, dpsiN, dws,
                     ws_bytes, &opt, with_grad);
  if (rc) return rc;
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return sfail(QOC_ERR_DEVICE, "execution: %s", hipGetErrorString(e));
  if (F) e = e ? e : hipMemcpy(F, dF, 8, hipMemcpyDeviceToHost);
  if (grad) e = e ? e : hipMemcpy(grad, dgrad, (size_t)m * N * 8, hipMemcpyDeviceToHost);
  if (psiN) e = e ? e : hipMemcpy(psiN, dpsiN, (size_t)d * 16, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return sfail(QOC_ERR_DEVICE, "download: %s", hipGetErrorString(e));
  return QOC_OK;
}

}  // namespace

extern "C" {

size_t qoc_state_workspace_size(int B, int d, int m, int N, int precision) {
  if (check_state_dims(B, d, m, N, precision)) return 0;
  return make_state_layout(B, d, m, N, precision).total;
}

int qoc_state_propagate(int d, int m, int N, const qoc_z* H0, const qoc_z* Hc, const double* u, double dt,
                        const qoc_z* psi0, qoc_z* psiN, const qoc_options* opt) {
  return run_state_host(d, m, N, H0, Hc, u, dt, psi0, nullptr, nullptr, nullptr, psiN, opt, false);
}

int qoc_state_gradient(int d, int m, int N, const qoc_z* H0, const qoc_z* Hc, const double* u, double dt,
                       const qoc_z* psi0, const qoc_z* chi, double* F, double* grad, const qoc_options* opt) {
  return run_state_host(d, m, N, H0, Hc, u, dt, psi0, chi, F, grad, nullptr, opt, true);
}

int qoc_state_propagate_dev(int B, int d, int m, int N, const void* H0, const void* Hc, const void* u, double dt,
                            const void* psi0, void* psiN, void* workspace, size_t ws_bytes, const qoc_options* opt) {
  return run_state_dev(B, d, m, N, H0, Hc, u, dt, psi0, nullptr, nullptr, nullptr, psiN, workspace, ws_bytes, opt,
                       false);
}

int qoc_state_gradient_dev(int B, int d, int m, int N, const void* H0, const void* Hc, const void* u, double dt,
                           const void* psi0, const void* chi, void* F, void* grad, void* workspace, size_t ws_bytes,
                           const qoc_options* opt) {
  return run_state_dev(B, d, m, N, H0, Hc, u, dt, psi0, chi, F, grad, nullptr, workspace, ws_bytes, opt, true);
}

}  // extern "C"
