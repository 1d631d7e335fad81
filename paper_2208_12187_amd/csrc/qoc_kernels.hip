// GRAPE hot path on gfx950: slice propagators by scaling-and-squaring Taylor
// series, chunked forward/backward propagator scans, fidelity in FP64 and the
// exact gradient through the block-triangular Frechet derivative.
//
// Notation (slice k = 0..N-1, slice 0 acts first; hbar = 1):
//   A_k = -i dt H_k,  H_k = H0 + sum_j u[j][k] Hc[j],  U_k = exp(A_k)
//   X_N = U_{N-1} ... U_0,  g = Tr(V^dag X_N),  F = |g|^2 / d^2
//   P_k = U_k ... U_0 (P_{-1} = I),  Q_k = U_{k+1}^dag ... U_{N-1}^dag V
//   W_k = Q_k P_{k-1}^dag
// GRAPE gradient (Khaneja et al. 2005), taken exactly: with L(A, E) the
// Frechet derivative of exp at A in direction E,
//   dg/du[j][k] = <W_k, L(A_k, -i dt Hc[j])>,   <X, Y> = Tr(X^dag Y).
// The adjoint identity <W, L(A, E)> = <L(A^dag, W), E> (L(A, E) is the
// integral of e^{sA} E e^{(1-s)A} over s in [0, 1]) turns the m derivatives
// of a slice into one: Z_k = L(A_k^dag, W_k) and
//   dF/du[j][k] = (2 dt / d^2) Im(conj(g) Tr(Z_k^dag Hc[j])).
// Z_k is the top-right block of exp([[A^dag, W], [0, A^dag]]) (Van Loan 1978;
// Goodwin and Kuprov 2015), evaluated with the same scaling and squaring as
// the propagator.  Everything runs in "delta form": the Taylor sum keeps
// T(X) - I and a squaring maps D to 2D + D^2, so that rounding errors scale
// with |A| rather than with |U| = 1.
#include "qoc_device.hpp"
#include "qoc_internal.hpp"
#include "qoc_plan.hpp"

namespace qoc {

// ---------------------------------------------------------------- work items

__device__ __forceinline__ int locate(const int* start, int n, int item) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (start[mid] <= item) lo = mid; else hi = mid;
  }
  return lo;
}

// Map a flat work item to (problem, local index).
__device__ __forceinline__ void split_item(int item, int uniform, const int* start, int n, int& p, int& k) {
  if (uniform > 0) {
    p = item / uniform;
    k = item - p * uniform;
  } else {
    p = locate(start, n, item);
    k = item - start[p];
  }
}

template <typename T, int D>
__device__ __forceinline__ T* pf_mat(void* base, int i) {
  return reinterpret_cast<T*>(base) + (size_t)i * Mat<T, D>::ELEMS;
}

// ---------------------------------------------------------------- prep

// Convert the caller's complex128 matrices to the compute precision: H0 and
// Hc[j] to planar D x D (zero padded), V to PF; also the FP64 one-norms
// (largest column sum of moduli) of H0 and Hc[j].
template <typename T, int D>
__global__ __launch_bounds__(256) void k_prep(const ProbDesc* __restrict__ descs) {
  const ProbDesc& P = descs[blockIdx.x];
  const int mat = blockIdx.y;
  const int d = P.d, m = P.m;
  if (mat > m + 1) return;
  __shared__ double colmax[256];
  if (mat <= m) {
    const double* src = mat == 0 ? P.H0z : P.Hcz + (size_t)(mat - 1) * 2 * d * d;
    T* dst = reinterpret_cast<T*>(P.Hint) + (size_t)mat * 2 * D * D;
    for (int e = threadIdx.x; e < D * D; e += 256) {
      int row = e / D, col = e % D;
      double re = 0, im = 0;
      if (row < d && col < d) {
        re = src[2 * (row * d + col)];
        im = src[2 * (row * d + col) + 1];
      }
      dst[e] = (T)re;
      dst[D * D + e] = (T)im;
    }
    double s = 0;
    if ((int)threadIdx.x < d)
      for (int row = 0; row < d; ++row) {
        double re = src[2 * (row * d + threadIdx.x)], im = src[2 * (row * d + threadIdx.x) + 1];
        s += sqrt(fma(re, re, im * im));
      }
    colmax[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) colmax[threadIdx.x] = fmax(colmax[threadIdx.x], colmax[threadIdx.x + o]);
      __syncthreads();
    }
    if (threadIdx.x == 0) P.norms[mat] = colmax[0];
  } else {
    if (P.Vz == nullptr || P.Vint == nullptr) return;
    T* dst = reinterpret_cast<T*>(P.Vint);
    for (int e = threadIdx.x; e < D * D; e += 256) {
      int row = e / D, col = e % D;
      double re = 0, im = 0;
      if (row < d && col < d) {
        re = P.Vz[2 * (row * d + col)];
        im = P.Vz[2 * (row * d + col) + 1];
      }
      int w = col >> 4, c16 = col & 15, rb = row >> 4, rr = row & 15;
      int r, g;
      if (sizeof(T) == 4) { g = rr >> 2; r = rr & 3; } else { r = rr >> 2; g = rr & 3; }
      int lane = 16 * g + c16, reg = 4 * rb + r;
      dst[pf_index<T, D>(w, 0, reg, lane)] = (T)re;
      dst[pf_index<T, D>(w, 1, reg, lane)] = (T)im;
    }
  }
}

// ---------------------------------------------------------------- plan

// Per slice: theta = dt (|H0|_1 + sum_j |u[j][k]| |Hc[j]|_1) in FP64, then the
// scaling exponent and Taylor degrees of choose_plan().
__global__ __launch_bounds__(256) void k_plan(const ProbDesc* __restrict__ descs, int nprob, int uniformN,
                                              const int* __restrict__ start, int total, double ur, int grad) {
  int item = blockIdx.x * 256 + threadIdx.x;
  if (item >= total) return;
  int p, k;
  split_item(item, uniformN, start, nprob, p, k);
  const ProbDesc& P = descs[p];
  double th = P.norms[0];
  for (int j = 0; j < P.m; ++j) th = fma(fabs(P.u[(size_t)j * P.N + k]), P.norms[j + 1], th);
  th *= P.dt;
  P.sq[k] = pack_plan(choose_plan(th, ur, grad != 0));
}

// ---------------------------------------------------------------- assembly

// lds <- sgn * (-i) * c * H_k  (sgn = +1: A_k / 2^s with c = dt / 2^s;
// sgn = -1: A_k^dag / 2^s).  H_k = H0 + sum_j u[j][k] Hc[j] in precision T.
template <typename T, int D>
__device__ __forceinline__ void assemble(T* lds, const ProbDesc& P, int k, double c, double sgn) {
  constexpr int NT = Mat<T, D>::NT;
  constexpr int EPT = D * D / NT;
  const T* H = reinterpret_cast<const T*>(P.Hint);
  T hr[EPT], hi[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    int e = threadIdx.x + i * NT;
    hr[i] = H[e];
    hi[i] = H[D * D + e];
  }
  for (int j = 0; j < P.m; ++j) {
    const T uj = (T)P.u[(size_t)j * P.N + k];
    const T* Hj = H + (size_t)(j + 1) * 2 * D * D;
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      int e = threadIdx.x + i * NT;
      hr[i] += uj * Hj[e];
      hi[i] += uj * Hj[D * D + e];
    }
  }
  const T f = (T)(sgn * c);
  T* im = lds + D * Mat<T, D>::SD;
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    int e = threadIdx.x + i * NT;
    int off = lds_off<T, D>(e / D, e % D);
    lds[off] = f * hi[i];   // -i f (hr + i hi) = f hi - i f hr
    im[off] = -f * hr[i];
  }
}

__device__ __forceinline__ void unpack_sq(int sq, int& s, int& q, int& qb) {
  s = sq & 255;
  q = (sq >> 8) & 255;
  qb = (sq >> 16) & 255;
}

// ---------------------------------------------------------------- slice propagators

// Delta_k = U_k - I for every slice: one workgroup per slice, D/16 wavefronts.
// Horner in delta form: R_q = I + X/q, R_i = I + X R_{i+1} / i, Delta = X R_2
// (X = A_k / 2^s), then s squarings Delta <- 2 Delta + Delta^2.
template <typename T, int D>
__global__ __launch_bounds__(4 * D) void k_expm(const ProbDesc* __restrict__ descs, int nprob,
                                                         int uniformN, const int* __restrict__ start, int total) {
  const int item = blockIdx.x;
  if (item >= total) return;
  int p, k;
  split_item(item, uniformN, start, nprob, p, k);
  const ProbDesc& P = descs[p];
  int s, q, qb;
  unpack_sq(P.sq[k], s, q, qb);
  __shared__ T lds[Mat<T, D>::LDS_ELEMS];
  Lane L;
  assemble<T, D>(lds, P, k, ldexp(P.dt, -s), 1.0);
  __syncthreads();
  Panel<T, D> R, acc;
  panel_from_lds(R, lds, L);
  if (q >= 2) {
    panel_scale(R, (T)(1.0 / q));
    panel_add_identity(R, L, (T)1);
    for (int i = q - 1; i >= 2; --i) {
      cgemm(acc, lds, R, L, true);
      R = acc;
      panel_scale(R, (T)(1.0 / i));
      panel_add_identity(R, L, (T)1);
    }
    cgemm(acc, lds, R, L, true);
    R = acc;
  }
  for (int j = 0; j < s; ++j) {
    __syncthreads();
    panel_to_lds(lds, R, L);
    __syncthreads();
    cgemm(acc, lds, R, L, true);
    panel_axpby(R, (T)1, acc, (T)2);
  }
  panel_store(pf_mat<T, D>(P.delta, k), R, L);
}

// ---------------------------------------------------------------- chunked scans

// One workgroup per (chunk, direction).  Forward (blockIdx.y = 0): running
// product S = U_k ... U_{k0}; stores xprev[k] = S before slice k and the chunk
// total.  Backward (blockIdx.y = 1): S = U_k^dag ... U_{k1-1}^dag; stores
// bloc[k] = S before slice k is applied and the chunk total.  Each step is
// S <- S + Delta S (or Delta^dag S) with Delta staged in LDS, double-buffered.
template <typename T, int D>
__global__ __launch_bounds__(4 * D) void k_scan_local(const ProbDesc* __restrict__ descs, int nprob,
                                                               int uniformP, const int* __restrict__ start,
                                                               int total) {
  const int item = blockIdx.x;
  if (item >= total) return;
  const int bwd = blockIdx.y;
  int p, c;
  split_item(item, uniformP, start, nprob, p, c);
  const ProbDesc& P = descs[p];
  const int k0 = c * P.L;
  const int k1 = min(P.N, k0 + P.L);
  __shared__ T lds[2][Mat<T, D>::LDS_ELEMS];
  Lane L;
  Panel<T, D> S, nxt, acc;
  panel_identity(S, L);
  const int n = k1 - k0;
  int k = bwd ? k1 - 1 : k0;
  panel_load(nxt, pf_mat<T, D>(P.delta, k), L);
  for (int i = 0; i < n; ++i) {
    T* buf = lds[i & 1];
    if (bwd) panel_to_lds_ct(buf, nxt, L); else panel_to_lds(buf, nxt, L);
    const int kn = bwd ? k - 1 : k + 1;
    if (i + 1 < n) panel_load(nxt, pf_mat<T, D>(P.delta, kn), L);
    panel_store(pf_mat<T, D>(bwd ? P.bloc : P.xprev, k), S, L);
    __syncthreads();
    cgemm(acc, buf, S, L, true);
    panel_axpby(S, (T)1, acc, (T)1);
    k = kn;
  }
  panel_store(pf_mat<T, D>(bwd ? P.tb : P.tf, c), S, L);
}

// One workgroup per (problem, direction): serial product over chunk totals.
// Forward: cf[c] = P_{k0(c)-1}, ending with X_N, its fidelity against V (FP64
// accumulation) and the unitarity residual |X_N^dag X_N - I|_F.  Backward:
// cb[c] = Q_{k1(c)-1}, starting from V.
template <typename T, int D>
__global__ __launch_bounds__(4 * D) void k_carry(const ProbDesc* __restrict__ descs) {
  const ProbDesc& P = descs[blockIdx.x];
  const int bwd = blockIdx.y;
  constexpr int NW = Mat<T, D>::NW;
  __shared__ T lds[2][Mat<T, D>::LDS_ELEMS];
  __shared__ double red[2 * NW];
  Lane L;
  Panel<T, D> S, nxt, acc;
  const int nc = P.P;
  if (bwd) panel_load(S, reinterpret_cast<const T*>(P.Vint), L); else panel_identity(S, L);
  int c = bwd ? nc - 1 : 0;
  panel_load(nxt, pf_mat<T, D>(bwd ? P.tb : P.tf, c), L);
  const int steps = bwd ? nc - 1 : nc;
  for (int i = 0; i < nc; ++i) {
    panel_store(pf_mat<T, D>(bwd ? P.cb : P.cf, c), S, L);
    if (i == steps) break;
    T* buf = lds[i & 1];
    panel_to_lds(buf, nxt, L);
    const int cn = bwd ? c - 1 : c + 1;
    if (i + 1 < steps) panel_load(nxt, pf_mat<T, D>(bwd ? P.tb : P.tf, cn), L);
    __syncthreads();
    cgemm(acc, buf, S, L, true);
    S = acc;
    c = cn;
  }
  if (bwd) return;
  // S = X_N.
  const int d = P.d;
  if (P.XN) {
#pragma unroll
    for (int rb = 0; rb < D / 16; ++rb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int row = 16 * rb + Prec<T>::rowmap(r, L.g), col = 16 * L.w + L.c16;
        if (row < d && col < d) {
          P.XN[2 * (row * d + col)] = (double)S.re[rb][r];
          P.XN[2 * (row * d + col) + 1] = (double)S.im[rb][r];
        }
      }
  }
  if (P.Vz) {
    double gr = 0, gi = 0;
#pragma unroll
    for (int rb = 0; rb < D / 16; ++rb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int row = 16 * rb + Prec<T>::rowmap(r, L.g), col = 16 * L.w + L.c16;
        if (row < d && col < d) {
          double vr = P.Vz[2 * (row * d + col)], vi = P.Vz[2 * (row * d + col) + 1];
          double xr = (double)S.re[rb][r], xi = (double)S.im[rb][r];
          gr += vr * xr + vi * xi;   // conj(v) x
          gi += vr * xi - vi * xr;
        }
      }
    gr = wave_sum(gr);
    gi = wave_sum(gi);
    if (L.lane == 0) { red[2 * L.w] = gr; red[2 * L.w + 1] = gi; }
    __syncthreads();
    if (threadIdx.x == 0) {
      double a = 0, b = 0;
      for (int w = 0; w < NW; ++w) { a += red[2 * w]; b += red[2 * w + 1]; }
      P.g[0] = a;
      P.g[1] = b;
      *P.F = (a * a + b * b) / ((double)d * d);
    }
  }
  // Unitarity residual of X_N (FP64 accumulation of |X^dag X - I|^2).
  __syncthreads();
  panel_to_lds_ct(lds[0], S, L);
  __syncthreads();
  cgemm(acc, lds[0], S, L, true);
  double e2 = 0;
#pragma unroll
  for (int rb = 0; rb < D / 16; ++rb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int row = 16 * rb + Prec<T>::rowmap(r, L.g), col = 16 * L.w + L.c16;
      if (row < d && col < d) {
        double xr = (double)acc.re[rb][r] - (row == col ? 1.0 : 0.0), xi = (double)acc.im[rb][r];
        e2 += xr * xr + xi * xi;
      }
    }
  e2 = wave_sum(e2);
  __syncthreads();
  if (L.lane == 0) red[L.w] = e2;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0;
    for (int w = 0; w < NW; ++w) a += red[w];
    P.diag[0] = sqrt(a);
  }
}

// mc[c] = cb[c] cf[c]^dag for every chunk, so that W_k = bloc[k] mc[c] xprev[k]^dag.
template <typename T, int D>
__global__ __launch_bounds__(4 * D) void k_mc(const ProbDesc* __restrict__ descs, int nprob, int uniformP,
                                                       const int* __restrict__ start, int total) {
  const int item = blockIdx.x;
  if (item >= total) return;
  int p, c;
  split_item(item, uniformP, start, nprob, p, c);
  const ProbDesc& P = descs[p];
  __shared__ T lds[2][Mat<T, D>::LDS_ELEMS];
  Lane L;
  Panel<T, D> a, b;
  panel_load(a, pf_mat<T, D>(P.cb, c), L);
  panel_to_lds(lds[0], a, L);
  panel_load(b, pf_mat<T, D>(P.cf, c), L);
  panel_to_lds(lds[1], b, L);
  __syncthreads();
  panel_from_lds_ct(b, lds[1], L);
  cgemm(a, lds[0], b, L, true);
  panel_store(pf_mat<T, D>(P.mc, c), a, L);
}

// ---------------------------------------------------------------- adjoint / gradient

// One workgroup per slice.
//  1. W_k = bloc[k] mc[c] xprev[k]^dag  (two products).
//  2. X = A_k^dag / 2^s in LDS buffer 0, E = W_k / 2^s in buffer 1.
//  3. Block Horner of degree qb on M = [[X, E], [0, X]] in delta form:
//     R = [[R1, R2], [0, R1]], R_qb = I + M/qb, R_i = I + M R_{i+1} / i, and
//     M R = [[X R1, X R2 + E R1], [0, X R1]].  Delta block = M R_2.
//  4. s squarings: [[I + D1, Q], [0, I + D1]]^2 gives D1 <- 2 D1 + D1^2 and
//     Q <- 2Q + D1 Q + Q D1.  Z_k = Q.
//  5. T_j = Tr(Z_k^dag Hc[j]) in FP64, grad = (2 dt / d^2) Im(conj(g) T_j).
template <typename T, int D>
__global__ __launch_bounds__(4 * D) void k_adjoint(const ProbDesc* __restrict__ descs, int nprob,
                                                            int uniformN, const int* __restrict__ start, int total) {
  const int item = blockIdx.x;
  if (item >= total) return;
  int p, k;
  split_item(item, uniformN, start, nprob, p, k);
  const ProbDesc& P = descs[p];
  constexpr int NW = Mat<T, D>::NW;
  int s, q, qb;
  unpack_sq(P.sq[k], s, q, qb);
  const int c = k / P.L;
  __shared__ T lds[2][Mat<T, D>::LDS_ELEMS];
  __shared__ double red[2][2 * NW];
  Lane L;
  Panel<T, D> R1, R2, A1, A2;

  // 1. W = bloc[k] (mc[c] xprev[k]^dag)
  panel_load(A1, pf_mat<T, D>(P.mc, c), L);
  panel_to_lds(lds[0], A1, L);
  panel_load(A2, pf_mat<T, D>(P.xprev, k), L);
  panel_to_lds(lds[1], A2, L);
  panel_load(R2, pf_mat<T, D>(P.bloc, k), L);
  __syncthreads();
  panel_from_lds_ct(A2, lds[1], L);
  cgemm(A1, lds[0], A2, L, true);
  __syncthreads();
  panel_to_lds(lds[0], R2, L);
  __syncthreads();
  cgemm(R2, lds[0], A1, L, true);  // R2 = W
  __syncthreads();

  // 2. E = W / 2^s, X = A^dag / 2^s
  const T scl = (T)ldexp(1.0, -s);
  panel_scale(R2, scl);
  panel_to_lds(lds[1], R2, L);
  assemble<T, D>(lds[0], P, k, ldexp(P.dt, -s), -1.0);
  __syncthreads();
  const T* X = lds[0];
  const T* E = lds[1];

  // 3. Horner on the block
  panel_from_lds(R1, X, L);
  panel_scale(R1, (T)(1.0 / qb));
  panel_add_identity(R1, L, (T)1);
  panel_scale(R2, (T)(1.0 / qb));
  for (int i = qb - 1; i >= 2; --i) {
    cgemm(A2, X, R2, L, true);
    cgemm(A2, E, R1, L, false);
    cgemm(A1, X, R1, L, true);
    const T inv = (T)(1.0 / i);
    R1 = A1;
    panel_scale(R1, inv);
    panel_add_identity(R1, L, (T)1);
    R2 = A2;
    panel_scale(R2, inv);
  }
  cgemm(A2, X, R2, L, true);
  cgemm(A2, E, R1, L, false);  // A2 = Q (top-right of the delta block)
  if (s > 0) cgemm(A1, X, R1, L, true);  // A1 = D1 (top-left)

  // 4. squarings
  for (int j = 0; j < s; ++j) {
    __syncthreads();
    panel_to_lds(lds[0], A1, L);
    panel_to_lds(lds[1], A2, L);
    __syncthreads();
    cgemm(R2, lds[0], A2, L, true);   // D1 Q
    cgemm(R2, lds[1], A1, L, false);  // + Q D1
    panel_axpby(R2, (T)2, A2, (T)1);  // R2 = 2Q + D1 Q + Q D1
    if (j + 1 < s) {
      cgemm(R1, lds[0], A1, L, true);
      panel_axpby(A1, (T)1, R1, (T)2);
    }
    A2 = R2;
  }

  // 5. inner products with the controls (FP64), then the gradient
  const T* H = reinterpret_cast<const T*>(P.Hint);
  const double gr = P.g[0], gi = P.g[1];
  const double pref = 2.0 * P.dt / ((double)P.d * P.d);
  for (int j = 0; j < P.m; ++j) {
    const T* Hr = H + (size_t)(j + 1) * 2 * D * D;
    const T* Hi = Hr + D * D;
    double tr = 0, ti = 0;
#pragma unroll
    for (int rb = 0; rb < D / 16; ++rb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int e = (16 * rb + Prec<T>::rowmap(r, L.g)) * D + 16 * L.w + L.c16;
        double zr = (double)A2.re[rb][r], zi = (double)A2.im[rb][r];
        double hr = (double)Hr[e], hi = (double)Hi[e];
        tr += zr * hr + zi * hi;  // conj(z) h
        ti += zr * hi - zi * hr;
      }
    tr = wave_sum(tr);
    ti = wave_sum(ti);
    double* rj = red[j & 1];
    if (L.lane == 0) { rj[2 * L.w] = tr; rj[2 * L.w + 1] = ti; }
    __syncthreads();
    if (threadIdx.x == 0) {
      double a = 0, b = 0;
      for (int w = 0; w < NW; ++w) { a += rj[2 * w]; b += rj[2 * w + 1]; }
      P.grad[(size_t)j * P.N + k] = pref * (gr * b - gi * a);
    }
  }
}

// ---------------------------------------------------------------- launcher

template <typename T, int D>
static hipError_t run(const Launch& L, double ur) {
  constexpr int NT = Mat<T, D>::NT;
  hipStream_t st = L.stream;
  const bool bwd = (L.flags & RUN_BWD) != 0;
  const bool grad = (L.flags & RUN_GRAD) != 0;
  stage_mark(ST_PREP, true, st);
  hipLaunchKernelGGL((k_prep<T, D>), dim3(L.nprob, L.max_m + 2), dim3(256), 0, st, L.descs);
  stage_mark(ST_PREP, false, st);
  stage_mark(ST_PLAN, true, st);
  hipLaunchKernelGGL(k_plan, dim3((L.total_slices + 255) / 256), dim3(256), 0, st, L.descs, L.nprob, L.uniformN,
                     L.slice_start, L.total_slices, ur, grad ? 1 : 0);
  stage_mark(ST_PLAN, false, st);
  stage_mark(ST_EXPM, true, st);
  hipLaunchKernelGGL((k_expm<T, D>), dim3(L.total_slices), dim3(NT), 0, st, L.descs, L.nprob, L.uniformN,
                     L.slice_start, L.total_slices);
  stage_mark(ST_EXPM, false, st);
  stage_mark(ST_SCAN, true, st);
  hipLaunchKernelGGL((k_scan_local<T, D>), dim3(L.total_chunks, bwd ? 2 : 1), dim3(NT), 0, st, L.descs, L.nprob,
                     L.uniformP, L.chunk_start, L.total_chunks);
  stage_mark(ST_SCAN, false, st);
  stage_mark(ST_CARRY, true, st);
  hipLaunchKernelGGL((k_carry<T, D>), dim3(L.nprob, bwd ? 2 : 1), dim3(NT), 0, st, L.descs);
  stage_mark(ST_CARRY, false, st);
  if (grad) {
    stage_mark(ST_MC, true, st);
    hipLaunchKernelGGL((k_mc<T, D>), dim3(L.total_chunks), dim3(NT), 0, st, L.descs, L.nprob, L.uniformP,
                       L.chunk_start, L.total_chunks);
    stage_mark(ST_MC, false, st);
    stage_mark(ST_ADJ, true, st);
    hipLaunchKernelGGL((k_adjoint<T, D>), dim3(L.total_slices), dim3(NT), 0, st, L.descs, L.nprob, L.uniformN,
                       L.slice_start, L.total_slices);
    stage_mark(ST_ADJ, false, st);
  }
  return hipGetLastError();
}

hipError_t launch_path(int precision, int D, const Launch& L) {
  const double ur64 = 0x1p-53, ur32 = 0x1p-24;
  if (precision == 0) {
    switch (D) {
      case 16: return run<double, 16>(L, ur64);
      case 32: return run<double, 32>(L, ur64);
      case 64: return run<double, 64>(L, ur64);
    }
  } else if (precision == 1) {
    switch (D) {
      case 16: return run<float, 16>(L, ur32);
      case 32: return run<float, 32>(L, ur32);
      case 64: return run<float, 64>(L, ur32);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace qoc
