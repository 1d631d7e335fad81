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
#include <type_traits>

#include "qoc_device.hpp"
#include "qoc_internal.hpp"
#include "qoc_plan.hpp"
#include "qoc_bf16.hpp"

namespace qoc {

// ---------------------------------------------------------------- work items

__device__ __forceinline__ int locate(const int* start, int n, int item) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (gp(start)[mid] <= item) lo = mid; else hi = mid;
  }
  return lo;
}

// Map a flat work item to (problem, slice or chunk index).  Uniform launches
// (count > 0) cover indices [lo, lo + count) of every problem; otherwise the
// items of problem p are [start[p], start[p + 1]).
__device__ __forceinline__ void split_item(int item, int lo, int count, const int* start, int n, int& p, int& k) {
  if (count > 0) {
    p = item / count;
    k = lo + (item - p * count);
  } else {
    p = locate(start, n, item);
    k = item - gp(start)[p];
  }
}

// The item counts of a launch (see Work).
struct Items {
  int nprob, total;
  const int* start;
  const int* slot;  // descriptor index of each problem (engine launches), else identity
  __device__ __forceinline__ explicit Items(const Work& W) {
    if (W.dyn) {
      nprob = gp(W.dyn)[0];
      total = gp(W.dyn)[1];
      start = W.dyn + 2;
      slot = W.dyn + 3 + nprob;
    } else {
      nprob = W.nprob;
      total = W.total;
      start = W.start;
      slot = nullptr;
    }
  }
  __device__ __forceinline__ int desc(int p) const { return slot ? gp(slot)[p] : p; }
};

template <typename T, int D>
__device__ __forceinline__ T* pf_mat(void* base, int i) {
  return reinterpret_cast<T*>(base) + (size_t)i * Mat<T, D>::ELEMS;
}

// ---------------------------------------------------------------- prep

// Row table of control j: for each row a, the column and value (in
// precision T, as the dense copy holds it) of its nonzero, and whether every
// row has at most one.  Such controls (Pauli strings, for instance) are then
// assembled and paired with Z_k entry by entry.  The table is written even
// when the control does not qualify; mok[j] says whether it may be used.
template <typename T, int D>
__device__ __forceinline__ void control_rows(const ProbDesc& P, int j, const double* src) {
  const int d = P.d;
  const int a = threadIdx.x;
  const bool gen = (P.flags & RUN_GENERAL) != 0;  // stored as i G (see prep_one)
  __shared__ int hits[D];  // rows whose entry lies in each column
  if (a < D) hits[a] = 0;
  __syncthreads();
  int multi = 0, col = a;
  {
    if (a < D) {
      int cnt = 0;
      T vr = 0, vi = 0;
      if (a < d)
        for (int c = 0; c < d; ++c) {
          const double sr = src[2 * (a * d + c)], si = src[2 * (a * d + c) + 1];
          const T r = (T)(gen ? -si : sr), i = (T)(gen ? sr : si);
          if (r != (T)0 || i != (T)0) {
            ++cnt;
            col = c;
            vr = r;
            vi = i;
          }
        }
      multi = cnt > 1;
      const size_t idx = (size_t)j * D + a;
      gp(P.mcol)[idx] = col;
      gp(reinterpret_cast<T*>(P.mval))[2 * idx] = vr;
      gp(reinterpret_cast<T*>(P.mval))[2 * idx + 1] = vi;
      atomicAdd(&hits[col], 1);
    }
  }
  // Whether control j - 1 puts its entries at the same columns (X_i and Y_i
  // do), from its source rows: then the entries of Z that both read are the
  // same (flag 4).
  int same = 1;
  if (j > 0 && a < d) {
    const double* prev = src - 2 * (size_t)d * d;
    int pc = a;
    for (int c = 0; c < d; ++c)
      if (prev[2 * (a * d + c)] != 0.0 || prev[2 * (a * d + c) + 1] != 0.0) pc = c;
    same = pc == col;
  }
  const int any = __syncthreads_or(multi);
  // A bijection when every column is hit once (empty rows count at their own
  // column, with a zero entry); then minv[j][col_j(a)] = a.
  const int bij = __syncthreads_and(a >= D || hits[a] == 1);
  const int all_same = __syncthreads_and(same) && j > 0;
  if (P.minv && a < D) gp(P.minv)[(size_t)j * D + col] = a;
  if (threadIdx.x == 0)
    gp(P.mok)[j] = (!any && !(P.flags & CTRL_DENSE)) ? (1 | (bij && P.minv ? 2 : 0) | (all_same ? 4 : 0)) : 0;
}

// True when every control of the problem has a usable row table (at most
// one nonzero per row, dense kernels not forced).  Uniform across the
// workgroup.
__device__ __forceinline__ bool controls_monomial(const ProbDesc& P) {
  for (int j = 0; j < P.m; ++j)
    if (!gp(P.mok)[j]) return false;
  return true;
}

// True when every control's row table is also a bijection from rows to
// columns (minv holds its inverse).  (All the flags are loaded together.)
__device__ __forceinline__ bool controls_permutation(const ProbDesc& P) {
  int all = 2;
  for (int j = 0; j < P.m; ++j) all &= gp(P.mok)[j];
  return all != 0;
}

// Bit 24 of a slice's packed plan: the FP32 adjoint may sample its last step
// there (s = 0 and permutation controls), so that the adjoint's two instances
// split the slices with the one load of the plan.
constexpr int kPlanSampled = 1 << 24;

// Convert the caller's complex128 matrices to the compute precision: H0 and
// Hc[j] to planar D x D (zero padded), V to PF; also the FP64 one-norms
// (largest column sum of moduli) of H0 and Hc[j].  With general generators
// (RUN_GENERAL) the caller's G is stored as H = i G, so that every kernel's
// A = -i dt H is dt G, and the norm is the larger of the one- and
// infinity-norms: the adjoint works with A^dag, whose one-norm is A's
// infinity-norm.
template <typename T, int D>
__device__ __forceinline__ void prep_one(const ProbDesc& P, int mat, double* colmax) {
  const int d = P.d, m = P.m;
  if (mat == 0 && threadIdx.x == 0) {
    P.diag[1] = 0.0;
    P.diag[2] = 0.0;
  }
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
      if (P.flags & RUN_GENERAL) {  // i (re + i im)
        const double t = re;
        re = -im;
        im = t;
      }
      dst[e] = (T)re;
      dst[D * D + e] = (T)im;
    }
    double s = 0;
    if ((int)threadIdx.x < d) {
      for (int row = 0; row < d; ++row) {
        double re = src[2 * (row * d + threadIdx.x)], im = src[2 * (row * d + threadIdx.x) + 1];
        s += sqrt(fma(re, re, im * im));
      }
      if (P.flags & RUN_GENERAL) {
        double r = 0;
        for (int col = 0; col < d; ++col) {
          double re = src[2 * (threadIdx.x * d + col)], im = src[2 * (threadIdx.x * d + col) + 1];
          r += sqrt(fma(re, re, im * im));
        }
        s = fmax(s, r);
      }
    }
    colmax[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) colmax[threadIdx.x] = fmax(colmax[threadIdx.x], colmax[threadIdx.x + o]);
      __syncthreads();
    }
    if (threadIdx.x == 0) P.norms[mat] = colmax[0];
    if (mat > 0) control_rows<T, D>(P, mat - 1, src);
    __syncthreads();
  } else if (P.Vz != nullptr && P.Vint != nullptr) {
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

// Convert the caller's complex128 matrices to the compute precision: H0 and
// Hc[j] to planar D x D (zero padded), V to PF; also the FP64 one-norms
// (largest column sum of moduli) of H0 and Hc[j].  Items: (problem, matrix
// index 0..m+1) with index m+1 standing for V; 256 threads per item.
template <typename T, int D>
__global__ __launch_bounds__(256) void k_prep(Work W) {
  __shared__ double colmax[256];
  const Items I(W);
  for (int item = blockIdx.x; item < I.total; item += gridDim.x) {
    int p, mat;
    split_item(item, 0, W.rg.s_n, I.start, I.nprob, p, mat);
    prep_one<T, D>(W.descs[I.desc(p)], mat, colmax);
  }
}

// ---------------------------------------------------------------- plan

// Per slice: theta = dt (|H0|_1 + sum_j |u[j][k]| |Hc[j]|_1) in FP64, then the
// scaling exponent and Taylor degrees of choose_plan().
// flags: bit 0 gradient, bit 1 the expm evaluates by Paterson-Stockmeyer
// (FP32 at D = 128).
__global__ __launch_bounds__(256) void k_plan(Work W, double ur, int flags) {
  const Items I(W);
  for (int item = blockIdx.x * 256 + threadIdx.x; item < I.total; item += gridDim.x * 256) {
    int p, k;
    split_item(item, W.rg.s_lo, W.rg.s_n, I.start, I.nprob, p, k);
    const ProbDesc P = W.descs[I.desc(p)];  // a copy: stores cannot alias it
    double th = P.norms[0];
    for (int j = 0; j < P.m; ++j) th = fma(fabs(gp(P.u)[(size_t)j * P.N + k]), gp(P.norms)[j + 1], th);
    th *= P.dt;
    const SlicePlan pl = choose_plan(th, ur, (flags & 1) != 0, (flags & 2) != 0);
    P.sq[k] = pack_plan(pl) | (pl.s == 0 && controls_permutation(P) ? kPlanSampled : 0);
  }
}

// ---------------------------------------------------------------- assembly

// The planar LDS layout of panel_to_lds (StdOps), which assemble's scatter
// form writes and reads directly.
template <typename T, int D, typename Ops>
constexpr bool kStdLds = std::is_same<Ops, StdOps<T, D>>::value;

// lds <- sgn * (-i) * c * H_k  (sgn = +1: A_k / 2^s with c = dt / 2^s;
// sgn = -1: A_k^dag / 2^s).  H_k = H0 + sum_j u[j][k] Hc[j] in precision T.
template <typename T, int D, typename Ops, int G = 1>
__device__ __forceinline__ void assemble(void* lds, const ProbDesc& P, int k, double c, double sgn, T* hk,
                                         bool mono, bool ct = false) {
  // The matrix is read as D^2/4 chunks of four consecutive row elements;
  // thread t owns chunks t, t + 4D, t + 8D, ... (D/16 of them), so that the
  // lanes of one 16-byte load read consecutive chunks.  The loads of G
  // controls are in flight together; indices past the last control are
  // clamped to it and weighted by zero, which leaves every sum unchanged.
  // Chunks are written to LDS four columns at a time.  When hk is not null,
  // H_k itself is also written there (planar, row-major) for the adjoint.
  // With mono (every control has at most one nonzero per row) each chunk
  // takes its row's entry of each control from the row tables instead: the
  // same products, minus those with structural zeros.
  using v4 = typename Prec<T>::v4;
  constexpr int NV = D / 16;
  constexpr int NT = 4 * D;
  const T* H = reinterpret_cast<const T*>(P.Hint);
  const int e0 = 4 * threadIdx.x;
  v4 hr[NV], hi[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    hr[v] = Prec<T>::gld4(H + e0 + 4 * NT * v);
    hi[v] = Prec<T>::gld4(H + D * D + e0 + 4 * NT * v);
  }
  const size_t tab_bytes = (size_t)P.m * D * (sizeof(int) + 2 * sizeof(T)) + (size_t)P.m * sizeof(T);
  if (mono && D >= 32 && !ct && kStdLds<T, D, Ops>) {
    // Scatter form (D >= 32, where the expm is the only row-table caller):
    // H0 goes to LDS unscaled; thread a < D then adds u_j Hc[j][a][col_j(a)]
    // to entry (a, col_j(a)) of its own row for j = 0 ... m - 1 (the dense
    // sum's nonzero terms in its order, so H_k is the same); every thread
    // then reads its chunks back.  O(m D) work instead of every thread
    // scanning every control for its chunks.
    T* pl = static_cast<T*>(lds);
    T* pi = pl + D * Mat<T, D>::SD;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int e = e0 + 4 * NT * v;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int off = lds_off<T, D>(e / D, e % D + i);
        pl[off] = hr[v][i];
        pi[off] = hi[v][i];
      }
    }
    __syncthreads();
    if ((int)threadIdx.x < D) {
      const int a = threadIdx.x;
      const T* mv = reinterpret_cast<const T*>(P.mval);
      for (int j = 0; j < P.m; ++j) {
        const size_t idx = (size_t)j * D + a;
        const T uj = (T)gp(P.u)[(size_t)j * P.N + k];
        const int off = lds_off<T, D>(a, gp(P.mcol)[idx]);
        pl[off] = fma(uj, gp(mv)[2 * idx], pl[off]);
        pi[off] = fma(uj, gp(mv)[2 * idx + 1], pi[off]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int e = e0 + 4 * NT * v;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int off = lds_off<T, D>(e / D, e % D + i);
        hr[v][i] = pl[off];
        hi[v][i] = pi[off];
      }
    }
  } else if (mono && tab_bytes <= (size_t)Ops::BYTES) {
    // The problem's row tables and the slice's amplitudes go through LDS (the
    // left-factor space, written below only after a barrier): one round trip
    // of coalesced loads instead of one per group of controls.
    const int mD = P.m * D;
    int* lc = static_cast<int*>(lds);
    T* lv = reinterpret_cast<T*>(lc + mD);
    T* lu = lv + 2 * mD;
    const T* mv = reinterpret_cast<const T*>(P.mval);
#pragma unroll 4
    for (int i = threadIdx.x; i < mD; i += NT) {
      lc[i] = gp(P.mcol)[i];
      lv[2 * i] = gp(mv)[2 * i];
      lv[2 * i + 1] = gp(mv)[2 * i + 1];
    }
    for (int j = threadIdx.x; j < P.m; j += NT) lu[j] = (T)gp(P.u)[(size_t)j * P.N + k];
    __syncthreads();
    for (int j = 0; j < P.m; ++j) {
      const T uj = lu[j];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int e = e0 + 4 * NT * v;
        const int idx = j * D + e / D, c0 = e % D;
        const int col = lc[idx];
        const T vr = lv[2 * idx], vi = lv[2 * idx + 1];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const T w = col == c0 + i ? uj : (T)0;
          hr[v][i] += w * vr;
          hi[v][i] += w * vi;
        }
      }
    }
    __syncthreads();  // the tables are read; the LDS takes the left factor next
  } else if (mono) {
    constexpr int GM = 4;  // controls whose table entries are loaded together
    const T* mv = reinterpret_cast<const T*>(P.mval);
    for (int j0 = 0; j0 < P.m; j0 += GM) {
      int col[GM][NV];
      T vr[GM][NV], vi[GM][NV], uw[GM];
#pragma unroll
      for (int jj = 0; jj < GM; ++jj) {
        const int j = min(j0 + jj, P.m - 1);
        uw[jj] = j0 + jj < P.m ? (T)gp(P.u)[(size_t)j * P.N + k] : (T)0;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const size_t idx = (size_t)j * D + (e0 + 4 * NT * v) / D;
          col[jj][v] = gp(P.mcol)[idx];
          vr[jj][v] = gp(mv)[2 * idx];
          vi[jj][v] = gp(mv)[2 * idx + 1];
        }
      }
#pragma unroll
      for (int jj = 0; jj < GM; ++jj)
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const int c0 = (e0 + 4 * NT * v) % D;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const T w = col[jj][v] == c0 + i ? uw[jj] : (T)0;
            hr[v][i] += w * vr[jj][v];
            hi[v][i] += w * vi[jj][v];
          }
        }
    }
  } else
  for (int j0 = 0; j0 < P.m; j0 += G) {
    v4 ar[G][NV], ai[G][NV];
    T uw[G];
#pragma unroll
    for (int jj = 0; jj < G; ++jj) {
      const int j = min(j0 + jj, P.m - 1);
      uw[jj] = j0 + jj < P.m ? (T)gp(P.u)[(size_t)j * P.N + k] : (T)0;
      const T* Hj = H + (size_t)(j + 1) * 2 * D * D + e0;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        ar[jj][v] = Prec<T>::gld4(Hj + 4 * NT * v);
        ai[jj][v] = Prec<T>::gld4(Hj + D * D + 4 * NT * v);
      }
    }
#pragma unroll
    for (int jj = 0; jj < G; ++jj)
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        hr[v] += uw[jj] * ar[jj][v];
        hi[v] += uw[jj] * ai[jj][v];
      }
  }
  const T f = (T)(sgn * c);
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int e = e0 + 4 * NT * v;
    if (ct) {
      // (-i (-f) H)^dag = -i f H^dag (see ham_put): element (col, row) is
      // -i f conj(H[row][col]) = -f hi - i f hr
#pragma unroll
      for (int i = 0; i < 4; ++i) Ops::put(lds, e % D + i, e / D, -f * hi[v][i], -f * hr[v][i]);
    } else {
      Ops::put4(lds, e / D, e % D, f * hi[v], -f * hr[v]);  // -i f (hr + i hi)
    }
    if (hk) {
      Prec<T>::gst4(hk + e, hr[v]);
      Prec<T>::gst4(hk + D * D + e, hi[v]);
    }
  }
}

// The slice's H_k as stored by k_expm: ham_load issues the loads of this
// thread's chunks (the same chunks as assemble), ham_put writes them to LDS,
// scaled, as assemble() writes its result.
template <typename T, int D>
struct HamRegs {
  typename Prec<T>::v4 hr[D / 16], hi[D / 16];
};

template <typename T, int D>
__device__ __forceinline__ void ham_load(HamRegs<T, D>& H, const T* hk) {
  constexpr int NT = 4 * D;
  const int e0 = 4 * threadIdx.x;
#pragma unroll
  for (int v = 0; v < D / 16; ++v) {
    H.hr[v] = Prec<T>::gld4(hk + e0 + 4 * NT * v);
    H.hi[v] = Prec<T>::gld4(hk + D * D + e0 + 4 * NT * v);
  }
}

// ct: write (-i (-sgn) c H_k)^dag instead of -i sgn c H_k.  The two agree
// when H_k is Hermitian; for general generators the adjoint's call
// (sgn = -1) then gets (-i c H_k)^dag = A_k^dag / 2^s.
template <typename T, int D, typename Ops>
__device__ __forceinline__ void ham_put(void* lds, const HamRegs<T, D>& H, double c, double sgn, bool ct = false) {
  constexpr int NT = 4 * D;
  const int e0 = 4 * threadIdx.x;
  const T f = (T)(sgn * c);
#pragma unroll
  for (int v = 0; v < D / 16; ++v) {
    const int e = e0 + 4 * NT * v;
    if (ct) {
#pragma unroll
      for (int i = 0; i < 4; ++i) Ops::put(lds, e % D + i, e / D, -f * H.hi[v][i], -f * H.hr[v][i]);
    } else {
      Ops::put4(lds, e / D, e % D, f * H.hi[v], -f * H.hr[v]);
    }
  }
}

__device__ __forceinline__ void unpack_sq(int sq, int& s, int& q, int& qb) {
  s = sq & 255;
  q = (sq >> 8) & 255;
  qb = (sq >> 16) & 255;
}

// ---------------------------------------------------------------- epilogues

// S = X_N (panel): write X_N if requested, then g = Tr(V^dag X_N) and
// F = |g|^2 / d^2 with FP64 accumulation.  red: 2 * D/16 doubles of LDS.
template <typename T, int D>
__device__ __forceinline__ void fidelity_epilogue(const ProbDesc& P, const Panel<T, D>& S, const Lane& L,
                                                  double* red) {
  constexpr int NW = D / 16;
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
          gr += vr * xr + vi * xi;  // conj(v) x
          gi += vr * xi - vi * xr;
        }
      }
    gr = wave_sum(gr);
    gi = wave_sum(gi);
    __syncthreads();
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
}

// G = S^dag S (panel): diag[0] = |G - I|_F over the d x d block, FP64 accumulation.
template <typename T, int D>
__device__ __forceinline__ void residual_epilogue(const ProbDesc& P, const Panel<T, D>& G, const Lane& L,
                                                  double* red) {
  constexpr int NW = D / 16;
  const int d = P.d;
  double e2 = 0;
#pragma unroll
  for (int rb = 0; rb < D / 16; ++rb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int row = 16 * rb + Prec<T>::rowmap(r, L.g), col = 16 * L.w + L.c16;
      if (row < d && col < d) {
        double xr = (double)G.re[rb][r] - (row == col ? 1.0 : 0.0), xi = (double)G.im[rb][r];
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

// Gradient from Z = Z_k: T_j = Tr(Z^dag Hc[j]) with FP64 accumulation and
// grad[j][k] = (2 dt / d^2) Im(conj(g) T_j).  Controls are taken in groups
// (kEpiGroup, or kEpiDense for the FP32 dense controls): every lane forms
// its partial sums for the whole group, one multi-value wavefront reduction
// combines them, one barrier publishes the per-wavefront totals and one
// thread per control adds those up.  Control indices past the last one are
// clamped to it, so every load stays in bounds, and their sums are
// discarded.  red: 2 x 2 G x (threads / 64) doubles of LDS for groups of G
// (double-buffered by group).
constexpr int kEpiGroup = 4;
// Controls reduced together by the FP32 dense-control epilogue.
constexpr int kEpiDense = 8;

// Stores the gradient entry (j, k) from T_j = a + i b.
__device__ __forceinline__ void grad_put(const ProbDesc& P, int j, int k, double a, double b) {
  if (P.flags & RUN_RAWDG) {
    // dg/du[j][k] = -i dt Tr(Z_k^dag Hc[j]), complex interleaved
    const size_t o = 2 * ((size_t)j * P.N + k);
    gp(P.grad)[o] = P.dt * b;
    gp(P.grad)[o + 1] = -P.dt * a;
  } else {
    const double pref = 2.0 * P.dt / ((double)P.d * P.d);
    gp(P.grad)[(size_t)j * P.N + k] = pref * (gp(P.g)[0] * b - gp(P.g)[1] * a);
  }
}

template <int NWAVES, int G = kEpiGroup>
__device__ __forceinline__ void epilogue_publish(const ProbDesc& P, int k, int j0, int grp, double (&v)[2 * G],
                                                 const Lane& L, double* red) {
  constexpr int V = 2 * G;
  constexpr int SH = 6 - __builtin_ctz(V);
  const int nj = min(G, P.m - j0);
  const double t = wave_sum_many<V>(v, L.lane);
  double* rg = red + (grp & 1) * V * NWAVES;
  if ((L.lane & ((1 << SH) - 1)) == 0) rg[(L.lane >> SH) * NWAVES + L.w] = t;
  __syncthreads();
  if ((int)threadIdx.x < nj) {
    const int jj = threadIdx.x;
    double a = 0, b = 0;
    for (int w = 0; w < NWAVES; ++w) {
      a += rg[(2 * jj) * NWAVES + w];
      b += rg[(2 * jj + 1) * NWAVES + w];
    }
    grad_put(P, j0 + jj, k, a, b);
  }
}

// D <= 64: Z goes through LDS (the caller's left-factor space, free once every
// wavefront has finished its products), so that thread t owns the chunks of
// four consecutive row elements t, t + 4D, t + 8D, ... and reads each
// control's matching chunks with 16-byte loads, consecutive across lanes.
// With mono (every control has at most one nonzero per row), Tr(Z^dag Hc[j])
// is the sum over rows a of conj(Z[a][col_j(a)]) val_j(a): thread t takes row
// t % D of control j0 + t / D of each group of four controls.
template <typename T, int D>
__device__ __forceinline__ void gradient_epilogue(const ProbDesc& P, int k, const Panel<T, D>& Z, const Lane& L,
                                                  void* lds, double* red, bool mono) {
  using v4 = typename Prec<T>::v4;
  constexpr int NV = D / 16;
  constexpr int EPT = 4 * NV;
  constexpr int NT = 4 * D;
  constexpr int SD = Mat<T, D>::SD;
  static_assert(NT == kEpiGroup * D, "one (control, row) pair per thread");
  T* zl = static_cast<T*>(lds);
  __syncthreads();  // every wavefront is done with the left factors
  panel_to_lds(zl, Z, L);
  __syncthreads();
  if (mono) {
    // The D threads of lane group jj = t / D (aligned inside one wavefront)
    // take row a = t % D of controls jj, jj + 4, jj + 8, jj + 12 of each
    // pass of 16, so that one control's sum stays inside one lane group: one
    // multi-value group reduction per pass and no barrier.
    constexpr int CPT = 4;
    constexpr int V = 2 * CPT;
    constexpr int GV = D / V;  // lanes per reduced value
    const int a = threadIdx.x % D, jj = threadIdx.x / D;
    const T* mv = reinterpret_cast<const T*>(P.mval);
    for (int j0 = 0; j0 < P.m; j0 += kEpiGroup * CPT) {
      double v[V];
#pragma unroll
      for (int i = 0; i < CPT; ++i) {
        const int j = j0 + jj + kEpiGroup * i;
        double tr = 0, ti = 0;
        if (j < P.m) {
          const size_t idx = (size_t)j * D + a;
          const int off = lds_off<T, D>(a, gp(P.mcol)[idx]);
          const double zr = (double)zl[off], zi = (double)zl[D * SD + off];
          const double x = (double)gp(mv)[2 * idx], y = (double)gp(mv)[2 * idx + 1];
          tr = zr * x + zi * y;  // conj(z) h
          ti = zr * y - zi * x;
        }
        v[2 * i] = tr;
        v[2 * i + 1] = ti;
      }
      const double t = group_sum_many<V, D>(v, L.lane);
      const double t1 = __shfl_xor(t, GV, 64);  // the other half of the complex sum
      const int vi = a / GV;
      if (a % GV == 0 && (vi & 1) == 0) {
        const int j = j0 + jj + kEpiGroup * (vi >> 1);
        if (j < P.m) grad_put(P, j, k, t, t1);
      }
    }
    return;
  }
  const int e0 = 4 * threadIdx.x;
  double zr[EPT], zi[EPT];
#pragma unroll
  for (int q = 0; q < NV; ++q)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int e = e0 + 4 * NT * q;
      const int off = lds_off<T, D>(e / D, e % D + i);
      zr[4 * q + i] = (double)zl[off];
      zi[4 * q + i] = (double)zl[D * SD + off];
    }
  // FP32 keeps the sums of kEpiDense controls together for one multi-value
  // reduction and one barrier; FP64 (whose values take twice the registers)
  // publishes every kEpiGroup controls.  LG controls' row segments are
  // loaded together.
  constexpr bool F32 = sizeof(T) == 4;
  constexpr int JG = F32 ? kEpiDense : kEpiGroup;
  constexpr int LG = 2;
  const T* H = reinterpret_cast<const T*>(P.Hint);
  for (int j0 = 0, grp = 0; j0 < P.m; j0 += JG, ++grp) {
    double v[2 * JG];
#pragma unroll
    for (int jb = 0; jb < JG; jb += LG) {
      double tr[LG], ti[LG];
#pragma unroll
      for (int jj = 0; jj < LG; ++jj) tr[jj] = ti[jj] = 0.0;
      if (!F32 || j0 + jb < P.m) {  // (FP32 groups: nothing to load past the last control)
        v4 hr[LG][NV], hi[LG][NV];
#pragma unroll
        for (int jj = 0; jj < LG; ++jj) {
          const int j = min(j0 + jb + jj, P.m - 1);
          const T* Hj = H + (size_t)(j + 1) * 2 * D * D + e0;
#pragma unroll
          for (int q = 0; q < NV; ++q) {
            hr[jj][q] = Prec<T>::gld4(Hj + 4 * NT * q);
            hi[jj][q] = Prec<T>::gld4(Hj + D * D + 4 * NT * q);
          }
        }
#pragma unroll
        for (int jj = 0; jj < LG; ++jj)
#pragma unroll
          for (int q = 0; q < NV; ++q)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const double a = zr[4 * q + i], b = zi[4 * q + i];
              const double x = (double)hr[jj][q][i], y = (double)hi[jj][q][i];
              tr[jj] += a * x + b * y;  // conj(z) h
              ti[jj] += a * y - b * x;
            }
      }
#pragma unroll
      for (int jj = 0; jj < LG; ++jj) {
        v[2 * (jb + jj)] = tr[jj];
        v[2 * (jb + jj) + 1] = ti[jj];
      }
    }
    epilogue_publish<D / 16, JG>(P, k, j0, grp, v, L, red);
  }
}

// ---------------------------------------------------------------- slice propagators

// Delta_k = U_k - I for every slice: one workgroup per slice, D/16 wavefronts.
// Horner in delta form: R_q = I + X/q, R_i = I + X R_{i+1} / i, Delta = X R_2
// (X = A_k / 2^s), then s squarings Delta <- 2 Delta + Delta^2.
// FP32 gradient runs at D >= 32 keep X^2 for the adjoint (keep_square).
// (Paterson-Stockmeyer in X^2, which would form X^2 as a product, needs the
// same two products at q = 3 but held 40 more VGPRs at d = 64, a workgroup
// per CU less, and was 0.4 ms slower on the d = 64 batch of 32.)
// The expm and scan kernels take the three-product form (Ops::gemm3) at
// D >= 32 with a floor of two waves per SIMD, which keeps the extra registers
// of that form from lowering their occupancy.
template <int D>
constexpr int kMinWaves = D >= 32 ? 2 : 1;

// The slice Hamiltonians are kept for the adjoint at D >= 32.  At D = 16 the
// adjoint re-assembles H_k from the (L2-resident) controls, which costs less
// than writing and reading it back through HBM.
template <int D>
constexpr bool kKeepH = D >= 32;

// The expm's products take their steps in pairs (cgemm3m) in FP32; in FP64
// the extra fragment registers would add to its spills.
template <typename T>
constexpr int kExpmPairs = sizeof(T) == 4 ? 2 : 1;
// FP32 keeps X2 = (A_k / 2^s)^2 for the adjoint at D >= 32 (where the
// workspace has room for it: not for the split-BF16 adjoint, P.x2 null); in
// FP64 the read-back would make the d = 64 adjoint spill, and it forms X2
// itself.
template <typename T>
constexpr bool kKeepX2 = sizeof(T) == 4;

// The first Horner product is P1 = X (I + X/q) = X + X^2/q, so
// X^2 = q (P1 - X) comes without a product of its own (X re-read from LDS).
// Its error, about q u |X| against |X^2|, enters the adjoint's Z only through
// terms of size |X^2| |E|, so Z keeps an error of order q u |X| |E|.  For
// Hermitian H_k the adjoint's X = A_k^dag / 2^s = -A_k / 2^s has the same
// square.
template <typename T, int D, typename Ops>
__device__ __forceinline__ void keep_square(T* out, const Panel<T, D>& P1, const void* lds, int q, const Lane& L) {
  Panel<T, D> X;
  Ops::load(X, lds, L);
  panel_axpby(X, (T)q, P1, (T)-q);
  panel_store(out, X, L);
}

// The FP32 d = 64 expm (one slice per workgroup) takes a floor of four waves
// per SIMD: it needs 130 VGPRs otherwise, and at 128 (two spilled) four
// workgroups share a CU instead of three (expm 1.88 -> 1.80 ms on the d = 64
// batch of 32).  The engine's persistent instance keeps the floor of two.
template <typename T, int D, bool PERSIST>
constexpr int kExpmWaves = (sizeof(T) == 4 && D == 64 && !PERSIST) ? 4 : kMinWaves<D>;

template <typename T, int D, typename Ops, bool PERSIST>
__global__ __launch_bounds__(4 * D) __attribute__((amdgpu_waves_per_eu(kExpmWaves<T, D, PERSIST>)))
void k_expm(Work W) {
  __shared__ __align__(16) unsigned char lds[Ops::BYTES];
  Lane L;
  const Items I(W);
  for (int item = blockIdx.x; item < I.total; item += gridDim.x) {
  int p, k;
  split_item(item, W.rg.s_lo, W.rg.s_n, I.start, I.nprob, p, k);
  const ProbDesc P = W.descs[I.desc(p)];  // a copy: stores cannot alias it
  int s, q, qb;
  unpack_sq(gp(P.sq)[k], s, q, qb);
  T* hk = (kKeepH<D> && (P.flags & RUN_GRAD)) ? pf_mat<T, D>(P.hk, k - W.rg.kbase) : nullptr;
  assemble<T, D, Ops>(lds, P, k, ldexp(P.dt, -s), 1.0, hk, controls_monomial(P));
  __syncthreads();
  Panel<T, D> R, acc;
  Ops::load(R, lds, L);
  T* x2 = (kKeepX2<T> && hk && P.x2) ? pf_mat<T, D>(P.x2, k - W.rg.kbase) : nullptr;
  if (q >= 2) {
    panel_scale(R, (T)(1.0 / q));
    panel_add_identity(R, L, (T)1);
    for (int i = q - 1; i >= 1; --i) {
      Ops::template gemm3<kExpmPairs<T>>(acc, lds, R, L, true);
      if (x2 && i == q - 1) keep_square<T, D, Ops>(x2, acc, lds, q, L);
      R = acc;
      if (i >= 2) {
        panel_scale(R, (T)(1.0 / i));
        panel_add_identity(R, L, (T)1);
      }
    }
  }
  for (int j = 0; j < s; ++j) {
    __syncthreads();
    Ops::store(lds, R, L);
    __syncthreads();
    Ops::template gemm3<kExpmPairs<T>>(acc, lds, R, L, true);
    panel_axpby(R, (T)1, acc, (T)2);
  }
  panel_store(pf_mat<T, D>(P.delta, k - W.rg.kbase), R, L);
  if constexpr (!PERSIST) break;  // one item per workgroup: a single-trip loop
  __syncthreads();
  }
}

// ---------------------------------------------------------------- re-unitarisation

// Check of a chunk product S (FP32 panel) in FP64: r = |S^dag S - I|_F over
// the d x d block, recorded as the largest residual of the problem.  When
// r > tol, one Newton-Schulz polar step S <- S (3I - S^dag S) / 2 (Higham
// 1986) moves S back towards the unitary group; the steps are counted.  The
// FP32 panel is moved into the FP64 register layout (and back) through LDS,
// which must hold one FP64 matrix.
template <int D>
__device__ __forceinline__ void reunitarise(const ProbDesc& P, Panel<float, D>& S, void* lds_raw, double* red,
                                            const Lane& L) {
  constexpr int NW = D / 16;
  double* M = static_cast<double*>(lds_raw);
  double* Mi = M + D * Mat<double, D>::SD;
  const int d = P.d;
  __syncthreads();
#pragma unroll
  for (int rb = 0; rb < D / 16; ++rb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int off = lds_off<double, D>(16 * rb + Prec<float>::rowmap(r, L.g), 16 * L.w + L.c16);
      M[off] = (double)S.re[rb][r];
      Mi[off] = (double)S.im[rb][r];
    }
  __syncthreads();
  Panel<double, D> Sd, G;
  panel_from_lds(Sd, M, L);
  __syncthreads();
  panel_to_lds_ct(M, Sd, L);
  __syncthreads();
  cgemm(G, M, Sd, L, true);  // G = S^dag S
  double e2 = 0;
#pragma unroll
  for (int rb = 0; rb < D / 16; ++rb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * rb + Prec<double>::rowmap(r, L.g), col = 16 * L.w + L.c16;
      if (row < d && col < d) {
        const double xr = G.re[rb][r] - (row == col ? 1.0 : 0.0), xi = G.im[rb][r];
        e2 += xr * xr + xi * xi;
      }
    }
  e2 = wave_sum(e2);
  if (L.lane == 0) red[L.w] = e2;
  __syncthreads();
  double tot = 0;
  for (int w = 0; w < NW; ++w) tot += red[w];
  const double res = sqrt(tot);
  if (threadIdx.x == 0)
    atomicMax(reinterpret_cast<unsigned long long*>(&P.diag[1]), (unsigned long long)__double_as_longlong(res));
  if (res > P.reun_tol) {
    // T = 3I - G, S <- S T / 2
    panel_scale(G, -1.0);
    panel_add_identity(G, L, 3.0);
    __syncthreads();
    panel_to_lds(M, Sd, L);
    __syncthreads();
    Panel<double, D> Sn;
    cgemm(Sn, M, G, L, true);
    panel_scale(Sn, 0.5);
    __syncthreads();
    panel_to_lds(M, Sn, L);
    __syncthreads();
#pragma unroll
    for (int rb = 0; rb < D / 16; ++rb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int off = lds_off<double, D>(16 * rb + Prec<float>::rowmap(r, L.g), 16 * L.w + L.c16);
        S.re[rb][r] = (float)M[off];
        S.im[rb][r] = (float)Mi[off];
      }
    if (threadIdx.x == 0) atomicAdd(reinterpret_cast<unsigned long long*>(&P.diag[2]), 1ull);
  }
  __syncthreads();
}

// ---------------------------------------------------------------- chunked scans

// One workgroup per chunk.  Forward pass (bwd = 0): running product
// S = U_k ... U_{k0}; stores xprev[k] = S before slice k and the chunk total
// tf[c].  Backward pass (bwd = 1, after the carry): S starts from
// mc[c] = cb[c] cf[c]^dag and becomes U_k^dag ... U_{k1-1}^dag mc[c]; stores
// bloc[k] = S before slice k is applied, so that the adjoint's
// W_k = bloc[k] xprev[k]^dag takes one product.  (The backward chunk total
// that the carry needs is tf[c]^dag.)  Each step is S <- S + Delta S (or
// Delta^dag S) with Delta staged in LDS (the next Delta is loaded into
// registers during a step).  The LDS buffer is double (no barrier before it
// is refilled) except in FP32 at D = 64, where one buffer and a barrier let
// three workgroups share a CU instead of two (measured on the d = 64 batch
// of 32: backward scans 1.00 -> 0.94 ms; FP64, held to one workgroup per CU
// by its registers, lost a third with one buffer).
template <typename T, int D>
constexpr int kScanBufs = (sizeof(T) == 4 && D == 64) ? 1 : 2;

template <typename T, int D, typename Ops, bool PERSIST>
__global__ __launch_bounds__(4 * D) __attribute__((amdgpu_waves_per_eu(kMinWaves<D>)))
void k_scan_local(Work W, int dir) {
  __shared__ __align__(16) unsigned char lds[kScanBufs<T, D>][Ops::BYTES];
  const int bwd = dir < 0 ? (int)blockIdx.y : dir;  // dir < 0: both passes, one per blockIdx.y
  Lane L;
  const Items I(W);
  for (int item = blockIdx.x; item < I.total; item += gridDim.x) {
  int p, c;
  split_item(item, W.rg.c_lo, W.rg.c_n, I.start, I.nprob, p, c);
  const ProbDesc P = W.descs[I.desc(p)];  // a copy: stores cannot alias it
  const int k0 = c * P.L;
  const int k1 = min(P.N, k0 + P.L);
  Panel<T, D> S, nxt, acc;
  if (bwd) panel_load(S, pf_mat<T, D>(P.mc, c), L); else panel_identity(S, L);
  const int n = k1 - k0;
  int k = bwd ? k1 - 1 : k0;
  panel_load(nxt, pf_mat<T, D>(P.delta, k - W.rg.kbase), L);
  for (int i = 0; i < n; ++i) {
    void* buf = lds[i % kScanBufs<T, D>];
    if (kScanBufs<T, D> == 1 && i > 0) __syncthreads();  // every wavefront is done with the previous factor
    if (bwd) Ops::store_ct(buf, nxt, L); else Ops::store(buf, nxt, L);
    const int kn = bwd ? k - 1 : k + 1;
    // the store of S before the prefetch of the next Delta, so that the wait
    // for the prefetch at the next step covers nothing issued after it
    panel_store(pf_mat<T, D>(bwd ? P.bloc : P.xprev, k - W.rg.kbase), S, L);
    if (i + 1 < n) panel_load(nxt, pf_mat<T, D>(P.delta, kn - W.rg.kbase), L);
    __syncthreads();
    Ops::gemm3(acc, buf, S, L, true);
    panel_axpby(S, (T)1, acc, (T)1);
    k = kn;
  }
  if (!bwd && !W.rg.recompute) panel_store(pf_mat<T, D>(P.tf, c), S, L);  // (k_reun follows in FP32)
  if constexpr (!PERSIST) break;  // one item per workgroup: a single-trip loop
  __syncthreads();
  }
}

// The re-unitarisation of the forward chunk totals tf[c] (FP32, problems with
// reun_tol >= 0), after the forward scans: one workgroup per chunk runs
// reunitarise() on the stored total.  A kernel of its own, so that the scan
// keeps the registers and LDS of its chain alone: inside it, the check's
// FP64 registers and its FP64 matrix in LDS cost the scan a workgroup per CU.
template <int D, bool PERSIST>
__global__ __launch_bounds__(4 * D) void k_reun(Work W) {
  __shared__ __align__(16) double lds[Mat<double, D>::LDS_ELEMS];
  __shared__ double red[D / 16];
  Lane L;
  const Items I(W);
  for (int item = blockIdx.x; item < I.total; item += gridDim.x) {
    int p, c;
    split_item(item, W.rg.c_lo, W.rg.c_n, I.start, I.nprob, p, c);
    const ProbDesc P = W.descs[I.desc(p)];  // a copy: stores cannot alias it
    if (P.reun_tol >= 0) {  // uniform over the workgroup
      Panel<float, D> S;
      panel_load(S, pf_mat<float, D>(P.tf, c), L);
      reunitarise<D>(P, S, lds, red, L);
      panel_store(pf_mat<float, D>(P.tf, c), S, L);
    }
    if constexpr (!PERSIST) break;  // one item per workgroup: a single-trip loop
    __syncthreads();
  }
}

// The carry over the chunk totals, in groups of CG chunks (carry_groups):
//   k_carry_grp: one workgroup per (group, direction), a serial chain over the
//     group's chunk totals that stores the carry from the group start into
//     each chunk (forward cf_loc[c] = tf[c-1] ... tf[g0] into cf, backward
//     cb_loc[c] = tf[c+1]^dag ... tf[g1-1]^dag into cb) and the group total;
//   k_carry_top: one workgroup per (problem, direction), a serial chain over
//     the group totals that stores the carry into each group (forward from I,
//     ending with X_N, its fidelity and unitarity residual; backward from V);
//   k_mc: mc[c] = cb[c] cf[c]^dag with cf[c] = cf_loc[c] gcf[g] and
//     cb[c] = cb_loc[c] gcb[g].
// The chains are serial and each runs as one workgroup, so they take the
// three-product form at D >= 32 regardless of its registers.

// n steps of S <- A_i S, storing S before each step to out[i] (i < nstore).
// A_i is the PF matrix src[i] (stride step) or, with ct, its conjugate
// transpose.  Double-buffered LDS; the next factor is loaded during a step.
template <typename T, int D>
__device__ __forceinline__ void carry_chain(Panel<T, D>& S, const T* src, int step, int n, bool ct, T* out,
                                            int ostep, int nstore, T (*lds)[Mat<T, D>::LDS_ELEMS], const Lane& L) {
  constexpr int EL = Mat<T, D>::ELEMS;
  Panel<T, D> nxt, acc;
  if (n > 0) panel_load(nxt, src, L);
  for (int i = 0; i < nstore || i < n; ++i) {
    if (i < nstore) panel_store(out + (ptrdiff_t)i * ostep * EL, S, L);
    if (i >= n) break;
    T* buf = lds[i & 1];
    if (ct) panel_to_lds_ct(buf, nxt, L); else panel_to_lds(buf, nxt, L);
    if (i + 1 < n) panel_load(nxt, src + (ptrdiff_t)(i + 1) * step * EL, L);
    __syncthreads();
    if constexpr (D >= 32) cgemm3m(acc, buf, S, L, true); else cgemm(acc, buf, S, L, true);
    S = acc;
  }
}

// Group matrices: [0, PG) forward totals, [PG, 2 PG) backward totals,
// [2 PG, 3 PG) forward carries, [3 PG, 4 PG) backward carries.
template <typename T, int D>
__device__ __forceinline__ T* grp_mat(const ProbDesc& P, int kind, int g) {
  return pf_mat<T, D>(P.grp, kind * P.PG + g);
}

template <typename T, int D>
__global__ __launch_bounds__(4 * D) void k_carry_grp(Work W) {
  __shared__ T lds[2][Mat<T, D>::LDS_ELEMS];
  Lane L;
  const int bwd = blockIdx.y;
  const Items I(W);
  for (int item = blockIdx.x; item < I.total; item += gridDim.x) {
  int p, g;
  split_item(item, 0, W.rg.c_n, I.start, I.nprob, p, g);
  const ProbDesc P = W.descs[I.desc(p)];  // a copy: stores cannot alias it
  const int c0 = g * P.CG;
  const int n = min(P.CG, P.P - c0);
  Panel<T, D> S;
  panel_identity(S, L);
  if (!bwd) {
    carry_chain<T, D>(S, pf_mat<T, D>(P.tf, c0), 1, n, false, pf_mat<T, D>(P.cf, c0), 1, n, lds, L);
    panel_store(grp_mat<T, D>(P, 0, g), S, L);
  } else {
    const int c1 = c0 + n - 1;  // the chain runs from the group's last chunk down
    carry_chain<T, D>(S, pf_mat<T, D>(P.tf, c1), -1, n, true, pf_mat<T, D>(P.cb, c1), -1, n, lds, L);
    panel_store(grp_mat<T, D>(P, 1, g), S, L);
  }
  __syncthreads();
  }
}

template <typename T, int D>
__global__ __launch_bounds__(4 * D) void k_carry_top(Work W) {
  constexpr int NW = Mat<T, D>::NW;
  __shared__ T lds[2][Mat<T, D>::LDS_ELEMS];
  __shared__ double red[2 * NW];
  Lane L;
  const int bwd = blockIdx.y;
  const Items I(W);
  for (int p = blockIdx.x; p < I.nprob; p += gridDim.x) {
  const ProbDesc P = W.descs[I.desc(p)];  // a copy: stores cannot alias it
  Panel<T, D> S, acc;
  const int ng = P.PG;
  if (!bwd) {
    panel_identity(S, L);
    carry_chain<T, D>(S, grp_mat<T, D>(P, 0, 0), 1, ng, false, grp_mat<T, D>(P, 2, 0), 1, ng, lds, L);
    fidelity_epilogue<T, D>(P, S, L, red);
    // Unitarity residual of X_N: S^dag S from the conjugate transpose in LDS.
    __syncthreads();
    panel_to_lds_ct(lds[0], S, L);
    __syncthreads();
    cgemm(acc, lds[0], S, L, true);
    residual_epilogue<T, D>(P, acc, L, red);
  } else {
    panel_load(S, reinterpret_cast<const T*>(P.Vint), L);
    carry_chain<T, D>(S, grp_mat<T, D>(P, 1, ng - 1), -1, ng - 1, false, grp_mat<T, D>(P, 3, ng - 1), -1, ng,
                      lds, L);
  }
  __syncthreads();
  }
}

// mc[c] = cb[c] cf[c]^dag for every chunk, the start of its backward scan, so
// that W_k = (local backward product) mc[c] xprev[k]^dag; cf[c] and cb[c] are
// formed here from the in-group carries and the group carries.
template <typename T, int D>
__global__ __launch_bounds__(4 * D) void k_mc(Work W) {
  __shared__ T lds[2][Mat<T, D>::LDS_ELEMS];
  Lane L;
  const Items I(W);
  for (int item = blockIdx.x; item < I.total; item += gridDim.x) {
  int p, c;
  split_item(item, W.rg.c_lo, W.rg.c_n, I.start, I.nprob, p, c);
  const ProbDesc P = W.descs[I.desc(p)];  // a copy: stores cannot alias it
  const int g = c / P.CG;
  Panel<T, D> a, b, x, y;
  // cf[c] = cf_loc[c] gcf[g] and cb[c] = cb_loc[c] gcb[g]
  panel_load(a, pf_mat<T, D>(P.cf, c), L);
  panel_load(b, pf_mat<T, D>(P.cb, c), L);
  panel_load(x, grp_mat<T, D>(P, 2, g), L);
  panel_load(y, grp_mat<T, D>(P, 3, g), L);
  panel_to_lds(lds[0], a, L);
  panel_to_lds(lds[1], b, L);
  __syncthreads();
  if constexpr (D >= 32) {
    cgemm3m(a, lds[0], x, L, true);
    cgemm3m(b, lds[1], y, L, true);
  } else {
    cgemm(a, lds[0], x, L, true);
    cgemm(b, lds[1], y, L, true);
  }
  // mc[c] = cb[c] cf[c]^dag
  __syncthreads();
  panel_to_lds(lds[0], b, L);
  panel_to_lds(lds[1], a, L);
  __syncthreads();
  panel_from_lds_ct(x, lds[1], L);
  cgemm(a, lds[0], x, L, true);
  panel_store(pf_mat<T, D>(P.mc, c), a, L);
  __syncthreads();
  }
}

// ---------------------------------------------------------------- adjoint / gradient

// The gradient from only the entries of Z = E + X2 C2 + S C1 that the
// controls read (s = 0, FP32, every control a weighted permutation: Pauli
// strings).  Control j reads Z[a][b] at b = col_j(a), once per column b, so
// the lane that holds column b of the panels (wavefront b / 16, lane b % 16
// of each lane group) forms z = Z[minv_j(b)][b] as the dot product of row
// minv_j(b) of X2 and of S (LDS) with its own entries of C2 and C1, the four
// lane groups each taking their 16 of the d rows and then summing.  E[a][b]
// of the first kSampleGather controls was gathered from LDS before S took
// E's place (sample_gather); later controls take it from the lane that holds
// it, inside the dot product.  That is 2 d m complex multiply-adds per column
// on the vector ALU in place of the last two products (d^3 each), then
// T_j = sum_b conj(z) val_j(minv_j(b)) in FP64 as in gradient_epilogue.
template <int D>
constexpr int kSampleGroup = 4;  // controls per reduction
// Controls whose entries E[minv_j(b)][b] are gathered (8 KB of LDS at D = 64,
// which still fits two workgroups per CU).
constexpr int kSampleGather = 16;

// Thread t: column t % D of controls t / D + 4 i.  The rows are loaded before
// the block's square is formed and the entries read after it, while E is
// still in LDS.
template <int D>
__device__ __forceinline__ void sample_rows(const ProbDesc& P, int (&ga)[kSampleGather / 4]) {
#pragma unroll
  for (int i = 0; i < kSampleGather / 4; ++i) {
    const int j = (int)threadIdx.x / D + 4 * i;
    ga[i] = j < P.m ? gp(P.minv)[(size_t)j * D + threadIdx.x % D] : 0;
  }
}

template <int D>
__device__ __forceinline__ void sample_gather(const ProbDesc& P, const int (&ga)[kSampleGather / 4], const void* elds,
                                              float* eg) {
  const float* er = static_cast<const float*>(elds);
  const float* ei = er + D * Mat<float, D>::SD;
  const int b = threadIdx.x % D;
#pragma unroll
  for (int i = 0; i < kSampleGather / 4; ++i) {
    const int j = (int)threadIdx.x / D + 4 * i;
    if (j < P.m) {
      const int off = lds_off<float, D>(ga[i], b);
      eg[2 * (j * D + b)] = er[off];
      eg[2 * (j * D + b) + 1] = ei[off];
    }
  }
}

// Partial sums of z over this lane group's rows; WITH_E also picks E[a][b]
// into (er, ei) in the lane that holds it (zero elsewhere), so that it is
// added after the sum over the lane groups, as the gathered entry is: the
// two forms give the same bits.
template <int D, bool WITH_E>
__device__ __forceinline__ void sampled_dot(float& zr, float& zi, float& er, float& ei, int a, const float* xr,
                                            const float* xi, const float* yr, const float* yi,
                                            const Panel<float, D>& E, const Panel<float, D>& C1,
                                            const Panel<float, D>& C2, const Lane& L) {
  constexpr int NV = D / 16;
  constexpr int SD = Mat<float, D>::SD;
  // LDS row a at the columns of this lane's panel rows 16 rb + 4 g + r
  const int base = a * SD + 4 * L.g;
  float pr[4] = {0.f, 0.f, 0.f, 0.f}, pi[4] = {0.f, 0.f, 0.f, 0.f};  // one chain per r
#pragma unroll
  for (int rb = 0; rb < NV; ++rb) {
    const f4 ar = Prec<float>::ld4(xr + base + 16 * rb), ai = Prec<float>::ld4(xi + base + 16 * rb);
    const f4 br = Prec<float>::ld4(yr + base + 16 * rb), bi = Prec<float>::ld4(yi + base + 16 * rb);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if constexpr (WITH_E) {
        const bool own = 16 * rb + 4 * L.g + r == a;
        er = own ? E.re[rb][r] : er;
        ei = own ? E.im[rb][r] : ei;
      }
      pr[r] = fmaf(ar[r], C2.re[rb][r], pr[r]);
      pr[r] = fmaf(-ai[r], C2.im[rb][r], pr[r]);
      pr[r] = fmaf(br[r], C1.re[rb][r], pr[r]);
      pr[r] = fmaf(-bi[r], C1.im[rb][r], pr[r]);
      pi[r] = fmaf(ar[r], C2.im[rb][r], pi[r]);
      pi[r] = fmaf(ai[r], C2.re[rb][r], pi[r]);
      pi[r] = fmaf(br[r], C1.im[rb][r], pi[r]);
      pi[r] = fmaf(bi[r], C1.re[rb][r], pi[r]);
    }
  }
  zr = (pr[0] + pr[1]) + (pr[2] + pr[3]);
  zi = (pi[0] + pi[1]) + (pi[2] + pi[3]);
}

// The sampled step's reduction: each group's per-wavefront sums go to their
// own slot of the reduction array (epilogue_publish's layout), and one
// barrier publishes every kSampleSlots groups at once.
constexpr int kSampleSlots = 2 * kEpiDense / kSampleGroup<64>;

template <int NWAVES, int G>
__device__ __forceinline__ void sample_stash(int slot, double (&v)[2 * G], const Lane& L, double* red) {
  constexpr int V = 2 * G;
  constexpr int SH = 6 - __builtin_ctz(V);
  const double t = wave_sum_many<V>(v, L.lane);
  if ((L.lane & ((1 << SH) - 1)) == 0) red[slot * V * NWAVES + (L.lane >> SH) * NWAVES + L.w] = t;
}

template <int NWAVES, int G>
__device__ __forceinline__ void sample_flush(const ProbDesc& P, int k, int j0, int nj, const double* red) {
  if ((int)threadIdx.x < nj) {
    const int jj = threadIdx.x;
    const double* rg = red + (jj / G) * 2 * G * NWAVES;
    const int q = jj % G;
    double a = 0, b = 0;
    for (int w = 0; w < NWAVES; ++w) {
      a += rg[(2 * q) * NWAVES + w];
      b += rg[(2 * q + 1) * NWAVES + w];
    }
    grad_put(P, j0 + jj, k, a, b);
  }
}

template <int D, bool GATHERED>
__device__ __forceinline__ void sampled_gradient(const ProbDesc& P, int k, const Panel<float, D>& E,
                                                 const Panel<float, D>& C1, const Panel<float, D>& C2,
                                                 const void* x2lds, const void* slds, const float* eg,
                                                 double* red, const Lane& L) {
  constexpr int G = kSampleGroup<D>;
  const float* xr = static_cast<const float*>(x2lds);
  const float* xi = xr + D * Mat<float, D>::SD;
  const float* yr = static_cast<const float*>(slds);
  const float* yi = yr + D * Mat<float, D>::SD;
  const int b = 16 * L.w + L.c16;
  const float* mv = reinterpret_cast<const float*>(P.mval);
  static_assert(G * kSampleSlots <= 4 * D, "one thread per control of a block");
  float zr = 0.f, zi = 0.f;
  for (int j0 = 0, grp = 0; j0 < P.m; j0 += G, ++grp) {
    const int slot = grp % kSampleSlots;
    if (slot == 0 && grp > 0) __syncthreads();  // the previous block's sums are read
    // the group's table entries first: two round trips per group, not per control
    int ag[G], fl[G];
    float hrg[G], hig[G];
#pragma unroll
    for (int jj = 0; jj < G; ++jj) {
      const int j = min(j0 + jj, P.m - 1);
      ag[jj] = gp(P.minv)[(size_t)j * D + b];
      fl[jj] = gp(P.mok)[j];
    }
#pragma unroll
    for (int jj = 0; jj < G; ++jj) {
      const size_t e = (size_t)min(j0 + jj, P.m - 1) * D + ag[jj];
      hrg[jj] = gp(mv)[2 * e];
      hig[jj] = gp(mv)[2 * e + 1];
    }
    double v[2 * G];
#pragma unroll
    for (int jj = 0; jj < G; ++jj) {
      // a control with the previous one's columns (in this group) reads the
      // same entries of Z: z is reused (uniform over the workgroup)
      if (jj == 0 || j0 + jj >= P.m || !(fl[jj] & 4)) {
        const int j = min(j0 + jj, P.m - 1);
        const bool gathered = GATHERED && j < kSampleGather;
        float er = 0.f, ei = 0.f;
        if constexpr (GATHERED) {
          if (gathered) sampled_dot<D, false>(zr, zi, er, ei, ag[jj], xr, xi, yr, yi, E, C1, C2, L);
          else sampled_dot<D, true>(zr, zi, er, ei, ag[jj], xr, xi, yr, yi, E, C1, C2, L);
        } else {
          sampled_dot<D, true>(zr, zi, er, ei, ag[jj], xr, xi, yr, yi, E, C1, C2, L);
        }
        zr += __shfl_xor(zr, 16, 64);
        zi += __shfl_xor(zi, 16, 64);
        zr += __shfl_xor(zr, 32, 64);
        zi += __shfl_xor(zi, 32, 64);
        if (gathered) {
          er = eg[2 * (j * D + b)];
          ei = eg[2 * (j * D + b) + 1];
        } else {  // one nonzero among the lane groups: the sum is exact
          er += __shfl_xor(er, 16, 64);
          ei += __shfl_xor(ei, 16, 64);
          er += __shfl_xor(er, 32, 64);
          ei += __shfl_xor(ei, 32, 64);
        }
        zr += er;
        zi += ei;
      }
      const float hr = hrg[jj], hi = hig[jj];
      double tr = 0, ti = 0;
      if (L.g == 0 && j0 + jj < P.m) {  // conj(z) h, once per column
        tr = (double)zr * hr + (double)zi * hi;
        ti = (double)zr * hi - (double)zi * hr;
      }
      v[2 * jj] = tr;
      v[2 * jj + 1] = ti;
    }
    sample_stash<D / 16, G>(slot, v, L, red);
    if (slot == kSampleSlots - 1 || j0 + G >= P.m) {
      __syncthreads();
      const int jb = j0 - slot * G;  // first control of the block
      sample_flush<D / 16, G>(P, k, jb, min(kSampleSlots * G, P.m - jb), red);
    }
  }
}

// Ops::gemm3 with P accumulator chain pairs where P > 1 (StdOps only).
template <int P, typename Ops, typename T, int D>
__device__ __forceinline__ void gemm3p(Panel<T, D>& acc, const void* lds, const Panel<T, D>& B, const Lane& L,
                                       bool zero_acc) {
  if constexpr (P > 1) Ops::template gemm3<P>(acc, lds, B, L, zero_acc);
  else Ops::gemm3(acc, lds, B, L, zero_acc);
}

template <typename T, int D, typename Ops>
constexpr bool kSampleLast = std::is_same<Ops, StdOps<float, D>>::value && D >= 32;

// One workgroup per slice.
//  1. W_k = bloc[k] xprev[k]^dag  (one product; bloc[k] carries mc[c]).
//  2. X = A_k^dag / 2^s in LDS buffer 0, E = W_k / 2^s in buffer 1.
//  3. The Taylor polynomial of degree qb of M = [[X, E], [0, X]] in delta
//     form, p(M) - I, by Paterson-Stockmeyer with M^2 as the step: the top
//     right block of exp(M) is the Frechet derivative L(X, E).
//  4. s squarings: [[I + D1, Q], [0, I + D1]]^2 gives D1 <- 2 D1 + D1^2 and
//     Q <- 2Q + D1 Q + Q D1.  Z_k = Q.
//  5. T_j = Tr(Z_k^dag Hc[j]) in FP64, grad = (2 dt / d^2) Im(conj(g) T_j).
// Two workgroups per CU (two waves per SIMD) where the LDS allows it, so
// that one workgroup's LDS and VALU work overlaps the other's MFMAs.  H_k is
// loaded together with the W factors where the extra registers cost no
// occupancy (FP32 at D = 64, FP64 at D = 32).
template <typename T, int D>
constexpr int kAdjWaves = ((sizeof(T) == 4 && D <= 64) || (sizeof(T) == 8 && D == 32)) ? 2 : 1;
template <typename T, int D>
constexpr bool kEarlyH = (sizeof(T) == 4 && D == 64) || (sizeof(T) == 8 && D == 32);

// MODE 0: every slice; where the sampled last step applies (kSampleLast), two
// instances split the slices: MODE 1 takes those where it does not apply,
// MODE 2 those where it does (s = 0, permutation controls), each returning at
// once for the others, so that neither carries the other's registers.
template <typename T, int D, typename Ops, bool PERSIST, int MODE = 0>
__global__ __launch_bounds__(4 * D) __attribute__((amdgpu_waves_per_eu(kAdjWaves<T, D>)))
void k_adjoint(Work W) {
  constexpr int NW = Mat<T, D>::NW;
  constexpr int AP = MODE == 2 ? 2 : 1;  // accumulator chain pairs of the sampling instance's products
  __shared__ __align__(16) unsigned char lds[2][Ops::BYTES];
  __shared__ double red[2 * kEpiDense * 2 * NW];
  // sample_gather (not in the persistent grid, whose registers it would spill)
  constexpr bool GATHER = MODE == 2 && !PERSIST;
  __shared__ __align__(16) float eg[GATHER ? 2 * kSampleGather * D : 1];
  Lane L;
  const Items I(W);
  for (int item = blockIdx.x; item < I.total; item += gridDim.x) {
  int p, k;
  split_item(item, W.rg.s_lo, W.rg.s_n, I.start, I.nprob, p, k);
  const ProbDesc P = W.descs[I.desc(p)];  // a copy: stores cannot alias it
  const int sqk = gp(P.sq)[k];
  int s, q, qb;
  unpack_sq(sqk, s, q, qb);
  if constexpr (MODE != 0) {
    const bool sampled = (sqk & kPlanSampled) != 0;  // uniform over the workgroup
    if (sampled != (MODE == 2)) {
      if constexpr (PERSIST) continue;
      else return;
    }
  }
  const bool mono = controls_monomial(P);
  Panel<T, D> R1, R2, A1, A2;

  // 1. W = bloc[k] xprev[k]^dag (bloc carries mc[c]).  The slice's global
  //    loads (xprev, bloc and, where the registers allow, H_k) are issued
  //    together.
  HamRegs<T, D> ham;
  if constexpr (kEarlyH<T, D>) ham_load<T, D>(ham, pf_mat<T, D>(P.hk, k - W.rg.kbase));
  panel_load(A2, pf_mat<T, D>(P.xprev, k - W.rg.kbase), L);
  panel_load(R2, pf_mat<T, D>(P.bloc, k - W.rg.kbase), L);
  Ops::store(lds[0], R2, L);
  Ops::store(lds[1], A2, L);
  __syncthreads();
  Ops::load_ct(A2, lds[1], L);
  gemm3p<AP, Ops>(R2, lds[0], A2, L, true);  // R2 = W
  __syncthreads();

  // 2. E = W / 2^s, X = A^dag / 2^s
  const T scl = (T)ldexp(1.0, -s);
  panel_scale(R2, scl);
  Ops::store(lds[1], R2, L);
  if constexpr (kKeepH<D>) {
    if constexpr (!kEarlyH<T, D>) ham_load<T, D>(ham, pf_mat<T, D>(P.hk, k - W.rg.kbase));
    ham_put<T, D, Ops>(lds[0], ham, ldexp(P.dt, -s), -1.0, (P.flags & RUN_GENERAL) != 0);
  } else {
    assemble<T, D, Ops, (sizeof(T) == 4 ? 4 : 2)>(lds[0], P, k, ldexp(P.dt, -s), -1.0, nullptr, mono,
                                                  (P.flags & RUN_GENERAL) != 0);
  }
  __syncthreads();
  const void* X = lds[0];
  const void* E = lds[1];

  // 3. Paterson-Stockmeyer on the block.  With M^2 = [[X2, S], [0, X2]],
  //    X2 = X X and S = X E + E X, the delta block is p(M) - I = M + M^2 C,
  //    C = sum_{n=2..qb} M^(n-2) / n!.  C runs Horner in M^2 over the digits
  //    D_t = I / (2t+2)! + M / (2t+3)! (terms above degree qb dropped):
  //    C <- D_t + M^2 C = [[D_t11 + X2 C1, b_t E + X2 C2 + S C1], [0, .]].
  //    Each block product by M^2 takes three d x d products, the last one
  //    only the blocks used next.
  Panel<T, D> R3;
  int ga[kSampleGather / 4];
  if constexpr (GATHER) sample_rows<D>(P, ga);
  Ops::load(R1, X, L);  // R1 = X, R2 = E
  // A1 = X2: kept by the expm pass where it keeps H_k and forms its own
  // square (q >= 2; for Hermitian H_k its X X equals this X X); general
  // generators form it here.
  if (kKeepH<D> && kKeepX2<T> && q >= 2 && P.x2 && !(P.flags & RUN_GENERAL))
    panel_load(A1, pf_mat<T, D>(P.x2, k - W.rg.kbase), L);
  else Ops::gemm3(A1, X, R1, L, true);
  gemm3p<AP, Ops>(A2, X, R2, L, true);
  gemm3p<AP, Ops>(A2, E, R1, L, false);  // A2 = S
  if constexpr (GATHER) sample_gather<D>(P, ga, E, eg);
  __syncthreads();                  // X and E are read: M^2 takes their place
  Ops::store(lds[0], A1, L);
  Ops::store(lds[1], A2, L);
  const int top = (qb - 2) / 2;  // index of the last digit
  int t;                         // next digit, folded in by a block product
  if (qb & 1) {                  // C = D_top = I / (qb-1)! + M / qb!
    t = top - 1;
    A1 = R1;
    panel_scale(A1, (T)inv_factorial(qb));
    panel_add_identity(A1, L, (T)inv_factorial(qb - 1));
    A2 = R2;
    panel_scale(A2, (T)inv_factorial(qb));
  } else if (top > 0) {  // D_top = I / qb!: C = D_{top-1} + M^2 / qb! without a product
    t = top - 2;
    panel_axpby(A1, (T)inv_factorial(qb - 1), R1, (T)inv_factorial(qb));
    panel_add_identity(A1, L, (T)inv_factorial(qb - 2));
    panel_axpby(A2, (T)inv_factorial(qb - 1), R2, (T)inv_factorial(qb));
  } else {  // qb = 2: C = I / 2
    t = -1;
    panel_zero(A1);
    panel_add_identity(A1, L, (T)0.5);
    panel_zero(A2);
  }
  __syncthreads();
  for (; t >= 0; --t) {
    const T a = (T)inv_factorial(2 * t + 2), b = (T)inv_factorial(2 * t + 3);
    R3 = R2;
    panel_scale(R3, b);
    Ops::gemm3(R3, lds[0], A2, L, false);
    Ops::gemm3(R3, lds[1], A1, L, false);  // R3 = b E + X2 C2 + S C1
    A2 = R1;
    panel_scale(A2, b);
    panel_add_identity(A2, L, a);
    Ops::gemm3(A2, lds[0], A1, L, false);  // A2 = a I + b X + X2 C1
    A1 = A2;
    A2 = R3;
  }
  if constexpr (MODE == 2) {
    // 4'-5'. only the entries of Z that the controls read
    sampled_gradient<D, GATHER>(P, k, R2, A1, A2, lds[0], lds[1], eg, red, L);
  } else {
  Ops::gemm3(R2, lds[0], A2, L, false);
  Ops::gemm3(R2, lds[1], A1, L, false);              // R2 = Q = E + X2 C2 + S C1
  if (s > 0) Ops::gemm3(R1, lds[0], A1, L, false);  // R1 = D1 = X + X2 C1
  A1 = R1;
  A2 = R2;

  // 4. squarings
  for (int j = 0; j < s; ++j) {
    __syncthreads();
    Ops::store(lds[0], A1, L);
    Ops::store(lds[1], A2, L);
    __syncthreads();
    Ops::gemm3(R2, lds[0], A2, L, true);   // D1 Q
    Ops::gemm3(R2, lds[1], A1, L, false);  // + Q D1
    panel_axpby(R2, (T)2, A2, (T)1);  // R2 = 2Q + D1 Q + Q D1
    if (j + 1 < s) {
      Ops::gemm3(R1, lds[0], A1, L, true);
      panel_axpby(A1, (T)1, R1, (T)2);
    }
    A2 = R2;
  }

  // 5. inner products with the controls (FP64), then the gradient
  gradient_epilogue<T, D>(P, k, A2, L, lds[0], red, mono);
  }
  if constexpr (!PERSIST) break;  // one item per workgroup: a single-trip loop
  __syncthreads();
  }
}

// ================================================================ d = 128
//
// A 128 x 128 complex matrix pair does not fit in LDS (one FP32 matrix is
// 132 KB with padding, one FP64 matrix 260 KB).  At D = 128 the state of every
// chain therefore lives in global scratch in PF layout (8 wavefronts, one
// 16-column panel each), each product accumulates one output panel per
// wavefront in registers, and the left factor is staged cooperatively into
// LDS, the whole matrix in FP32 and one 64-column half at a time in FP64.
// The grids are persistent (at most kScratchSlots workgroups), so that each
// workgroup owns a fixed scratch region.

template <typename T>
struct K128 {
  static constexpr int D = 128, NW = 8, RB = 8;
  static constexpr int HALVES = sizeof(T) == 8 ? 2 : 1;
  static constexpr int HC = D / HALVES;             // columns staged at once
  static constexpr int SD = HC + Prec<T>::PAD;      // LDS row stride
  static constexpr int LDS_ELEMS = 2 * D * SD;
  static constexpr int ELEMS = 2 * D * D;
  static constexpr int KBH = HC / 16;               // k blocks per staged part
  static constexpr int WPH = NW / HALVES;           // panels per staged part
};

// acc <- acc + a * (this wavefront's panel of the PF matrix M), one row block
// at a time so that no second panel is held in registers.
template <typename T>
__device__ __forceinline__ void panel_axpy_pf(Panel<T, 128>& acc, T a, const T* M, const Lane& L) {
#pragma unroll
  for (int rb = 0; rb < 8; ++rb) {
    typename Prec<T>::v4 re, im;
    pf_rb_load<T>(re, im, M, L.w, rb, L.lane);
    acc.re[rb] += a * re;
    acc.im[rb] += a * im;
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Stage part h (columns [h HC, (h+1) HC)) of M (CT = false) or of M^dag
// (CT = true) into LDS; M is a PF matrix.  Layout as for the D <= 64 LDS
// matrices, restricted to HC columns.
template <typename T, bool CT>
__device__ __forceinline__ void stage128(T* lds, const T* M, int h, const Lane& L) {
  using K = K128<T>;
  using v4 = typename Prec<T>::v4;
  T* lim = lds + K::D * K::SD;
  // Row blocks are loaded NB at a time, all NB loads in flight before the
  // LDS writes, so that the staging waits for RB / NB global round trips.
  constexpr int NB = sizeof(T) == 4 ? 4 : 2;
  if constexpr (!CT) {
    if (L.w / K::WPH != h) return;
    const int lw = L.w - h * K::WPH;
#pragma unroll
    for (int b0 = 0; b0 < K::RB; b0 += NB) {
      v4 re[NB], im[NB];
#pragma unroll
      for (int i = 0; i < NB; ++i) pf_rb_load<T>(re[i], im[i], M, L.w, b0 + i, L.lane);
#pragma unroll
      for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int off = (16 * (b0 + i) + Prec<T>::rowmap(r, L.g)) * K::SD + 16 * lw + Prec<T>::perm(L.c16);
          lds[off] = re[i][r];
          lim[off] = im[i][r];
        }
      __builtin_amdgcn_sched_barrier(0);
    }
  } else {
    // M^dag[16w + c16][16 rb + rowmap(r, g)] = conj(M[16 rb + rowmap(r, g)][16w + c16])
    constexpr int RL = K::RB / K::HALVES;
#pragma unroll
    for (int b0 = 0; b0 < RL; b0 += NB) {
      v4 re[NB], im[NB];
#pragma unroll
      for (int i = 0; i < NB; ++i) pf_rb_load<T>(re[i], im[i], M, L.w, h * RL + b0 + i, L.lane);
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        int off = (16 * L.w + L.c16) * K::SD + 16 * (b0 + i) + 4 * L.g;
        Prec<T>::st4(lds + off, re[i]);
        Prec<T>::st4(lim + off, -im[i]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// acc (+)= M B, M (or M^dag when CT) staged through LDS part by part, B this
// wavefront's panel of a PF matrix.  Every part is staged between two
// workgroup barriers, so M may have been written by any wavefront.  With
// stage = false and the whole matrix in one part (FP32), M is taken to be in
// LDS already from the previous product, which had the same left factor and
// no LDS writes since: one barrier (which also completes this wavefront's
// stores of B) and no staging.  G3 selects the three-product form of the
// complex product (as cgemm3m: T1 in acc.re, T3 in acc.im starting at
// acc.im + acc.re, T2 apart).
template <typename T, bool CT, bool G3 = false>
__device__ __forceinline__ void gemm128(Panel<T, 128>& acc, T* lds, const T* M, const T* B, const Lane& L,
                                        bool zero_acc, bool stage = true) {
  using K = K128<T>;
  using v4 = typename Prec<T>::v4;
  const T* lim = lds + K::D * K::SD;
  if (zero_acc) panel_zero(acc);
  v4 t2[G3 ? K::RB : 1];
  if constexpr (G3) {
#pragma unroll
    for (int rb = 0; rb < K::RB; ++rb) {
      t2[rb] = (v4){0, 0, 0, 0};
      if (!zero_acc) acc.im[rb] += acc.re[rb];
    }
  }
  const int base = L.c16 * K::SD + 4 * L.g;
#pragma unroll
  for (int h = 0; h < K::HALVES; ++h) {
    __syncthreads();
    if (stage || K::HALVES > 1) {
      stage128<T, CT>(lds, M, h, L);
      __syncthreads();
    }
    constexpr int STEPS = K::KBH * K::RB;
    v4 ar[2], ai[2], br[2], bi[2];
    ar[0] = Prec<T>::ld4(lds + base);
    ai[0] = Prec<T>::ld4(lim + base);
    pf_rb_load<T>(br[0], bi[0], B, L.w, h * K::KBH, L.lane);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int st = 0; st < STEPS; ++st) {
      const int kbl = st / K::RB, mb = st % K::RB;
      const int cur = st & 1, kcur = kbl & 1;
      if (st + 1 < STEPS) {
        const int kn = (st + 1) / K::RB, mn = (st + 1) % K::RB;
        const int off = base + 16 * mn * K::SD + 16 * kn;
        ar[cur ^ 1] = Prec<T>::ld4(lds + off);
        ai[cur ^ 1] = Prec<T>::ld4(lim + off);
        if (mb == 0 && kbl + 1 < K::KBH) pf_rb_load<T>(br[kcur ^ 1], bi[kcur ^ 1], B, L.w, h * K::KBH + kbl + 1, L.lane);
      }
      if constexpr (G3) {
        const v4 as = ar[cur] + ai[cur];
        const v4 bs = br[kcur] + bi[kcur];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          acc.re[mb] = Prec<T>::mfma(ar[cur][r], br[kcur][r], acc.re[mb]);
          t2[mb] = Prec<T>::mfma(ai[cur][r], bi[kcur][r], t2[mb]);
          acc.im[mb] = Prec<T>::mfma(as[r], bs[r], acc.im[mb]);
        }
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const T b_r = br[kcur][r];
          const T b_i = bi[kcur][r];
          acc.re[mb] = Prec<T>::mfma(ar[cur][r], b_r, acc.re[mb]);
          acc.im[mb] = Prec<T>::mfma(ar[cur][r], b_i, acc.im[mb]);
          acc.re[mb] = Prec<T>::mfma(-ai[cur][r], b_i, acc.re[mb]);
          acc.im[mb] = Prec<T>::mfma(ai[cur][r], b_r, acc.im[mb]);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  if constexpr (G3) {
#pragma unroll
    for (int rb = 0; rb < K::RB; ++rb) {
      acc.im[rb] = acc.im[rb] - acc.re[rb] - t2[rb];
      acc.re[rb] = acc.re[rb] - t2[rb];
    }
  }
}

// out = M^dag (both PF), through LDS part by part.
template <typename T>
__device__ __forceinline__ void transpose128(T* out, T* lds, const T* M, const Lane& L) {
  using K = K128<T>;
  const T* lim = lds + K::D * K::SD;
  for (int h = 0; h < K::HALVES; ++h) {
    __syncthreads();
    stage128<T, true>(lds, M, h, L);
    __syncthreads();
    if (L.w / K::WPH == h) {
      const int lw = L.w - h * K::WPH;
      Panel<T, 128> P;
#pragma unroll
      for (int rb = 0; rb < K::RB; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int off = (16 * rb + Prec<T>::rowmap(r, L.g)) * K::SD + 16 * lw + Prec<T>::perm(L.c16);
          P.re[rb][r] = lds[off];
          P.im[rb][r] = lim[off];
        }
      panel_store(out, P, L);
    }
  }
}

// X <- sgn * (-i) * c * H_k (this wavefront's panel, in registers) with
// H_k = H0 + sum_j u_jk Hc[j].  The matrix is read as chunks of four
// consecutive row elements, chunk t + 512 i by thread t, so that every
// 16-byte load is consecutive across lanes and a control's loads are all in
// flight together; the chunks then go through LDS (row-major, the layout of
// the staged left factors) to the panels, which are also stored to the PF
// matrix out.  FP32 takes all rows at once, FP64 one half of the rows per
// pass (one FP64 matrix does not fit in LDS); FP64 writes each half's rows of
// the panel to out and reads the panel back at the end, so that no panel is
// held across the passes.  Starts and ends with a workgroup barrier.
// With mono (every control has at most one nonzero per row) the chunks of H0
// go to LDS unscaled, one thread per row then adds the row's entry of each
// control in turn (the same sums, minus the structural zeros), and a last
// pass over the chunks applies the scale.
template <typename T>
__device__ __forceinline__ void assemble128(Panel<T, 128>& X, T* out, T* lds, const ProbDesc& P, int k, double c,
                                            double sgn, const Lane& L, bool mono) {
  using v4 = typename Prec<T>::v4;
  constexpr int D = 128, NT = 512;
  constexpr int PASSES = sizeof(T) == 4 ? 1 : 2;
  constexpr int NV = D * D / 4 / NT / PASSES;
  constexpr int ROWS = D / PASSES;
  constexpr int SD = D + Prec<T>::PAD;
  static_assert(2 * ROWS * SD <= K128<T>::LDS_ELEMS, "LDS too small");
  T* lim = lds + ROWS * SD;
  const T* H = reinterpret_cast<const T*>(P.Hint);
  const T f = (T)(sgn * c);
#pragma unroll
  for (int pass = 0; pass < PASSES; ++pass) {
    const int e0 = 4 * (threadIdx.x + pass * NV * NT);
    v4 hr[NV], hi[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      hr[v] = Prec<T>::gld4(H + e0 + 4 * NT * v);
      hi[v] = Prec<T>::gld4(H + D * D + e0 + 4 * NT * v);
    }
    if (!mono)
    for (int j = 0; j < P.m; ++j) {
      const T uj = (T)gp(P.u)[(size_t)j * P.N + k];
      const T* Hj = H + (size_t)(j + 1) * 2 * D * D + e0;
      v4 ar[NV], ai[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        ar[v] = Prec<T>::gld4(Hj + 4 * NT * v);
        ai[v] = Prec<T>::gld4(Hj + D * D + 4 * NT * v);
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        hr[v] += uj * ar[v];
        hi[v] += uj * ai[v];
      }
    }
    __syncthreads();  // LDS free
    if (mono) {
      // H0 unscaled, then each row's control entries, then the scale
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int e = e0 + 4 * NT * v;
        const int row = e / D - pass * ROWS, col = e % D;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int off = row * SD + ((col + i) & ~15) + Prec<T>::perm((col + i) & 15);
          lds[off] = hr[v][i];
          lim[off] = hi[v][i];
        }
      }
      __syncthreads();
      if ((int)threadIdx.x < ROWS) {
        const int a = pass * ROWS + threadIdx.x;
        const T* mv = reinterpret_cast<const T*>(P.mval);
        for (int j = 0; j < P.m; ++j) {
          const T uj = (T)gp(P.u)[(size_t)j * P.N + k];
          const size_t idx = (size_t)j * D + a;
          const int col = gp(P.mcol)[idx];
          const int off = (int)threadIdx.x * SD + (col & ~15) + Prec<T>::perm(col & 15);
          lds[off] += uj * gp(mv)[2 * idx];
          lim[off] += uj * gp(mv)[2 * idx + 1];
        }
      }
      __syncthreads();
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int e = e0 + 4 * NT * v;
        const int row = e / D - pass * ROWS, col = e % D;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int off = row * SD + ((col + i) & ~15) + Prec<T>::perm((col + i) & 15);
          const T r = lds[off], im = lim[off];
          lds[off] = f * im;  // -i f (r + i im)
          lim[off] = -f * r;
        }
      }
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int e = e0 + 4 * NT * v;
        const int row = e / D - pass * ROWS, col = e % D;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int off = row * SD + ((col + i) & ~15) + Prec<T>::perm((col + i) & 15);
          lds[off] = f * hi[v][i];   // -i f (hr + i hi)
          lim[off] = -f * hr[v][i];
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 8 / PASSES; ++i) {
      const int rb = pass * (8 / PASSES) + i;
      v4 re, im;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int off = (16 * i + Prec<T>::rowmap(r, L.g)) * SD + 16 * L.w + Prec<T>::perm(L.c16);
        re[r] = lds[off];
        im[r] = lim[off];
      }
      if constexpr (PASSES == 1) {
        X.re[rb] = re;
        X.im[rb] = im;
      } else {
        pf_rb_store<T>(out, re, im, L.w, rb, L.lane);
      }
    }
  }
  if constexpr (PASSES == 1) panel_store(out, X, L);
  else panel_load(X, out, L);  // own panel
  __syncthreads();
}

// The gradient epilogue at D = 128 (512 threads), as gradient_epilogue: Z goes
// through LDS so that thread t owns the chunks of four consecutive row
// elements t + 512 i and reads each control's chunks with 16-byte loads,
// consecutive across lanes.  The chunks are taken in two passes over the row
// halves (registers); FP32 stages all of Z once, FP64 stages the half of each
// pass (one FP64 matrix does not fit in LDS).  Z is read from the PF matrix
// Zpf, in which every wavefront has stored its own panel (so the staging
// needs no barrier before its reads and holds no panel in registers).
// With mono (every control has at most one nonzero per row) thread t takes
// row t % 128 of control j0 + t / 128 of each group of four controls and
// reads its one entry of Z from Zpf directly, after a barrier.  FP32 only:
// the branch doubles the FP64 adjoint's register spills, which costs more
// than the dense inner products.
template <typename T>
__device__ __forceinline__ void gradient_epilogue128(const ProbDesc& P, int k, const T* Zpf, const Lane& L,
                                                     T* lds, double* red, bool mono) {
  using v4 = typename Prec<T>::v4;
  constexpr int D = 128, NT = 512, NV = 4;
  static_assert(NT == kEpiGroup * D, "one (control, row) pair per thread");
  if (sizeof(T) == 4 && mono) {
    __syncthreads();  // every wavefront's panel of Z is in Zpf
    const int a = threadIdx.x % D, jj = threadIdx.x / D;
    const T* mv = reinterpret_cast<const T*>(P.mval);
    // PF position of row a: row block, and register / lane group within it
    const int rb = a >> 4, rr = a & 15;
    const int g = sizeof(T) == 4 ? rr >> 2 : rr & 3;
    const int r = sizeof(T) == 4 ? rr & 3 : rr >> 2;
    for (int j0 = 0, grp = 0; j0 < P.m; j0 += kEpiGroup, ++grp) {
      double v[2 * kEpiGroup];
      double tr = 0, ti = 0;
      if (j0 + jj < P.m) {
        const size_t idx = (size_t)(j0 + jj) * D + a;
        const int col = gp(P.mcol)[idx];
        const int lane = 16 * g + (col & 15);
        const double zr = (double)gp(Zpf)[pf_index<T, D>(col >> 4, 0, 4 * rb + r, lane)];
        const double zi = (double)gp(Zpf)[pf_index<T, D>(col >> 4, 1, 4 * rb + r, lane)];
        const double x = (double)gp(mv)[2 * idx], y = (double)gp(mv)[2 * idx + 1];
        tr = zr * x + zi * y;  // conj(z) h
        ti = zr * y - zi * x;
      }
#pragma unroll
      for (int q = 0; q < kEpiGroup; ++q) {
        v[2 * q] = q == jj ? tr : 0.0;
        v[2 * q + 1] = q == jj ? ti : 0.0;
      }
      epilogue_publish<8>(P, k, j0, grp, v, L, red);
    }
    return;
  }
  constexpr bool RESTAGE = sizeof(T) == 8;
  constexpr int ROWS = RESTAGE ? 64 : 128;  // rows staged at once
  constexpr int SD = D + Prec<T>::PAD;
  static_assert(2 * ROWS * SD <= K128<T>::LDS_ELEMS, "LDS too small");
  constexpr int LG = sizeof(T) == 4 ? 2 : 1;  // controls loaded together
  T* lim = lds + ROWS * SD;
  // Stage row blocks [rb0, rb0 + ROWS / 16) of Z, at local rows from 0.
  auto stage = [&](int rb0) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ROWS / 16; ++i) {
      v4 re, im;
      pf_rb_load<T>(re, im, Zpf, L.w, rb0 + i, L.lane);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int off = (16 * i + Prec<T>::rowmap(r, L.g)) * SD + 16 * L.w + Prec<T>::perm(L.c16);
        lds[off] = re[r];
        lim[off] = im[r];
      }
    }
    __syncthreads();
  };
  if (!RESTAGE) stage(0);
  const T* H = reinterpret_cast<const T*>(P.Hint);
  for (int j0 = 0, grp = 0; j0 < P.m; j0 += kEpiGroup, ++grp) {
    double v[2 * kEpiGroup];
#pragma unroll
    for (int i = 0; i < 2 * kEpiGroup; ++i) v[i] = 0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (RESTAGE) stage(4 * h);
      const int e0 = 4 * (threadIdx.x + h * NV * NT);
      const int row0 = RESTAGE ? 64 * h : 0;
      double zr[4 * NV], zi[4 * NV];
#pragma unroll
      for (int q = 0; q < NV; ++q)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int e = e0 + 4 * NT * q;
          const int col = e % D + i;
          const int off = (e / D - row0) * SD + (col & ~15) + Prec<T>::perm(col & 15);
          zr[4 * q + i] = (double)lds[off];
          zi[4 * q + i] = (double)lim[off];
        }
#pragma unroll
      for (int jb = 0; jb < kEpiGroup; jb += LG) {
        v4 hr[LG][NV], hi[LG][NV];
#pragma unroll
        for (int jj = 0; jj < LG; ++jj) {
          const int j = min(j0 + jb + jj, P.m - 1);
          const T* Hj = H + (size_t)(j + 1) * 2 * D * D + e0;
#pragma unroll
          for (int q = 0; q < NV; ++q) {
            hr[jj][q] = Prec<T>::gld4(Hj + 4 * NT * q);
            hi[jj][q] = Prec<T>::gld4(Hj + D * D + 4 * NT * q);
          }
        }
#pragma unroll
        for (int jj = 0; jj < LG; ++jj) {
          double tr = 0, ti = 0;
#pragma unroll
          for (int q = 0; q < NV; ++q)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const double a = zr[4 * q + i], b = zi[4 * q + i];
              const double x = (double)hr[jj][q][i], y = (double)hi[jj][q][i];
              tr += a * x + b * y;  // conj(z) h
              ti += a * y - b * x;
            }
          v[2 * (jb + jj)] += tr;
          v[2 * (jb + jj) + 1] += ti;
        }
      }
    }
    epilogue_publish<8>(P, k, j0, grp, v, L, red);
  }
}

// The three-product form in the FP32 expm and adjoint products at D = 128
// (their registers allow it; the FP64 kernels already spill).
template <typename T>
constexpr bool k128Gauss = sizeof(T) == 4;

template <typename T>
__device__ __forceinline__ T* slot_mat(void* scratch, int i) {
  return reinterpret_cast<T*>(scratch) + ((size_t)blockIdx.x * kScratchMats + i) * K128<T>::ELEMS;
}

template <typename T>
__global__ __launch_bounds__(512) void k_expm128(Work W, void* scratch) {
  __shared__ T lds[K128<T>::LDS_ELEMS];
  Lane L;
  T* SX = slot_mat<T>(scratch, 0);
  T* SR = slot_mat<T>(scratch, 1);
  const Items I(W);
  for (int item = blockIdx.x; item < I.total; item += gridDim.x) {
    int p, k;
    split_item(item, W.rg.s_lo, W.rg.s_n, I.start, I.nprob, p, k);
    const ProbDesc P = W.descs[I.desc(p)];  // a copy: stores cannot alias it
    int s, q, qb;
    unpack_sq(gp(P.sq)[k], s, q, qb);
    Panel<T, 128> acc;
    assemble128<T>(acc, SX, lds, P, k, ldexp(P.dt, -s), 1.0, L, controls_monomial(P));  // SX: the left factor
    // For the adjoint: X = A_k / 2^s in PF layout (its X, A_k^dag / 2^s, is
    // the exact negation), one coalesced store of this wavefront's panel.
    if (P.flags & RUN_GRAD) panel_store(pf_mat<T, 128>(P.hk, k - W.rg.kbase), acc, L);
    // FP32: Paterson-Stockmeyer with X2 = X X as the step, X2 in slot 2 (and
    // kept for the adjoint in gradient runs), C in SR:
    //   p(X) - I = X + X2 C,  C = sum_{n=2..q} X^(n-2) / n!,  C <- D_t + X2 C,
    //   D_t = I / (2t+2)! + X / (2t+3)!
    // (as k_adjoint's block polynomial): expm_products(q) products instead
    // of Horner's q - 1, and X2 on the way.  (Taking X2 from Horner's first
    // product as k_expm does cost this kernel more in scratch traffic than
    // the products it saves.)  FP64, whose kernels spill, runs Horner.
    if (kKeepX2<T> && q >= 2) {
      T* S2 = slot_mat<T>(scratch, 2);
      gemm128<T, false, k128Gauss<T>>(acc, lds, SX, SX, L, true);
      if ((P.flags & RUN_GRAD) && P.x2) panel_store(pf_mat<T, 128>(P.x2, k - W.rg.kbase), acc, L);
      if (q == 2) {
        panel_scale(acc, (T)0.5);
        panel_axpy_pf(acc, (T)1, SX, L);  // X + X2 / 2
      } else {
        panel_store(S2, acc, L);
        const int top = (q - 2) / 2;
        int t;
        if (q & 1) {  // C = I / (q-1)! + X / q!
          t = top - 1;
          panel_load(acc, SX, L);
          panel_scale(acc, (T)inv_factorial(q));
          panel_add_identity(acc, L, (T)inv_factorial(q - 1));
        } else {  // C = I / (q-2)! + X / (q-1)! + X2 / q!
          t = top - 2;
          panel_scale(acc, (T)inv_factorial(q));
          panel_axpy_pf(acc, (T)inv_factorial(q - 1), SX, L);
          panel_add_identity(acc, L, (T)inv_factorial(q - 2));
        }
        panel_store(SR, acc, L);
        bool staged = false;  // X2 already in LDS (from the previous product)
        for (; t >= 0; --t) {  // C <- D_t + X2 C
          panel_load(acc, SX, L);
          panel_scale(acc, (T)inv_factorial(2 * t + 3));
          panel_add_identity(acc, L, (T)inv_factorial(2 * t + 2));
          gemm128<T, false, k128Gauss<T>>(acc, lds, S2, SR, L, false, !staged);
          staged = true;
          panel_store(SR, acc, L);
        }
        panel_load(acc, SX, L);
        gemm128<T, false, k128Gauss<T>>(acc, lds, S2, SR, L, false, !staged);  // X + X2 C
      }
    } else if (q >= 2) {
      panel_scale(acc, (T)(1.0 / q));
      panel_add_identity(acc, L, (T)1);
      panel_store(SR, acc, L);
      for (int i = q - 1; i >= 2; --i) {
        gemm128<T, false, k128Gauss<T>>(acc, lds, SX, SR, L, true);
        panel_scale(acc, (T)(1.0 / i));
        panel_add_identity(acc, L, (T)1);
        panel_store(SR, acc, L);
      }
      gemm128<T, false, k128Gauss<T>>(acc, lds, SX, SR, L, true);
    }
    for (int j = 0; j < s; ++j) {
      panel_store(SR, acc, L);
      gemm128<T, false, k128Gauss<T>>(acc, lds, SR, SR, L, true);
      panel_axpy_pf(acc, (T)2, SR, L);
    }
    panel_store(pf_mat<T, 128>(P.delta, k - W.rg.kbase), acc, L);
  }
}

// The re-unitarisation check of a forward chunk total at D = 128 (FP32): as
// reunitarise(), with G = Y^dag Y formed in FP64 on the vector ALU from Y
// staged in LDS (one FP64 matrix does not fit there): thread t owns the 4 x 8
// tile of G at rows 4 (t / 16), columns 8 (t % 16).  When r > tol, the factor
// (3I - G) / 2 is written in FP32 to Tpf (a PF matrix free during the forward
// scans) and Y <- Y (3I - G) / 2 replaces the chunk total at Ypf.
__device__ __noinline__ void reunitarise128(const ProbDesc& P, float* Ypf, float* Tpf, float* lds, double* red,
                                               const Lane& L) {
  using K = K128<float>;
  constexpr int D = 128, SD = K::SD;
  static_assert(2 * D * SD <= K::LDS_ELEMS, "LDS too small");
  float* yr = lds;
  float* yi = lds + D * SD;
  __syncthreads();  // every wavefront's panel of Y is stored; the LDS is free
#pragma unroll
  for (int rb = 0; rb < 8; ++rb) {
    typename Prec<float>::v4 re, im;
    pf_rb_load<float>(re, im, Ypf, L.w, rb, L.lane);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int off = (16 * rb + Prec<float>::rowmap(r, L.g)) * SD + 16 * L.w + L.c16;
      yr[off] = re[r];
      yi[off] = im[r];
    }
  }
  __syncthreads();
  const int i0 = 4 * (threadIdx.x / 16), j0 = 8 * (threadIdx.x % 16);
  double gr[4][8], gi[4][8];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b) gr[a][b] = gi[a][b] = 0.0;
  for (int k = 0; k < D; ++k) {
    double ar[4], ai[4], br[8], bi[8];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      ar[a] = (double)yr[k * SD + i0 + a];
      ai[a] = (double)yi[k * SD + i0 + a];
    }
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      br[b] = (double)yr[k * SD + j0 + b];
      bi[b] = (double)yi[k * SD + j0 + b];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 8; ++b) {  // conj(Y[k][i]) Y[k][j]
        gr[a][b] += ar[a] * br[b] + ai[a] * bi[b];
        gi[a][b] += ar[a] * bi[b] - ai[a] * br[b];
      }
  }
  const int d = P.d;
  double e2 = 0;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b)
      if (i0 + a < d && j0 + b < d) {
        const double xr = gr[a][b] - (i0 + a == j0 + b ? 1.0 : 0.0), xi = gi[a][b];
        e2 += xr * xr + xi * xi;
      }
  e2 = wave_sum(e2);
  if (L.lane == 0) red[L.w] = e2;
  __syncthreads();
  double tot = 0;
  for (int w = 0; w < 8; ++w) tot += red[w];
  const double res = sqrt(tot);
  if (threadIdx.x == 0)
    atomicMax(reinterpret_cast<unsigned long long*>(&P.diag[1]), (unsigned long long)__double_as_longlong(res));
  if (res > P.reun_tol) {
    // T = (3I - G) / 2 in PF layout: row i is register 4 (i / 16) + r of lane
    // group g (rowmap), column j is lane 16 g + j % 16 of panel j / 16
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int i = i0 + a, rr = i & 15;
      const int g = rr >> 2, r = rr & 3;  // FP32 rowmap(r, g) = 4 g + r
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const int j = j0 + b;
        const int lane = 16 * g + (j & 15);
        gp(Tpf)[pf_index<float, D>(j >> 4, 0, 4 * (i >> 4) + r, lane)] =
            (float)(0.5 * ((i == j ? 3.0 : 0.0) - gr[a][b]));
        gp(Tpf)[pf_index<float, D>(j >> 4, 1, 4 * (i >> 4) + r, lane)] = (float)(-0.5 * gi[a][b]);
      }
    }
    __syncthreads();  // the factor is complete
    Panel<float, D> acc;
    gemm128<float, false>(acc, lds, Ypf, Tpf, L, true);  // Y (3I - G) / 2
    panel_store(Ypf, acc, L);
    if (threadIdx.x == 0) atomicAdd(reinterpret_cast<unsigned long long*>(&P.diag[2]), 1ull);
  }
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(512) void k_scan128(Work W, int dir) {
  __shared__ T lds[K128<T>::LDS_ELEMS];
  __shared__ double red[8];
  const int bwd = dir < 0 ? (int)blockIdx.y : dir;  // dir < 0: both passes, one per blockIdx.y
  Lane L;
  const Items I(W);
  for (int item = blockIdx.x; item < I.total; item += gridDim.x) {
    int p, c;
    split_item(item, W.rg.c_lo, W.rg.c_n, I.start, I.nprob, p, c);
    const ProbDesc P = W.descs[I.desc(p)];  // a copy: stores cannot alias it
    const int k0 = c * P.L;
    const int k1 = min(P.N, k0 + P.L);
    Panel<T, 128> acc;
    if (bwd) panel_load(acc, pf_mat<T, 128>(P.mc, c), L); else panel_identity(acc, L);
    if (!bwd) {
      panel_store(pf_mat<T, 128>(P.xprev, k0 - W.rg.kbase), acc, L);
      for (int k = k0; k < k1; ++k) {
        T* cur = pf_mat<T, 128>(P.xprev, k - W.rg.kbase);
        gemm128<T, false>(acc, lds, pf_mat<T, 128>(P.delta, k - W.rg.kbase), cur, L, true);
        panel_axpy_pf(acc, (T)1, cur, L);
        panel_store(k + 1 < k1 ? pf_mat<T, 128>(P.xprev, k + 1 - W.rg.kbase) : pf_mat<T, 128>(P.tf, c), acc, L);
      }
      if constexpr (sizeof(T) == 4) {
        if (P.reun_tol >= 0 && !W.rg.recompute)
          reunitarise128(P, pf_mat<T, 128>(P.tf, c), pf_mat<T, 128>(P.cf, c), reinterpret_cast<float*>(lds), red, L);
      }
    } else {
      panel_store(pf_mat<T, 128>(P.bloc, k1 - 1 - W.rg.kbase), acc, L);
      for (int k = k1 - 1; k >= k0; --k) {
        T* cur = pf_mat<T, 128>(P.bloc, k - W.rg.kbase);
        gemm128<T, true>(acc, lds, pf_mat<T, 128>(P.delta, k - W.rg.kbase), cur, L, true);
        panel_axpy_pf(acc, (T)1, cur, L);
        if (k > k0) panel_store(pf_mat<T, 128>(P.bloc, k - 1 - W.rg.kbase), acc, L);
      }
    }
    __syncthreads();
  }
}

// The grouped carry at D = 128 (the steps of k_carry_grp, k_carry_top and
// k_mc); every product reads both factors from stored PF matrices.
template <typename T>
__device__ __forceinline__ T* grp_mat128(const ProbDesc& P, int kind, int g) {
  return pf_mat<T, 128>(P.grp, kind * P.PG + g);
}

template <typename T>
__global__ __launch_bounds__(512) void k_carry_grp128(Work W, int dirs, void* scratch) {
  __shared__ T lds[K128<T>::LDS_ELEMS];
  Lane L;
  const Items I(W);
  for (int item = blockIdx.x; item < I.total * dirs; item += gridDim.x) {
    const int bwd = item % dirs;
    int p, g;
    split_item(item / dirs, 0, W.rg.c_n, I.start, I.nprob, p, g);
    const ProbDesc P = W.descs[I.desc(p)];  // a copy: stores cannot alias it
    const int c0 = g * P.CG;
    const int c1 = min(P.P, c0 + P.CG) - 1;
    Panel<T, 128> acc;
    panel_identity(acc, L);
    if (!bwd) {
      panel_store(pf_mat<T, 128>(P.cf, c0), acc, L);
      for (int c = c0; c <= c1; ++c) {
        gemm128<T, false>(acc, lds, pf_mat<T, 128>(P.tf, c), pf_mat<T, 128>(P.cf, c), L, true);
        panel_store(c < c1 ? pf_mat<T, 128>(P.cf, c + 1) : grp_mat128<T>(P, 0, g), acc, L);
      }
    } else {
      panel_store(pf_mat<T, 128>(P.cb, c1), acc, L);
      for (int c = c1; c >= c0; --c) {
        gemm128<T, true>(acc, lds, pf_mat<T, 128>(P.tf, c), pf_mat<T, 128>(P.cb, c), L, true);  // tf[c]^dag cb_loc[c]
        panel_store(c > c0 ? pf_mat<T, 128>(P.cb, c - 1) : grp_mat128<T>(P, 1, g), acc, L);
      }
    }
    __syncthreads();
  }
  (void)scratch;
}

template <typename T>
__global__ __launch_bounds__(512) void k_carry_top128(Work W, int dirs, void* scratch) {
  __shared__ T lds[K128<T>::LDS_ELEMS];
  __shared__ double red[2 * 8];
  Lane L;
  const Items I(W);
  for (int item = blockIdx.x; item < I.nprob * dirs; item += gridDim.x) {
    const int bwd = item % dirs;
    const ProbDesc P = W.descs[I.desc(item / dirs)];  // a copy: stores cannot alias it
    const int ng = P.PG;
    Panel<T, 128> acc;
    if (!bwd) {
      panel_identity(acc, L);
      panel_store(grp_mat128<T>(P, 2, 0), acc, L);
      for (int g = 0; g < ng; ++g) {
        gemm128<T, false>(acc, lds, grp_mat128<T>(P, 0, g), grp_mat128<T>(P, 2, g), L, true);
        if (g + 1 < ng) panel_store(grp_mat128<T>(P, 2, g + 1), acc, L);
      }
      fidelity_epilogue<T, 128>(P, acc, L, red);
      T* SXN = slot_mat<T>(scratch, 0);
      panel_store(SXN, acc, L);
      gemm128<T, true>(acc, lds, SXN, SXN, L, true);
      residual_epilogue<T, 128>(P, acc, L, red);
    } else {
      panel_load(acc, reinterpret_cast<const T*>(P.Vint), L);
      panel_store(grp_mat128<T>(P, 3, ng - 1), acc, L);
      for (int g = ng - 1; g >= 1; --g) {
        gemm128<T, false>(acc, lds, grp_mat128<T>(P, 1, g), grp_mat128<T>(P, 3, g), L, true);
        panel_store(grp_mat128<T>(P, 3, g - 1), acc, L);
      }
    }
    __syncthreads();
  }
}

// mc[c] = cb[c] cf[c]^dag with cf[c] = cf_loc[c] gcf[g], cb[c] = cb_loc[c] gcb[g].
template <typename T>
__global__ __launch_bounds__(512) void k_mc128(Work W, void* scratch) {
  __shared__ T lds[K128<T>::LDS_ELEMS];
  Lane L;
  T* S0 = slot_mat<T>(scratch, 0);
  T* S1 = slot_mat<T>(scratch, 1);
  T* S2 = slot_mat<T>(scratch, 2);
  const Items I(W);
  for (int item = blockIdx.x; item < I.total; item += gridDim.x) {
    int p, c;
    split_item(item, W.rg.c_lo, W.rg.c_n, I.start, I.nprob, p, c);
    const ProbDesc P = W.descs[I.desc(p)];  // a copy: stores cannot alias it
    const int g = c / P.CG;
    Panel<T, 128> acc;
    gemm128<T, false>(acc, lds, pf_mat<T, 128>(P.cf, c), grp_mat128<T>(P, 2, g), L, true);
    panel_store(S1, acc, L);  // cf[c]
    gemm128<T, false>(acc, lds, pf_mat<T, 128>(P.cb, c), grp_mat128<T>(P, 3, g), L, true);
    panel_store(S2, acc, L);  // cb[c]
    transpose128<T>(S0, lds, S1, L);
    gemm128<T, false>(acc, lds, S2, S0, L, true);
    panel_store(pf_mat<T, 128>(P.mc, c), acc, L);
    __syncthreads();
  }
}

// The sampled last step at D = 128 (FP32, s = 0, permutation controls, at most
// kSample128Max controls): as sampled_gradient, with the operands in scratch.
// X2 and S take the LDS in turn (the whole FP32 matrix fits), so every
// column set's partial sums stay in registers between the two passes: pass 1
// adds X2 C2, pass 2 S C1 and E; C1, C2 and E are read one row block of this
// wavefront's own panels at a time.
constexpr int kSample128Max = 16;

__device__ __forceinline__ void sampled_gradient128(const ProbDesc& P, int k, const Lane& L, float* lds, double* red,
                                                    const float* X2, const float* S, const float* C1,
                                                    const float* C2, const float* E, bool x2_staged) {
  using K = K128<float>;
  constexpr int MS = kSample128Max;
  constexpr int G = kEpiGroup;
  const float* lim = lds + K::D * K::SD;
  const int b = 16 * L.w + L.c16;
  const int m = P.m;
  int aj[MS];
  unsigned fresh = 0;  // bit j: control j starts a column set (else it reuses j - 1's)
#pragma unroll
  for (int j = 0; j < MS; ++j) {
    aj[j] = j < m ? gp(P.minv)[(size_t)j * K::D + b] : 0;
    if (j < m && (j % G == 0 || !(gp(P.mok)[j] & 4))) fresh |= 1u << j;
  }
  float zr[MS], zi[MS];
#pragma unroll
  for (int j = 0; j < MS; ++j) zr[j] = zi[j] = 0.f;
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 1 || !x2_staged) {
      __syncthreads();
      stage128<float, false>(lds, pass == 0 ? X2 : S, 0, L);
      __syncthreads();
    }
    const float* Cp = pass == 0 ? C2 : C1;
#pragma unroll 1
    for (int rb = 0; rb < K::RB; ++rb) {
      f4 cr, ci, er, ei;
      pf_rb_load<float>(cr, ci, Cp, L.w, rb, L.lane);
      if (pass == 1) pf_rb_load<float>(er, ei, E, L.w, rb, L.lane);
      const int col = 16 * rb + 4 * L.g;
#pragma unroll
      for (int j = 0; j < MS; ++j) {
        if (fresh & (1u << j)) {  // uniform over the workgroup
          const f4 ar = Prec<float>::ld4(lds + aj[j] * K::SD + col), ai = Prec<float>::ld4(lim + aj[j] * K::SD + col);
          float pr = zr[j], pi = zi[j];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            if (pass == 1 && col + r == aj[j]) {
              pr += er[r];
              pi += ei[r];
            }
            pr = fmaf(ar[r], cr[r], pr);
            pr = fmaf(-ai[r], ci[r], pr);
            pi = fmaf(ar[r], ci[r], pi);
            pi = fmaf(ai[r], cr[r], pi);
          }
          zr[j] = pr;
          zi[j] = pi;
        }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < MS; ++j) {
    if (fresh & (1u << j)) {
      zr[j] += __shfl_xor(zr[j], 16, 64);
      zi[j] += __shfl_xor(zi[j], 16, 64);
      zr[j] += __shfl_xor(zr[j], 32, 64);
      zi[j] += __shfl_xor(zi[j], 32, 64);
    } else if (j > 0) {
      zr[j] = zr[j - 1];
      zi[j] = zi[j - 1];
    }
  }
  const float* mv = reinterpret_cast<const float*>(P.mval);
#pragma unroll
  for (int j0 = 0; j0 < MS; j0 += G) {
    if (j0 >= m) break;
    double v[2 * G];
#pragma unroll
    for (int jj = 0; jj < G; ++jj) {
      const int j = j0 + jj;
      double tr = 0, ti = 0;
      if (L.g == 0 && j < m) {  // conj(z) h, once per column
        const size_t e = (size_t)j * K::D + aj[j];
        const float hr = gp(mv)[2 * e], hi = gp(mv)[2 * e + 1];
        tr = (double)zr[j] * hr + (double)zi[j] * hi;
        ti = (double)zr[j] * hi - (double)zi[j] * hr;
      }
      v[2 * jj] = tr;
      v[2 * jj + 1] = ti;
    }
    epilogue_publish<8, G>(P, k, j0, j0 / G, v, L, red);
  }
}

// Same steps as k_adjoint, with the chain state in scratch (see above).
template <typename T>
__global__ __launch_bounds__(512) void k_adjoint128(Work W, void* scratch) {
  __shared__ T lds[K128<T>::LDS_ELEMS];
  __shared__ double red[2 * kEpiGroup * 2 * 8];
  Lane L;
  T* S0 = slot_mat<T>(scratch, 0);
  T* S1 = slot_mat<T>(scratch, 1);
  T* SE = slot_mat<T>(scratch, 2);
  T* SX = slot_mat<T>(scratch, 3);
  T* SR1 = slot_mat<T>(scratch, 4);
  T* SR2 = slot_mat<T>(scratch, 5);
  const Items I(W);
  for (int item = blockIdx.x; item < I.total; item += gridDim.x) {
    int p, k;
    split_item(item, W.rg.s_lo, W.rg.s_n, I.start, I.nprob, p, k);
    const ProbDesc P = W.descs[I.desc(p)];  // a copy: stores cannot alias it
    const int sqk = gp(P.sq)[k];
    int s, q, qb;
    unpack_sq(sqk, s, q, qb);
    Panel<T, 128> acc;
    // W = bloc[k] xprev[k]^dag (bloc carries mc[c])
    transpose128<T>(S0, lds, pf_mat<T, 128>(P.xprev, k - W.rg.kbase), L);
    gemm128<T, false, k128Gauss<T>>(acc, lds, pf_mat<T, 128>(P.bloc, k - W.rg.kbase), S0, L, true);
    // E = W / 2^s
    panel_scale(acc, (T)ldexp(1.0, -s));
    panel_store(SE, acc, L);
    // X = A^dag / 2^s: the expm pass's A / 2^s negated (A = -i dt H_k with H_k
    // Hermitian), or its conjugate transpose for general generators (own
    // panel; the barrier at the start of the next product publishes SX)
    if (P.flags & RUN_GENERAL) {
      transpose128<T>(SX, lds, pf_mat<T, 128>(P.hk, k - W.rg.kbase), L);
    } else {
      panel_load(acc, pf_mat<T, 128>(P.hk, k - W.rg.kbase), L);
      panel_scale(acc, (T)-1);
      panel_store(SX, acc, L);
    }
    // The block polynomial by Paterson-Stockmeyer as in k_adjoint: M^2 =
    // [[X2, S], [0, X2]] into S0 (X2) and S1 (S), the running C = [[C1, C2],
    // [0, C1]] in SR1 and SR2.
    if (kKeepX2<T> && q >= 2 && P.x2 && !(P.flags & RUN_GENERAL))
      panel_load(acc, pf_mat<T, 128>(P.x2, k - W.rg.kbase), L);  // kept by the expm
    else gemm128<T, false, k128Gauss<T>>(acc, lds, SX, SX, L, true);
    panel_store(S0, acc, L);
    gemm128<T, false, k128Gauss<T>>(acc, lds, SX, SE, L, true);
    gemm128<T, false, k128Gauss<T>>(acc, lds, SE, SX, L, false);
    panel_store(S1, acc, L);
    const int top = (qb - 2) / 2;
    int t;
    if (qb & 1) {  // C = I / (qb-1)! + M / qb!
      t = top - 1;
      panel_load(acc, SX, L);
      panel_scale(acc, (T)inv_factorial(qb));
      panel_add_identity(acc, L, (T)inv_factorial(qb - 1));
      panel_store(SR1, acc, L);
      panel_load(acc, SE, L);
      panel_scale(acc, (T)inv_factorial(qb));
      panel_store(SR2, acc, L);
    } else if (top > 0) {  // C = I / (qb-2)! + M / (qb-1)! + M^2 / qb!
      t = top - 2;
      panel_load(acc, SX, L);
      panel_scale(acc, (T)inv_factorial(qb - 1));
      panel_axpy_pf(acc, (T)inv_factorial(qb), S0, L);
      panel_add_identity(acc, L, (T)inv_factorial(qb - 2));
      panel_store(SR1, acc, L);
      panel_load(acc, SE, L);
      panel_scale(acc, (T)inv_factorial(qb - 1));
      panel_axpy_pf(acc, (T)inv_factorial(qb), S1, L);
      panel_store(SR2, acc, L);
    } else {  // qb = 2: C = I / 2
      t = -1;
      panel_zero(acc);
      panel_store(SR2, acc, L);
      panel_add_identity(acc, L, (T)0.5);
      panel_store(SR1, acc, L);
    }
    // Products with X2 as the left factor follow each other where they can
    // (S C1 first in a step), so that X2 stays in LDS between them (FP32).
    bool x2_staged = false;
    for (; t >= 0; --t) {  // C <- D_t + M^2 C (own panels of SR1, SR2 only)
      const T a = (T)inv_factorial(2 * t + 2), b = (T)inv_factorial(2 * t + 3);
      panel_load(acc, SE, L);
      panel_scale(acc, b);
      gemm128<T, false, k128Gauss<T>>(acc, lds, S1, SR1, L, false);
      gemm128<T, false, k128Gauss<T>>(acc, lds, S0, SR2, L, false);
      panel_store(SR2, acc, L);  // b E + S C1 + X2 C2
      panel_load(acc, SX, L);
      panel_scale(acc, b);
      panel_add_identity(acc, L, a);
      gemm128<T, false, k128Gauss<T>>(acc, lds, S0, SR1, L, false, false);
      panel_store(SR1, acc, L);  // a I + b X + X2 C1
      x2_staged = true;
    }
    if constexpr (sizeof(T) == 4) {
      if ((sqk & kPlanSampled) && P.m <= kSample128Max) {  // s = 0: only the entries the controls read
        sampled_gradient128(P, k, L, lds, red, S0, S1, SR1, SR2, SE, x2_staged);
        __syncthreads();
        continue;
      }
    }
    // Q = E + X2 C2 + S C1 and, when squaring follows, D1 = X + X2 C1 (into
    // S1 once every wavefront has staged S; Q waits in the own panel of SE).
    panel_load(acc, SE, L);
    gemm128<T, false, k128Gauss<T>>(acc, lds, S0, SR2, L, false, !x2_staged);
    gemm128<T, false, k128Gauss<T>>(acc, lds, S1, SR1, L, false);
    if (s > 0) {
      panel_store(SE, acc, L);
      panel_load(acc, SX, L);
      gemm128<T, false, k128Gauss<T>>(acc, lds, S0, SR1, L, false);
      panel_store(S1, acc, L);
      panel_load(acc, SE, L);
    }
    for (int j = 0; j < s; ++j) {
      panel_store(S0, acc, L);                        // Q
      gemm128<T, false, k128Gauss<T>>(acc, lds, S1, S0, L, true);   // D1 Q
      gemm128<T, false, k128Gauss<T>>(acc, lds, S0, S1, L, false);  // + Q D1
      panel_axpy_pf(acc, (T)2, S0, L);                // Q <- 2Q + D1 Q + Q D1
      if (j + 1 < s) {
        // Every wavefront's staging of the old Q and D1 ended before the
        // barrier inside the last product, so own panels may be replaced.
        panel_store(S0, acc, L);
        gemm128<T, false, k128Gauss<T>>(acc, lds, S1, S1, L, true);
        panel_axpy_pf(acc, (T)2, S1, L);              // D1 <- 2 D1 + D1^2
        panel_store(S1, acc, L);
        panel_load(acc, S0, L);
      }
    }
    panel_store(S0, acc, L);  // Z (own panel)
    gradient_epilogue128<T>(P, k, S0, L, lds, red, sizeof(T) == 4 && controls_monomial(P));
    __syncthreads();
  }
}

// ---------------------------------------------------------------- launchers

// Work of an API launch over range rg: uniform counts when rg says so,
// otherwise the prefix arrays of the launch.
static inline Work slice_work(const Launch& L, const Range& rg) {
  return Work{L.descs, L.nprob, rg.s_n > 0 ? L.nprob * rg.s_n : L.total_slices, rg.s_n > 0 ? nullptr : L.slice_start,
              rg, nullptr};
}
static inline Work chunk_work(const Launch& L, const Range& rg) {
  return Work{L.descs, L.nprob, rg.c_n > 0 ? L.nprob * rg.c_n : L.total_chunks, rg.c_n > 0 ? nullptr : L.chunk_start,
              rg, nullptr};
}
static inline int grid_of(const Launch& L, int items, int cap) {
  if (L.dyn_grid > 0) return L.dyn_grid;
  return items < 1 ? 1 : (cap > 0 && items > cap ? cap : items);
}

template <typename T, int D, typename Ops>
static void stage_small(int stage, const Launch& L, const Range& rg, double ur) {
  constexpr int NT = Mat<T, D>::NT;
  hipStream_t st = L.stream;
  const int dirs = (L.flags & RUN_BWD) ? 2 : 1;
  const int grad = (L.flags & RUN_GRAD) ? 1 : 0;
  const Range all = {0, L.uniformN, 0, L.uniformP, rg.kbase};
  const Work dyn = L.dyn ? Work{L.descs, 0, 0, nullptr, Range{0, 0, 0, 0, 0}, L.dyn} : Work{};
  switch (stage) {
    case ST_PREP: {
      Work w = L.dyn ? dyn : Work{L.descs, L.nprob, L.nprob * (L.max_m + 2), nullptr,
                                  Range{0, L.max_m + 2, 0, 0, 0}, nullptr};
      hipLaunchKernelGGL((k_prep<T, D>), dim3(grid_of(L, w.total, 0)), dim3(256), 0, st, w);
      break;
    }
    case ST_PLAN: {
      Work w = L.dyn ? dyn : slice_work(L, all);
      hipLaunchKernelGGL(k_plan, dim3(L.dyn ? L.dyn_grid : (w.total + 255) / 256), dim3(256), 0, st, w, ur, grad);
      break;
    }
    case ST_EXPM: {
      // the split-BF16 policy serves the adjoint only (launch_stage)
      if constexpr (kStdLds<T, D, Ops>) {
      Work w = L.dyn ? dyn : slice_work(L, rg);
      if (L.dyn) hipLaunchKernelGGL((k_expm<T, D, Ops, true>), dim3(grid_of(L, w.total, 0)), dim3(NT), 0, st, w);
      else hipLaunchKernelGGL((k_expm<T, D, Ops, false>), dim3(grid_of(L, w.total, 0)), dim3(NT), 0, st, w);
      }
      break;
    }
    case ST_SCAN:
    case ST_BSCAN: {
      if constexpr (kStdLds<T, D, Ops>) {
      Work w = L.dyn ? dyn : chunk_work(L, rg);
      // a recompute sweep runs the forward and backward passes of a segment
      // together (they are independent once mc is known)
      const bool both = stage == ST_SCAN && rg.recompute && !L.dyn;
      const int dir = stage == ST_BSCAN ? 1 : (both ? -1 : 0);
      const dim3 grid(grid_of(L, w.total, 0), both ? 2 : 1);
      if (L.dyn) hipLaunchKernelGGL((k_scan_local<T, D, Ops, true>), grid, dim3(NT), 0, st, w, dir);
      else hipLaunchKernelGGL((k_scan_local<T, D, Ops, false>), grid, dim3(NT), 0, st, w, dir);
      if constexpr (sizeof(T) == 4) {
        if (stage == ST_SCAN && !rg.recompute) {
          if (L.dyn) hipLaunchKernelGGL((k_reun<D, true>), dim3(grid.x), dim3(NT), 0, st, w);
          else hipLaunchKernelGGL((k_reun<D, false>), dim3(grid.x), dim3(NT), 0, st, w);
        }
      }
      }
      break;
    }
    case ST_CARRY: {
      int CG, PG;
      carry_groups(L.uniformP, CG, PG);
      Work wg = L.dyn ? dyn : Work{L.descs, L.nprob, L.nprob * PG, nullptr, Range{0, 0, 0, PG, 0}, nullptr};
      hipLaunchKernelGGL((k_carry_grp<T, D>), dim3(grid_of(L, wg.total, 0), dirs), dim3(NT), 0, st, wg);
      Work w = L.dyn ? dyn : Work{L.descs, L.nprob, L.nprob, nullptr, all, nullptr};
      hipLaunchKernelGGL((k_carry_top<T, D>), dim3(grid_of(L, L.nprob, 0), dirs), dim3(NT), 0, st, w);
      break;
    }
    case ST_MC: {
      Work w = L.dyn ? dyn : chunk_work(L, all);
      hipLaunchKernelGGL((k_mc<T, D>), dim3(grid_of(L, w.total, 0)), dim3(NT), 0, st, w);
      break;
    }
    case ST_ADJ: {
      Work w = L.dyn ? dyn : slice_work(L, rg);
      const dim3 grid(grid_of(L, w.total, 0));
      if constexpr (kSampleLast<T, D, Ops>) {
        if (L.dyn) {
          hipLaunchKernelGGL((k_adjoint<T, D, Ops, true, 2>), grid, dim3(NT), 0, st, w);
          hipLaunchKernelGGL((k_adjoint<T, D, Ops, true, 1>), grid, dim3(NT), 0, st, w);
        } else {
          hipLaunchKernelGGL((k_adjoint<T, D, Ops, false, 2>), grid, dim3(NT), 0, st, w);
          hipLaunchKernelGGL((k_adjoint<T, D, Ops, false, 1>), grid, dim3(NT), 0, st, w);
        }
      } else {
        if (L.dyn) hipLaunchKernelGGL((k_adjoint<T, D, Ops, true>), grid, dim3(NT), 0, st, w);
        else hipLaunchKernelGGL((k_adjoint<T, D, Ops, false>), grid, dim3(NT), 0, st, w);
      }
      break;
    }
  }
}

template <typename T>
static void stage_128(int stage, const Launch& L, const Range& rg, double ur) {
  hipStream_t st = L.stream;
  const int dirs = (L.flags & RUN_BWD) ? 2 : 1;
  const int grad = (L.flags & RUN_GRAD) ? 1 : 0;
  const Range all = {0, L.uniformN, 0, L.uniformP, rg.kbase};
  const Work dyn = L.dyn ? Work{L.descs, 0, 0, nullptr, Range{0, 0, 0, 0, 0}, L.dyn} : Work{};
  const int cap = kScratchSlots;
  switch (stage) {
    case ST_PREP: {
      Work w = L.dyn ? dyn : Work{L.descs, L.nprob, L.nprob * (L.max_m + 2), nullptr,
                                  Range{0, L.max_m + 2, 0, 0, 0}, nullptr};
      hipLaunchKernelGGL((k_prep<T, 128>), dim3(grid_of(L, w.total, 0)), dim3(256), 0, st, w);
      break;
    }
    case ST_PLAN: {
      Work w = L.dyn ? dyn : slice_work(L, all);
      hipLaunchKernelGGL(k_plan, dim3(L.dyn ? L.dyn_grid : (w.total + 255) / 256), dim3(256), 0, st, w, ur,
                         grad | (kKeepX2<T> ? 2 : 0));
      break;
    }
    case ST_EXPM: {
      Work w = L.dyn ? dyn : slice_work(L, rg);
      hipLaunchKernelGGL(k_expm128<T>, dim3(grid_of(L, w.total, cap)), dim3(512), 0, st, w, L.scratch);
      break;
    }
    case ST_SCAN:
    case ST_BSCAN: {
      Work w = L.dyn ? dyn : chunk_work(L, rg);
      const bool both = stage == ST_SCAN && rg.recompute && !L.dyn;
      const int dir = stage == ST_BSCAN ? 1 : (both ? -1 : 0);
      hipLaunchKernelGGL(k_scan128<T>, dim3(grid_of(L, w.total, 0), both ? 2 : 1), dim3(512), 0, st, w, dir);
      break;
    }
    case ST_CARRY: {
      int CG, PG;
      carry_groups(L.uniformP, CG, PG);
      Work wg = L.dyn ? dyn : Work{L.descs, L.nprob, L.nprob * PG, nullptr, Range{0, 0, 0, PG, 0}, nullptr};
      hipLaunchKernelGGL(k_carry_grp128<T>, dim3(grid_of(L, wg.total * dirs, cap)), dim3(512), 0, st, wg, dirs,
                         L.scratch);
      Work w = L.dyn ? dyn : Work{L.descs, L.nprob, L.nprob, nullptr, all, nullptr};
      hipLaunchKernelGGL(k_carry_top128<T>, dim3(grid_of(L, L.nprob * dirs, cap)), dim3(512), 0, st, w, dirs,
                         L.scratch);
      break;
    }
    case ST_MC: {
      Work w = L.dyn ? dyn : chunk_work(L, all);
      hipLaunchKernelGGL(k_mc128<T>, dim3(grid_of(L, w.total, cap)), dim3(512), 0, st, w, L.scratch);
      break;
    }
    case ST_ADJ: {
      Work w = L.dyn ? dyn : slice_work(L, rg);
      hipLaunchKernelGGL(k_adjoint128<T>, dim3(grid_of(L, w.total, cap)), dim3(512), 0, st, w, L.scratch);
      break;
    }
  }
}

hipError_t launch_stage(int precision, int D, int stage, const Launch& L, const Range& rg) {
  const double ur64 = 0x1p-53, ur32 = 0x1p-24;
  stage_mark(stage, true, L.stream);
  bool ok = true;
  if (precision == 0) {
    switch (D) {
      case 16: stage_small<double, 16, StdOps<double, 16>>(stage, L, rg, ur64); break;
      case 32: stage_small<double, 32, StdOps<double, 32>>(stage, L, rg, ur64); break;
      case 64: stage_small<double, 64, StdOps<double, 64>>(stage, L, rg, ur64); break;
      case 128: stage_128<double>(stage, L, rg, ur64); break;
      default: ok = false;
    }
  } else if (precision == 1) {
    switch (D) {
      case 16: stage_small<float, 16, StdOps<float, 16>>(stage, L, rg, ur32); break;
      case 32: stage_small<float, 32, StdOps<float, 32>>(stage, L, rg, ur32); break;
      case 64: stage_small<float, 64, StdOps<float, 64>>(stage, L, rg, ur32); break;
      case 128: stage_128<float>(stage, L, rg, ur32); break;
      default: ok = false;
    }
  } else if (precision == 2) {
    // split-BF16 products in the adjoint (the Frechet series and its trace
    // contractions, the dominant kernel); the exponentials, scans, carries and
    // chunk products stay FP32.  Split products in the forward chain as well
    // leave an absolute error in Tr(V^dag X_N) several times larger, which
    // the gradient of a member with a small |g| cannot absorb.
    const bool adj = stage == ST_ADJ;
    switch (D) {
      case 32:
        if (adj) stage_small<float, 32, Bf3Ops<32>>(stage, L, rg, ur32);
        else stage_small<float, 32, StdOps<float, 32>>(stage, L, rg, ur32);
        break;
      case 64:
        if (adj) stage_small<float, 64, Bf3Ops<64>>(stage, L, rg, ur32);
        else stage_small<float, 64, StdOps<float, 64>>(stage, L, rg, ur32);
        break;
      default: ok = false;
    }
  } else {
    ok = false;
  }
  stage_mark(stage, false, L.stream);
  if (!ok) return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace qoc
