// Device building blocks for the GRAPE kernels on gfx950 (CDNA4).
//
// A D x D complex matrix is processed by D/16 wavefronts; wavefront w owns the
// 16-column panel [16w, 16w + 16).  A panel is held in registers in the output
// ("C") layout of the 16x16x4 MFMA: for row block rb (16 rows) each lane holds
// four values per real plane.  Lane l = 16 g + c16 holds column 16w + c16 and
// rows 16 rb + rowmap(r, g), r = 0..3, where rowmap is the accumulator layout
// of the instruction (FP32: 4g + r; FP64: 4r + g).
//
// A panel in that layout is fed straight back as the B operand of the next
// MFMA: register r of row block rb supplies K index g (= lane / 16), which
// stands for matrix row 16 rb + rowmap(r, g).  The A operand is read from LDS
// with the matching permutation of its columns, so chained products
// (Horner steps, scan steps) keep their state in registers and only the
// left factor is staged in LDS.  Complex products use four real MFMA
// products (cgemm), Re += Ar Br - Ai Bi and Im += Ar Bi + Ai Br, or three
// (cgemm3m, the Gauss form below).
//
// LDS matrices are row-major with separate real and imaginary planes, a row
// stride of D + pad elements (16 bytes of padding) and, within each 16-column
// block, the column permutation perm() under which the four A values a lane
// needs for one row block are contiguous (one 16-byte read for FP32, two for
// FP64).
//
// Stored matrices ("PF" layout) keep the register order of a panel so that a
// wavefront loads or stores its panel with fully coalesced 16-byte accesses:
//   index(w, plane, reg, lane) = ((w*2 + plane) * (D/4/G) + reg/G) * 64 * G + lane * G + reg % G
// with reg = 4 rb + r and G = 16 / sizeof(T) elements per 16-byte access.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qoc {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

// Global-memory accesses go through address space 1, so that the compiler
// issues global_* instructions.  Through a generic pointer it issues flat_*
// ones, which may also address LDS; it then has to wait for every
// outstanding memory operation around them (a prefetch issued before a store
// would be waited for at once).
#define QOC_GLOBAL __attribute__((address_space(1)))

template <typename T>
__device__ __forceinline__ const QOC_GLOBAL T* gp(const T* p) {
  return (const QOC_GLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ QOC_GLOBAL T* gp(T* p) {
  return (QOC_GLOBAL T*)p;
}

template <typename T>
struct Prec;

template <>
struct Prec<float> {
  using v4 = f4;
  static constexpr int PAD = 4;
  __device__ static __forceinline__ int rowmap(int r, int g) { return 4 * g + r; }
  __device__ static __forceinline__ int perm(int c) { return c; }
  __device__ static __forceinline__ v4 mfma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ v4 ld4(const float* p) { return *reinterpret_cast<const f4*>(p); }
  __device__ static __forceinline__ void st4(float* p, v4 v) { *reinterpret_cast<f4*>(p) = v; }
  // the same from / to global memory
  __device__ static __forceinline__ v4 gld4(const float* p) { return *(const QOC_GLOBAL f4*)p; }
  __device__ static __forceinline__ void gst4(float* p, v4 v) { *(QOC_GLOBAL f4*)p = v; }
};

template <>
struct Prec<double> {
  using v4 = d4;
  static constexpr int PAD = 2;
  __device__ static __forceinline__ int rowmap(int r, int g) { return 4 * r + g; }
  __device__ static __forceinline__ int perm(int c) { return 4 * (c & 3) + (c >> 2); }
  __device__ static __forceinline__ v4 mfma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ v4 ld4(const double* p) {
    d2 lo = *reinterpret_cast<const d2*>(p);
    d2 hi = *reinterpret_cast<const d2*>(p + 2);
    v4 v;
    v.x = lo.x; v.y = lo.y; v.z = hi.x; v.w = hi.y;
    return v;
  }
  __device__ static __forceinline__ void st4(double* p, v4 v) {
    d2 lo, hi;
    lo.x = v.x; lo.y = v.y; hi.x = v.z; hi.y = v.w;
    *reinterpret_cast<d2*>(p) = lo;
    *reinterpret_cast<d2*>(p + 2) = hi;
  }
  // the same from / to global memory
  __device__ static __forceinline__ v4 gld4(const double* p) {
    d2 lo = *(const QOC_GLOBAL d2*)p;
    d2 hi = *(const QOC_GLOBAL d2*)(p + 2);
    v4 v;
    v.x = lo.x; v.y = lo.y; v.z = hi.x; v.w = hi.y;
    return v;
  }
  __device__ static __forceinline__ void gst4(double* p, v4 v) {
    d2 lo, hi;
    lo.x = v.x; lo.y = v.y; hi.x = v.z; hi.y = v.w;
    *(QOC_GLOBAL d2*)p = lo;
    *(QOC_GLOBAL d2*)(p + 2) = hi;
  }
};

// Elements of one stored matrix (both planes).
template <typename T, int D>
struct Mat {
  static constexpr int SD = D + Prec<T>::PAD;  // LDS row stride
  static constexpr int LDS_ELEMS = 2 * D * SD;  // one LDS matrix, both planes
  static constexpr int ELEMS = 2 * D * D;       // one stored matrix
  static constexpr int RB = D / 16;             // row blocks per panel
  static constexpr int NW = D / 16;             // wavefronts per matrix
  static constexpr int NT = 64 * NW;            // threads per matrix
};

template <typename T, int D>
struct Panel {
  using v4 = typename Prec<T>::v4;
  v4 re[D / 16];
  v4 im[D / 16];
};

struct Lane {
  int w, g, c16, lane;
  __device__ __forceinline__ Lane() {
    lane = threadIdx.x & 63;
    w = threadIdx.x >> 6;
    g = lane >> 4;
    c16 = lane & 15;
  }
};

// LDS offset of logical element (row, col).
template <typename T, int D>
__device__ __forceinline__ int lds_off(int row, int col) {
  return row * Mat<T, D>::SD + (col & ~15) + Prec<T>::perm(col & 15);
}

template <typename T, int D>
__device__ __forceinline__ void panel_zero(Panel<T, D>& P) {
#pragma unroll
  for (int rb = 0; rb < D / 16; ++rb) {
    P.re[rb] = 0;
    P.im[rb] = 0;
  }
}

// The constant 1 passed through an empty asm, so that the compiler cannot
// hoist a whole identity panel out of a loop and keep it live in registers.
template <typename T>
__device__ __forceinline__ T opaque_one() {
  T one = T(1);
  asm volatile("" : "+v"(one));
  return one;
}

template <typename T, int D>
__device__ __forceinline__ void panel_identity(Panel<T, D>& P, const Lane& L) {
  const T one = opaque_one<T>();
#pragma unroll
  for (int rb = 0; rb < D / 16; ++rb) {
#pragma unroll
    for (int r = 0; r < 4; ++r) P.re[rb][r] = (rb == L.w && Prec<T>::rowmap(r, L.g) == L.c16) ? one : T(0);
    P.im[rb] = 0;
  }
}

// P += a * I
template <typename T, int D>
__device__ __forceinline__ void panel_add_identity(Panel<T, D>& P, const Lane& L, T a) {
#pragma unroll
  for (int r = 0; r < 4; ++r)
    if (Prec<T>::rowmap(r, L.g) == L.c16) {
#pragma unroll
      for (int rb = 0; rb < D / 16; ++rb)
        if (rb == L.w) P.re[rb][r] += a;
    }
}

// Y = a * X + b * Y  (elementwise on panels)
template <typename T, int D>
__device__ __forceinline__ void panel_axpby(Panel<T, D>& Y, T a, const Panel<T, D>& X, T b) {
#pragma unroll
  for (int rb = 0; rb < D / 16; ++rb) {
    Y.re[rb] = a * X.re[rb] + b * Y.re[rb];
    Y.im[rb] = a * X.im[rb] + b * Y.im[rb];
  }
}

template <typename T, int D>
__device__ __forceinline__ void panel_scale(Panel<T, D>& Y, T a) {
#pragma unroll
  for (int rb = 0; rb < D / 16; ++rb) {
    Y.re[rb] *= a;
    Y.im[rb] *= a;
  }
}

// ---------------------------------------------------------------- LDS <-> panel

// Panel of the matrix stored in LDS (same orientation).
template <typename T, int D>
__device__ __forceinline__ void panel_from_lds(Panel<T, D>& P, const T* lds, const Lane& L) {
  const T* im = lds + D * Mat<T, D>::SD;
#pragma unroll
  for (int rb = 0; rb < D / 16; ++rb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int off = lds_off<T, D>(16 * rb + Prec<T>::rowmap(r, L.g), 16 * L.w + L.c16);
      P.re[rb][r] = lds[off];
      P.im[rb][r] = im[off];
    }
}

// Panel of the conjugate transpose of the matrix stored in LDS.  Element
// (row, col) of M^dag is conj(M[col][row]); the four values of one row block
// sit contiguously in LDS row 16w + c16, so each plane takes one vector read.
template <typename T, int D>
__device__ __forceinline__ void panel_from_lds_ct(Panel<T, D>& P, const T* lds, const Lane& L) {
  const T* im = lds + D * Mat<T, D>::SD;
#pragma unroll
  for (int rb = 0; rb < D / 16; ++rb) {
    int off = (16 * L.w + L.c16) * Mat<T, D>::SD + 16 * rb + 4 * L.g;
    P.re[rb] = Prec<T>::ld4(lds + off);
    P.im[rb] = -Prec<T>::ld4(im + off);
  }
}

template <typename T, int D>
__device__ __forceinline__ void panel_to_lds(T* lds, const Panel<T, D>& P, const Lane& L) {
  T* im = lds + D * Mat<T, D>::SD;
#pragma unroll
  for (int rb = 0; rb < D / 16; ++rb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int off = lds_off<T, D>(16 * rb + Prec<T>::rowmap(r, L.g), 16 * L.w + L.c16);
      lds[off] = P.re[rb][r];
      im[off] = P.im[rb][r];
    }
}

// Store the conjugate transpose of the panel's matrix into LDS.
template <typename T, int D>
__device__ __forceinline__ void panel_to_lds_ct(T* lds, const Panel<T, D>& P, const Lane& L) {
  T* im = lds + D * Mat<T, D>::SD;
#pragma unroll
  for (int rb = 0; rb < D / 16; ++rb) {
    int off = (16 * L.w + L.c16) * Mat<T, D>::SD + 16 * rb + 4 * L.g;
    Prec<T>::st4(lds + off, P.re[rb]);
    Prec<T>::st4(im + off, -P.im[rb]);
  }
}

// ---------------------------------------------------------------- MFMA product

// acc = A * P (zero_acc) or acc += A * P, with A a D x D matrix in LDS and P a
// panel.  Each wavefront computes its own 16 output columns; no barrier inside.
// The product runs over (k block, output row block) steps; the A fragment of
// the next step is read from LDS while the 16 MFMAs of the current step issue,
// and scheduling barriers keep the compiler from hoisting every LDS read to
// the top (which would cost one register set per step).
template <typename T, int D>
__device__ __forceinline__ void cgemm(Panel<T, D>& acc, const T* A, const Panel<T, D>& P, const Lane& L,
                                      bool zero_acc) {
  using v4 = typename Prec<T>::v4;
  constexpr int RB = D / 16;
  constexpr int SD = Mat<T, D>::SD;
  constexpr int STEPS = RB * RB;
  const T* Ai = A + D * SD;
  const int base = L.c16 * SD + 4 * L.g;
  __builtin_amdgcn_sched_barrier(0);
  if (zero_acc) panel_zero(acc);
  v4 ar[2], ai[2];
  ar[0] = Prec<T>::ld4(A + base);
  ai[0] = Prec<T>::ld4(Ai + base);
#pragma unroll
  for (int st = 0; st < STEPS; ++st) {
    const int kb = st / RB, mb = st % RB;
    const int cur = st & 1;
    if (st + 1 < STEPS) {
      const int kn = (st + 1) / RB, mn = (st + 1) % RB;
      const int off = base + 16 * mn * SD + 16 * kn;
      ar[cur ^ 1] = Prec<T>::ld4(A + off);
      ai[cur ^ 1] = Prec<T>::ld4(Ai + off);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const T br = P.re[kb][r];
      const T bi = P.im[kb][r];
      acc.re[mb] = Prec<T>::mfma(ar[cur][r], br, acc.re[mb]);
      acc.im[mb] = Prec<T>::mfma(ar[cur][r], bi, acc.im[mb]);
      acc.re[mb] = Prec<T>::mfma(-ai[cur][r], bi, acc.re[mb]);
      acc.im[mb] = Prec<T>::mfma(ai[cur][r], br, acc.im[mb]);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// The same product with three real products per complex one (Gauss; the "3M" method):
// T1 = Ar Br, T2 = Ai Bi, T3 = (Ar + Ai)(Br + Bi), Re = T1 - T2 and
// Im = T3 - T1 - T2.  T1 accumulates in acc.re and T3 in acc.im, which
// starts at acc.im + acc.re so that the final Im = T3 - T1 - T2 keeps the
// incoming acc.im; its error bound is a small multiple of that of the
// four-product form (Higham, Accuracy and Stability of Numerical Algorithms,
// 2nd ed., sec. 23.2.4).
//
// It needs two more register sets (the B sums and T2) than cgemm, so kernels
// use it where their occupancy allows.  PAIRS = 2 takes the steps two at a
// time, so that six accumulator chains are independent within each group of
// MFMAs instead of three (measured: the expm 4% faster, the scans 3% slower;
// chosen per caller).
template <typename T, int D, int PAIRS = 1>
__device__ __forceinline__ void cgemm3m(Panel<T, D>& acc, const T* A, const Panel<T, D>& P, const Lane& L,
                                      bool zero_acc) {
  using v4 = typename Prec<T>::v4;
  constexpr int RB = D / 16;
  constexpr int SD = Mat<T, D>::SD;
  constexpr int STEPS = RB * RB;
  const T* Ai = A + D * SD;
  const int base = L.c16 * SD + 4 * L.g;
  __builtin_amdgcn_sched_barrier(0);
  v4 bs[RB], t2[RB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    bs[rb] = P.re[rb] + P.im[rb];
    t2[rb] = (v4){0, 0, 0, 0};
    if (zero_acc) {
      acc.re[rb] = (v4){0, 0, 0, 0};
      acc.im[rb] = (v4){0, 0, 0, 0};
    } else {
      acc.im[rb] += acc.re[rb];
    }
  }
  if constexpr (PAIRS == 2) {
    static_assert(STEPS % 2 == 0, "pairs of steps");
    v4 pr[2][2], pi[2][2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int off = base + 16 * (h % RB) * SD + 16 * (h / RB);
      pr[0][h] = Prec<T>::ld4(A + off);
      pi[0][h] = Prec<T>::ld4(Ai + off);
    }
#pragma unroll
    for (int sp = 0; sp < STEPS; sp += 2) {
      const int cur = (sp / 2) & 1;
      if (sp + 2 < STEPS) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int sn = sp + 2 + h;
          const int off = base + 16 * (sn % RB) * SD + 16 * (sn / RB);
          pr[cur ^ 1][h] = Prec<T>::ld4(A + off);
          pi[cur ^ 1][h] = Prec<T>::ld4(Ai + off);
        }
      }
      const int kb0 = sp / RB, mb0 = sp % RB, kb1 = (sp + 1) / RB, mb1 = (sp + 1) % RB;
      const v4 as0 = pr[cur][0] + pi[cur][0];
      const v4 as1 = pr[cur][1] + pi[cur][1];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        acc.re[mb0] = Prec<T>::mfma(pr[cur][0][r], P.re[kb0][r], acc.re[mb0]);
        acc.re[mb1] = Prec<T>::mfma(pr[cur][1][r], P.re[kb1][r], acc.re[mb1]);
        t2[mb0] = Prec<T>::mfma(pi[cur][0][r], P.im[kb0][r], t2[mb0]);
        t2[mb1] = Prec<T>::mfma(pi[cur][1][r], P.im[kb1][r], t2[mb1]);
        acc.im[mb0] = Prec<T>::mfma(as0[r], bs[kb0][r], acc.im[mb0]);
        acc.im[mb1] = Prec<T>::mfma(as1[r], bs[kb1][r], acc.im[mb1]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  } else {
  v4 ar[2], ai[2];
  ar[0] = Prec<T>::ld4(A + base);
  ai[0] = Prec<T>::ld4(Ai + base);
#pragma unroll
  for (int st = 0; st < STEPS; ++st) {
    const int kb = st / RB, mb = st % RB;
    const int cur = st & 1;
    if (st + 1 < STEPS) {
      const int kn = (st + 1) / RB, mn = (st + 1) % RB;
      const int off = base + 16 * mn * SD + 16 * kn;
      ar[cur ^ 1] = Prec<T>::ld4(A + off);
      ai[cur ^ 1] = Prec<T>::ld4(Ai + off);
    }
    const v4 as = ar[cur] + ai[cur];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      acc.re[mb] = Prec<T>::mfma(ar[cur][r], P.re[kb][r], acc.re[mb]);
      t2[mb] = Prec<T>::mfma(ai[cur][r], P.im[kb][r], t2[mb]);
      acc.im[mb] = Prec<T>::mfma(as[r], bs[kb][r], acc.im[mb]);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  }
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    acc.im[rb] = acc.im[rb] - acc.re[rb] - t2[rb];
    acc.re[rb] = acc.re[rb] - t2[rb];
  }
}

// ---------------------------------------------------------------- stored (PF) matrices

template <typename T, int D>
__host__ __device__ constexpr int pf_index(int w, int plane, int reg, int lane) {
  constexpr int G = 16 / sizeof(T);
  return ((w * 2 + plane) * (D / 4 / G) + reg / G) * 64 * G + lane * G + reg % G;
}

// Offset of one row block of a d = 128 PF panel access.  It passes through an
// empty asm statement, so that each access's address is formed where the
// access is issued: otherwise the compiler precomputes the 64-bit addresses
// of all sixteen row blocks of a product, spills them, and every reload waits
// for all outstanding memory operations.
__device__ __forceinline__ int pf_site_offset(int off) {
  asm volatile("" : "+v"(off));
  return off;
}

// Row block rb of this wavefront's panel of a PF matrix, addressed at the
// access site (pf_site_offset).
template <typename T>
__device__ __forceinline__ void pf_rb_load(typename Prec<T>::v4& re, typename Prec<T>::v4& im, const T* M, int w,
                                           int rb, int lane) {
  constexpr int PLANE = pf_index<T, 128>(0, 1, 0, 0);  // offset of the imaginary plane
  const int off = pf_site_offset(pf_index<T, 128>(w, 0, 4 * rb, lane));
  if constexpr (sizeof(T) == 4) {
    re = *(const QOC_GLOBAL f4*)(M + off);
    im = *(const QOC_GLOBAL f4*)(M + off + PLANE);
  } else {
    constexpr int R2 = pf_index<T, 128>(0, 0, 2, 0);  // offset of registers 2 and 3
#pragma unroll
    for (int plane = 0; plane < 2; ++plane) {
      d2 a = *(const QOC_GLOBAL d2*)(M + off + plane * PLANE);
      d2 b = *(const QOC_GLOBAL d2*)(M + off + plane * PLANE + R2);
      d4 v;
      v.x = a.x; v.y = a.y; v.z = b.x; v.w = b.y;
      if (plane == 0) re = v; else im = v;
    }
  }
}

// Store row block rb of this wavefront's panel of a PF matrix (the layout of
// pf_rb_load).
template <typename T>
__device__ __forceinline__ void pf_rb_store(T* M, const typename Prec<T>::v4& re, const typename Prec<T>::v4& im,
                                            int w, int rb, int lane) {
  constexpr int PLANE = pf_index<T, 128>(0, 1, 0, 0);
  const int off = pf_site_offset(pf_index<T, 128>(w, 0, 4 * rb, lane));
  if constexpr (sizeof(T) == 4) {
    *(QOC_GLOBAL f4*)(M + off) = re;
    *(QOC_GLOBAL f4*)(M + off + PLANE) = im;
  } else {
    constexpr int R2 = pf_index<T, 128>(0, 0, 2, 0);
    *(QOC_GLOBAL d2*)(M + off) = d2{re.x, re.y};
    *(QOC_GLOBAL d2*)(M + off + R2) = d2{re.z, re.w};
    *(QOC_GLOBAL d2*)(M + off + PLANE) = d2{im.x, im.y};
    *(QOC_GLOBAL d2*)(M + off + PLANE + R2) = d2{im.z, im.w};
  }
}

template <typename T, int D>
__device__ __forceinline__ void panel_load(Panel<T, D>& P, const T* M, const Lane& L) {
  if constexpr (D == 128) {
#pragma unroll
    for (int rb = 0; rb < D / 16; ++rb) pf_rb_load<T>(P.re[rb], P.im[rb], M, L.w, rb, L.lane);
  } else if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int rb = 0; rb < D / 16; ++rb) {
      P.re[rb] = *(const QOC_GLOBAL f4*)(M + pf_index<T, D>(L.w, 0, 4 * rb, L.lane));
      P.im[rb] = *(const QOC_GLOBAL f4*)(M + pf_index<T, D>(L.w, 1, 4 * rb, L.lane));
    }
  } else {
#pragma unroll
    for (int rb = 0; rb < D / 16; ++rb) {
#pragma unroll
      for (int plane = 0; plane < 2; ++plane) {
        d2 a = *(const QOC_GLOBAL d2*)(M + pf_index<T, D>(L.w, plane, 4 * rb, L.lane));
        d2 b = *(const QOC_GLOBAL d2*)(M + pf_index<T, D>(L.w, plane, 4 * rb + 2, L.lane));
        d4 v;
        v.x = a.x; v.y = a.y; v.z = b.x; v.w = b.y;
        if (plane == 0) P.re[rb] = v; else P.im[rb] = v;
      }
    }
  }
}

template <typename T, int D>
__device__ __forceinline__ void panel_store(T* M, const Panel<T, D>& P, const Lane& L) {
  if constexpr (D == 128) {
#pragma unroll
    for (int rb = 0; rb < D / 16; ++rb) pf_rb_store<T>(M, P.re[rb], P.im[rb], L.w, rb, L.lane);
  } else if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int rb = 0; rb < D / 16; ++rb) {
      *(QOC_GLOBAL f4*)(M + pf_index<T, D>(L.w, 0, 4 * rb, L.lane)) = P.re[rb];
      *(QOC_GLOBAL f4*)(M + pf_index<T, D>(L.w, 1, 4 * rb, L.lane)) = P.im[rb];
    }
  } else {
#pragma unroll
    for (int rb = 0; rb < D / 16; ++rb) {
#pragma unroll
      for (int plane = 0; plane < 2; ++plane) {
        d4 v = plane == 0 ? P.re[rb] : P.im[rb];
        d2 a, b;
        a.x = v.x; a.y = v.y; b.x = v.z; b.y = v.w;
        *(QOC_GLOBAL d2*)(M + pf_index<T, D>(L.w, plane, 4 * rb, L.lane)) = a;
        *(QOC_GLOBAL d2*)(M + pf_index<T, D>(L.w, plane, 4 * rb + 2, L.lane)) = b;
      }
    }
  }
}

// ---------------------------------------------------------------- reductions

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sums each of V values of every lane over the wavefront in log2(V) halving
// exchanges plus 6 - log2(V) plain ones.  At the halving exchange with offset
// o a lane keeps the half of its values selected by (lane & o) and adds its
// partner's copy of that half.  Afterwards lane l holds the total of value
// l >> (6 - log2 V).
template <int V>
__device__ __forceinline__ double wave_sum_many(double (&v)[V], int lane) {
  static_assert(V >= 1 && V <= 64 && (V & (V - 1)) == 0, "V must be a power of two up to 64");
  constexpr int LOG = __builtin_ctz(V);
#pragma unroll
  for (int s = 0; s < LOG; ++s) {
    const int o = 32 >> s;
    const int H = V >> (s + 1);
    const bool up = (lane & o) != 0;
#pragma unroll
    for (int i = 0; i < H; ++i) {
      double lo = v[i], hi = v[i + H];
      // opaque to the optimiser: the selects below stay selects of values
      // (folded into one load through a selected address, they would keep
      // the array in scratch memory)
      asm volatile("" : "+v"(lo), "+v"(hi));
      const double keep = up ? hi : lo;
      const double give = up ? lo : hi;
      v[i] = keep + __shfl_xor(give, o, 64);
    }
  }
  double t = v[0];
#pragma unroll
  for (int o = 32 >> LOG; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
  return t;
}

// The same over the G consecutive lanes of each aligned lane group
// (V <= G <= 64, both powers of two): afterwards lane l holds its group's
// total of value (l % G) / (G / V).
template <int V, int G>
__device__ __forceinline__ double group_sum_many(double (&v)[V], int lane) {
  static_assert(V >= 1 && V <= G && G <= 64 && (V & (V - 1)) == 0 && (G & (G - 1)) == 0, "powers of two");
  constexpr int LOG = __builtin_ctz(V);
#pragma unroll
  for (int s = 0; s < LOG; ++s) {
    const int o = (G / 2) >> s;
    const int H = V >> (s + 1);
    const bool up = (lane & o) != 0;
#pragma unroll
    for (int i = 0; i < H; ++i) {
      double lo = v[i], hi = v[i + H];
      // opaque to the optimiser: the selects below stay selects of values
      // (folded into one load through a selected address, they would keep
      // the array in scratch memory)
      asm volatile("" : "+v"(lo), "+v"(hi));
      const double keep = up ? hi : lo;
      const double give = up ? lo : hi;
      v[i] = keep + __shfl_xor(give, o, 64);
    }
  }
  double t = v[0];
#pragma unroll
  for (int o = (G / 2) >> LOG; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
  return t;
}

}  // namespace qoc

namespace qoc {

// LDS policy of the FP64 / FP32 products: planar matrices of T as above.
// Kernels that stage left factors in LDS go through one of these policies,
// so that the split-BF16 products can use their own LDS format.
template <typename T, int D>
struct StdOps {
  using Tp = T;
  static constexpr int BYTES = Mat<T, D>::LDS_ELEMS * (int)sizeof(T);
  __device__ static __forceinline__ void put(void* lds, int row, int col, T re, T im) {
    T* p = static_cast<T*>(lds);
    const int off = lds_off<T, D>(row, col);
    p[off] = re;
    p[D * Mat<T, D>::SD + off] = im;
  }
  // Four consecutive columns col..col+3 of one row (col a multiple of 4).
  __device__ static __forceinline__ void put4(void* lds, int row, int col, typename Prec<T>::v4 re,
                                              typename Prec<T>::v4 im) {
    T* p = static_cast<T*>(lds);
    if constexpr (sizeof(T) == 4) {
      const int off = lds_off<T, D>(row, col);
      Prec<T>::st4(p + off, re);
      Prec<T>::st4(p + D * Mat<T, D>::SD + off, im);
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) put(lds, row, col + i, re[i], im[i]);
    }
  }
  __device__ static __forceinline__ void store(void* lds, const Panel<T, D>& P, const Lane& L) {
    panel_to_lds(static_cast<T*>(lds), P, L);
  }
  __device__ static __forceinline__ void store_ct(void* lds, const Panel<T, D>& P, const Lane& L) {
    panel_to_lds_ct(static_cast<T*>(lds), P, L);
  }
  __device__ static __forceinline__ void load(Panel<T, D>& P, const void* lds, const Lane& L) {
    panel_from_lds(P, static_cast<const T*>(lds), L);
  }
  __device__ static __forceinline__ void load_ct(Panel<T, D>& P, const void* lds, const Lane& L) {
    panel_from_lds_ct(P, static_cast<const T*>(lds), L);
  }
  __device__ static __forceinline__ void gemm(Panel<T, D>& acc, const void* lds, const Panel<T, D>& P, const Lane& L,
                                              bool zero_acc) {
    cgemm(acc, static_cast<const T*>(lds), P, L, zero_acc);
  }
  // The same product in the three-product form where it pays (D >= 32; at
  // D = 16 the extra registers cost more occupancy than the saved MFMAs).
  template <int PAIRS = 1>
  __device__ static __forceinline__ void gemm3(Panel<T, D>& acc, const void* lds, const Panel<T, D>& P,
                                               const Lane& L, bool zero_acc) {
    if constexpr (D >= 32) cgemm3m<T, D, PAIRS>(acc, static_cast<const T*>(lds), P, L, zero_acc);
    else cgemm(acc, static_cast<const T*>(lds), P, L, zero_acc);
  }
};

}  // namespace qoc
