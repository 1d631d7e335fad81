// Split-BF16 ("BF16x3") complex products on the 16x16x32 BF16 MFMA with FP32
// accumulation (Henry, Tang and Heinecke, ARITH 2019).
//
// Every FP32 value x is split into hi = bf16(x) and lo = bf16(x - hi)
// (round to nearest even; x - hi is exact in FP32), and a real product is
// taken as A_hi B_hi + A_hi B_lo + A_lo B_hi, dropping A_lo B_lo (relative
// size about 2^-16).  A complex product is four real ones, so one
// (k step, row block) step issues 12 MFMAs, each of K = 32.
//
// Register panels stay FP32 in the accumulator layout (rows 16 rb + 4g + r).
// For K step t the B operand of lane (g, c16) is the 8 values of row blocks
// 2t and 2t+1 it holds: K index 8g + j stands for matrix row
// 32t + 16 (j / 4) + 4g + (j % 4).  The left factor is staged in LDS as four
// BF16 planes (re hi, re lo, im hi, im lo), row stride D + 8, with the columns
// of each 32-column block permuted by phys() so that those 8 K values of a
// row are contiguous: one 16-byte read per plane and step.
#pragma once

#include "qoc_device.hpp"

namespace qoc {

typedef short s8v __attribute__((ext_vector_type(8)));
typedef short s4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned bf16_rne(float x) {
  const unsigned u = __float_as_uint(x);
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

__device__ __forceinline__ void bf16_split(float x, unsigned& hi, unsigned& lo) {
  hi = bf16_rne(x);
  lo = bf16_rne(x - __uint_as_float(hi << 16));
}

__device__ __forceinline__ float bf16_join(unsigned short hi, unsigned short lo) {
  return __uint_as_float((unsigned)hi << 16) + __uint_as_float((unsigned)lo << 16);
}

template <int D>
struct Bf3Ops {
  using Tp = float;
  static constexpr int SB = D + 8;          // row stride in BF16 elements
  static constexpr int PLANE = D * SB;      // elements per plane
  static constexpr int BYTES = 4 * PLANE * 2;
  static_assert(D % 32 == 0, "split-BF16 products need D to be a multiple of 32");

  __device__ static __forceinline__ int phys(int c) {
    const int c32 = c & 31;
    return (c & ~31) + 8 * ((c32 & 15) >> 2) + 4 * (c32 >> 4) + (c32 & 3);
  }
  __device__ static __forceinline__ unsigned short* plane(void* lds, int i) {
    return static_cast<unsigned short*>(lds) + i * PLANE;
  }
  __device__ static __forceinline__ const unsigned short* plane(const void* lds, int i) {
    return static_cast<const unsigned short*>(lds) + i * PLANE;
  }

  __device__ static __forceinline__ void put(void* lds, int row, int col, float re, float im) {
    const int off = row * SB + phys(col);
    unsigned h, l;
    bf16_split(re, h, l);
    plane(lds, 0)[off] = (unsigned short)h;
    plane(lds, 1)[off] = (unsigned short)l;
    bf16_split(im, h, l);
    plane(lds, 2)[off] = (unsigned short)h;
    plane(lds, 3)[off] = (unsigned short)l;
  }

  __device__ static __forceinline__ void store(void* lds, const Panel<float, D>& P, const Lane& L) {
#pragma unroll
    for (int rb = 0; rb < D / 16; ++rb)
#pragma unroll
      for (int r = 0; r < 4; ++r) put(lds, 16 * rb + 4 * L.g + r, 16 * L.w + L.c16, P.re[rb][r], P.im[rb][r]);
  }

  // Conjugate transpose: M^dag[16w + c16][16 rb + 4g + r]; the four r are
  // contiguous after phys(), so each plane takes one 8-byte write.
  __device__ static __forceinline__ void store_ct(void* lds, const Panel<float, D>& P, const Lane& L) {
#pragma unroll
    for (int rb = 0; rb < D / 16; ++rb) {
      const int off = (16 * L.w + L.c16) * SB + phys(16 * rb + 4 * L.g);
      s4v rh, rl, ih, il;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        unsigned h, l;
        bf16_split(P.re[rb][r], h, l);
        rh[r] = (short)h;
        rl[r] = (short)l;
        bf16_split(-P.im[rb][r], h, l);
        ih[r] = (short)h;
        il[r] = (short)l;
      }
      *reinterpret_cast<s4v*>(plane(lds, 0) + off) = rh;
      *reinterpret_cast<s4v*>(plane(lds, 1) + off) = rl;
      *reinterpret_cast<s4v*>(plane(lds, 2) + off) = ih;
      *reinterpret_cast<s4v*>(plane(lds, 3) + off) = il;
    }
  }

  __device__ static __forceinline__ void load(Panel<float, D>& P, const void* lds, const Lane& L) {
#pragma unroll
    for (int rb = 0; rb < D / 16; ++rb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int off = (16 * rb + 4 * L.g + r) * SB + phys(16 * L.w + L.c16);
        P.re[rb][r] = bf16_join(plane(lds, 0)[off], plane(lds, 1)[off]);
        P.im[rb][r] = bf16_join(plane(lds, 2)[off], plane(lds, 3)[off]);
      }
  }

  __device__ static __forceinline__ void load_ct(Panel<float, D>& P, const void* lds, const Lane& L) {
#pragma unroll
    for (int rb = 0; rb < D / 16; ++rb) {
      const int off = (16 * L.w + L.c16) * SB + phys(16 * rb + 4 * L.g);
      const s4v rh = *reinterpret_cast<const s4v*>(plane(lds, 0) + off);
      const s4v rl = *reinterpret_cast<const s4v*>(plane(lds, 1) + off);
      const s4v ih = *reinterpret_cast<const s4v*>(plane(lds, 2) + off);
      const s4v il = *reinterpret_cast<const s4v*>(plane(lds, 3) + off);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        P.re[rb][r] = bf16_join(rh[r], rl[r]);
        P.im[rb][r] = -bf16_join(ih[r], il[r]);
      }
    }
  }

  __device__ static __forceinline__ f4 mfma(s8v a, s8v b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }

  // acc (+)= A P with A the LDS matrix: per K step t the panel's 8 values are
  // split once; per row block 4 x 16-byte reads and 12 MFMAs.
  __device__ static __forceinline__ void gemm(Panel<float, D>& acc, const void* lds, const Panel<float, D>& P,
                                              const Lane& L, bool zero_acc) {
    constexpr int RB = D / 16;
    constexpr int KT = D / 32;
    __builtin_amdgcn_sched_barrier(0);
    if (zero_acc) panel_zero(acc);
    const int base = L.c16 * SB + 8 * L.g;
#pragma unroll
    for (int t = 0; t < KT; ++t) {
      s8v brh, brl, bih, bil, nih, nil;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const float xr = j < 4 ? P.re[2 * t][j] : P.re[2 * t + 1][j - 4];
        const float xi = j < 4 ? P.im[2 * t][j] : P.im[2 * t + 1][j - 4];
        unsigned h, l;
        bf16_split(xr, h, l);
        brh[j] = (short)h;
        brl[j] = (short)l;
        bf16_split(xi, h, l);
        bih[j] = (short)h;
        bil[j] = (short)l;
        nih[j] = (short)(h ^ 0x8000u);
        nil[j] = (short)(l ^ 0x8000u);
      }
      s8v a[2][4];
      {
        const int off = base + 32 * t;
#pragma unroll
        for (int pl = 0; pl < 4; ++pl) a[0][pl] = *reinterpret_cast<const s8v*>(plane(lds, pl) + off);
      }
#pragma unroll
      for (int mb = 0; mb < RB; ++mb) {
        const int cur = mb & 1;
        if (mb + 1 < RB) {
          const int off = base + 16 * (mb + 1) * SB + 32 * t;
#pragma unroll
          for (int pl = 0; pl < 4; ++pl) a[cur ^ 1][pl] = *reinterpret_cast<const s8v*>(plane(lds, pl) + off);
        }
        const s8v arh = a[cur][0], arl = a[cur][1], aih = a[cur][2], ail = a[cur][3];
        f4 re = acc.re[mb], im = acc.im[mb];
        re = mfma(arh, brh, re);
        im = mfma(arh, bih, im);
        re = mfma(arh, brl, re);
        im = mfma(arh, bil, im);
        re = mfma(arl, brh, re);
        im = mfma(arl, bih, im);
        re = mfma(aih, nih, re);
        im = mfma(aih, brh, im);
        re = mfma(aih, nil, re);
        im = mfma(aih, brl, im);
        re = mfma(ail, nih, re);
        im = mfma(ail, brh, im);
        acc.re[mb] = re;
        acc.im[mb] = im;
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
};

}  // namespace qoc
