// Split-BF16 ("BF16x3") complex products on the 16x16x32 BF16 MFMA with FP32
// accumulation (Henry, Tang and Heinecke, ARITH 2019).
//
// Every FP32 value x is split into hi = bf16(x) and lo = bf16(x - hi)
// (round to nearest even; x - hi is exact in FP32), and a real product is
// taken as A_hi B_hi + A_hi B_lo + A_lo B_hi, dropping A_lo B_lo (relative
// size about 2^-16).  A complex product is taken as four real ones (the
// three-product form would need BF16 splits of Ar + Ai as well), so one
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
typedef unsigned u2v __attribute__((ext_vector_type(2)));
typedef unsigned u4v __attribute__((ext_vector_type(4)));

typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));

// Split two FP32 values at once: hi = bf16(x) with round to nearest even
// (one v_cvt_pk_bf16_f32 on gfx950), lo = bf16(x - hi).  Element 0 sits in
// the low 16 bits of the packed results.
__device__ __forceinline__ void bf16_split2(float x0, float x1, unsigned& hi, unsigned& lo) {
  const f2v v = {x0, x1};
  hi = __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2v));
  const f2v r = {x0 - __uint_as_float(hi << 16), x1 - __uint_as_float(hi & 0xffff0000u)};
  lo = __builtin_bit_cast(unsigned, __builtin_convertvector(r, bf16x2v));
}

__device__ __forceinline__ void bf16_split(float x, unsigned& hi, unsigned& lo) {
  unsigned h, l;
  bf16_split2(x, 0.0f, h, l);
  hi = h & 0xffffu;
  lo = l & 0xffffu;
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

  // Four consecutive columns col..col+3 of one row (col a multiple of 4):
  // contiguous after phys(), one 8-byte write per plane.
  __device__ static __forceinline__ void put4(void* lds, int row, int col, f4 re, f4 im) {
    const int off = row * SB + phys(col);
    u2v rh, rl, ih, il;
    unsigned h, l;
    bf16_split2(re[0], re[1], h, l);
    rh[0] = h;
    rl[0] = l;
    bf16_split2(re[2], re[3], h, l);
    rh[1] = h;
    rl[1] = l;
    bf16_split2(im[0], im[1], h, l);
    ih[0] = h;
    il[0] = l;
    bf16_split2(im[2], im[3], h, l);
    ih[1] = h;
    il[1] = l;
    *reinterpret_cast<u2v*>(plane(lds, 0) + off) = rh;
    *reinterpret_cast<u2v*>(plane(lds, 1) + off) = rl;
    *reinterpret_cast<u2v*>(plane(lds, 2) + off) = ih;
    *reinterpret_cast<u2v*>(plane(lds, 3) + off) = il;
  }

  __device__ static __forceinline__ void store(void* lds, const Panel<float, D>& P, const Lane& L) {
    const int pc = phys(16 * L.w + L.c16);
#pragma unroll
    for (int rb = 0; rb < D / 16; ++rb)
#pragma unroll
      for (int r = 0; r < 4; r += 2) {
        unsigned rh, rl, ih, il;
        bf16_split2(P.re[rb][r], P.re[rb][r + 1], rh, rl);
        bf16_split2(P.im[rb][r], P.im[rb][r + 1], ih, il);
        const int o0 = (16 * rb + 4 * L.g + r) * SB + pc, o1 = o0 + SB;
        plane(lds, 0)[o0] = (unsigned short)rh;
        plane(lds, 0)[o1] = (unsigned short)(rh >> 16);
        plane(lds, 1)[o0] = (unsigned short)rl;
        plane(lds, 1)[o1] = (unsigned short)(rl >> 16);
        plane(lds, 2)[o0] = (unsigned short)ih;
        plane(lds, 2)[o1] = (unsigned short)(ih >> 16);
        plane(lds, 3)[o0] = (unsigned short)il;
        plane(lds, 3)[o1] = (unsigned short)(il >> 16);
      }
  }

  // Conjugate transpose: M^dag[16w + c16][16 rb + 4g + r]; the four r are
  // contiguous after phys(), so each plane takes one 8-byte write.
  __device__ static __forceinline__ void store_ct(void* lds, const Panel<float, D>& P, const Lane& L) {
#pragma unroll
    for (int rb = 0; rb < D / 16; ++rb) {
      const int off = (16 * L.w + L.c16) * SB + phys(16 * rb + 4 * L.g);
      u2v rh, rl, ih, il;
#pragma unroll
      for (int r = 0; r < 4; r += 2) {
        unsigned h, l;
        bf16_split2(P.re[rb][r], P.re[rb][r + 1], h, l);
        rh[r / 2] = h;
        rl[r / 2] = l;
        bf16_split2(-P.im[rb][r], -P.im[rb][r + 1], h, l);
        ih[r / 2] = h;
        il[r / 2] = l;
      }
      *reinterpret_cast<u2v*>(plane(lds, 0) + off) = rh;
      *reinterpret_cast<u2v*>(plane(lds, 1) + off) = rl;
      *reinterpret_cast<u2v*>(plane(lds, 2) + off) = ih;
      *reinterpret_cast<u2v*>(plane(lds, 3) + off) = il;
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

  __device__ static __forceinline__ void gemm3(Panel<float, D>& acc, const void* lds, const Panel<float, D>& P,
                                               const Lane& L, bool zero_acc) {
    gemm(acc, lds, P, L, zero_acc);
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
      u4v rh, rl, ih, il, nh, nl;
#pragma unroll
      for (int jp = 0; jp < 4; ++jp) {
        const int rb = 2 * t + (jp >> 1), r = 2 * (jp & 1);
        unsigned h, l;
        bf16_split2(P.re[rb][r], P.re[rb][r + 1], h, l);
        rh[jp] = h;
        rl[jp] = l;
        bf16_split2(P.im[rb][r], P.im[rb][r + 1], h, l);
        ih[jp] = h;
        il[jp] = l;
        nh[jp] = h ^ 0x80008000u;
        nl[jp] = l ^ 0x80008000u;
      }
      const s8v brh = __builtin_bit_cast(s8v, rh), brl = __builtin_bit_cast(s8v, rl);
      const s8v bih = __builtin_bit_cast(s8v, ih), bil = __builtin_bit_cast(s8v, il);
      const s8v nih = __builtin_bit_cast(s8v, nh), nil = __builtin_bit_cast(s8v, nl);
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
