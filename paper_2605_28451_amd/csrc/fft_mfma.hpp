// Radix-16 Stockham passes on the gfx950 matrix cores (v_mfma_f32_16x16x32_f16)
// for N = 4096 = 16^3: FP16 operands, FP32 accumulation.
//
// A radix-16 butterfly is the dense product Y = F16 x (16 complex inputs ->
// 16 complex outputs).  Over the reals with interleaved (re, im) components,
// 16 butterflies form one 32 x 16 FP16 operand B (K = 32 real inputs, one
// column per butterfly), and the DFT matrix splits into two 16 x 32 FP16
// operands A_lo / A_hi (rows: real and imaginary parts of 8 outputs each).
// Per wavefront and pass: 4 groups of 16 butterflies x 2 MFMAs.
//
// Lane layout of v_mfma_f32_16x16x32_f16 (lane l, c = l % 16, g = l / 16):
//   A: A[c][8g + k'], B: B[8g + k'][c], D: D[4g + k''][c]  (k' < 8, k'' < 4).
// With K ordered as k = 2r + (re, im) of input r, lane (c, g) supplies inputs
// r = 4g..4g+3 of butterfly c as four packed FP16 pairs.  A_lo holds outputs
// {0,1,4,5,8,9,12,13} and A_hi {2,3,6,7,10,11,14,15}, so lane (c, g) receives
// outputs q = 4g..4g+3: the slots of its inputs, which lets one transform hand
// its last pass to the next transform's first pass in registers.
//
// Thread t = 64 w + l of a 256-thread workgroup owns, for m, i = 0..3,
// butterfly j = 64 w + 16 m + c and slot r = 4 g + i: element position
// j + 256 r at the input and output of every pass.  The Stockham scatter
// between passes goes through LDS with the address swizzle
//   p -> p ^ b67 ^ (b67 << 4) ^ (b1011 << 4),  b67 = p[7:6], b1011 = p[11:10],
// which is conflict-free on 64 banks for every access below (checked by
// simulation); each access resolves to four per-lane base registers plus
// compile-time offsets.
//
// The operand slices and the dot-product-form twiddles come from a host
// table built in FP64 and rounded once (see mfma4096_table).
#pragma once

#include "fft_device.hpp"

namespace bfp {

typedef f16 half8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

struct Mfma4096 {
  static constexpr int N = 4096;
  static constexpr int TW_OFFSET_HALVES = 1024;  // twiddles follow the operand slices

  half8 alo, ahi;              // DFT16 operand slices of this lane
  const uint4 *tw;             // dot2-form twiddles, 8 bytes per entry
  int w, c, g;

  __device__ __forceinline__ Mfma4096(const void *table, int tid) {
    const int lane = tid & 63;
    w = tid >> 6;
    c = lane & 15;
    g = lane >> 4;
    const uint4 *a = reinterpret_cast<const uint4 *>(static_cast<const uint16_t *>(table) + 16 * lane);
    const uint4 lo = a[0], hi = a[1];
    alo = __builtin_bit_cast(half8, lo);
    ahi = __builtin_bit_cast(half8, hi);
    tw = reinterpret_cast<const uint4 *>(static_cast<const uint16_t *>(table) + TW_OFFSET_HALVES);
  }

  // element position of slot (m, i)
  __device__ __forceinline__ unsigned pos(int m, int i) const {
    return (unsigned)(64 * w + 16 * m + c + 256 * (4 * g + i));
  }

  // 64 butterflies: x[4m + i] (FP16) -> y[4m + i] (FP32)
  __device__ __forceinline__ void dft(const h2 (&x)[16], c32 (&y)[16]) const {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      half8 b;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        b[2 * i] = x[4 * m + i].x;
        b[2 * i + 1] = x[4 * m + i].y;
      }
      const f4 z = {0.0f, 0.0f, 0.0f, 0.0f};
      const f4 dlo = __builtin_amdgcn_mfma_f32_16x16x32_f16(alo, b, z, 0, 0, 0);
      const f4 dhi = __builtin_amdgcn_mfma_f32_16x16x32_f16(ahi, b, z, 0, 0, 0);
      y[4 * m + 0] = c32{dlo[0], dlo[1]};
      y[4 * m + 1] = c32{dlo[2], dlo[3]};
      y[4 * m + 2] = c32{dhi[0], dhi[1]};
      y[4 * m + 3] = c32{dhi[2], dhi[3]};
    }
  }

  // Outputs of the pass of span 1 to LDS: position 16 j + q.
  __device__ __forceinline__ void scatter1(const c32 (&y)[16], h2 *lds) const {
    const int c2 = c >> 2;
    const int base = 1024 * w + 64 * c2 + 16 * ((c & 3) ^ c2 ^ w) + 4 * g;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      h2 *p = lds + base + (i ^ c2);
#pragma unroll
      for (int m = 0; m < 4; ++m) p[256 * m] = c32_to_h2(y[4 * m + i]);
    }
  }

  // Outputs of the pass of span 16 to LDS: position 256 (j/16) + j%16 + 16 q.
  __device__ __forceinline__ void scatter16(const c32 (&y)[16], h2 *lds) const {
    const int s = g ^ w;
    const int base = 1024 * w + 64 * g + ((c & 3) ^ g) + 4 * (c >> 2);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      h2 *p = lds + base + 16 * (i ^ s);
#pragma unroll
      for (int m = 0; m < 4; ++m) p[256 * m] = c32_to_h2(y[4 * m + i]);
    }
  }

  // Inputs of the pass of span NS (16 or 256) from LDS, times the twiddles
  // W_{16 NS}^{(j mod NS) r} with FP16 operands and FP32 accumulation.
  template <int NS, int TW_ROW0>
  __device__ __forceinline__ void gather(h2 (&x)[16], const h2 *lds) const {
    const int s = w ^ g;
    const int base = 64 * w + 1024 * g + (c ^ w);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int j = 64 * w + 16 * m + c;
      const uint4 *tp = tw + (TW_ROW0 + (j & (NS - 1)) * 16 + 4 * g) / 2;  // 2 entries per uint4
      const uint4 t01 = tp[0], t23 = tp[1];
      h2 wt[8];
      __builtin_memcpy(&wt[0], &t01, 16);
      __builtin_memcpy(&wt[4], &t23, 16);
      const h2 *p = lds + base + 16 * (m ^ s);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const h2 v = p[256 * i];
        const float re = __builtin_amdgcn_fdot2(v, wt[2 * i], 0.0f, false);
        const float im = __builtin_amdgcn_fdot2(v, wt[2 * i + 1], 0.0f, false);
        x[4 * m + i] = h2{(f16)re, (f16)im};
      }
    }
  }

  // The transform: x = inputs at pos(m, i) (FP16) -> y = outputs X[pos(m, i)]
  // (FP32).  lds: 4096 FP16 pairs per workgroup.
  __device__ __forceinline__ void run(h2 (&x)[16], c32 (&y)[16], h2 *lds) const {
    dft(x, y);  // span 1: no twiddles
    __syncthreads();
    scatter1(y, lds);
    __syncthreads();
    gather<16, 0>(x, lds);
    dft(x, y);
    __syncthreads();
    scatter16(y, lds);
    __syncthreads();
    gather<256, 256>(x, lds);
    dft(x, y);
  }
};

}  // namespace bfp
