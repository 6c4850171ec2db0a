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
// compile-time offsets.  Two LDS buffers alternate between the exchanges, so
// one barrier per exchange orders every write after the reads of the
// buffer's previous contents.
//
// Twiddles W_{16 NS}^{(j mod NS) r} are applied to the FP16 inputs of the
// passes of span 16 and 256 as two v_dot2_f32_f16 per element (FP16 products,
// FP32 sum) and rounded once to FP16.  The span-16 rows depend only on
// (c, g), so each lane keeps its four for the whole kernel; the span-256
// rows are fetched one pass ahead.
//
// Block-floating-point shift of the inverse (Eq. (1)): the first pass of a
// BFP inverse uses S = F16 . 2^-12 instead of F16.  Every entry of F16 is 0
// or has magnitude >= sin(pi/8), so S is exact in FP16, and because the FP16
// x FP16 products are exact in FP32, the pass computes exactly
// 2^-12 (F16 x) with FP32 accumulation: the shift costs no instruction and
// no extra rounding.
//
// The operand slices and the twiddles come from a host table built in FP64
// and rounded once (mfma4096_table).
#pragma once

#include "fft_device.hpp"

namespace bfp {

typedef f16 half8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Table layout in FP16 units (see mfma4096_table): F16 slices (64 lanes x
// 16), S slices (64 x 16), span-16 twiddles (256 entries x 4), span-256
// twiddles (4096 entries x 4); a twiddle entry is the pair of dot-product
// operands (Re w, -Im w), (Im w, Re w).
constexpr int kMfmaTwOffsetHalves = 2048;
constexpr int kMfmaTw256OffsetHalves = kMfmaTwOffsetHalves + 4 * 256;

// Twiddles of one pass for one lane: slot i of group m in t[2 m + i / 2]
// (two entries per 16 bytes).
struct MfmaTw {
  uint4 t[8];
};

struct Mfma4096 {
  static constexpr int N = 4096;

  half8 alo, ahi;  // F16 operand slices of this lane
  half8 slo, shi;  // F16 . 2^-12
  uint4 tw16[2];   // span-16 twiddles of this lane (slots 0..3)
  const uint4 *tw256;
  int w, c, g;

  __device__ __forceinline__ Mfma4096(const void *table, int tid) {
    const int lane = tid & 63;
    w = tid >> 6;
    c = lane & 15;
    g = lane >> 4;
    const uint16_t *tab = static_cast<const uint16_t *>(table);
    const uint4 *a = reinterpret_cast<const uint4 *>(tab + 16 * lane);
    const uint4 *s = reinterpret_cast<const uint4 *>(tab + 1024 + 16 * lane);
    alo = __builtin_bit_cast(half8, a[0]);
    ahi = __builtin_bit_cast(half8, a[1]);
    slo = __builtin_bit_cast(half8, s[0]);
    shi = __builtin_bit_cast(half8, s[1]);
    // span 16: row j mod 16 = c for every group, entries r = 4g..4g+3
    const uint4 *t16 = reinterpret_cast<const uint4 *>(tab + kMfmaTwOffsetHalves) + (c * 16 + 4 * g) / 2;
    tw16[0] = t16[0];
    tw16[1] = t16[1];
    tw256 = reinterpret_cast<const uint4 *>(tab + kMfmaTw256OffsetHalves);
  }

  // element position of slot (m, i)
  __device__ __forceinline__ unsigned pos(int m, int i) const {
    return (unsigned)(64 * w + 16 * m + c + 256 * (4 * g + i));
  }

  // Twiddles of the pass of span 256: row j = 64 w + 16 m + c, entries r = 4g..4g+3.
  __device__ __forceinline__ void load_tw256(MfmaTw &t) const {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const uint4 *p = tw256 + ((64 * w + 16 * m + c) * 16 + 4 * g) / 2;
      t.t[2 * m] = p[0];
      t.t[2 * m + 1] = p[1];
    }
  }

  // 64 butterflies: x[4m + i] (FP16) -> y[4m + i] (FP32); SCALED selects S.
  template <bool SCALED>
  __device__ __forceinline__ void dft(const h2 (&x)[16], c32 (&y)[16]) const {
    const half8 lo = SCALED ? slo : alo;
    const half8 hi = SCALED ? shi : ahi;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      half8 b;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        b[2 * i] = x[4 * m + i].x;
        b[2 * i + 1] = x[4 * m + i].y;
      }
      const f4 z = {0.0f, 0.0f, 0.0f, 0.0f};
      const f4 dlo = __builtin_amdgcn_mfma_f32_16x16x32_f16(lo, b, z, 0, 0, 0);
      const f4 dhi = __builtin_amdgcn_mfma_f32_16x16x32_f16(hi, b, z, 0, 0, 0);
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

  // v . w as FP16 products with an FP32 sum, rounded once to FP16; tw holds
  // the two dot-product forms of w.
  static __device__ __forceinline__ h2 twiddle(h2 v, uint2 tw) {
    const h2 w0 = __builtin_bit_cast(h2, tw.x), w1 = __builtin_bit_cast(h2, tw.y);
    return c32_to_h2(c32{__builtin_amdgcn_fdot2(v, w0, 0.0f, false),
                         __builtin_amdgcn_fdot2(v, w1, 0.0f, false)});
  }

  // Inputs of the pass of span 16 from LDS, times W_256^{(j mod 16) r}.
  __device__ __forceinline__ void gather16(h2 (&x)[16], const h2 *lds) const {
    const int s = w ^ g;
    const int base = 64 * w + 1024 * g + (c ^ w);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const h2 *p = lds + base + 16 * (m ^ s);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint4 t = tw16[i >> 1];
        x[4 * m + i] = twiddle(p[256 * i], (i & 1) ? uint2{t.z, t.w} : uint2{t.x, t.y});
      }
    }
  }

  // Inputs of the pass of span 256 from LDS, times W_4096^{j r}.
  __device__ __forceinline__ void gather256(h2 (&x)[16], const h2 *lds, const MfmaTw &tw) const {
    const int s = w ^ g;
    const int base = 64 * w + 1024 * g + (c ^ w);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const h2 *p = lds + base + 16 * (m ^ s);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint4 t = tw.t[2 * m + (i >> 1)];
        x[4 * m + i] = twiddle(p[256 * i], (i & 1) ? uint2{t.z, t.w} : uint2{t.x, t.y});
      }
    }
  }

  // The transform: x = inputs at pos(m, i) (FP16) -> y = outputs X[pos(m, i)]
  // (FP32), scaled by 2^-12 when SCALED.  lds0, lds1: 4096 FP16 pairs each.
  template <bool SCALED>
  __device__ __forceinline__ void run(h2 (&x)[16], c32 (&y)[16], h2 *lds0, h2 *lds1) const {
    MfmaTw t;
    load_tw256(t);  // in flight during the first two passes
    dft<SCALED>(x, y);
    scatter1(y, lds0);
    __syncthreads();
    gather16(x, lds0);
    dft<false>(x, y);
    scatter16(y, lds1);
    __syncthreads();
    gather256(x, lds1, t);
    dft<false>(x, y);
  }
};

}  // namespace bfp
