// Device building blocks of the gfx950 FFT: complex arithmetic in FP32 and
// packed FP16, constant-twiddle radix-2/4/8/16 DFTs, storage conversions
// (FP32, FP16, OCP FP8 E4M3/E5M2) and the precision-mode policies.
//
// Everything here is device code compiled for gfx950 only.  No twiddle or
// filter table is evaluated on the device: twiddles come from host-built FP64
// tables rounded once (the paper, Sec. III-A, ties the poor "42 dB" FP16
// folklore to recurrence-built tables), and the few radix constants below are
// exact decimal expansions rounded by the compiler.  The only device
// trigonometry is per row or per pulse, outside the transforms: the autofocus
// phasor exp(i phi_m) (FP64 sincos, sar.hip) and the three migration phasors
// per row of the RCMC compression (FP32 sincospif, rows.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bfp {

typedef _Float16 f16;
typedef f16 h2 __attribute__((ext_vector_type(2)));  // (re, im) in one VGPR

struct __attribute__((aligned(8))) c32 {
  float x, y;
};

// ------------------------------------------------------------ FP32 ops ---
// Contraction is off in these helpers and the complex products use explicit
// FMAs: with the compiler free to fuse a product into whichever neighbouring
// add it finds, two kernels doing the same arithmetic on the same data
// (one row or two rows per thread, a fused or a separate pass) could round
// differently.  Written out, every kernel gets the same bits.
#define BFP_NO_CONTRACT _Pragma("clang fp contract(off)")
__device__ __forceinline__ c32 mk(float x, float y) { return c32{x, y}; }
__device__ __forceinline__ c32 cadd(c32 a, c32 b) { return c32{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ c32 csub(c32 a, c32 b) { return c32{a.x - b.x, a.y - b.y}; }
// a - i b and a + i b
__device__ __forceinline__ c32 csub_i(c32 a, c32 b) { return c32{a.x + b.y, a.y - b.x}; }
__device__ __forceinline__ c32 cadd_i(c32 a, c32 b) { return c32{a.x - b.y, a.y + b.x}; }
__device__ __forceinline__ c32 cmul(c32 a, c32 b) {
  BFP_NO_CONTRACT
  return c32{__builtin_fmaf(a.x, b.x, -(a.y * b.y)), __builtin_fmaf(a.x, b.y, a.y * b.x)};
}
__device__ __forceinline__ c32 cscale(c32 a, float s) {
  BFP_NO_CONTRACT
  return c32{a.x * s, a.y * s};
}
__device__ __forceinline__ c32 cconj(c32 a) { return c32{a.x, -a.y}; }
__device__ __forceinline__ c32 mul_mi(c32 a) { return c32{a.y, -a.x}; }   // x (-i)
__device__ __forceinline__ c32 mul_pi(c32 a) { return c32{-a.y, a.x}; }   // x (+i)
__device__ __forceinline__ c32 cneg(c32 a) { return c32{-a.x, -a.y}; }
// x (c + i s) with compile-time constants
__device__ __forceinline__ c32 cmulk(c32 a, float c, float s) {
  BFP_NO_CONTRACT
  return c32{__builtin_fmaf(a.x, c, -(a.y * s)), __builtin_fmaf(a.x, s, a.y * c)};
}
// x k (1 - i), x k (-1 - i), x k (-1 + i), x k (1 + i)
__device__ __forceinline__ c32 mul_1mi(c32 a, float k) {
  BFP_NO_CONTRACT
  return c32{(a.x + a.y) * k, (a.y - a.x) * k};
}
__device__ __forceinline__ c32 mul_m1mi(c32 a, float k) {
  BFP_NO_CONTRACT
  return c32{(a.y - a.x) * k, -(a.x + a.y) * k};
}
__device__ __forceinline__ c32 mul_m1pi(c32 a, float k) {
  BFP_NO_CONTRACT
  return c32{-(a.x + a.y) * k, (a.x - a.y) * k};
}
__device__ __forceinline__ c32 mul_1pi(c32 a, float k) {
  BFP_NO_CONTRACT
  return c32{(a.x - a.y) * k, (a.x + a.y) * k};
}

// ----------------------------------------------------- packed FP16 ops ---
__device__ __forceinline__ h2 cadd(h2 a, h2 b) { return a + b; }
__device__ __forceinline__ h2 csub(h2 a, h2 b) { return a - b; }
__device__ __forceinline__ h2 csub_i(h2 a, h2 b) { return a + h2{b.y, -b.x}; }
__device__ __forceinline__ h2 cadd_i(h2 a, h2 b) { return a + h2{-b.y, b.x}; }
__device__ __forceinline__ h2 cmul(h2 a, h2 b) {
  // a b = b.y (-ay, ax) + b.x (ax, ay): both products take b's halves as
  // broadcasts and a's as a swizzle, all source modifiers of the packed
  // instructions.  The swizzled product comes first: with register-held
  // twiddles the compiler then needs no wait state between the two
  // instructions (the other order costs one per product)
  const h2 t = h2{-a.y, a.x} * h2{b.y, b.y};
  return __builtin_elementwise_fma(a, h2{b.x, b.x}, t);
}
__device__ __forceinline__ h2 cscale(h2 a, float s) { return a * h2{(f16)s, (f16)s}; }
__device__ __forceinline__ h2 cconj(h2 a) { return h2{a.x, -a.y}; }
__device__ __forceinline__ h2 mul_mi(h2 a) { return h2{a.y, -a.x}; }
__device__ __forceinline__ h2 mul_pi(h2 a) { return h2{-a.y, a.x}; }
__device__ __forceinline__ h2 cneg(h2 a) { return -a; }
__device__ __forceinline__ h2 cmulk(h2 a, float c, float s) {
  return cmul(a, h2{(f16)c, (f16)s});
}
__device__ __forceinline__ h2 mul_1mi(h2 a, float k) { return (a + h2{a.y, -a.x}) * h2{(f16)k, (f16)k}; }
__device__ __forceinline__ h2 mul_m1mi(h2 a, float k) { return (h2{a.y, -a.x} - a) * h2{(f16)k, (f16)k}; }
__device__ __forceinline__ h2 mul_m1pi(h2 a, float k) { return (h2{-a.y, a.x} - a) * h2{(f16)k, (f16)k}; }
__device__ __forceinline__ h2 mul_1pi(h2 a, float k) { return (a + h2{-a.y, a.x}) * h2{(f16)k, (f16)k}; }

// Exact power-of-two scaling a . 2^-K (the block-floating-point shift) as an
// ldexp instruction: exact for normal results, round-to-nearest-even into
// subnormals, and never contracted into a neighbouring FMA, so the shifted
// value is the same in every kernel.
__device__ __forceinline__ f16 ldexp16(f16 v, int k) {
  return (f16)__builtin_amdgcn_ldexph((__fp16)v, k);
}
template <int K>
__device__ __forceinline__ c32 pow2(c32 a) {
  if constexpr (K == 0) return a;
  else return c32{__builtin_ldexpf(a.x, -K), __builtin_ldexpf(a.y, -K)};
}
// Packed FP16 variant: one v_pk_mul_f16 by (2^-K, +/-2^-K), the same
// correctly rounded product as ldexp.  Contraction is off for this product,
// so the compiler cannot fuse it into a neighbouring FMA.
__device__ __forceinline__ h2 pk_scale(h2 a, h2 s) {
#pragma clang fp contract(off)
  return a * s;
}
template <int K>
__device__ __forceinline__ h2 pow2(h2 a) {
  static_assert(K >= 0 && K <= 14, "2^-K must be a normal FP16 number");
  if constexpr (K == 0) return a;
  else return pk_scale(a, h2{(f16)(1.0f / (1 << K)), (f16)(1.0f / (1 << K))});
}
// conj(a) as a sign flip (one instruction on a packed FP16 pair)
__device__ __forceinline__ c32 conj_store(c32 a) { return c32{a.x, -a.y}; }
__device__ __forceinline__ h2 conj_store(h2 a) {
  return __builtin_bit_cast(h2, __builtin_bit_cast(uint32_t, a) ^ 0x80000000u);
}
// conj(a) . 2^-K
template <int K>
__device__ __forceinline__ c32 conj_pow2(c32 a) {
  if constexpr (K == 0) return c32{a.x, -a.y};
  else return c32{__builtin_ldexpf(a.x, -K), -__builtin_ldexpf(a.y, -K)};
}
template <int K>
__device__ __forceinline__ h2 conj_pow2(h2 a) {
  static_assert(K >= 0 && K <= 14, "2^-K must be a normal FP16 number");
  if constexpr (K == 0) return h2{a.x, -a.y};
  else return pk_scale(a, h2{(f16)(1.0f / (1 << K)), (f16)(-1.0f / (1 << K))});
}

// ------------------------------------------------- radix constants ------
// cos(pi/4), cos(pi/8), sin(pi/8) to 20 significant digits.
#define BFP_C8 0.70710678118654752440f
#define BFP_C16 0.92387953251128675613f
#define BFP_S16 0.38268343236508977173f

// a * W_R^e, W_R = exp(-2 pi i / R), e a compile-time constant
template <int R, int E, class C>
__device__ __forceinline__ C mulw(C a) {
  constexpr int e = ((E % R) + R) % R;
  if constexpr (e == 0) {
    return a;
  } else if constexpr (4 * e == R) {
    return mul_mi(a);
  } else if constexpr (2 * e == R) {
    return cneg(a);
  } else if constexpr (4 * e == 3 * R) {
    return mul_pi(a);
  } else if constexpr (8 * e == R) {
    return mul_1mi(a, BFP_C8);       // e^{-i pi/4}
  } else if constexpr (8 * e == 3 * R) {
    return mul_m1mi(a, BFP_C8);      // e^{-3i pi/4}
  } else if constexpr (8 * e == 5 * R) {
    return mul_m1pi(a, BFP_C8);      // e^{-5i pi/4}
  } else if constexpr (8 * e == 7 * R) {
    return mul_1pi(a, BFP_C8);       // e^{-7i pi/4}
  } else {
    static_assert(R == 16, "generic constant twiddles only for radix 16");
    // e odd: angle = 2 pi e / 16 = e pi / 8
    constexpr int q = e;  // 1,3,5,7,9,11,13,15
    constexpr float c = (q == 1 || q == 15) ? BFP_C16
                      : (q == 3 || q == 13) ? BFP_S16
                      : (q == 5 || q == 11) ? -BFP_S16
                                            : -BFP_C16;  // 7, 9
    constexpr float s = (q == 1 || q == 7) ? -BFP_S16
                      : (q == 3 || q == 5) ? -BFP_C16
                      : (q == 9 || q == 15) ? BFP_S16
                                            : BFP_C16;   // 11, 13
    return cmulk(a, c, s);
  }
}

// ------------------------------------------------------------ DFTs ------
// In-place length-R DFT (forward sign), natural order in and out.
// CJ = true returns the conjugated outputs: the last combining step takes
// conjugated operands (conj(x + y) = conj x + conj y, conj(-i y) = i conj y),
// which the packed adds apply as source negations, so the conjugate at the
// end of an inverse transform costs no instruction.
template <bool CJ = false, class C>
__device__ __forceinline__ void dft2(C &a, C &b) {
  C t = CJ ? cconj(a) : a;
  C u = CJ ? cconj(b) : b;
  a = cadd(t, u);
  b = csub(t, u);
}

template <bool CJ = false, class C>
__device__ __forceinline__ void dft4(C &a, C &b, C &c, C &d) {
  C s0 = cadd(a, c), s1 = csub(a, c), s2 = cadd(b, d), s3 = csub(b, d);
  if constexpr (CJ) {
    s0 = cconj(s0);
    s1 = cconj(s1);
    s2 = cconj(s2);
    s3 = cconj(s3);
    a = cadd(s0, s2);
    c = csub(s0, s2);
    b = cadd_i(s1, s3);  // conj((a-c) - i(b-d))
    d = csub_i(s1, s3);  // conj((a-c) + i(b-d))
  } else {
    a = cadd(s0, s2);
    c = csub(s0, s2);
    b = csub_i(s1, s3);  // (a-c) - i(b-d)
    d = cadd_i(s1, s3);  // (a-c) + i(b-d)
  }
}

template <int R, bool CJ = false, class C>
__device__ __forceinline__ void dft(C *v) {
  if constexpr (R == 2) {
    dft2<CJ>(v[0], v[1]);
  } else if constexpr (R == 4) {
    dft4<CJ>(v[0], v[1], v[2], v[3]);
  } else if constexpr (R == 8) {
    // n = n2 + 2 n1 (n2 < 2, n1 < 4), k = k1 + 4 k2
    dft4(v[0], v[2], v[4], v[6]);  // n2 = 0 -> slots 0,2,4,6 hold k1 = 0..3
    dft4(v[1], v[3], v[5], v[7]);  // n2 = 1
    v[3] = mulw<8, 1>(v[3]);
    v[5] = mulw<8, 2>(v[5]);
    v[7] = mulw<8, 3>(v[7]);
    C y[8];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      const C p = CJ ? cconj(v[2 * k1]) : v[2 * k1];
      const C q = CJ ? cconj(v[2 * k1 + 1]) : v[2 * k1 + 1];
      y[k1] = cadd(p, q);
      y[k1 + 4] = csub(p, q);
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = y[i];
  } else if constexpr (R == 16) {
    // n = n2 + 4 n1, k = k1 + 4 k2: DFT4 over n1, twiddle W16^{n2 k1},
    // DFT4 over n2.
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) dft4(v[n2], v[n2 + 4], v[n2 + 8], v[n2 + 12]);
    // slot n2 + 4 k1 now holds Y[n2][k1]
    v[5] = mulw<16, 1>(v[5]);
    v[6] = mulw<16, 2>(v[6]);
    v[7] = mulw<16, 3>(v[7]);
    v[9] = mulw<16, 2>(v[9]);
    v[10] = mulw<16, 4>(v[10]);
    v[11] = mulw<16, 6>(v[11]);
    v[13] = mulw<16, 3>(v[13]);
    v[14] = mulw<16, 6>(v[14]);
    v[15] = mulw<16, 9>(v[15]);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) dft4<CJ>(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
    // slot k2 + 4 k1 holds X[k1 + 4 k2]: transpose the 4x4 slot grid
    C y[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) y[k1 + 4 * k2] = v[k2 + 4 * k1];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = y[i];
  } else {
    static_assert(R == 2 || R == 4 || R == 8 || R == 16, "radix");
  }
}

// ----------------------------------------------------- storage types ----
struct __attribute__((aligned(2))) fp8x2 {
  uint8_t x, y;
};

// OCP FP8 codec on gfx950's conversion instructions: v_cvt_pk_f32_fp8 /
// v_cvt_pk_f32_bf8 decode two bytes exactly (E4M3: bias 7, 3 mantissa bits,
// 0x7F/0xFF NaN; E5M2: bias 15, 2 mantissa bits, exponent 31 = inf/NaN), and
// v_cvt_pk_fp8_f32 / v_cvt_pk_bf8_f32 round two FP32 values to nearest-even.
// Saturation (|x| above the largest finite value maps to it, sign kept, NaN
// stays NaN) is a compare and select ahead of the rounding: a comparison
// with NaN is false, so NaN reaches the instruction, which keeps it NaN.
// The codec is checked bit for bit against the host encoder over the whole
// range, subnormals, saturation and NaN included.
typedef float f32x2 __attribute__((ext_vector_type(2)));
template <int MANT>
struct Fp8Codec {
  static_assert(MANT == 3 || MANT == 2, "E4M3 or E5M2");
  static constexpr float kMax = MANT == 3 ? 448.0f : 57344.0f;
  static __device__ __forceinline__ float sat(float x) {
    return __builtin_fabsf(x) > kMax ? __builtin_copysignf(kMax, x) : x;
  }
  // bytes 0 and 1 of `bits` -> (x, y)
  static __device__ __forceinline__ c32 decode2(uint32_t bits) {
    f32x2 v;
    if constexpr (MANT == 3) v = __builtin_amdgcn_cvt_pk_f32_fp8((int)bits, false);
    else v = __builtin_amdgcn_cvt_pk_f32_bf8((int)bits, false);
    return c32{v.x, v.y};
  }
  // (x, y) -> bytes 0 and 1
  static __device__ __forceinline__ uint32_t encode2(float x, float y) {
    if constexpr (MANT == 3) return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(sat(x), sat(y), 0, false) & 0xFFFFu;
    else return (uint32_t)__builtin_amdgcn_cvt_pk_bf8_f32(sat(x), sat(y), 0, false) & 0xFFFFu;
  }
};

// ------------------------------------------------------ streaming I/O ---
// Row data is read once and written once: nontemporal loads and stores keep
// it from displacing the twiddle and filter tables in the caches.
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
template <class T>
__device__ __forceinline__ T ld_stream(const T *p) {
  static_assert(sizeof(T) == 2 || sizeof(T) == 4 || sizeof(T) == 8, "unsupported element size");
  if constexpr (sizeof(T) == 2)
    return __builtin_bit_cast(T, __builtin_nontemporal_load(reinterpret_cast<const uint16_t *>(p)));
  else if constexpr (sizeof(T) == 4)
    return __builtin_bit_cast(T, __builtin_nontemporal_load(reinterpret_cast<const uint32_t *>(p)));
  else
    return __builtin_bit_cast(T, __builtin_nontemporal_load(reinterpret_cast<const u32x2 *>(p)));
}
template <class T>
__device__ __forceinline__ void st_stream(T *p, T v) {
  static_assert(sizeof(T) == 2 || sizeof(T) == 4 || sizeof(T) == 8, "unsupported element size");
  if constexpr (sizeof(T) == 2)
    __builtin_nontemporal_store(__builtin_bit_cast(uint16_t, v), reinterpret_cast<uint16_t *>(p));
  else if constexpr (sizeof(T) == 4)
    __builtin_nontemporal_store(__builtin_bit_cast(uint32_t, v), reinterpret_cast<uint32_t *>(p));
  else
    __builtin_nontemporal_store(__builtin_bit_cast(u32x2, v), reinterpret_cast<u32x2 *>(p));
}

// The same through a pointer known to address global memory: a uniform base
// can then stay in scalar registers (global loads and stores take a scalar
// base, a 32-bit lane offset and an immediate).
template <class T>
using global_ptr = __attribute__((address_space(1))) T *;
template <class T>
__device__ __forceinline__ T ld_stream_g(global_ptr<const T> p) {
  static_assert(sizeof(T) == 2 || sizeof(T) == 4 || sizeof(T) == 8, "unsupported element size");
  if constexpr (sizeof(T) == 2)
    return __builtin_bit_cast(T, __builtin_nontemporal_load(reinterpret_cast<global_ptr<const uint16_t>>(p)));
  else if constexpr (sizeof(T) == 4)
    return __builtin_bit_cast(T, __builtin_nontemporal_load(reinterpret_cast<global_ptr<const uint32_t>>(p)));
  else
    return __builtin_bit_cast(T, __builtin_nontemporal_load(reinterpret_cast<global_ptr<const u32x2>>(p)));
}
template <class T>
__device__ __forceinline__ T ld_cached_g(global_ptr<const T> p) {
  static_assert(sizeof(T) == 2 || sizeof(T) == 4 || sizeof(T) == 8, "unsupported element size");
  if constexpr (sizeof(T) == 2)
    return __builtin_bit_cast(T, *reinterpret_cast<global_ptr<const uint16_t>>(p));
  else if constexpr (sizeof(T) == 4)
    return __builtin_bit_cast(T, *reinterpret_cast<global_ptr<const uint32_t>>(p));
  else
    return __builtin_bit_cast(T, *reinterpret_cast<global_ptr<const u32x2>>(p));
}
template <class T>
__device__ __forceinline__ void st_stream_g(global_ptr<T> p, T v) {
  static_assert(sizeof(T) == 2 || sizeof(T) == 4 || sizeof(T) == 8, "unsupported element size");
  if constexpr (sizeof(T) == 2)
    __builtin_nontemporal_store(__builtin_bit_cast(uint16_t, v), reinterpret_cast<global_ptr<uint16_t>>(p));
  else if constexpr (sizeof(T) == 4)
    __builtin_nontemporal_store(__builtin_bit_cast(uint32_t, v), reinterpret_cast<global_ptr<uint32_t>>(p));
  else
    __builtin_nontemporal_store(__builtin_bit_cast(u32x2, v), reinterpret_cast<global_ptr<u32x2>>(p));
}

// --------------------------------------------------- precision policies --
// Each mode defines:
//   Store: HBM element; Lds: on-chip element between passes;
//   Comp: register arithmetic type; Tw: twiddle table element;
//   Filt: filter element.
// and the conversions/multiplies the engine needs.

struct ModeFP32 {
  typedef c32 Store; typedef c32 Lds; typedef c32 Comp; typedef c32 Tw; typedef c32 Filt;
  static __device__ __forceinline__ Comp decode(Store s) { return s; }
  static __device__ __forceinline__ Store encode(Comp v) { return v; }
  static __device__ __forceinline__ Comp load(const Store *p, unsigned i) { return ld_stream(p + i); }
  static __device__ __forceinline__ void store(Store *p, unsigned i, Comp v) { st_stream(p + i, v); }
  static __device__ __forceinline__ Lds to_lds(Comp v) { return v; }
  static __device__ __forceinline__ Comp from_lds(Lds v) { return v; }
  static __device__ __forceinline__ Comp twiddle(Lds v, Tw w) { return cmul(v, w); }
  static __device__ __forceinline__ Comp fmul(Comp v, Filt h) { return cmul(v, h); }
  static __device__ __forceinline__ Comp round_store(Comp v) { return v; }
};

struct ModeFP16 {  // pure packed FP16
  typedef h2 Store; typedef h2 Lds; typedef h2 Comp; typedef h2 Tw; typedef h2 Filt;
  static __device__ __forceinline__ Comp decode(Store s) { return s; }
  static __device__ __forceinline__ Store encode(Comp v) { return v; }
  static __device__ __forceinline__ Comp load(const Store *p, unsigned i) { return ld_stream(p + i); }
  static __device__ __forceinline__ void store(Store *p, unsigned i, Comp v) { st_stream(p + i, v); }
  static __device__ __forceinline__ Lds to_lds(Comp v) { return v; }
  static __device__ __forceinline__ Comp from_lds(Lds v) { return v; }
  static __device__ __forceinline__ Comp twiddle(Lds v, Tw w) { return cmul(v, w); }
  static __device__ __forceinline__ Comp fmul(Comp v, Filt h) { return cmul(v, h); }
  static __device__ __forceinline__ Comp round_store(Comp v) { return v; }
};

__device__ __forceinline__ c32 h2_to_c32(h2 v) { return c32{(float)v.x, (float)v.y}; }

// Natural logarithm of a positive FP32 value from the hardware base-2
// logarithm (v_log_f32, about 1 ulp) and one multiply, instead of the
// library's correctly-scaled sequence (about 11 instructions more).  The
// hardware instruction does not take denormal inputs, so arguments below the
// smallest normal number are raised to it: for an image power p that small
// the terms p ln p and p (ln p + c) are below 1e-36.
__device__ __forceinline__ float ln_pos(float a) {
  return __builtin_amdgcn_logf(fmaxf(a, 1.17549435e-38f)) * 0.693147180559945309f;
}
__device__ __forceinline__ h2 c32_to_h2(c32 v) { return h2{(f16)v.x, (f16)v.y}; }

struct ModeF16StoreF32 {
  typedef h2 Store; typedef h2 Lds; typedef c32 Comp; typedef c32 Tw; typedef h2 Filt;
  static __device__ __forceinline__ Comp decode(Store s) { return h2_to_c32(s); }
  static __device__ __forceinline__ Store encode(Comp v) { return c32_to_h2(v); }
  static __device__ __forceinline__ Comp load(const Store *p, unsigned i) { return h2_to_c32(ld_stream(p + i)); }
  static __device__ __forceinline__ void store(Store *p, unsigned i, Comp v) { st_stream(p + i, c32_to_h2(v)); }
  static __device__ __forceinline__ Lds to_lds(Comp v) { return c32_to_h2(v); }
  static __device__ __forceinline__ Comp from_lds(Lds v) { return h2_to_c32(v); }
  static __device__ __forceinline__ Comp twiddle(Lds v, Tw w) { return cmul(h2_to_c32(v), w); }
  static __device__ __forceinline__ Comp fmul(Comp v, Filt h) { return cmul(v, h2_to_c32(h)); }
  static __device__ __forceinline__ Comp round_store(Comp v) { return h2_to_c32(c32_to_h2(v)); }
};

// FP16 operands, FP32 accumulation: (a.x, a.y) . (b.x, -b.y) and
// (a.x, a.y) . (b.y, b.x) with v_dot2_f32_f16.
__device__ __forceinline__ c32 cmul_dot2(h2 a, h2 b) {
  float re = __builtin_amdgcn_fdot2(a, h2{b.x, -b.y}, 0.0f, false);
  float im = __builtin_amdgcn_fdot2(a, h2{b.y, b.x}, 0.0f, false);
  return c32{re, im};
}

struct ModeF16MulF32Acc {
  typedef h2 Store; typedef h2 Lds; typedef c32 Comp; typedef h2 Tw; typedef h2 Filt;
  static __device__ __forceinline__ Comp decode(Store s) { return h2_to_c32(s); }
  static __device__ __forceinline__ Store encode(Comp v) { return c32_to_h2(v); }
  static __device__ __forceinline__ Comp load(const Store *p, unsigned i) { return h2_to_c32(ld_stream(p + i)); }
  static __device__ __forceinline__ void store(Store *p, unsigned i, Comp v) { st_stream(p + i, c32_to_h2(v)); }
  static __device__ __forceinline__ Lds to_lds(Comp v) { return c32_to_h2(v); }
  static __device__ __forceinline__ Comp from_lds(Lds v) { return h2_to_c32(v); }
  static __device__ __forceinline__ Comp twiddle(Lds v, Tw w) { return cmul_dot2(v, w); }
  static __device__ __forceinline__ Comp fmul(Comp v, Filt h) { return cmul_dot2(c32_to_h2(v), h); }
  static __device__ __forceinline__ Comp round_store(Comp v) { return h2_to_c32(c32_to_h2(v)); }
};

template <int MANT, int BIAS>
struct ModeFP8 {
  typedef fp8x2 Store; typedef c32 Lds; typedef c32 Comp; typedef c32 Tw; typedef c32 Filt;
  typedef Fp8Codec<MANT> Codec;
  static __device__ __forceinline__ Comp decode(Store b) {
    return Codec::decode2(__builtin_bit_cast(uint16_t, b));
  }
  static __device__ __forceinline__ Comp load(const Store *p, unsigned i) { return decode(ld_stream(p + i)); }
  static __device__ __forceinline__ Store encode(Comp v) {
    return __builtin_bit_cast(fp8x2, (uint16_t)Codec::encode2(v.x, v.y));
  }
  static __device__ __forceinline__ void store(Store *p, unsigned i, Comp v) { st_stream(p + i, encode(v)); }
  static __device__ __forceinline__ Lds to_lds(Comp v) { return v; }
  static __device__ __forceinline__ Comp from_lds(Lds v) { return v; }
  static __device__ __forceinline__ Comp twiddle(Lds v, Tw w) { return cmul(v, w); }
  static __device__ __forceinline__ Comp fmul(Comp v, Filt h) { return cmul(v, h); }
  static __device__ __forceinline__ Comp round_store(Comp v) { return decode(encode(v)); }
};
typedef ModeFP8<3, 7> ModeE4M3;
typedef ModeFP8<2, 15> ModeE5M2;

__device__ __forceinline__ c32 to_c32(c32 v) { return v; }
__device__ __forceinline__ c32 to_c32(h2 v) { return h2_to_c32(v); }

__device__ __forceinline__ bool finite_c(c32 v) {
  return __builtin_isfinite(v.x) && __builtin_isfinite(v.y);
}
__device__ __forceinline__ bool finite_c(h2 v) {
  return __builtin_isfinite((float)v.x) && __builtin_isfinite((float)v.y);
}

}  // namespace bfp
