// Row kernels: batched forward FFT, BFP inverse and fused matched-filter
// compression for one precision mode.  This file is compiled once per mode
// with -DBFP_MODE_ID=<bfp_precision>; each object defines
// launch_rows_mode<ID>(), which the dispatcher in dispatch.cpp calls.
//
// Inverse (paper Eq. (1)): y = conj(FFT(conj(z . H) . 2^-log2N)).  The
// 2^-log2N factor and the conjugate are applied to each element as it is
// loaded, before the first radix pass, so no intermediate of the inverse
// exceeds O(N) max|z . H|.  With KF_NAIVE the factor is instead applied after
// the inverse, to the value already rounded to the storage format (the
// conventional schedule whose overflow Sec. III-B describes).
//
// Compression (Fig. 1): x -> [x exp(i phi_m)] -> FFT -> x H -> conj . 2^-log2N
// -> FFT -> conj, entirely in registers/LDS: one HBM read and one HBM write
// per row.  The forward FFT's last pass leaves X[k] at the positions the
// inverse's first pass reads, so no data moves between the two transforms.
#include "fft_engine.hpp"
#include "fft_mfma.hpp"
#include "internal.hpp"

#ifndef BFP_MODE_ID
#error "BFP_MODE_ID must be defined"
#endif

namespace bfp {

#if BFP_MODE_ID == 0
typedef ModeFP32 MODE;
#elif BFP_MODE_ID == 1
typedef ModeFP16 MODE;
#elif BFP_MODE_ID == 2
typedef ModeF16StoreF32 MODE;
#elif BFP_MODE_ID == 3
typedef ModeF16MulF32Acc MODE;
#elif BFP_MODE_ID == 4
typedef ModeE4M3 MODE;
#elif BFP_MODE_ID == 5
typedef ModeE5M2 MODE;
#else
#error "unknown BFP_MODE_ID"
#endif

__device__ __forceinline__ c32 mul_c32(c32 v, c32 p) { return cmul(v, p); }
__device__ __forceinline__ h2 mul_c32(h2 v, c32 p) { return cmul(v, c32_to_h2(p)); }

// Compile-time variants of the inverse / compression kernels (no runtime
// selects in the per-element code): conventional post-scaling (debug),
// conjugated filter (adjoint), per-pulse phasor at load.
enum Variant { V_PLAIN = 0, V_NAIVE = 1, V_CONJ = 2, V_PHASOR = 4 };

template <class M, int LOG2N, int OP, int V, bool OUT32>
__global__ void __launch_bounds__(Geometry<LOG2N>::WG) row_kernel(RowArgs a) {
  typedef Geometry<LOG2N> G;
  typedef Engine<M, LOG2N> EN;
  typedef typename M::Comp Comp;
  typedef typename M::Store Store;
  typedef typename M::Filt Filt;
  typedef typename M::Tw Tw;
  constexpr int E = G::E, T = G::T, N = G::N;
  constexpr bool naive = (V & V_NAIVE) != 0;
  constexpr bool conj_f = (V & V_CONJ) != 0;
  constexpr bool phasor = (V & V_PHASOR) != 0;

  __shared__ typename M::Lds lds_all[G::TPW * G::LDS_N];
  // one transform per workgroup for N >= 4096: keep the row index uniform
  const int local = G::TPW == 1 ? 0 : (int)(threadIdx.x / T);
  const unsigned t = threadIdx.x & (T - 1);
  typename M::Lds *lds = lds_all + local * G::LDS_N;
  const Tw *tw = static_cast<const Tw *>(a.tw);
  // workgroups loop over groups of TPW rows (one iteration unless the grid
  // was limited to a persistent size); every thread takes the same trips
  const int groups = (a.rows + G::TPW - 1) / G::TPW;
  for (int grp = blockIdx.x; grp < groups; grp += gridDim.x) {
  const long long row = (long long)grp * G::TPW + local;
  const bool active = row < a.rows;

  Comp v[E];
  if (active) {
    // one per-thread base, element offsets T e as immediates
    const Store *src = static_cast<const Store *>(a.in) + row * N + t;
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = M::load(src, (unsigned)(T * e));
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = Comp{};
  }

  if constexpr (OP == OP_FWD) {
    EN::run(v, lds, tw, t);
  } else {
    if constexpr (OP == OP_COMPRESS) {
      if constexpr (phasor) {
        const c32 *ph = static_cast<const c32 *>(a.phasor) + t;
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = mul_c32(v[e], ph[T * e]);
      }
      EN::run(v, lds, tw, t);
    }
    // BFP fold at the inverse's load: conj(z . H) . 2^-log2N, or with the
    // conjugated filter conj(z . conj H) = conj(z) . H
    constexpr int K = naive ? 0 : LOG2N;  // block shift 2^-log2N
    const Filt *f = static_cast<const Filt *>(a.filter);
    if (f) {
      const Filt *ft = f + t;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const Filt h = ft[T * e];
        v[e] = conj_f ? pow2<K>(M::fmul(cconj(v[e]), h)) : conj_pow2<K>(M::fmul(v[e], h));
      }
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = conj_pow2<K>(v[e]);
    }
    EN::run(v, lds, tw, t);
    if constexpr (naive) {
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = pow2<LOG2N>(M::round_store(cconj(v[e])));
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = conj_store(v[e]);
    }
  }

  if (active) {
    if constexpr (OUT32) {
      c32 *dst = static_cast<c32 *>(a.out) + row * N + t;
#pragma unroll
      for (int e = 0; e < E; ++e) dst[(unsigned)(T * e)] = to_c32(v[e]);
    } else {
      Store *dst = static_cast<Store *>(a.out) + row * N + t;
#pragma unroll
      for (int e = 0; e < E; ++e) M::store(dst, (unsigned)(T * e), v[e]);
    }
    if (a.flags & KF_CHECK_FINITE) {
      unsigned bad = 0;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        c32 s = OUT32 ? to_c32(v[e]) : to_c32(M::round_store(v[e]));
        bad += finite_c(s) ? 0u : 1u;
      }
      if (bad) atomicAdd(a.nonfinite, (unsigned long long)bad);
    }
  }
  }  // row groups
}

#if BFP_MODE_ID == 3
// FP16 multiply / FP32 accumulate at N = 4096 on the matrix cores: the same
// operations as row_kernel (forward, BFP inverse, fused compression), every
// radix-16 pass evaluated by MFMA (fft_mfma.hpp).  One transform per
// 256-thread workgroup; the plan's table holds the MFMA operands.
//
// Products with the filter take FP16 operands: X is rounded to FP16 as the
// two dot-product forms (Re X, -Im X) and (Im X, Re X), so
// Re(X H) = (Re X, -Im X) . H and Im(X H) = (Im X, Re X) . H accumulate in
// FP32; conj(X) H uses (Re X, Im X) and (-Im X, Re X).
template <int OP, int V, bool OUT32>
__global__ void __launch_bounds__(256) row_kernel_mfma(RowArgs a) {
  constexpr int N = 4096;
  constexpr bool naive = (V & V_NAIVE) != 0;
  constexpr bool conj_f = (V & V_CONJ) != 0;
  constexpr bool phasor = (V & V_PHASOR) != 0;
  __shared__ h2 lds[N];
  const Mfma4096 E(a.tw, threadIdx.x);
  for (long long row = blockIdx.x; row < a.rows; row += gridDim.x) {
  h2 x[16];
  c32 y[16];
  const h2 *src = static_cast<const h2 *>(a.in) + row * N;
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int i = 0; i < 4; ++i) x[4 * m + i] = src[E.pos(m, i)];

  if constexpr (OP != OP_FWD) {
    if constexpr (OP == OP_COMPRESS) {
      if constexpr (phasor) {
        const c32 *ph = static_cast<const c32 *>(a.phasor);
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
          for (int i = 0; i < 4; ++i)
            x[4 * m + i] = c32_to_h2(cmul(h2_to_c32(x[4 * m + i]), ph[E.pos(m, i)]));
      }
      E.run(x, y, lds);
    } else {
#pragma unroll
      for (int k = 0; k < 16; ++k) y[k] = h2_to_c32(x[k]);
    }
    // BFP fold: conj(z . H) . 2^-12 (exact), FP16 operands, FP32 sums
    constexpr int K = naive ? 0 : 12;  // block shift 2^-12
    const h2 *f = static_cast<const h2 *>(a.filter);
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k = 4 * m + i;
        c32 z;
        if (f) {
          const h2 h = f[E.pos(m, i)];
          if constexpr (conj_f) {
            const h2 xa = c32_to_h2(c32{y[k].x, y[k].y}), xb = c32_to_h2(c32{-y[k].y, y[k].x});
            z = pow2<K>(c32{__builtin_amdgcn_fdot2(xa, h, 0.0f, false),
                            __builtin_amdgcn_fdot2(xb, h, 0.0f, false)});
          } else {
            const h2 xa = c32_to_h2(c32{y[k].x, -y[k].y}), xb = c32_to_h2(c32{y[k].y, y[k].x});
            z = conj_pow2<K>(c32{__builtin_amdgcn_fdot2(xa, h, 0.0f, false),
                                 __builtin_amdgcn_fdot2(xb, h, 0.0f, false)});
          }
        } else {
          z = conj_pow2<K>(y[k]);
        }
        x[k] = c32_to_h2(z);
      }
  }
  E.run(x, y, lds);
  if constexpr (OP != OP_FWD) {
#pragma unroll
    for (int k = 0; k < 16; ++k)
      y[k] = naive ? pow2<12>(h2_to_c32(c32_to_h2(cconj(y[k])))) : cconj(y[k]);
  }

  if constexpr (OUT32) {
    c32 *dst = static_cast<c32 *>(a.out) + row * N;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int i = 0; i < 4; ++i) dst[E.pos(m, i)] = y[4 * m + i];
  } else {
    h2 *dst = static_cast<h2 *>(a.out) + row * N;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int i = 0; i < 4; ++i) dst[E.pos(m, i)] = c32_to_h2(y[4 * m + i]);
  }
  if (a.flags & KF_CHECK_FINITE) {
    unsigned bad = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) bad += finite_c(OUT32 ? y[k] : h2_to_c32(c32_to_h2(y[k]))) ? 0u : 1u;
    if (bad) atomicAdd(a.nonfinite, (unsigned long long)bad);
  }
  }  // rows
}

template <int OP, int V, bool OUT32>
static hipError_t launch_mfma(const RowArgs &a, hipStream_t s) {
  if (a.rows <= 0) return hipSuccess;
  unsigned grid = (unsigned)a.rows;
  if (a.grid_limit > 0 && grid > (unsigned)a.grid_limit) grid = (unsigned)a.grid_limit;
  hipLaunchKernelGGL((row_kernel_mfma<OP, V, OUT32>), dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}
#endif

template <int LOG2N, int OP, int V, bool OUT32>
static hipError_t launch_one(const RowArgs &a, hipStream_t s) {
  typedef Geometry<LOG2N> G;
  if (a.rows <= 0) return hipSuccess;
#if BFP_MODE_ID == 3
  if constexpr (LOG2N == 12) {
    if (a.engine == 0) return launch_mfma<OP, V, OUT32>(a, s);
  }
#endif
  unsigned grid = (unsigned)((a.rows + G::TPW - 1) / G::TPW);
  if (a.grid_limit > 0 && grid > (unsigned)a.grid_limit) grid = (unsigned)a.grid_limit;
  hipLaunchKernelGGL((row_kernel<MODE, LOG2N, OP, V, OUT32>), dim3(grid), dim3(G::WG), 0, s, a);
  return hipGetLastError();
}

// Variant selection; combinations outside this table are rejected by the
// C layer before launch.
template <int LOG2N>
static hipError_t launch_size(int op, bool out32, const RowArgs &a, hipStream_t s) {
  const bool naive = (a.flags & KF_NAIVE) != 0;
  const bool conj = (a.flags & KF_CONJ_FILTER) != 0;
  const bool ph = a.phasor != nullptr;
  switch (op) {
    case OP_FWD:
      return out32 ? launch_one<LOG2N, OP_FWD, V_PLAIN, true>(a, s)
                   : launch_one<LOG2N, OP_FWD, V_PLAIN, false>(a, s);
    case OP_INV:
      if (out32 || ph || (naive && conj)) return hipErrorInvalidValue;
      if (naive) return launch_one<LOG2N, OP_INV, V_NAIVE, false>(a, s);
      if (conj) return launch_one<LOG2N, OP_INV, V_CONJ, false>(a, s);
      return launch_one<LOG2N, OP_INV, V_PLAIN, false>(a, s);
    case OP_COMPRESS:
      if ((naive && (conj || ph)) || (conj && ph)) return hipErrorInvalidValue;
      if (naive) return out32 ? hipErrorInvalidValue : launch_one<LOG2N, OP_COMPRESS, V_NAIVE, false>(a, s);
      if (conj) return out32 ? hipErrorInvalidValue : launch_one<LOG2N, OP_COMPRESS, V_CONJ, false>(a, s);
      if (ph)
        return out32 ? launch_one<LOG2N, OP_COMPRESS, V_PHASOR, true>(a, s)
                     : launch_one<LOG2N, OP_COMPRESS, V_PHASOR, false>(a, s);
      return out32 ? launch_one<LOG2N, OP_COMPRESS, V_PLAIN, true>(a, s)
                   : launch_one<LOG2N, OP_COMPRESS, V_PLAIN, false>(a, s);
  }
  return hipErrorInvalidValue;
}

#define BFP_CAT2(a, b) a##b
#define BFP_CAT(a, b) BFP_CAT2(a, b)

hipError_t BFP_CAT(launch_rows_mode, BFP_MODE_ID)(int log2n, int op, bool out32, const RowArgs &a,
                                                 hipStream_t s) {
  switch (log2n) {
    case 8: return launch_size<8>(op, out32, a, s);
    case 9: return launch_size<9>(op, out32, a, s);
    case 10: return launch_size<10>(op, out32, a, s);
    case 11: return launch_size<11>(op, out32, a, s);
    case 12: return launch_size<12>(op, out32, a, s);
    case 13: return launch_size<13>(op, out32, a, s);
    case 14: return launch_size<14>(op, out32, a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace bfp
