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

template <class M, int LOG2N, int OP, bool OUT32>
__global__ void __launch_bounds__(Geometry<LOG2N>::WG) row_kernel(RowArgs a) {
  typedef Geometry<LOG2N> G;
  typedef Engine<M, LOG2N> EN;
  typedef typename M::Comp Comp;
  typedef typename M::Store Store;
  typedef typename M::Filt Filt;
  typedef typename M::Tw Tw;
  constexpr int E = G::E, T = G::T, N = G::N;
  constexpr float inv_n = 1.0f / (float)N;  // 2^-LOG2N, exact

  __shared__ typename M::Lds lds_all[G::TPW * G::LDS_N];
  const int local = threadIdx.x / T;
  const int t = threadIdx.x & (T - 1);
  const long long row = (long long)blockIdx.x * G::TPW + local;
  const bool active = row < a.rows;
  typename M::Lds *lds = lds_all + local * G::LDS_N;
  const Tw *tw = static_cast<const Tw *>(a.tw);
  const bool naive = (a.flags & KF_NAIVE) != 0;
  const bool conj_f = (a.flags & KF_CONJ_FILTER) != 0;

  Comp v[E];
  if (active) {
    const Store *src = static_cast<const Store *>(a.in) + row * N;
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = M::load(src, t + T * e);
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = Comp{};
  }

  if constexpr (OP == OP_FWD) {
    EN::run(v, lds, tw, t);
  } else {
    if constexpr (OP == OP_COMPRESS) {
      if (a.phasor) {
        const c32 *ph = static_cast<const c32 *>(a.phasor);
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = mul_c32(v[e], ph[t + T * e]);
      }
      EN::run(v, lds, tw, t);
    }
    // BFP fold: conj(z . H) . 2^-log2N at the inverse's load
    const Filt *f = static_cast<const Filt *>(a.filter);
    if (f) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        Filt h = f[t + T * e];
        if (conj_f) h = cconj(h);
        v[e] = M::fmul(v[e], h);
      }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = naive ? cconj(v[e]) : cscale(cconj(v[e]), inv_n);
    EN::run(v, lds, tw, t);
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = cconj(v[e]);
    if (naive) {
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = cscale(M::round_store(v[e]), inv_n);
    }
  }

  if (active) {
    if constexpr (OUT32) {
      c32 *dst = static_cast<c32 *>(a.out) + row * N;
#pragma unroll
      for (int e = 0; e < E; ++e) dst[t + T * e] = to_c32(v[e]);
    } else {
      Store *dst = static_cast<Store *>(a.out) + row * N;
#pragma unroll
      for (int e = 0; e < E; ++e) M::store(dst, t + T * e, v[e]);
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
}

template <int LOG2N, int OP, bool OUT32>
static hipError_t launch_one(const RowArgs &a, hipStream_t s) {
  typedef Geometry<LOG2N> G;
  if (a.rows <= 0) return hipSuccess;
  const unsigned grid = (unsigned)((a.rows + G::TPW - 1) / G::TPW);
  hipLaunchKernelGGL((row_kernel<MODE, LOG2N, OP, OUT32>), dim3(grid), dim3(G::WG), 0, s, a);
  return hipGetLastError();
}

template <int LOG2N>
static hipError_t launch_size(int op, bool out32, const RowArgs &a, hipStream_t s) {
  switch (op) {
    case OP_FWD:
      return out32 ? launch_one<LOG2N, OP_FWD, true>(a, s) : launch_one<LOG2N, OP_FWD, false>(a, s);
    case OP_INV:
      return out32 ? launch_one<LOG2N, OP_INV, true>(a, s) : launch_one<LOG2N, OP_INV, false>(a, s);
    case OP_COMPRESS:
      return out32 ? launch_one<LOG2N, OP_COMPRESS, true>(a, s)
                   : launch_one<LOG2N, OP_COMPRESS, false>(a, s);
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
