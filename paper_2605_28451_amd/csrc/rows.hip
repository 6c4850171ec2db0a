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
#include <type_traits>

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
// conjugated filter (adjoint), per-pulse phasor at load, or, with V_POST,
// applied to the output instead (the adjoint of a phase-corrected
// compression: A = C diag(e^{i phi}) has A^H = diag(e^{-i phi}) C^H, and C^H
// is the same chain with the conjugated filter).
enum Variant { V_PLAIN = 0, V_NAIVE = 1, V_CONJ = 2, V_PHASOR = 4, V_TRANS = 8, V_ENT = 16,
               V_ADAPT = 32, V_RAMP = 64, V_POST = 128 };

// Range cell migration correction folded into the range compression (the
// RCMC step of the range-Doppler pipeline, Sec. VI): row r (one Doppler
// bin) multiplies its spectrum by H[k] exp(+2 pi i k' s_r / N), k' the
// signed bin (k - N for k >= N/2), which is the band-limited (periodic sinc)
// interpolation moving the compressed row s_r bins toward smaller range.
// A thread's bins are k' = t + T e (e < E/2) and t + T e - N (e >= E/2), so
// its phasors are base . step^e (times a wrap phasor for the upper half):
// three sincospif per row (phases reduced to [-1/2, 1/2] cycles) and FP32
// complex products (the error of 16 products stays below 1e-6); the product
// with H is formed in FP32 and rounded once to the filter type.
__device__ __forceinline__ c32 cycles_phasor(float cyc) {
  cyc -= rintf(cyc);
  float sn, cs;
  sincospif(2.0f * cyc, &sn, &cs);
  return c32{cs, sn};
}
__device__ __forceinline__ void filt_from_c32(c32 v, c32 &h) { h = v; }
__device__ __forceinline__ void filt_from_c32(c32 v, h2 &h) { h = c32_to_h2(v); }

// Adaptive block shift of one transform (the per-block exponents the paper
// leaves as future work, Sec. VIII): with M the largest |Re| or |Im| of the
// inverse's input z (after the filter product), every partial sum of the
// inverse is bounded by sqrt(2) N M 2^-k after a shift 2^-k, so the
// smallest k with sqrt(2) N M 2^-k < 2^15 keeps all of them below 2^15 (half
// the FP16 range) while scaling weak rows up instead of pushing them toward
// the FP16 subnormals as the fixed k = log2 N does.  With sqrt(2) N M =
// f 2^x, 1/2 <= f < 1: k = x - 15, kept in [-15, 14] (2^15 and 2^-14 are
// normal FP16 numbers; k = -15 for an all-zero row).  The stored output is the normalised inverse times 2^(log2N - k);
// the kernel writes row_exp = k - log2 N, so true value = stored 2^row_exp.
template <int LOG2N>
__device__ __forceinline__ int adaptive_shift(float m) {
  int x = 0;
  (void)frexpf(1.41421356f * (float)(1 << LOG2N) * m, &x);
  const int k = x - 15;
  return k < -15 ? -15 : (k > 14 ? 14 : k);
}
__device__ __forceinline__ float max_component(c32 v) { return fmaxf(fabsf(v.x), fabsf(v.y)); }
__device__ __forceinline__ float max_component(h2 v) {
  return fmaxf(fabsf((float)v.x), fabsf((float)v.y));
}
// conj(v) . 2^-k for a run-time k (exact: a power of two, never contracted)
__device__ __forceinline__ c32 conj_scale(c32 v, float s) { return c32{v.x * s, -(v.y * s)}; }
__device__ __forceinline__ h2 conj_scale(h2 v, float s) {
  return pk_scale(v, h2{(f16)s, (f16)(-s)});
}

// Order of the row groups of a transposed store.  Workgroups are dispatched
// to the 8 XCDs in turn (workgroup w on XCD w mod 8), so the groups of
// iterations it = x, x + 8, ... (one XCD) are given consecutive rows: the
// 4-byte stores that neighbouring rows make into one output line then meet
// in that XCD's L2 instead of eight.  A bijection of [0, groups) (the
// mapping only moves work; any dispatch order gives the same result).
__device__ __forceinline__ int xcd_group(int it, int groups) {
  const int q = groups >> 3, rem = groups & 7, x = it & 7, i = it >> 3;
  return x * q + (x < rem ? x : rem) + i;
}

// The image entropy sums of a workgroup: a fixed-order tree of the threads'
// (S, Q) in `sh` (2 * WG doubles of LDS, free once the caller's barrier has
// passed), written as the workgroup's partial; a second kernel adds the
// partials.  (Finishing the total in the workgroup that arrives last would
// need a device-scope release per workgroup, an L2 writeback in the middle
// of the image's streaming stores: it made the autofocus step 1.7x slower.)
template <int WG>
__device__ __forceinline__ void entropy_sums(const RowArgs &a, double es, double eq, double *sh) {
  sh[threadIdx.x] = es;
  sh[WG + threadIdx.x] = eq;
  __syncthreads();
  for (int w = WG / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sh[threadIdx.x] += sh[threadIdx.x + w];
      sh[WG + threadIdx.x] += sh[WG + threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    a.ent_partial[2 * blockIdx.x] = sh[0];
    a.ent_partial[2 * blockIdx.x + 1] = sh[WG];
  }
}

// PIPE (persistent grids, where the engine keeps its twiddles in registers):
// the twiddle rows are loaded once per workgroup, and the next row group's
// data is loaded into registers while the current group is transformed, so
// HBM reads overlap the arithmetic instead of alternating with it.
template <class M, int LOG2N, int OP, int V, bool OUT32, bool PIPE>
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
  constexpr bool post = (V & V_POST) != 0;
  static_assert(!post || (phasor && OP == OP_COMPRESS && (V & ~(V_PHASOR | V_POST | V_CONJ)) == 0),
                "the output phasor is a variant of the (conjugate-filter) compression");
  constexpr bool trans = (V & V_TRANS) != 0;
  static_assert(!trans || (OP == OP_COMPRESS && V == V_TRANS && !OUT32),
                "the transposed store is a variant of the plain compression");
  // entropy sums of the FP32 output (autofocus image): per workgroup
  // S = sum |I|^2 and Q = sum |I|^2 ln |I|^2 over the rows it wrote
  constexpr bool ent = (V & V_ENT) != 0;
  static_assert(!ent || (OP == OP_COMPRESS && (V & ~V_PHASOR) == V_ENT && OUT32),
                "entropy sums are a variant of the (phase-corrected) compression to FP32");
  double es = 0.0, eq = 0.0;
  // adaptive block shift (V_ADAPT): per-transform max through LDS
  constexpr bool adapt = (V & V_ADAPT) != 0;
  static_assert(!adapt || ((OP == OP_INV || OP == OP_COMPRESS) && V == V_ADAPT && !OUT32),
                "the adaptive shift is a variant of the plain inverse and compression");
  __shared__ unsigned amax[adapt ? G::TPW : 1];
  constexpr bool ramp = (V & V_RAMP) != 0;
  static_assert(!ramp || (OP == OP_COMPRESS && V == V_RAMP && !OUT32),
                "the migration ramp is a variant of the plain compression");

  // the pipelined kernel alternates two LDS buffers (one barrier per exchange)
  __shared__ typename M::Lds lds_all[(PIPE ? 2 : 1) * G::TPW * G::LDS_N];
  // one transform per workgroup for N >= 4096: keep the row index uniform
  const int local = G::TPW == 1 ? 0 : (int)(threadIdx.x / T);
  const unsigned t = threadIdx.x & (T - 1);
  typename M::Lds *lds = lds_all + local * G::LDS_N;
  typename M::Lds *const buf[2] = {lds, lds + (PIPE ? G::TPW * G::LDS_N : 0)};
  unsigned xch = 0;  // LDS exchanges so far (pipelined kernel)
  const Tw *tw = static_cast<const Tw *>(a.tw);
  // A 4-byte filter (FP16 pairs) is the same for every row: its E values
  // per thread are loaded once, ahead of the row loop, so no row waits on
  // them.  Wider filters are read per row to keep registers free, and so is
  // the pure-FP16 filter at N >= 8192: without its E registers those kernels
  // fit 8 wavefronts per SIMD (two 1024-thread workgroups per CU at
  // N = 16384 instead of one).
  const Filt *f = static_cast<const Filt *>(a.filter);
  // row I/O through load_row / store_row (not in the pipelined kernel; FP8
  // rows keep the per-element decode, which needs fewer registers)
  constexpr bool kRowIo = !PIPE && sizeof(Store) >= 4;
  constexpr bool kHoist = sizeof(Filt) == 4 && OP != OP_FWD &&
                          (LOG2N <= 12 || !std::is_same<M, ModeFP16>::value);
  Filt hf[kHoist ? E : 1];
  if constexpr (kHoist) {
    if (f) {
#pragma unroll
      for (int e = 0; e < E; ++e) hf[e] = f[t + T * e];
    }
  }
  // workgroups loop over groups of TPW rows (one iteration unless the grid
  // was limited to a persistent size); every thread takes the same trips
  const int groups = (a.rows + G::TPW - 1) / G::TPW;
  static_assert(!PIPE || EN::kTwRegs, "the pipelined kernel keeps its twiddles in registers");
  typename EN::TwRegs W;
  Store nx[PIPE ? E : 1];
  auto group_of = [&](int it) { return trans ? xcd_group(it, groups) : it; };
  if constexpr (PIPE) {
    EN::load_tw_regs(tw, t, W);
    const long long row0 = (long long)group_of(blockIdx.x) * G::TPW + local;
    if ((int)blockIdx.x < groups && row0 < a.rows) {
      const Store *src = static_cast<const Store *>(a.in) + row0 * N + t;
#pragma unroll
      for (int e = 0; e < E; ++e) nx[e] = ld_stream(src + (unsigned)(T * e));
    }
  }
  auto transform = [&](Comp (&x)[E], unsigned tt) {
    if constexpr (PIPE) EN::run_regs(x, buf, xch, tt, W);
    else EN::run(x, lds, tw, tt);
  };
  // the inverse's transform, its final conjugate folded into the last pass
  auto transform_conj = [&](Comp (&x)[E], unsigned tt) {
    if constexpr (PIPE) EN::template run_regs<true>(x, buf, xch, tt, W);
    else EN::template run<true>(x, lds, tw, tt);
  };
  for (int it = blockIdx.x; it < groups; it += gridDim.x) {
  const int grp = group_of(it);
  const long long row = (long long)grp * G::TPW + local;
  const bool active = row < a.rows;
  // the thread index, made opaque per row group: otherwise the compiler
  // hoists every pass's LDS addresses out of the loop into registers (the
  // empty statement emits no instruction)
  unsigned tt = t;
  asm volatile("" : "+v"(tt));
  if constexpr (adapt) {
    // the previous row read amax before its inverse transform, whose
    // barriers every thread has passed; the forward transform's barriers
    // (compression) or this one (inverse) order the reset before the maxima
    if (tt == 0) amax[local] = 0u;
    if constexpr (OP == OP_INV) __syncthreads();
  }
  if constexpr (PIPE) {
    // likewise the register twiddles and filter: hoisted, each FP16 pair
    // would be kept twice, pre-broadcast as (re, re) and (im, im), instead
    // of broadcast by the packed instructions' operand selects
#pragma unroll
    for (int p = 0; p < (int)(sizeof(W.w) / sizeof(W.w[0])); ++p)
#pragma unroll
      for (int e = 0; e < E; ++e) asm volatile("" : "+v"(W.w[p][e]));
    if constexpr (kHoist) {
#pragma unroll
      for (int e = 0; e < E; ++e) asm volatile("" : "+v"(hf[e]));
    }
  }

  Comp v[E];
  if (active) {
    if constexpr (PIPE) {
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = M::decode(nx[e]);
    } else {
      if constexpr (kRowIo) {
        Store raw[E];
        load_row<G>(raw, a.in, row, tt & (T - 1));
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = M::decode(raw[e]);
      } else {
        const Store *src = static_cast<const Store *>(a.in) + row * N + tt;
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = M::load(src, (unsigned)(T * e));
      }
    }
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = Comp{};
  }
  if constexpr (OP == OP_COMPRESS && phasor && !post) {
    if (active) {
      const c32 *ph = static_cast<const c32 *>(a.phasor) + tt;
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = mul_c32(v[e], ph[T * e]);
    }
  }
  if constexpr (PIPE) {
    // the next group's data, in flight during this group's transforms
    const int nit = it + (int)gridDim.x;
    const long long nrow = nit < groups ? (long long)group_of(nit) * G::TPW + local : a.rows;
    if (nrow < a.rows) {
      const Store *src = static_cast<const Store *>(a.in) + nrow * N + tt;
#pragma unroll
      for (int e = 0; e < E; ++e) nx[e] = ld_stream(src + (unsigned)(T * e));
    }
  }

  if constexpr (OP == OP_FWD) {
    transform(v, tt);
  } else {
    if constexpr (OP == OP_COMPRESS) transform(v, tt);
    // BFP fold at the inverse's load: conj(z . H) . 2^-log2N, or with the
    // conjugated filter conj(z . conj H) = conj(z) . H
    constexpr int K = naive ? 0 : LOG2N;  // block shift 2^-log2N
    // compression always carries a filter (checked by the C layer), so its
    // kernels have no run-time branch here
    if constexpr (adapt) {
      if (OP == OP_COMPRESS || f) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
          Filt h;
          if constexpr (kHoist) h = hf[e];
          else h = f[tt + T * e];
          v[e] = M::fmul(v[e], h);
        }
      }
      // the largest component of the transform's z (non-negative floats
      // order like their bit patterns)
      float m = 0.0f;
#pragma unroll
      for (int e = 0; e < E; ++e) m = fmaxf(m, max_component(v[e]));
      atomicMax(&amax[local], __float_as_uint(m));
      __syncthreads();
      const int k = adaptive_shift<LOG2N>(__uint_as_float(amax[local]));
      if (active && tt == 0) a.row_exp[row] = k - LOG2N;
      const float sc = __uint_as_float((unsigned)(127 - k) << 23);  // 2^-k
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = conj_scale(v[e], sc);
    } else if constexpr (ramp) {
      const float sr = active ? a.shift[row] : 0.0f;
      c32 r = cycles_phasor((float)tt * sr * (1.0f / N));
      const c32 step = cycles_phasor(sr * ((float)T / N));
      const c32 wrap = cycles_phasor(-sr);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        if (e == E / 2) r = cmul(r, wrap);
        Filt h;
        if constexpr (kHoist) h = hf[e];
        else h = f[tt + T * e];
        filt_from_c32(cmul(to_c32(h), r), h);
        v[e] = conj_pow2<K>(M::fmul(v[e], h));
        r = cmul(r, step);
      }
    } else if (OP == OP_COMPRESS || f) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        Filt h;
        if constexpr (kHoist) h = hf[e];
        else h = f[tt + T * e];
        v[e] = conj_f ? pow2<K>(M::fmul(cconj(v[e]), h)) : conj_pow2<K>(M::fmul(v[e], h));
      }
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = conj_pow2<K>(v[e]);
    }
    if constexpr (naive) {
      transform(v, tt);
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = pow2<LOG2N>(M::round_store(cconj(v[e])));
    } else {
      transform_conj(v, tt);
    }
  }
  if constexpr (post) {
    if (active) {
      const c32 *ph = static_cast<const c32 *>(a.phasor) + tt;
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = mul_c32(v[e], ph[T * e]);
    }
  }

  if (active) {
    if constexpr (trans) {
      // out[k][row] for k = t + T e: plain (cached) stores, so the rows of
      // one output line merge in L2 before the line goes to HBM
      Store *dst = static_cast<Store *>(a.out) + row + (long long)tt * a.rows;
      const long long step = (long long)T * a.rows;
#pragma unroll
      for (int e = 0; e < E; ++e) dst[e * step] = M::encode(v[e]);
    } else if constexpr (OUT32) {
      if constexpr (PIPE) {
        c32 *dst = static_cast<c32 *>(a.out) + row * N + tt;
#pragma unroll
        for (int e = 0; e < E; ++e) st_stream(dst + (unsigned)(T * e), to_c32(v[e]));
      } else {
        c32 o[E];
#pragma unroll
        for (int e = 0; e < E; ++e) o[e] = to_c32(v[e]);
        store_row<G>(a.out, row, tt & (T - 1), o);
      }
      if constexpr (ent) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const c32 z = to_c32(v[e]);
          const float p = z.x * z.x + z.y * z.y;
          es += p;
          eq += (double)p * (double)ln_pos(p);  // 0 ln 0 = 0: ln_pos(0) is finite
        }
      }
    } else {
      if constexpr (!kRowIo) {
        Store *dst = static_cast<Store *>(a.out) + row * N + tt;
#pragma unroll
        for (int e = 0; e < E; ++e) M::store(dst, (unsigned)(T * e), v[e]);
      } else {
        Store o[E];
#pragma unroll
        for (int e = 0; e < E; ++e) o[e] = M::encode(v[e]);
        store_row<G>(a.out, row, tt & (T - 1), o);
      }
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
  if constexpr (ent) {
    __shared__ double esh[2 * G::WG];
    entropy_sums<G::WG>(a, es, eq, esh);
  }
}

// Several rows per thread: the plain forward transform, the BFP inverse
// (with or without a filter, or its conjugate) and the compression (plain,
// conjugated filter, phasor before the chain) with RR rows of a group
// transformed together (Engine::pass_rr: shared twiddles, one barrier per
// exchange for all RR rows, one row's LDS latency covered by the others'
// arithmetic).  The arithmetic of each row is that of row_kernel, so the
// results are the same bits.  PIPE (register twiddles, persistent grids):
// the next group's rows are loaded while the current group is transformed.
// Otherwise the twiddles come from the table one pass ahead and a group's
// rows are loaded at its start.  NB LDS buffers per row (2: one barrier per
// exchange; 1: two, half the LDS).  With RR = 1, NB = 1 and PIPE this is
// also the pipelined pure-FP16 kernel at 4096 points.  Group g holds rows
// g TPW RR + q TPW + local, q < RR.
template <class M, int LOG2N, int OP, int V, bool OUT32, int RR, int NB, bool PIPE, int PLAN = 0>
__global__ void __launch_bounds__((Geometry<LOG2N, PLAN>::WG)) row_kernel_rr(RowArgs a) {
  typedef Geometry<LOG2N, PLAN> G;
  typedef Engine<M, LOG2N, PLAN> EN;
  typedef typename M::Comp Comp;
  typedef typename M::Store Store;
  typedef typename M::Filt Filt;
  typedef typename M::Tw Tw;
  constexpr int E = G::E, T = G::T, N = G::N;
  constexpr bool conj_f = (V & V_CONJ) != 0;
  constexpr bool phasor = (V & V_PHASOR) != 0;
  constexpr bool ent = (V & V_ENT) != 0;
  static_assert((V & ~(V_CONJ | V_PHASOR | V_ENT)) == 0, "plain, conjugated-filter, phasor and entropy variants only");
  static_assert(!phasor || OP == OP_COMPRESS, "the phasor belongs to the compression");
  static_assert(!ent || (OP == OP_COMPRESS && OUT32 && !conj_f),
                "entropy sums are a variant of the (phase-corrected) compression to FP32");
  double es = 0.0, eq = 0.0;
  static_assert(!PIPE || EN::kTwRegs, "the pipelined form keeps its twiddles in registers");
  __shared__ __align__(16) typename M::Lds lds_all[NB * G::TPW * RR * G::LDS_N];
  const int local = G::TPW == 1 ? 0 : (int)(threadIdx.x / T);
  const unsigned t = threadIdx.x & (T - 1);
  typename M::Lds *lds = lds_all + local * RR * G::LDS_N;
  typename M::Lds *const buf[2] = {lds, lds + (NB == 2 ? G::TPW * RR * G::LDS_N : 0)};
  unsigned xch = 0;
  const Tw *tw = static_cast<const Tw *>(a.tw);
  const Filt *f = static_cast<const Filt *>(a.filter);
  constexpr bool kHoist = sizeof(Filt) == 4 && OP != OP_FWD;
  Filt hf[kHoist ? E : 1];
  if constexpr (kHoist) {
    if (f) {
#pragma unroll
      for (int e = 0; e < E; ++e) hf[e] = f[t + T * e];
    }
  }
  constexpr int ROWS = G::TPW * RR;
  const int groups = (a.rows + ROWS - 1) / ROWS;
  auto row_of = [&](int g, int q) { return (long long)g * ROWS + q * G::TPW + local; };
  typename EN::TwRegs W;
  Store nx[PIPE ? RR : 1][E];
  if constexpr (PIPE) {
    EN::load_tw_regs(tw, t, W);
#pragma unroll
    for (int q = 0; q < RR; ++q) {
      const long long r0 = row_of(blockIdx.x, q);
      if ((int)blockIdx.x < groups && r0 < a.rows) {
        const Store *src = static_cast<const Store *>(a.in) + r0 * N + t;
#pragma unroll
        for (int e = 0; e < E; ++e) nx[q][e] = ld_stream(src + (unsigned)(T * e));
      }
    }
  }
  for (int it = blockIdx.x; it < groups; it += gridDim.x) {
    // opaque per group: the thread index (else every pass's LDS addresses are
    // hoisted into registers), the register twiddles and the hoisted filter
    // (else each FP16 pair is kept twice, pre-broadcast)
    unsigned tt = t;
    asm volatile("" : "+v"(tt));
    if constexpr (PIPE) {
#pragma unroll
      for (int p = 0; p < (int)(sizeof(W.w) / sizeof(W.w[0])); ++p)
#pragma unroll
        for (int e = 0; e < E; ++e) asm volatile("" : "+v"(W.w[p][e]));
    }
    if constexpr (kHoist) {
#pragma unroll
      for (int e = 0; e < E; ++e) asm volatile("" : "+v"(hf[e]));
    }
    Comp v[RR][E];
#pragma unroll
    for (int q = 0; q < RR; ++q) {
      const long long row = row_of(it, q);
      if (row < a.rows) {
        if constexpr (PIPE) {
#pragma unroll
          for (int e = 0; e < E; ++e) v[q][e] = M::decode(nx[q][e]);
        } else {
          const Store *src = static_cast<const Store *>(a.in) + row * N + tt;
#pragma unroll
          for (int e = 0; e < E; ++e) v[q][e] = M::load(src, (unsigned)(T * e));
        }
      } else {
#pragma unroll
        for (int e = 0; e < E; ++e) v[q][e] = Comp{};
      }
    }
    if constexpr (phasor) {
      const c32 *ph = static_cast<const c32 *>(a.phasor) + tt;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const c32 p = ph[T * e];
#pragma unroll
        for (int q = 0; q < RR; ++q) v[q][e] = mul_c32(v[q][e], p);
      }
    }
    if constexpr (PIPE) {
      const int nit = it + (int)gridDim.x;
#pragma unroll
      for (int q = 0; q < RR; ++q) {
        const long long nrow = nit < groups ? row_of(nit, q) : a.rows;
        if (nrow < a.rows) {
          const Store *src = static_cast<const Store *>(a.in) + nrow * N + tt;
#pragma unroll
          for (int e = 0; e < E; ++e) nx[q][e] = ld_stream(src + (unsigned)(T * e));
        }
      }
    }
    auto run = [&](auto cj) {
      if constexpr (PIPE) EN::template run_regs_rr<decltype(cj)::value, RR, NB>(v, buf, xch, tt, W);
      else EN::template run_rr<decltype(cj)::value, RR, NB>(v, buf, xch, tw, tt);
    };
    if constexpr (OP == OP_FWD) {
      run(std::false_type{});
    } else {
      if constexpr (OP == OP_COMPRESS) run(std::false_type{});
      // BFP fold at the inverse's load: conj(z . H) . 2^-log2N, or with the
      // conjugated filter conj(z . conj H) = conj(z) . H
      if (OP == OP_COMPRESS || f) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
          Filt h;
          if constexpr (kHoist) h = hf[e];
          else h = f[tt + T * e];
#pragma unroll
          for (int q = 0; q < RR; ++q)
            v[q][e] = conj_f ? pow2<LOG2N>(M::fmul(cconj(v[q][e]), h)) : conj_pow2<LOG2N>(M::fmul(v[q][e], h));
        }
      } else {
#pragma unroll
        for (int q = 0; q < RR; ++q)
#pragma unroll
          for (int e = 0; e < E; ++e) v[q][e] = conj_pow2<LOG2N>(v[q][e]);
      }
      run(std::true_type{});
    }
    unsigned bad = 0;
#pragma unroll
    for (int q = 0; q < RR; ++q) {
      const long long row = row_of(it, q);
      if (row < a.rows) {
        if constexpr (OUT32) {
          c32 *dst = static_cast<c32 *>(a.out) + row * N + tt;
#pragma unroll
          for (int e = 0; e < E; ++e) st_stream(dst + (unsigned)(T * e), to_c32(v[q][e]));
          if constexpr (ent) {
            // as in row_kernel: |I|^2 and |I|^2 ln |I|^2 in FP32, sums in FP64
#pragma unroll
            for (int e = 0; e < E; ++e) {
              const c32 z = to_c32(v[q][e]);
              const float p = z.x * z.x + z.y * z.y;
              es += p;
              eq += (double)p * (double)ln_pos(p);
            }
          }
        } else {
          Store *dst = static_cast<Store *>(a.out) + row * N + tt;
#pragma unroll
          for (int e = 0; e < E; ++e) M::store(dst, (unsigned)(T * e), v[q][e]);
        }
        if (a.flags & KF_CHECK_FINITE) {
#pragma unroll
          for (int e = 0; e < E; ++e) {
            c32 z = OUT32 ? to_c32(v[q][e]) : to_c32(M::round_store(v[q][e]));
            bad += finite_c(z) ? 0u : 1u;
          }
        }
      }
    }
    if (bad) atomicAdd(a.nonfinite, (unsigned long long)bad);
  }
  if constexpr (ent) {
    // fixed-order tree over the workgroup; one (S, Q) per workgroup, in the
    // exchange buffer once every thread has read its last exchange (no
    // LDS of its own: 16 B per thread more would cost resident workgroups)
    static_assert(sizeof(lds_all) >= 2 * G::WG * sizeof(double), "the reduction fits the exchange buffer");
    double *esh = reinterpret_cast<double *>(lds_all);
    __syncthreads();
    entropy_sums<G::WG>(a, es, eq, esh);
  }
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
// FP32; conj(X) H uses (Re X, Im X) and (-Im X, Re X).  The conjugated
// product is rounded once to FP16, and the exact 2^-12 shift of Eq. (1) is
// the scaled operand of the inverse's first pass.
template <int OP, int V, bool OUT32>
__global__ void __launch_bounds__(256) row_kernel_mfma(RowArgs a) {
  constexpr int N = 4096;
  constexpr bool naive = (V & V_NAIVE) != 0;
  constexpr bool conj_f = (V & V_CONJ) != 0;
  constexpr bool phasor = (V & V_PHASOR) != 0;
  __shared__ h2 lds[2][N];
  const Mfma4096 E(a.tw, threadIdx.x);
  // the filter is the same for every row: its 16 values per thread are
  // loaded once, ahead of the row loop, so no row waits on them
  const h2 *f = static_cast<const h2 *>(a.filter);
  h2 hf[16];
  if constexpr (OP != OP_FWD) {
    if (f) {
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int i = 0; i < 4; ++i) hf[4 * m + i] = f[E.pos(m, i)];
    }
  }
  for (long long row = blockIdx.x; row < a.rows; row += gridDim.x) {
  h2 x[16];
  c32 y[16];
  const h2 *src = static_cast<const h2 *>(a.in) + row * N;
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int i = 0; i < 4; ++i) x[4 * m + i] = ld_stream(src + E.pos(m, i));

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
      E.run<false>(x, y, lds[0], lds[1]);
    } else {
#pragma unroll
      for (int k = 0; k < 16; ++k) y[k] = h2_to_c32(x[k]);
    }
    // BFP fold: conj(z . H) (or conj(z) . H) here, 2^-12 in the next pass;
    // compression always carries a filter (checked by the C layer)
    if (OP == OP_COMPRESS || f) {
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const h2 h = hf[k];
        if constexpr (conj_f) {
          const h2 xa = c32_to_h2(c32{y[k].x, y[k].y}), xb = c32_to_h2(c32{-y[k].y, y[k].x});
          x[k] = c32_to_h2(c32{__builtin_amdgcn_fdot2(xa, h, 0.0f, false),
                               __builtin_amdgcn_fdot2(xb, h, 0.0f, false)});
        } else {
          const h2 xa = c32_to_h2(c32{y[k].x, -y[k].y}), xb = c32_to_h2(c32{y[k].y, y[k].x});
          x[k] = c32_to_h2(c32{__builtin_amdgcn_fdot2(xa, h, 0.0f, false),
                               -__builtin_amdgcn_fdot2(xb, h, 0.0f, false)});
        }
      }
    } else {
#pragma unroll
      for (int k = 0; k < 16; ++k) x[k] = c32_to_h2(cconj(y[k]));
    }
  }
  E.run<OP != OP_FWD && !naive>(x, y, lds[0], lds[1]);
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
      for (int i = 0; i < 4; ++i) st_stream(dst + E.pos(m, i), y[4 * m + i]);
  } else {
    h2 *dst = static_cast<h2 *>(a.out) + row * N;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int i = 0; i < 4; ++i) st_stream(dst + E.pos(m, i), c32_to_h2(y[4 * m + i]));
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
  if (a.grid_out) *a.grid_out = (int)grid;
  hipLaunchKernelGGL((row_kernel_mfma<OP, V, OUT32>), dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}
#endif

// Workgroups of `kernel` (WG threads) resident on one CU, by the occupancy
// calculator; at least 1.
template <class K>
static unsigned resident_per_cu(K kernel, int wg) {
  int b = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, kernel, wg, 0) != hipSuccess || b < 1) b = 1;
  return (unsigned)b;
}

// The image-entropy variants (V_ENT) without a grid of their own
// (a.resident_cus > 0): one round of the kernel's resident workgroups,
// looping over the row groups (4096 x 4096 with FP16 storage: 66 against
// 70-76 us for one workgroup per row pair); `occ` is the kernel's resident
// count per CU.
template <int V>
static unsigned image_grid(const RowArgs &a, unsigned grid, unsigned occ) {
  if constexpr ((V & V_ENT) != 0) {
    if (a.grid_limit <= 0 && a.resident_cus > 0) {
      const unsigned r = occ * (unsigned)a.resident_cus;
      if (grid > r) grid = r;
    }
  }
  return grid;
}

template <int LOG2N, int OP, int V, bool OUT32>
static hipError_t launch_vector(const RowArgs &a, hipStream_t s) {
  typedef Geometry<LOG2N> G;
  unsigned grid = (unsigned)((a.rows + G::TPW - 1) / G::TPW);
  if (a.grid_limit > 0 && grid > (unsigned)a.grid_limit) grid = (unsigned)a.grid_limit;
  if constexpr ((V & V_ENT) != 0) {
    static const unsigned occ = resident_per_cu(row_kernel<MODE, LOG2N, OP, V, OUT32, false>, G::WG);
    grid = image_grid<V>(a, grid, occ);
  }
  if (a.grid_out) *a.grid_out = (int)grid;
  if constexpr (Engine<MODE, LOG2N>::kTwRegs) {
    if (a.grid_limit > 0) {
      // pure FP16 at 4096 points: the pipelined kernel with one LDS buffer
      // (two barriers per exchange, 17 KiB: 5 workgroups per CU, as many as
      // its 88 VGPRs allow, against 4 with two buffers) measured 1.5%
      // faster on the 2048 x 4096 compression (17.6 against 17.9 us), with
      // the same bits
      constexpr bool kOneBuf = LOG2N == 12 && std::is_same<MODE, ModeFP16>::value && !OUT32 &&
                               (V & ~(V_CONJ | V_PHASOR)) == 0 && (!(V & V_PHASOR) || OP == OP_COMPRESS);
      if constexpr (kOneBuf)
        hipLaunchKernelGGL((row_kernel_rr<MODE, LOG2N, OP, V, OUT32, 1, 1, true>), dim3(grid), dim3(G::WG), 0, s, a);
      else
        hipLaunchKernelGGL((row_kernel<MODE, LOG2N, OP, V, OUT32, true>), dim3(grid), dim3(G::WG), 0, s, a);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((row_kernel<MODE, LOG2N, OP, V, OUT32, false>), dim3(grid), dim3(G::WG), 0, s, a);
  return hipGetLastError();
}

// The multi-row kernel for RR = a.rows_per_thread > 1, where it covers the
// variant (returns false otherwise).
template <int LOG2N, int OP, int V, bool OUT32>
static bool launch_rr(const RowArgs &a, hipStream_t s, hipError_t &err) {
  typedef Geometry<LOG2N> G;
  if constexpr ((V & ~(V_CONJ | V_PHASOR | V_ENT)) != 0 || ((V & V_PHASOR) && OP != OP_COMPRESS)) {
    return false;
  } else {
    constexpr int RR = 2;
    // LDS per buffer set; two workgroups must fit a CU (160 KiB), else no
    // multi-row kernel.  One buffer per row (two barriers per exchange)
    // except for the pipelined pure-FP16 form: with FP32 arithmetic the LDS
    // saved, twice the workgroups per CU, is worth more than the barrier
    // (FP16 storage / FP32 arithmetic at 4096 points: 60.0 against 64.7 us
    // for 4096 x 4096 compressions, and the autofocus image 72-75 against
    // 80-85 us)
    constexpr long kSet = (long)G::TPW * RR * G::LDS_N * sizeof(typename MODE::Lds);
    constexpr int NB = (Engine<MODE, LOG2N>::kTwRegs && 2 * kSet <= 80 * 1024) ? 2 : 1;
    if constexpr (kSet > 80 * 1024) {
      return false;
    } else {
      if (a.rows_per_thread != 2) return false;
      unsigned grid = (unsigned)((a.rows + G::TPW * RR - 1) / (G::TPW * RR));
      if (a.grid_limit > 0 && grid > (unsigned)a.grid_limit) grid = (unsigned)a.grid_limit;
      constexpr bool kPipe = Engine<MODE, LOG2N>::kTwRegs && NB == 2;
      if constexpr ((V & V_ENT) != 0) {
        static const unsigned occ =
            resident_per_cu(row_kernel_rr<MODE, LOG2N, OP, V, OUT32, RR, NB, false>, G::WG);
        grid = image_grid<V>(a, grid, occ);
      }
      if (a.grid_out) *a.grid_out = (int)grid;
      if (kPipe && a.grid_limit > 0)
        hipLaunchKernelGGL((row_kernel_rr<MODE, LOG2N, OP, V, OUT32, RR, 2, kPipe>), dim3(grid), dim3(G::WG), 0, s, a);
      else
        hipLaunchKernelGGL((row_kernel_rr<MODE, LOG2N, OP, V, OUT32, RR, NB, false>), dim3(grid), dim3(G::WG), 0, s, a);
      err = hipGetLastError();
      return true;
    }
  }
}

// The second radix plan (a.radix_plan == 1): the multi-row kernel with
// a.rows_per_thread rows, for the plain forward transform, the BFP inverse
// and the compression with a filter, its conjugate or a phasor (storage-type
// output); returns false where it does not apply (other variants, sizes with
// one plan, rows whose LDS would not leave two workgroups per CU).  The
// FP32-output image with its entropy sums stays on plan 0, which measured
// 76 against 81 us at 4096 x 4096.
template <int LOG2N, int OP, int V, bool OUT32>
static bool launch_plan1(const RowArgs &a, hipStream_t s, hipError_t &err) {
  if constexpr (!has_second_plan(LOG2N) || OUT32 || (V & ~(V_CONJ | V_PHASOR)) != 0 ||
                ((V & V_PHASOR) && OP != OP_COMPRESS)) {
    return false;
  } else {
    typedef Geometry<LOG2N, 1> G;
    constexpr long kRow = (long)G::TPW * G::LDS_N * sizeof(typename MODE::Lds);
    if (a.radix_plan != 1 || !a.tw_alt) return false;
    RowArgs b = a;
    b.tw = a.tw_alt;
    auto go = [&](auto rr) {
      constexpr int RR = decltype(rr)::value;
      constexpr int NB = 2 * RR * kRow <= 80 * 1024 ? 2 : 1;
      unsigned grid = (unsigned)((a.rows + G::TPW * RR - 1) / (G::TPW * RR));
      if (a.grid_limit > 0 && grid > (unsigned)a.grid_limit) grid = (unsigned)a.grid_limit;
      if (a.grid_out) *a.grid_out = (int)grid;
      hipLaunchKernelGGL((row_kernel_rr<MODE, LOG2N, OP, V, OUT32, RR, NB, false, 1>), dim3(grid),
                         dim3(G::WG), 0, s, b);
      err = hipGetLastError();
    };
    if constexpr (2 * kRow <= 80 * 1024) {
      if (a.rows_per_thread == 2) {
        go(std::integral_constant<int, 2>{});
        return true;
      }
    }
    if constexpr (kRow > 80 * 1024) {
      return false;
    } else {
      go(std::integral_constant<int, 1>{});
      return true;
    }
  }
}

// a.tw is the plan's table.  Where a matrix-core engine exists, that table
// starts with the matrix-core operands and the vector engine's twiddles
// follow at kMfmaTableBytes: variants without a matrix-core kernel run on
// the vector engine whatever the plan's engine, with its table.
template <int LOG2N, int OP, int V, bool OUT32>
static hipError_t launch_one(const RowArgs &a, hipStream_t s) {
  if (a.rows <= 0) return hipSuccess;
  {
    hipError_t err = hipSuccess;
    if (launch_plan1<LOG2N, OP, V, OUT32>(a, s, err)) return err;
  }
#if BFP_MODE_ID == 3
  if constexpr (LOG2N == 12) {
    if constexpr ((V & (V_TRANS | V_ADAPT | V_RAMP | V_POST)) == 0) {
      if (a.engine == 0) return launch_mfma<OP, V, OUT32>(a, s);
    }
    RowArgs b = a;
    b.tw = static_cast<const unsigned char *>(a.tw) + kMfmaTableBytes;
    hipError_t err = hipSuccess;
    if (launch_rr<LOG2N, OP, V, OUT32>(b, s, err)) return err;
    return launch_vector<LOG2N, OP, V, OUT32>(b, s);
  }
#endif
  hipError_t err = hipSuccess;
  if (launch_rr<LOG2N, OP, V, OUT32>(a, s, err)) return err;
  return launch_vector<LOG2N, OP, V, OUT32>(a, s);
}

// Variant selection; combinations outside this table are rejected by the
// C layer before launch.
template <int LOG2N>
static hipError_t launch_size(int op, bool out32, const RowArgs &a, hipStream_t s) {
  const bool naive = (a.flags & KF_NAIVE) != 0;
  const bool conj = (a.flags & KF_CONJ_FILTER) != 0;
  const bool ph = a.phasor != nullptr;
  const bool post = (a.flags & KF_POST_PHASOR) != 0;
  switch (op) {
    case OP_FWD:
      return out32 ? launch_one<LOG2N, OP_FWD, V_PLAIN, true>(a, s)
                   : launch_one<LOG2N, OP_FWD, V_PLAIN, false>(a, s);
    case OP_INV:
      if (a.flags & KF_ADAPT) {
        if (out32 || ph || naive || conj || !a.row_exp) return hipErrorInvalidValue;
#if BFP_MODE_ID >= 1 && BFP_MODE_ID <= 3
        return launch_one<LOG2N, OP_INV, V_ADAPT, false>(a, s);
#else
        return hipErrorInvalidValue;
#endif
      }
      if (out32 || ph || (naive && conj)) return hipErrorInvalidValue;
      if (naive) return launch_one<LOG2N, OP_INV, V_NAIVE, false>(a, s);
      if (conj) return launch_one<LOG2N, OP_INV, V_CONJ, false>(a, s);
      return launch_one<LOG2N, OP_INV, V_PLAIN, false>(a, s);
    case OP_COMPRESS:
      if (a.flags & KF_RAMP) {
        if (out32 || ph || naive || conj || a.ent_partial || (a.flags & (KF_TRANSPOSED | KF_ADAPT)) ||
            !a.shift)
          return hipErrorInvalidValue;
        return launch_one<LOG2N, OP_COMPRESS, V_RAMP, false>(a, s);
      }
      if (a.flags & KF_ADAPT) {
        if (out32 || ph || naive || conj || a.ent_partial || (a.flags & KF_TRANSPOSED) || !a.row_exp)
          return hipErrorInvalidValue;
#if BFP_MODE_ID >= 1 && BFP_MODE_ID <= 3
        return launch_one<LOG2N, OP_COMPRESS, V_ADAPT, false>(a, s);
#else
        return hipErrorInvalidValue;
#endif
      }
      if (a.flags & KF_TRANSPOSED) {
        if (naive || conj || ph || out32) return hipErrorInvalidValue;
        return launch_one<LOG2N, OP_COMPRESS, V_TRANS, false>(a, s);
      }
      if (post && !ph) return hipErrorInvalidValue;
      if (naive && (conj || ph)) return hipErrorInvalidValue;
      if (naive) return out32 ? hipErrorInvalidValue : launch_one<LOG2N, OP_COMPRESS, V_NAIVE, false>(a, s);
      if (a.ent_partial) {
        if (!out32 || conj || post) return hipErrorInvalidValue;
#if BFP_MODE_ID == 0 || BFP_MODE_ID == 2
        return ph ? launch_one<LOG2N, OP_COMPRESS, V_PHASOR | V_ENT, true>(a, s)
                  : launch_one<LOG2N, OP_COMPRESS, V_ENT, true>(a, s);
#else
        return hipErrorInvalidValue;
#endif
      }
      if (ph && (conj || post)) {
        // phase-corrected compression with the conjugated filter, and the
        // adjoints (output phasor) of both filter choices
        if (out32) return hipErrorInvalidValue;
        if (!post) return launch_one<LOG2N, OP_COMPRESS, V_PHASOR | V_CONJ, false>(a, s);
        return conj ? launch_one<LOG2N, OP_COMPRESS, V_PHASOR | V_POST | V_CONJ, false>(a, s)
                    : launch_one<LOG2N, OP_COMPRESS, V_PHASOR | V_POST, false>(a, s);
      }
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
    case 3: return launch_size<3>(op, out32, a, s);
    case 4: return launch_size<4>(op, out32, a, s);
    case 5: return launch_size<5>(op, out32, a, s);
    case 6: return launch_size<6>(op, out32, a, s);
    case 7: return launch_size<7>(op, out32, a, s);
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
