// Single-pass, LDS-resident Stockham FFT engine for gfx950.
//
// One transform of N = 2^LOG2N points is processed by T = N / E threads that
// each hold E complex values in registers.  N is factored into radix passes
// (16 x 16 x 16 for N = 4096).  Pass p with radix R and span NS (the length of
// the sub-transforms already combined) applies, to each of the N / R
// butterflies j, the twiddles W_{NS R}^{(j mod NS) r} (r = 1..R-1), a
// constant-twiddle DFT_R in registers, and writes the R results to positions
// (j / NS) NS R + (j mod NS) + r NS of the LDS buffer: the self-sorting
// (Stockham) order, so the final pass leaves X[k] in natural order.  Every
// pass reads thread t's inputs from positions t + T e (e = 0..E-1), so the
// first pass reads HBM and the last pass writes HBM with unit stride across
// the threads of a wavefront (coalesced), and only the interior passes touch
// LDS.  Each exchange has its own padded layout (Pad) that keeps both the
// scattered Stockham writes and the reads free of bank conflicts.
//
// Twiddles come from a per-plan table in HBM (L2/L1-resident after the first
// wavefronts): pass p owns NS_p x R_p entries W_{NS R}^{m r}, m < NS, r < R,
// built on the host in FP64 and rounded once to the mode's twiddle type.
#pragma once

#include "fft_device.hpp"

namespace bfp {

// Radix plans per size: E values per thread, up to 4 passes.  Plan 0 (the
// default) takes radix-16 passes where it can; below 256 points a transform
// takes 1 (N <= 16) to 8 threads and a workgroup holds 256 / T transforms,
// and N = 8 and 16 need no exchange at all.  Plan 1 is the second candidate
// the autotuner times: radix-8 passes with 8 values per thread (half the
// registers, one pass more) from 32 to 4096 points, and at 512, 8192 and
// 16384 points another radix-16 order (16 16 2; 16 16 8 4; 4 16 16 16).
// N <= 16 has one plan (a single in-register DFT): plan 1 equals plan 0.
template <int LOG2N, int PLAN = 0> struct Shape;
template <> struct Shape<3, 0>  { static constexpr int E = 8,  P = 1, R0 = 8,  R1 = 1,  R2 = 1, R3 = 1; };
template <> struct Shape<4, 0>  { static constexpr int E = 16, P = 1, R0 = 16, R1 = 1,  R2 = 1, R3 = 1; };
template <> struct Shape<5, 0>  { static constexpr int E = 16, P = 2, R0 = 16, R1 = 2,  R2 = 1, R3 = 1; };
template <> struct Shape<6, 0>  { static constexpr int E = 16, P = 2, R0 = 16, R1 = 4,  R2 = 1, R3 = 1; };
template <> struct Shape<7, 0>  { static constexpr int E = 16, P = 2, R0 = 16, R1 = 8,  R2 = 1, R3 = 1; };
template <> struct Shape<8, 0>  { static constexpr int E = 16, P = 2, R0 = 16, R1 = 16, R2 = 1, R3 = 1; };
template <> struct Shape<9, 0>  { static constexpr int E = 8,  P = 3, R0 = 8,  R1 = 8,  R2 = 8, R3 = 1; };
template <> struct Shape<10, 0> { static constexpr int E = 16, P = 3, R0 = 16, R1 = 16, R2 = 4, R3 = 1; };
template <> struct Shape<11, 0> { static constexpr int E = 16, P = 3, R0 = 16, R1 = 16, R2 = 8, R3 = 1; };
template <> struct Shape<12, 0> { static constexpr int E = 16, P = 3, R0 = 16, R1 = 16, R2 = 16, R3 = 1; };
template <> struct Shape<13, 0> { static constexpr int E = 16, P = 4, R0 = 16, R1 = 16, R2 = 16, R3 = 2; };
template <> struct Shape<14, 0> { static constexpr int E = 16, P = 4, R0 = 16, R1 = 16, R2 = 16, R3 = 4; };
template <> struct Shape<3, 1> : Shape<3, 0> {};
template <> struct Shape<4, 1> : Shape<4, 0> {};
template <> struct Shape<5, 1>  { static constexpr int E = 8,  P = 2, R0 = 8,  R1 = 4,  R2 = 1, R3 = 1; };
template <> struct Shape<6, 1>  { static constexpr int E = 8,  P = 2, R0 = 8,  R1 = 8,  R2 = 1, R3 = 1; };
template <> struct Shape<7, 1>  { static constexpr int E = 8,  P = 3, R0 = 8,  R1 = 8,  R2 = 2, R3 = 1; };
template <> struct Shape<8, 1>  { static constexpr int E = 8,  P = 3, R0 = 8,  R1 = 8,  R2 = 4, R3 = 1; };
template <> struct Shape<9, 1>  { static constexpr int E = 16, P = 3, R0 = 16, R1 = 16, R2 = 2, R3 = 1; };
template <> struct Shape<10, 1> { static constexpr int E = 8,  P = 4, R0 = 8,  R1 = 8,  R2 = 8, R3 = 2; };
template <> struct Shape<11, 1> { static constexpr int E = 8,  P = 4, R0 = 8,  R1 = 8,  R2 = 8, R3 = 4; };
template <> struct Shape<12, 1> { static constexpr int E = 8,  P = 4, R0 = 8,  R1 = 8,  R2 = 8, R3 = 8; };
template <> struct Shape<13, 1> { static constexpr int E = 16, P = 4, R0 = 16, R1 = 16, R2 = 8, R3 = 4; };
template <> struct Shape<14, 1> { static constexpr int E = 16, P = 4, R0 = 4,  R1 = 16, R2 = 16, R3 = 16; };
// whether a size has a second plan distinct from the first
constexpr bool has_second_plan(int log2n) { return log2n >= 5 && log2n <= 14; }

// LDS layout of exchange X (written by pass X, read by pass X + 1): element
// i sits at slot i + C (i >> S).  Each half-wavefront's 32 lanes then hit 32
// different banks both in the Stockham scatter of pass X and in the reads at
// t + T e of pass X + 1 (checked by simulation for every size and plan; the
// bank conflict counter confirms 32 banks per half-wavefront): plan 0 after a
// span-1 pass, (C, S) = (1, 5); after a span-16 radix-16 pass, (4, 6) ((8, 6)
// after span 8 at N = 512); after a span-256 pass the scatter is
// conflict-free unpadded (C = 0).  N = 256 (four transforms per wavefront)
// keeps one pad slot per 16.  One pad slot per 16 in every exchange made
// each read 2-way.  Below 256 points (at most 8 threads per transform) the
// single exchange is unpadded.  Plan 1: (1, 5) after the first pass, then
// (4, 5) after a second radix-8 pass or (2, 5) after a second radix-16 or
// radix-4 one, unpadded after the third; from 32 to 128 points (1, 3),
// (1, 2) and (2, 3), which leave the 2-way conflicts of 4 to 16 threads per
// transform.
template <int LOG2N, int X, int PLAN = 0>
struct Pad {
  static constexpr int C0 = LOG2N < 8 ? 0 : LOG2N == 8 ? 1 : X == 0 ? 1 : X == 1 ? (LOG2N == 9 ? 8 : 4) : 0;
  static constexpr int S0 = LOG2N == 8 ? 4 : X == 0 ? 5 : 6;
  static constexpr int C1 = LOG2N == 5 ? 0
                          : LOG2N == 6 ? 1
                          : LOG2N == 7 ? (X == 0 ? 1 : 2)
                          : X == 0 ? 1
                          : X == 1 ? ((LOG2N == 9 || LOG2N >= 13) ? 2 : 4)
                          : 0;
  static constexpr int S1 = LOG2N == 6 ? 3 : LOG2N == 7 ? (X == 0 ? 2 : 3) : 5;
  static constexpr int C = (PLAN == 0 || LOG2N <= 4) ? C0 : C1;
  static constexpr int S = (PLAN == 0 || LOG2N <= 4) ? S0 : S1;
  static __host__ __device__ constexpr int at(int i) { return i + C * (i >> S); }
};

template <int LOG2N, int PLAN = 0>
struct Geometry {
  typedef Shape<LOG2N, PLAN> S;
  static constexpr int N = 1 << LOG2N;
  static constexpr int E = S::E;
  static constexpr int T = N / E;                    // threads per transform
  static constexpr int WG = T < 256 ? 256 : T;       // threads per workgroup
  static constexpr int TPW = WG / T;                 // transforms per workgroup
  // padded LDS elements: the largest exchange layout, at least N + N / 16
  static constexpr int LDS_N = [] {
    int m = N + N / 16;
    for (int x = 0; x + 1 < S::P; ++x) {
      const int slots = (x == 0 ? Pad<LOG2N, 0, PLAN>::at(N - 1)
                         : x == 1 ? Pad<LOG2N, 1, PLAN>::at(N - 1) : Pad<LOG2N, 2, PLAN>::at(N - 1)) + 1;
      m = slots > m ? slots : m;
    }
    return m;
  }();
  static constexpr int radix(int p) {
    return p == 0 ? S::R0 : p == 1 ? S::R1 : p == 2 ? S::R2 : S::R3;
  }
  static constexpr int span(int p) {  // NS of pass p
    int ns = 1;
    for (int q = 0; q < p; ++q) ns *= radix(q);
    return ns;
  }
  // offset of pass p's twiddle block in the plan table (passes with NS > 1)
  static constexpr int tw_offset(int p) {
    int off = 0;
    for (int q = 1; q < p; ++q) off += span(q) * radix(q);
    return off;
  }
  static constexpr int tw_entries() { return tw_offset(S::P); }
};

// Offset of element d in a layout, relative to a base whose position is a
// multiple of 2^S or whose low bits never carry into bit S with d (see
// pad_splits): d + C (d >> S).
template <class P>
__host__ __device__ constexpr int pad_off(int d) { return d + P::C * (d >> P::S); }

// Slot of element t + T e in layout P.  T is a multiple of 2^S (or C = 0),
// so P(t + T e) = P(t) + pad_off(T e): one base register per thread and a
// compile-time offset per element.
template <class P, int T>
__device__ __forceinline__ constexpr int lds_slot(int tpad, int e) {
  static_assert(P::C == 0 || T % (1 << P::S) == 0, "the pad split needs T to be a multiple of 2^S");
  return tpad + pad_off<P>(T * e);
}

// Slot of butterfly j's first output in a Stockham pass of radix R and span
// NS: position (j / NS) NS R + j mod NS (unsigned: shifts, no signed
// division fix-up).
template <class P, int R, int NS>
__device__ __forceinline__ int stockham_base(unsigned j) {
  return P::at((int)((j / NS) * NS * R + (j & (NS - 1))));
}

// True when, for every butterfly j of an N-point pass, P(base_j + r NS) =
// P(base_j) + pad_off(r NS): then the R scattered writes of a butterfly use
// one address register and compile-time offsets.
template <class P, int N, int R, int NS>
constexpr bool pad_splits() {
  for (int j = 0; j < N / R; ++j) {
    const int base = (j / NS) * NS * R + (j % NS);
    for (int r = 0; r < R; ++r)
      if (P::at(base + r * NS) != P::at(base) + pad_off<P>(r * NS)) return false;
  }
  return true;
}

// Elements t + T e of one row, raw (storage type).  With one transform per
// workgroup the row's base is uniform: each group of four elements takes a
// base in scalar registers and the immediates 0, T, 2T, 3T elements, so all
// sixteen accesses share one 32-bit lane offset (ti, which must be < T).
// STREAM: nontemporal (row data read or written once); otherwise cached
// (tables every row reads, such as a filter or a phasor: row = 0).
// (The pipelined row kernel keeps per-lane pointers: there the compiler
// turns this form into 64-bit address arithmetic per store.)
template <class G, bool STREAM = true, class X>
__device__ __forceinline__ void load_row(X (&x)[G::E], const void *base, long long row, unsigned ti) {
  static_assert(G::E % 4 == 0, "elements go in groups of four");
  const X *src = static_cast<const X *>(base) + row * G::N;
#pragma unroll
  for (int e = 0; e < G::E; e += 4) {
    const X *grp = src + G::T * e;
    if constexpr (G::TPW == 1) asm volatile("" : "+s"(grp));
    const global_ptr<const X> g = (global_ptr<const X>)grp;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if constexpr (STREAM) x[e + k] = ld_stream_g(g + (ti + (unsigned)(G::T * k)));
      else x[e + k] = ld_cached_g(g + (ti + (unsigned)(G::T * k)));
    }
  }
}
template <class G, class X>
__device__ __forceinline__ void store_row(void *base, long long row, unsigned ti, const X (&x)[G::E]) {
  static_assert(G::E % 4 == 0, "elements go in groups of four");
  X *dst = static_cast<X *>(base) + row * G::N;
#pragma unroll
  for (int e = 0; e < G::E; e += 4) {
    X *grp = dst + G::T * e;
    if constexpr (G::TPW == 1) asm volatile("" : "+s"(grp));
    const global_ptr<X> g = (global_ptr<X>)grp;
#pragma unroll
    for (int k = 0; k < 4; ++k) st_stream_g(g + (ti + (unsigned)(G::T * k)), x[e + k]);
  }
}

template <class M, int LOG2N, int PLAN = 0>
struct Engine {
  typedef Geometry<LOG2N, PLAN> G;
  typedef typename M::Comp Comp;
  typedef typename M::Lds Lds;
  typedef typename M::Tw Tw;
  static constexpr int E = G::E;
  static constexpr int T = G::T;
  // Conjugated outputs (CJ) are folded into the last pass when it ends in a
  // DFT4 stage (radix 4 or 16), whose outputs are sums of sums: conj of a
  // sum is then exactly the sum of conjugates.  A radix-2 or radix-8 last
  // pass adds products, which the compiler may contract into FMAs
  // differently once conjugates sit in between, so there the conjugate
  // follows the transform and every kernel rounds alike.
  static constexpr int kLastRadix = G::radix(G::S::P - 1);
  static constexpr bool kFoldConj = kLastRadix == 4 || kLastRadix == 16;

  // Twiddle rows of pass PASS for this thread: butterfly b uses row
  // (t + T b) mod NS, entries r = 0..R-1, kept at w[b R + r].
  template <int PASS>
  static __device__ __forceinline__ void load_tw(const Tw *__restrict__ tw, int t, Tw (&w)[E]) {
    if constexpr (PASS > 0 && PASS < G::S::P) {
      constexpr int R = G::radix(PASS);
      constexpr int NS = G::span(PASS);
      constexpr int B = E / R;
      const Tw *twp = tw + G::tw_offset(PASS);
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const Tw *row = twp + ((t + T * b) & (NS - 1)) * R;
#pragma unroll
        for (int r = 0; r < R; ++r) w[b * R + r] = row[r];
      }
    }
  }

  // One Stockham pass.  On entry v[e] holds this thread's inputs (pass 0)
  // or nothing (later passes, which read LDS), and w this pass's twiddle
  // rows; the next pass's rows are loaded into w as soon as this pass has
  // consumed its own, so their latency overlaps the butterflies and the LDS
  // exchange.  On exit v[e] holds the outputs (last pass) or the outputs
  // have been written to LDS.
  template <int PASS, bool PREFETCH = true, bool CJ = false>
  static __device__ __forceinline__ void pass(Comp (&v)[E], Lds *lds, const Tw *__restrict__ tw,
                                              int t, Tw (&w)[E]) {
    constexpr int R = G::radix(PASS);
    constexpr int NS = G::span(PASS);
    constexpr int B = E / R;
    constexpr bool LAST = (PASS == G::S::P - 1);
    if constexpr (PASS > 0) {
      typedef Pad<LOG2N, PASS - 1, PLAN> In;
      Lds raw[E];
      const int tp = In::at(t);
#pragma unroll
      for (int e = 0; e < E; ++e) raw[e] = lds[lds_slot<In, T>(tp, e)];
#pragma unroll
      for (int b = 0; b < B; ++b) {
        v[b] = M::from_lds(raw[b]);
#pragma unroll
        for (int r = 1; r < R; ++r) v[b + B * r] = M::twiddle(raw[b + B * r], w[b * R + r]);
      }
    }
    if constexpr (PREFETCH) load_tw<PASS + 1>(tw, t, w);
#pragma unroll
    for (int b = 0; b < B; ++b) {
      Comp u[R];
#pragma unroll
      for (int r = 0; r < R; ++r) u[r] = v[b + B * r];
      dft<R, CJ && LAST && kFoldConj>(u);
#pragma unroll
      for (int r = 0; r < R; ++r) v[b + B * r] = u[r];
    }
    if constexpr (!LAST) {
      typedef Pad<LOG2N, PASS, PLAN> Out;
      static_assert(pad_splits<Out, G::N, R, NS>(), "padded offsets of a butterfly must not straddle a pad");
      __syncthreads();  // all reads of the previous contents are done
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const int pbase = stockham_base<Out, R, NS>((unsigned)t + T * b);
        // Out(base + r NS) = Out(base) + pad_off(r NS) (see pad_splits)
#pragma unroll
        for (int r = 0; r < R; ++r) lds[pbase + pad_off<Out>(r * NS)] = M::to_lds(v[b + B * r]);
      }
      __syncthreads();
    }
  }

  // Full forward transform: v[e] = x[t + T e] in, v[e] = X[t + T e] out
  // (CJ: conj(X[t + T e]), see kFoldConj).
  template <bool CJ = false>
  static __device__ __forceinline__ void run(Comp (&v)[E], Lds *lds, const Tw *__restrict__ tw,
                                             int t) {
    Tw w[E];
    load_tw<1>(tw, t, w);
    pass<0, true, CJ>(v, lds, tw, t, w);
    if constexpr (G::S::P > 1) pass<1, true, CJ>(v, lds, tw, t, w);
    if constexpr (G::S::P > 2) pass<2, true, CJ>(v, lds, tw, t, w);
    if constexpr (G::S::P > 3) pass<3, true, CJ>(v, lds, tw, t, w);
    conj_unfolded<CJ>(v);
  }

  template <bool CJ>
  static __device__ __forceinline__ void conj_unfolded(Comp (&v)[E]) {
    if constexpr (CJ && !kFoldConj) {
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = conj_store(v[e]);
    }
  }

  // ---- twiddles held in registers for a whole persistent kernel ----
  // The rows of every pass (E values each), loaded once; a row then issues
  // no global loads but its own data, so a load of the next row can stay in
  // flight across the whole transform without any wait on the
  // vector-memory counter catching it.  Used where the rows fit the
  // register budget next to the data: packed FP16 data and twiddles and at
  // most 3 passes.
  static constexpr bool kTwRegs = sizeof(Tw) == 4 && sizeof(Comp) == 4 && G::S::P <= 3;
  struct TwRegs {
    Tw w[G::S::P > 1 ? G::S::P - 1 : 1][E];
  };
  static __device__ __forceinline__ void load_tw_regs(const Tw *__restrict__ tw, int t, TwRegs &W) {
    if constexpr (G::S::P > 1) load_tw<1>(tw, t, W.w[0]);
    if constexpr (G::S::P > 2) load_tw<2>(tw, t, W.w[1]);
  }
  // One pass with two alternating LDS buffers: exchange x (a count kept by
  // the caller across passes, transforms and rows, uniform in the
  // workgroup) writes buf[x & 1] and the next pass reads it back.  The
  // previous reads of buf[x & 1] belong to the gather after exchange x - 2,
  // which every wave finished before reaching the barrier of exchange x - 1,
  // so one barrier per exchange (after the writes) orders everything.
  template <int PASS, bool CJ = false>
  static __device__ __forceinline__ void pass_db(Comp (&v)[E], Lds *const (&buf)[2], unsigned &x,
                                                 int t, const Tw (&w)[E]) {
    constexpr int R = G::radix(PASS);
    constexpr int NS = G::span(PASS);
    constexpr int B = E / R;
    constexpr bool LAST = (PASS == G::S::P - 1);
    if constexpr (PASS > 0) {
      const Lds *rd = buf[(x - 1) & 1];
      typedef Pad<LOG2N, PASS - 1, PLAN> In;
      Lds raw[E];
      const int tp = In::at(t);
#pragma unroll
      for (int e = 0; e < E; ++e) raw[e] = rd[lds_slot<In, T>(tp, e)];
#pragma unroll
      for (int b = 0; b < B; ++b) {
        v[b] = M::from_lds(raw[b]);
#pragma unroll
        for (int r = 1; r < R; ++r) v[b + B * r] = M::twiddle(raw[b + B * r], w[b * R + r]);
      }
    }
#pragma unroll
    for (int b = 0; b < B; ++b) {
      Comp u[R];
#pragma unroll
      for (int r = 0; r < R; ++r) u[r] = v[b + B * r];
      dft<R, CJ && LAST && kFoldConj>(u);
#pragma unroll
      for (int r = 0; r < R; ++r) v[b + B * r] = u[r];
    }
    if constexpr (!LAST) {
      typedef Pad<LOG2N, PASS, PLAN> Out;
      static_assert(pad_splits<Out, G::N, R, NS>(), "padded offsets of a butterfly must not straddle a pad");
      Lds *wr = buf[x & 1];
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const int pbase = stockham_base<Out, R, NS>((unsigned)t + T * b);
#pragma unroll
        for (int r = 0; r < R; ++r) wr[pbase + pad_off<Out>(r * NS)] = M::to_lds(v[b + B * r]);
      }
      __syncthreads();
      ++x;
    }
  }

  // ---- several rows per thread ----
  // RR independent transforms (rows) per thread: every pass reads, twiddles
  // and butterflies all RR rows before the next exchange, so the rows share
  // the twiddle registers and one barrier per exchange, and one row's LDS
  // latency is covered by the other rows' arithmetic.  Row r of a buffer
  // sits at buf[b] + r LDS_N.  NB = 2: buffers alternate as in pass_db (one
  // barrier per exchange); NB = 1: one buffer, a barrier before its writes
  // too.  MID() runs between the twiddle products and the butterflies (the
  // next pass's twiddle loads, where twiddles come from memory).
  template <int PASS, bool CJ, int RR, int NB, class Mid>
  static __device__ __forceinline__ void pass_rr(Comp (&v)[RR][E], Lds *const (&buf)[2], unsigned &x,
                                                 int t, const Tw (&w)[E], Mid mid) {
    constexpr int R = G::radix(PASS);
    constexpr int NS = G::span(PASS);
    constexpr int B = E / R;
    constexpr bool LAST = (PASS == G::S::P - 1);
    if constexpr (PASS > 0) {
      const Lds *rd = buf[NB == 2 ? ((x - 1) & 1) : 0];
      typedef Pad<LOG2N, PASS - 1, PLAN> In;
      const int tp = In::at(t);
#pragma unroll
      for (int q = 0; q < RR; ++q) {
        Lds raw[E];
#pragma unroll
        for (int e = 0; e < E; ++e) raw[e] = rd[q * G::LDS_N + lds_slot<In, T>(tp, e)];
#pragma unroll
        for (int b = 0; b < B; ++b) {
          v[q][b] = M::from_lds(raw[b]);
#pragma unroll
          for (int r = 1; r < R; ++r) v[q][b + B * r] = M::twiddle(raw[b + B * r], w[b * R + r]);
        }
      }
    }
    mid();
#pragma unroll
    for (int q = 0; q < RR; ++q) {
#pragma unroll
      for (int b = 0; b < B; ++b) {
        Comp u[R];
#pragma unroll
        for (int r = 0; r < R; ++r) u[r] = v[q][b + B * r];
        dft<R, CJ && LAST && kFoldConj>(u);
#pragma unroll
        for (int r = 0; r < R; ++r) v[q][b + B * r] = u[r];
      }
    }
    if constexpr (!LAST) {
      typedef Pad<LOG2N, PASS, PLAN> Out;
      static_assert(pad_splits<Out, G::N, R, NS>(), "padded offsets of a butterfly must not straddle a pad");
      if constexpr (NB == 1) __syncthreads();  // the reads of the previous exchange are done
      Lds *wr = buf[NB == 2 ? (x & 1) : 0];
#pragma unroll
      for (int q = 0; q < RR; ++q) {
#pragma unroll
        for (int b = 0; b < B; ++b) {
          const int pbase = stockham_base<Out, R, NS>((unsigned)t + T * b);
#pragma unroll
          for (int r = 0; r < R; ++r)
            wr[q * G::LDS_N + pbase + pad_off<Out>(r * NS)] = M::to_lds(v[q][b + B * r]);
        }
      }
      __syncthreads();
      ++x;
    }
  }

  template <bool CJ, int RR>
  static __device__ __forceinline__ void conj_unfolded_rr(Comp (&v)[RR][E]) {
    if constexpr (CJ && !kFoldConj) {
#pragma unroll
      for (int q = 0; q < RR; ++q)
#pragma unroll
        for (int e = 0; e < E; ++e) v[q][e] = conj_store(v[q][e]);
    }
  }

  // RR rows with register twiddles, NB buffers per row (2: one barrier per
  // exchange; 1: two).
  template <bool CJ, int RR, int NB = 2>
  static __device__ __forceinline__ void run_regs_rr(Comp (&v)[RR][E], Lds *const (&buf)[2], unsigned &x,
                                                     int t, TwRegs &W) {
    static_assert(kTwRegs, "register twiddles need packed FP16 data and twiddles and at most 3 passes");
    auto none = [] {};
    pass_rr<0, CJ, RR, NB>(v, buf, x, t, W.w[0], none);
    if constexpr (G::S::P > 1) pass_rr<1, CJ, RR, NB>(v, buf, x, t, W.w[0], none);
    if constexpr (G::S::P > 2) pass_rr<2, CJ, RR, NB>(v, buf, x, t, W.w[1], none);
    conj_unfolded_rr<CJ>(v);
  }

  // RR rows with twiddles loaded from the plan's table one pass ahead.
  template <bool CJ, int RR, int NB>
  static __device__ __forceinline__ void run_rr(Comp (&v)[RR][E], Lds *const (&buf)[2], unsigned &x,
                                                const Tw *__restrict__ tw, int t) {
    Tw w[E];
    load_tw<1>(tw, t, w);
    pass_rr<0, CJ, RR, NB>(v, buf, x, t, w, [] {});
    if constexpr (G::S::P > 1) pass_rr<1, CJ, RR, NB>(v, buf, x, t, w, [&] { load_tw<2>(tw, t, w); });
    if constexpr (G::S::P > 2) pass_rr<2, CJ, RR, NB>(v, buf, x, t, w, [&] { load_tw<3>(tw, t, w); });
    if constexpr (G::S::P > 3) pass_rr<3, CJ, RR, NB>(v, buf, x, t, w, [] {});
    conj_unfolded_rr<CJ>(v);
  }

  // Forward transform with register twiddles and two LDS buffers (CJ as in
  // run).
  template <bool CJ = false>
  static __device__ __forceinline__ void run_regs(Comp (&v)[E], Lds *const (&buf)[2], unsigned &x,
                                                  int t, TwRegs &W) {
    static_assert(kTwRegs, "register twiddles need packed FP16 data and twiddles and at most 3 passes");
    pass_db<0, CJ>(v, buf, x, t, W.w[0]);
    if constexpr (G::S::P > 1) pass_db<1, CJ>(v, buf, x, t, W.w[0]);
    if constexpr (G::S::P > 2) pass_db<2, CJ>(v, buf, x, t, W.w[1]);
    conj_unfolded<CJ>(v);
  }
};

}  // namespace bfp
