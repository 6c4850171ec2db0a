// Differentiable azimuth compression for entropy autofocus.
//
// Forward (done by the row kernels): z[r][m] = rc_t[r][m] exp(i phi_m),
// I = A(z) with A(v) = IDFT(DFT(v) . H_a) per range bin r.
// Image entropy: E = -sum p ln p, p = |I|^2 / S, S = sum |I|^2; computed here
// as E = ln S - Q / S with Q = sum |I|^2 ln |I|^2 (0 ln 0 = 0).
// Gradient of a real loss L with respect to I as a real pair
// (dL/dRe I + i dL/dIm I): for L = E it is G_I = -(2/S)(ln p + E) I.
// Adjoint: A^H = IDFT . diag(conj H_a) . DFT (the same BFP chain with the
// conjugated filter), so G_z = A^H(G_I), and since dz/dphi_m = i z,
// dL/dphi_m = sum_r Im(G_z[r][m] conj(z[r][m])).
//
// phase_grad_kernel fuses, per range row: (optionally) forming G_I from the
// image and the entropy statistics, the adjoint chain in FP32, the
// re-formation of z from the FP16/FP32 range-compressed data and the phasor,
// and the per-pulse accumulation of Im(G_z conj z).  Each workgroup
// accumulates its rows in registers and writes one partial row; a second
// kernel sums the partial rows in a fixed order (deterministic).
#include <mutex>

#include "fft_engine.hpp"
#include "internal.hpp"

namespace bfp {

// ------------------------------------------------------------- entropy ----
constexpr int ENT_BLOCKS = 1024;

__global__ void __launch_bounds__(256) entropy_partial_kernel(const c32 *__restrict__ img,
                                                              long long count,
                                                              double *__restrict__ partial) {
  __shared__ double sh[2][256];
  double s = 0.0, q = 0.0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
    const c32 v = img[i];
    // |I|^2 and its logarithm in FP32 (the image is FP32; ln_pos), sums in FP64
    const float a = v.x * v.x + v.y * v.y;
    s += a;
    q += (double)a * (double)ln_pos(a);  // 0 ln 0 = 0: ln_pos(0) is finite
  }
  sh[0][threadIdx.x] = s;
  sh[1][threadIdx.x] = q;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + w];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = sh[0][0];
    partial[2 * blockIdx.x + 1] = sh[1][0];
  }
}

__global__ void __launch_bounds__(256) entropy_final_kernel(const double *__restrict__ partial,
                                                            int blocks, double *__restrict__ stats) {
  __shared__ double sh[2][256];
  double s = 0.0, q = 0.0;
  for (int b = threadIdx.x; b < blocks; b += 256) {
    s += partial[2 * b];
    q += partial[2 * b + 1];
  }
  sh[0][threadIdx.x] = s;
  sh[1][threadIdx.x] = q;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + w];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double S = sh[0][0], Q = sh[1][0];
    stats[0] = S;
    stats[1] = Q;
    stats[2] = S > 0.0 ? log(S) - Q / S : 0.0;
  }
}

hipError_t launch_entropy_final(const double *partial, int blocks, double *stats, hipStream_t s) {
  if (blocks < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(entropy_final_kernel, dim3(1), dim3(256), 0, s, partial, blocks, stats);
  return hipGetLastError();
}

hipError_t launch_entropy(const void *img, long long count, double *partial, double *stats,
                          hipStream_t s) {
  long long blocks = (count + 255) / 256;
  if (blocks > ENT_BLOCKS) blocks = ENT_BLOCKS;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(entropy_partial_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                     static_cast<const c32 *>(img), count, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(entropy_final_kernel, dim3(1), dim3(256), 0, s, partial, (int)blocks, stats);
  return hipGetLastError();
}

// ------------------------------------------- entropy without allocation ----
// The plan-free variant of launch_entropy: the per-workgroup (S, Q) partials
// live in this file-scope device array instead of a plan's workspace.  Each
// GPU holds its own copy at its own address, found once per device with
// hipGetSymbolAddress (the array's name in host code is only a stand-in for
// the symbol, never a device address).  Every launch writes the partials of
// all the workgroups it uses before the final kernel reads them, so nothing
// needs clearing; calls that overlap on one GPU share the array and race.
static __device__ __align__(256) double scratch[2 * kEntropyNoAllocPartials];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t entropy_scratch(void **ptr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return hipSuccess;
}

hipError_t launch_entropy_noalloc(const void *img, long long count, double *stats, hipStream_t s) {
  static_assert(ENT_BLOCKS <= kEntropyNoAllocPartials, "the partials must fit the scratch array");
  void *ptr = nullptr;
  hipError_t e = entropy_scratch(&ptr);
  if (e != hipSuccess) return e;
  return launch_entropy(img, count, static_cast<double *>(ptr), stats, s);
}

// dE/dI scaled by an upstream factor: G = g (-2/S)(ln|I|^2 - ln S + E) I
// (no branch: at I = 0 the factor is finite, since ln_pos is, and G = 0)
__device__ __forceinline__ c32 entropy_grad_of(c32 v, double S, double E, float g) {
  const float a = v.x * v.x + v.y * v.y;
  const float c = (float)(-2.0 / S) * ((ln_pos(a) - (float)log(S)) + (float)E) * g;
  return c32{c * v.x, c * v.y};
}

__global__ void __launch_bounds__(256) entropy_grad_kernel(const c32 *__restrict__ img,
                                                           const double *__restrict__ stats,
                                                           const float *__restrict__ scale,
                                                           c32 *__restrict__ grad, long long count) {
  const double S = stats[0], E = stats[2];
  const float g = scale ? scale[0] : 1.0f;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
    grad[i] = entropy_grad_of(img[i], S, E, g);
}

hipError_t launch_entropy_grad(const void *img, const double *stats, const float *scale, void *grad,
                               long long count, hipStream_t s) {
  long long blocks = (count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) return hipSuccess;
  hipLaunchKernelGGL(entropy_grad_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                     static_cast<const c32 *>(img), stats, scale, static_cast<c32 *>(grad), count);
  return hipGetLastError();
}

// ------------------------------------------------------ Adam update ----

// One Adam step (Kingma & Ba, 2015, Algorithm 1) on the n per-pulse phases,
// its moments and step counter kept in device memory, so that consecutive
// autofocus steps need no host round trip and can be replayed from a graph.
// One workgroup: the counter is read once, and written back after every
// element has used it.
// lr_sched (device, sched_len values) replaces lr when given: step k uses
// lr_sched[min(k, sched_len) - 1]; an entry that is not finite and >= 0
// gives a zero step.
__global__ void __launch_bounds__(1024) adam_kernel(float *phase, const float *grad, float *m, float *v,
                                                    unsigned *step, int n, float lr, float b1,
                                                    float b2, float eps, const float *lr_sched,
                                                    int sched_len) {
  __shared__ unsigned k_s;
  __shared__ float lr_s;
  if (threadIdx.x == 0) {
    const unsigned k = step[0] + 1u;
    k_s = k;
    float l = lr;
    if (lr_sched) {
      l = lr_sched[(k < (unsigned)sched_len ? k : (unsigned)sched_len) - 1u];
      if (!(l >= 0.0f && l < 1e30f)) l = 0.0f;
    }
    lr_s = l;
  }
  __syncthreads();
  lr = lr_s;
  // bias corrections 1 - beta^k, in FP64: near k = 1, 1 - beta^k is small
  // and an FP32 power's last-place error would be a large part of it
  const float c1 = (float)(1.0 - pow((double)b1, (double)k_s));
  const float c2 = (float)(1.0 - pow((double)b2, (double)k_s));
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const float g = grad[i];
    const float mi = b1 * m[i] + (1.0f - b1) * g;
    const float vi = b2 * v[i] + (1.0f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    phase[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
  __syncthreads();
  if (threadIdx.x == 0) step[0] = k_s;
}

hipError_t launch_adam(float *phase, const float *grad, float *m, float *v, unsigned *step, int n,
                       float lr, float b1, float b2, float eps, const float *lr_sched, int sched_len,
                       hipStream_t s) {
  hipLaunchKernelGGL(adam_kernel, dim3(1), dim3(1024), 0, s, phase, grad, m, v, step, n, lr, b1, b2,
                     eps, lr_sched, sched_len);
  return hipGetLastError();
}

// ------------------------------------------------------ phase gradient ----

// RR range rows per thread and iteration (Engine::run_rr: the rows share
// the twiddles and the barriers of each LDS exchange); the per-pulse sums of
// the RR rows go into the same registers, row by row in order.  NB LDS
// buffers per row (2: one barrier per exchange).
template <class StoreT, int LOG2N, bool FUSED, int RR, int NB, int PLAN = 0>
__global__ void __launch_bounds__((Geometry<LOG2N, PLAN>::WG)) phase_grad_kernel(PhaseGradArgs a) {
  typedef Geometry<LOG2N, PLAN> G;
  typedef Engine<ModeFP32, LOG2N, PLAN> EN;
  constexpr int E = G::E, T = G::T, N = G::N;
  constexpr int ROWS = G::TPW * RR;
  __shared__ c32 lds_all[NB * ROWS * G::LDS_N];
  // one transform per workgroup for N >= 4096: keep the row index uniform
  const int local = G::TPW == 1 ? 0 : (int)(threadIdx.x / T);
  c32 *lds = lds_all + local * RR * G::LDS_N;
  c32 *const buf[2] = {lds, lds + (NB == 2 ? ROWS * G::LDS_N : 0)};
  unsigned xch = 0;
  const c32 *tw = static_cast<const c32 *>(PLAN == 0 ? a.tw32 : a.tw32_alt);
  const StoreT *flt = static_cast<const StoreT *>(a.filter);
  const c32 *ph = static_cast<const c32 *>(a.phasor);
  const c32 *gin = static_cast<const c32 *>(a.gimg);
  const StoreT *rc = static_cast<const StoreT *>(a.rc_t);
  double S = 0.0, Ent = 0.0;
  if constexpr (FUSED) {
    S = a.stats[0];
    Ent = a.stats[2];
  }
  float acc[E];
#pragma unroll
  for (int e = 0; e < E; ++e) acc[e] = 0.0f;
  const int groups = (a.rows + ROWS - 1) / ROWS;
  for (int g = blockIdx.x; g < groups; g += gridDim.x) {
    // the thread index, made opaque per group: otherwise the compiler hoists
    // every pass's LDS and twiddle addresses out of the loop into registers
    // (the empty statement emits no instruction)
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int t = tid & (T - 1);
    const unsigned ti = (unsigned)t;
    c32 v[RR][E];
#pragma unroll
    for (int q = 0; q < RR; ++q) {
      const long long row = (long long)g * ROWS + q * G::TPW + local;
      if (row < a.rows) {
        load_row<G>(v[q], gin, row, ti);
        if constexpr (FUSED) {
#pragma unroll
          for (int e = 0; e < E; ++e) v[q][e] = entropy_grad_of(v[q][e], S, Ent, 1.0f);
        }
      } else {
#pragma unroll
        for (int e = 0; e < E; ++e) v[q][e] = c32{0.0f, 0.0f};
      }
    }
    EN::template run_rr<false, RR, NB>(v, buf, xch, tw, t);
    {
      StoreT h[E];
      load_row<G, false>(h, flt, 0, ti);
#pragma unroll
      for (int e = 0; e < E; ++e)  // adjoint: conj(H_a), then the block shift
#pragma unroll
        for (int q = 0; q < RR; ++q) v[q][e] = conj_pow2<LOG2N>(cmul(v[q][e], cconj(to_c32(h[e]))));
    }
    EN::template run_rr<false, RR, NB>(v, buf, xch, tw, t);
    c32 p[E];
    load_row<G, false>(p, ph, 0, ti);
#pragma unroll
    for (int q = 0; q < RR; ++q) {
      const long long row = (long long)g * ROWS + q * G::TPW + local;
      if (row < a.rows) {
        StoreT r[E];
        load_row<G>(r, rc, row, ti);
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const c32 gz = cconj(v[q][e]);
          const c32 z = cmul(to_c32(r[e]), p[e]);
          acc[e] += gz.y * z.x - gz.x * z.y;  // Im(gz conj z)
        }
      }
    }
  }
  const int t = threadIdx.x & (T - 1);
  float *dst = a.partial + ((long long)blockIdx.x * G::TPW + local) * N;
#pragma unroll
  for (int e = 0; e < E; ++e) dst[t + T * e] = acc[e];
}

// out[m] = sum over p of partial[p][m] in a fixed order, in two steps:
// partial_sum_kernel adds part chunk c (parts [c P/C, (c+1) P/C)) of 64
// columns per workgroup, 4 interleaved slices per column combined in slice
// order, into stage[c][m]; the same kernel over the C stage rows (one chunk)
// gives out[m].  (One launch whose last-arriving workgroup per column block
// adds the stage rows needs a device-scope release fence per workgroup, an
// L2 writeback each: it made an autofocus iteration 229 instead of 162 us;
// a single pass of 64 column blocks of 1024 threads over all partial rows
// took 153.6 against 150.1 us per iteration.)
constexpr int kSumChunks = 16;

__global__ void __launch_bounds__(256) partial_sum_kernel(const float *__restrict__ partial, int parts,
                                                          int n, float *__restrict__ out) {
  __shared__ double sh[4][64];
  const int c = threadIdx.x & 63, slice = threadIdx.x >> 6;
  const int m = blockIdx.x * 64 + c;
  const int chunks = gridDim.y;
  const int p0 = (int)(((long long)parts * blockIdx.y) / chunks);
  const int p1 = (int)(((long long)parts * (blockIdx.y + 1)) / chunks);
  double s = 0.0;
  if (m < n)
    for (int p = p0 + slice; p < p1; p += 4) s += partial[(long long)p * n + m];
  sh[slice][c] = s;
  __syncthreads();
  if (slice == 0 && m < n)
    out[(long long)blockIdx.y * n + m] = (float)(((sh[0][c] + sh[1][c]) + sh[2][c]) + sh[3][c]);
}

template <class StoreT, int LOG2N, int RR, int NB, int PLAN = 0>
static hipError_t launch_pg_rr(const PhaseGradArgs &a, bool fused, hipStream_t s) {
  typedef Geometry<LOG2N, PLAN> G;
  const int groups = (a.rows + G::TPW * RR - 1) / (G::TPW * RR);
  const int grid = groups < kPhaseGradBlocks ? (groups < 1 ? 1 : groups) : kPhaseGradBlocks;
  if (fused)
    hipLaunchKernelGGL((phase_grad_kernel<StoreT, LOG2N, true, RR, NB, PLAN>), dim3(grid), dim3(G::WG), 0, s, a);
  else
    hipLaunchKernelGGL((phase_grad_kernel<StoreT, LOG2N, false, RR, NB, PLAN>), dim3(grid), dim3(G::WG), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int n = G::N;
  const int parts = grid * G::TPW;
  float *stage = a.partial + (long long)kPhaseGradBlocks * G::TPW * n;  // kSumChunks rows
  hipLaunchKernelGGL(partial_sum_kernel, dim3((n + 63) / 64, kSumChunks), dim3(256), 0, s, a.partial,
                     parts, n, stage);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(partial_sum_kernel, dim3((n + 63) / 64, 1), dim3(256), 0, s, stage, kSumChunks,
                     n, a.grad);
  return hipGetLastError();
}

// Two rows per iteration where the plan asks for it and their FP32 exchange
// buffers leave LDS for two workgroups per CU (n <= 4096); one otherwise.
// The plan's radix plan 1 where that plan's workgroups hold no more
// transforms than plan 0's (the partials are sized for plan 0).
template <class StoreT, int LOG2N, int PLAN>
static hipError_t launch_pg_plan(const PhaseGradArgs &a, bool fused, hipStream_t s) {
  typedef Geometry<LOG2N, PLAN> G;
  constexpr long kSet2 = (long)G::TPW * 2 * G::LDS_N * sizeof(c32);
  if constexpr (kSet2 <= 80 * 1024) {
    if (a.rows_per_thread == 2) return launch_pg_rr<StoreT, LOG2N, 2, 1, PLAN>(a, fused, s);
  }
  return launch_pg_rr<StoreT, LOG2N, 1, 1, PLAN>(a, fused, s);
}
template <class StoreT, int LOG2N>
static hipError_t launch_pg(const PhaseGradArgs &a, bool fused, hipStream_t s) {
  if constexpr (has_second_plan(LOG2N) && Geometry<LOG2N, 1>::TPW <= Geometry<LOG2N, 0>::TPW) {
    if (a.radix_plan == 1 && a.tw32_alt) return launch_pg_plan<StoreT, LOG2N, 1>(a, fused, s);
  }
  return launch_pg_plan<StoreT, LOG2N, 0>(a, fused, s);
}

long long phase_grad_scratch_floats(int log2n) {
  const int T = threads_per_transform(log2n);
  const int wg = T < 256 ? 256 : T;
  // per-workgroup partial rows, then the kSumChunks rows of the first sum
  return ((long long)kPhaseGradBlocks * (wg / T) + kSumChunks) * (1ll << log2n);
}

hipError_t launch_phase_grad(bool fp16_storage, int log2n, const PhaseGradArgs &a, bool fused,
                             hipStream_t s) {
#define BFP_PG_CASE(L)                                                              \
  case L:                                                                           \
    return fp16_storage ? launch_pg<h2, L>(a, fused, s) : launch_pg<c32, L>(a, fused, s);
  switch (log2n) {
    BFP_PG_CASE(8)
    BFP_PG_CASE(9)
    BFP_PG_CASE(10)
    BFP_PG_CASE(11)
    BFP_PG_CASE(12)
    BFP_PG_CASE(13)
    BFP_PG_CASE(14)
  }
#undef BFP_PG_CASE
  return hipErrorInvalidValue;
}

}  // namespace bfp
