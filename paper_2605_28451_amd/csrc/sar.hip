// Data-movement and helper kernels of the SAR chain: the LDS-tiled corner
// turn, storage-format conversion and the per-pulse phasor table used by the
// autofocus phase correction.
#include "fft_device.hpp"
#include "internal.hpp"

namespace bfp {

// ------------------------------------------------------------ corner turn --
// out[c][r] = in[r][c].  A 256-thread workgroup moves a 64 x 64 tile: it is
// read row by row (coalesced), staged in LDS with one element of padding per
// row (so the column reads hit distinct banks), and written row by row of the
// output.  Tiles are assigned row-major over the output so that consecutive
// workgroups write neighbouring output rows.
//
// Vector form (rows and cols multiples of V, V elements = 8 or 16 bytes per
// lane): each lane reads V consecutive elements of an input row and writes V
// consecutive elements of an output row.  The tile is 64 input rows by TC
// input columns: with TC = 128 each input row segment is 512 bytes (4-byte
// elements), which measured 5% faster on 4096 x 4096 than 64 x 64 tiles
// (25.0 against 26.4 us) although the staging writes into LDS then meet
// 2-way bank conflicts; the reads out of LDS stay conflict-free at the
// padded stride (bank of tile[r][c] = r + c mod 64).
template <class T, int V, int TC = 64>
__global__ void __launch_bounds__(256) transpose_vec_kernel(const T *__restrict__ in, T *__restrict__ out,
                                                            int rows, int cols) {
  typedef T vec __attribute__((ext_vector_type(V)));
  constexpr int CH = TC / V;    // V-chunks per tile row
  constexpr int RPI = 256 / CH; // tile rows per iteration
  constexpr int CHO = 64 / V;   // V-chunks per output row of the tile
  constexpr int RPO = 256 / CHO;
  static_assert(256 % CH == 0 && 64 % RPI == 0 && TC % RPO == 0, "tile shape");
  __shared__ T tile[64][TC + 1];
  const int tiles_r = (rows + 63) / 64;
  const int tc = blockIdx.x / tiles_r;
  const int tr = blockIdx.x % tiles_r;
  const int r0 = tr * 64, c0 = tc * TC;
  const int ch = threadIdx.x % CH, rl = threadIdx.x / CH;
#pragma unroll
  for (int k = 0; k < 64 / RPI; ++k) {
    const int rr = rl + RPI * k;
    const int r = r0 + rr, c = c0 + V * ch;
    if (r < rows && c < cols) {
      const vec x = __builtin_nontemporal_load(reinterpret_cast<const vec *>(in + (size_t)r * cols + c));
#pragma unroll
      for (int u = 0; u < V; ++u) tile[rr][V * ch + u] = x[u];
    }
  }
  __syncthreads();
  const int cho = threadIdx.x % CHO, ro = threadIdx.x / CHO;
#pragma unroll
  for (int k = 0; k < TC / RPO; ++k) {
    const int oc = ro + RPO * k;      // output row within the tile = input column
    const int orow = c0 + oc, ocol = r0 + V * cho;
    if (orow < cols && ocol < rows) {
      vec x;
#pragma unroll
      for (int u = 0; u < V; ++u) x[u] = tile[V * cho + u][oc];
      __builtin_nontemporal_store(x, reinterpret_cast<vec *>(out + (size_t)orow * rows + ocol));
    }
  }
}

// Element form for any shape.
template <class T>
__global__ void __launch_bounds__(256) transpose_kernel(const T *__restrict__ in, T *__restrict__ out,
                                                        int rows, int cols) {
  __shared__ T tile[64][65];
  const int tiles_r = (rows + 63) / 64;
  const int tc = blockIdx.x / tiles_r;  // tile column (input) = tile row of output
  const int tr = blockIdx.x % tiles_r;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;  // 0..3
  const int r0 = tr * 64, c0 = tc * 64;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int r = r0 + wv + 4 * i, c = c0 + lane;
    if (r < rows && c < cols) tile[wv + 4 * i][lane] = in[(size_t)r * cols + c];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int oc = c0 + wv + 4 * i;  // output row = input column
    const int orr = r0 + lane;       // output column = input row
    if (oc < cols && orr < rows) out[(size_t)oc * rows + orr] = tile[lane][wv + 4 * i];
  }
}

hipError_t launch_transpose(const void *in, void *out, int rows, int cols, int bytes,
                            hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  const long long tiles = (long long)((rows + 63) / 64) * ((cols + 63) / 64);
  const long long tiles_w = (long long)((rows + 63) / 64) * ((cols + 127) / 128);  // 64 x 128 tiles
  if (tiles > 0x7fffffffLL) return hipErrorInvalidValue;
  dim3 grid((unsigned)tiles), grid_w((unsigned)tiles_w), block(256);
  // the vector form needs whole, aligned V-element chunks
  const uintptr_t align = (uintptr_t)in | (uintptr_t)out;
  switch (bytes) {
    case 2:
      if (rows % 4 == 0 && cols % 4 == 0 && align % 8 == 0)
        hipLaunchKernelGGL((transpose_vec_kernel<uint16_t, 4, 128>), grid_w, block, 0, s,
                           (const uint16_t *)in, (uint16_t *)out, rows, cols);
      else
        hipLaunchKernelGGL(transpose_kernel<uint16_t>, grid, block, 0, s,
                           (const uint16_t *)in, (uint16_t *)out, rows, cols);
      break;
    case 4:
      if (rows % 4 == 0 && cols % 4 == 0 && align % 16 == 0)
        hipLaunchKernelGGL((transpose_vec_kernel<uint32_t, 4, 128>), grid_w, block, 0, s,
                           (const uint32_t *)in, (uint32_t *)out, rows, cols);
      else
        hipLaunchKernelGGL(transpose_kernel<uint32_t>, grid, block, 0, s,
                           (const uint32_t *)in, (uint32_t *)out, rows, cols);
      break;
    case 8:
      if (rows % 2 == 0 && cols % 2 == 0 && align % 16 == 0)
        hipLaunchKernelGGL((transpose_vec_kernel<uint64_t, 2>), grid, block, 0, s,
                           (const uint64_t *)in, (uint64_t *)out, rows, cols);
      else
        hipLaunchKernelGGL(transpose_kernel<uint2>, grid, block, 0, s, (const uint2 *)in,
                           (uint2 *)out, rows, cols);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ------------------------------------------------------------- convert ----
__device__ __forceinline__ c32 load_fmt(const void *p, long long i, int fmt) {
  switch (fmt) {
    case 0: return static_cast<const c32 *>(p)[i];
    case 1: return h2_to_c32(static_cast<const h2 *>(p)[i]);
    case 2: return Fp8Codec<3>::decode2(static_cast<const uint16_t *>(p)[i]);
    default: return Fp8Codec<2>::decode2(static_cast<const uint16_t *>(p)[i]);
  }
}

// FP32 -> FP16 rounds once (RNE); FP16/FP8 inputs are exact in FP32, so
// every conversion below is a single correct rounding of the input value.
__device__ __forceinline__ void store_fmt(void *p, long long i, int fmt, c32 v) {
  switch (fmt) {
    case 0: static_cast<c32 *>(p)[i] = v; break;
    case 1: static_cast<h2 *>(p)[i] = c32_to_h2(v); break;
    case 2: static_cast<uint16_t *>(p)[i] = (uint16_t)Fp8Codec<3>::encode2(v.x, v.y); break;
    default: static_cast<uint16_t *>(p)[i] = (uint16_t)Fp8Codec<2>::encode2(v.x, v.y); break;
  }
}

__global__ void __launch_bounds__(256) convert_kernel(const void *in, int in_fmt, void *out,
                                                      int out_fmt, long long count) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
    store_fmt(out, i, out_fmt, load_fmt(in, i, in_fmt));
}

hipError_t launch_convert(const void *in, int in_fmt, void *out, int out_fmt, long long count,
                          hipStream_t s) {
  if (count <= 0) return hipSuccess;
  long long blocks = (count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(convert_kernel, dim3((unsigned)blocks), dim3(256), 0, s, in, in_fmt, out,
                     out_fmt, count);
  return hipGetLastError();
}

// -------------------------------------------------------------- phasor ----
// p[m] = exp(+/- i phase[m]) for the per-pulse phase correction; evaluated in
// FP64 from the FP32 radians and rounded once to FP32.
__global__ void __launch_bounds__(256) phasor_kernel(const float *__restrict__ phase,
                                                     c32 *__restrict__ p, int n, int negate) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    double s, c;
    sincos((double)phase[i], &s, &c);
    p[i] = c32{(float)c, (float)(negate ? -s : s)};
  }
}

hipError_t launch_phasor(const float *phase, void *phasor, int n, int negate, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(phasor_kernel, dim3((n + 255) / 256), dim3(256), 0, s, phase,
                     static_cast<c32 *>(phasor), n, negate);
  return hipGetLastError();
}

// ------------------------------------------------------------- copy ------
// Plain streaming copy: the reference for achievable HBM bandwidth and for
// calibrating memory counters.  Each thread keeps four 16-byte loads in
// flight (the workgroup moves 16 KiB per trip, lanes contiguous within each
// 4 KiB slice); the tail that is not a whole 16 KiB chunk is copied by a
// second, element-wise loop.
constexpr int kCopyUnroll = 4;
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) copy_kernel(const u32x4 *__restrict__ in,
                                                   u32x4 *__restrict__ out, long long n16) {
  const long long chunk = 256LL * kCopyUnroll;
  const long long chunks = n16 / chunk;
  for (long long c = blockIdx.x; c < chunks; c += gridDim.x) {
    const u32x4 *src = in + c * chunk + threadIdx.x;
    u32x4 *dst = out + c * chunk + threadIdx.x;
    u32x4 v[kCopyUnroll];
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) v[u] = __builtin_nontemporal_load(src + 256 * u);
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) __builtin_nontemporal_store(v[u], dst + 256 * u);
  }
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = chunks * chunk + (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n16;
       i += stride)
    out[i] = in[i];
}

hipError_t launch_copy(const void *in, void *out, long long bytes, hipStream_t s) {
  const long long n16 = bytes / 16;
  if (n16 <= 0) return hipSuccess;
  long long blocks = (n16 + 256LL * kCopyUnroll - 1) / (256LL * kCopyUnroll);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                     static_cast<const u32x4 *>(in), static_cast<u32x4 *>(out), n16);
  return hipGetLastError();
}

}  // namespace bfp
