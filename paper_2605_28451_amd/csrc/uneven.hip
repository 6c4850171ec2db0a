// Persistent kernel for a batch of transforms of uneven length and mixed
// direction, one launch for the whole batch.  Compiled once per precision
// mode with -DBFP_MODE_ID.
//
// The host groups transforms of equal length into work items that fill one
// 1024-thread workgroup (16384/N transforms of length N, 16 elements per
// thread; 16 transforms of 512 with 8 per thread) and orders the items
// longest transform first.  A grid sized to the resident occupancy pulls
// items from a device counter until the queue is empty, so the load balances
// across the 256 CUs without a second launch.  Every workgroup leaves the
// loop when the counter passes the item count, so the grid always drains.
// A grid of at least one workgroup per item (the hardware queues the
// workgroups beyond the resident ones, longest items first) takes each item
// by its workgroup index and makes no claims.
#include <type_traits>

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

constexpr int UNEVEN_WG = 1024;
constexpr int UNEVEN_LDS = 16384 + 16384 / 16;  // largest per-item LDS (elements)

// One item: d.y transforms of length 2^LOG2N and one direction (INV: the
// BFP inverse, the fold of Eq. (1) at the load and the final conjugate in
// the last pass), each thread holding E elements of one transform.  From
// 64 threads per transform (N >= 1024) a wavefront lies in one transform:
// its offset is made scalar and each group of four elements takes a base in
// scalar registers and one 32-bit lane offset, as the row kernels' load_row
// does (1% faster on the 20,000-transform batch, same bits).  Below that,
// OFF32: the packed batch spans less than 4 GiB, so every access is a
// uniform base plus a 32-bit byte offset (one 32-bit add per access instead
// of a 64-bit address per lane).
template <class M, int LOG2N, bool INV, bool OFF32>
__device__ __forceinline__ void uneven_item(const UnevenArgs &a, int4 d, typename M::Lds *lds_all,
                                            int tid) {
  typedef Geometry<LOG2N> G;
  typedef Engine<M, LOG2N> EN;
  typedef typename M::Comp Comp;
  typedef typename M::Store Store;
  constexpr int E = G::E, T = G::T;
  constexpr unsigned SZ = sizeof(Store);
  static_assert((UNEVEN_WG / T) * G::LDS_N <= UNEVEN_LDS, "item exceeds LDS");
  const int local = tid / T;
  const int t = tid & (T - 1);
  const bool active = local < d.y;
  // element offset of this thread's transform (the word's low bit, the
  // direction, is the item's)
  long long off = active ? (a.xform[d.x + local] >> 1) : 0;
  constexpr bool kWave = T >= 64 && T % 64 == 0;  // one transform per wavefront
  static_assert(!kWave || E % 4 == 0, "elements go in groups of four");
  if constexpr (kWave) {
    // the same value in every lane of the wavefront (and `active` too)
    const unsigned long long u = (unsigned long long)off;
    off = (long long)(((unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane((int)(u >> 32)) << 32) |
                      (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)u));
  }
  const unsigned b0 = ((unsigned)off + (unsigned)t) * SZ;
  Comp v[E];
  if (active) {
    const Store *src = static_cast<const Store *>(a.in) + off;
    const global_ptr<const char> gb = (global_ptr<const char>)a.in;
    if constexpr (kWave) {
#pragma unroll
      for (int e = 0; e < E; e += 4) {
        const Store *grp = src + T * e;
        asm volatile("" : "+s"(grp));
        const global_ptr<const Store> g = (global_ptr<const Store>)grp;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const Comp z = M::decode(ld_stream_g(g + ((unsigned)t + (unsigned)(T * k))));
          v[e + k] = INV ? conj_pow2<LOG2N>(z) : z;  // BFP fold for inverse transforms
        }
      }
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        Comp z;
        if constexpr (OFF32) z = M::decode(ld_stream_g((global_ptr<const Store>)(gb + (b0 + (unsigned)(T * e) * SZ))));
        else z = M::load(src, t + T * e);
        v[e] = INV ? conj_pow2<LOG2N>(z) : z;
      }
    }
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = Comp{};
  }
  EN::template run<INV>(v, lds_all + local * G::LDS_N, static_cast<const typename M::Tw *>(a.tw[LOG2N - 8]), t);
  if (active) {
    Store *dst = static_cast<Store *>(a.out) + off;
    const global_ptr<char> gb = (global_ptr<char>)a.out;
    if constexpr (kWave) {
#pragma unroll
      for (int e = 0; e < E; e += 4) {
        Store *grp = dst + T * e;
        asm volatile("" : "+s"(grp));
        const global_ptr<Store> g = (global_ptr<Store>)grp;
#pragma unroll
        for (int k = 0; k < 4; ++k) st_stream_g(g + ((unsigned)t + (unsigned)(T * k)), M::encode(v[e + k]));
      }
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        if constexpr (OFF32) st_stream_g((global_ptr<Store>)(gb + (b0 + (unsigned)(T * e) * SZ)), M::encode(v[e]));
        else M::store(dst, t + T * e, v[e]);
      }
    }
    // the check as a branch of its own (inside the store loop the compiler
    // evaluates it for every element whatever the flag)
    if (a.flags & KF_CHECK_FINITE) {
      unsigned bad = 0;
#pragma unroll
      for (int e = 0; e < E; ++e) bad += finite_c(to_c32(M::round_store(v[e]))) ? 0u : 1u;
      if (bad) atomicAdd(a.nonfinite, (unsigned long long)bad);
    }
  }
}

template <class M, int LOG2N, bool OFF32>
__device__ __forceinline__ void uneven_dir(const UnevenArgs &a, int4 d, typename M::Lds *lds, int tid) {
  if (d.w) uneven_item<M, LOG2N, true, OFF32>(a, d, lds, tid);
  else uneven_item<M, LOG2N, false, OFF32>(a, d, lds, tid);
}

template <class M>
__global__ void uneven_reset_kernel(unsigned *queue) { *queue = 0u; }

// Waves per SIMD the kernel is compiled for.  Pure FP16 fits two
// 1024-thread workgroups per CU (8 waves per SIMD: 64 VGPRs, and 2 x 68 KiB
// of LDS) without spills, so one workgroup's loads overlap the other's
// arithmetic; compiled without the bound it takes 77 VGPRs (each size alone
// needs at most 63) and one workgroup per CU.  The FP32-compute modes
// would spill at 64, and the FP32 / FP8 modes' LDS holds one workgroup.
template <class M>
constexpr int uneven_waves_per_simd() {
  return std::is_same<M, ModeFP16>::value ? 8 : 1;
}

template <class M, bool OFF32>
__global__ void __launch_bounds__(UNEVEN_WG, uneven_waves_per_simd<M>()) uneven_kernel(UnevenArgs a) {
  __shared__ typename M::Lds lds[UNEVEN_LDS];
  __shared__ int item_s;
  // the first item of each workgroup is its own index (no queue round trip
  // before the first load); later items come from the counter, past the
  // grid's first gridDim.x
  for (int it = blockIdx.x;;) {
    if (it >= a.n_items) break;
    const int4 d = a.items[it];
    // The thread index, made opaque per item: otherwise the compiler hoists
    // the LDS and twiddle addresses of all seven sizes out of the loop and
    // spills them (the empty statement emits no instruction).
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    switch (d.z) {
      case 8: uneven_dir<M, 8, OFF32>(a, d, lds, tid); break;
      case 9: uneven_dir<M, 9, OFF32>(a, d, lds, tid); break;
      case 10: uneven_dir<M, 10, OFF32>(a, d, lds, tid); break;
      case 11: uneven_dir<M, 11, OFF32>(a, d, lds, tid); break;
      case 12: uneven_dir<M, 12, OFF32>(a, d, lds, tid); break;
      case 13: uneven_dir<M, 13, OFF32>(a, d, lds, tid); break;
      case 14: uneven_dir<M, 14, OFF32>(a, d, lds, tid); break;
      default: break;
    }
    if ((int)gridDim.x >= a.n_items) break;  // one workgroup per item: no queue
    if (threadIdx.x == 0) item_s = (int)(gridDim.x + atomicAdd(a.queue, 1u));
    __syncthreads();  // LDS of this item is free, and item_s is written
    it = item_s;
    __syncthreads();  // every thread has read item_s before it is rewritten
  }
}

#define BFP_CAT2(a, b) a##b
#define BFP_CAT(a, b) BFP_CAT2(a, b)

hipError_t BFP_CAT(launch_uneven_mode, BFP_MODE_ID)(const UnevenArgs &a, int grid, hipStream_t s) {
  if (a.n_items <= 0) return hipSuccess;
  // only a grid smaller than the item count claims from the queue
  if (grid < a.n_items) {
    hipLaunchKernelGGL(uneven_reset_kernel<MODE>, dim3(1), dim3(1), 0, s, a.queue);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (a.off32)
    hipLaunchKernelGGL((uneven_kernel<MODE, true>), dim3(grid), dim3(UNEVEN_WG), 0, s, a);
  else
    hipLaunchKernelGGL((uneven_kernel<MODE, false>), dim3(grid), dim3(UNEVEN_WG), 0, s, a);
  return hipGetLastError();
}

int BFP_CAT(uneven_blocks_per_cu_mode, BFP_MODE_ID)() {
  // the resident workgroups of the form with fewer
  int b32 = 0, b64 = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b32, uneven_kernel<MODE, true>, UNEVEN_WG, 0) !=
          hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&b64, uneven_kernel<MODE, false>, UNEVEN_WG, 0) !=
          hipSuccess)
    return 1;
  const int blocks = b32 < b64 ? b32 : b64;
  return blocks < 1 ? 1 : blocks;
}

}  // namespace bfp
