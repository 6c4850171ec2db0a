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

template <class M, int LOG2N>
__device__ __forceinline__ void uneven_item(const UnevenArgs &a, int4 d, typename M::Lds *lds_all,
                                            int tid) {
  typedef Geometry<LOG2N> G;
  typedef Engine<M, LOG2N> EN;
  typedef typename M::Comp Comp;
  typedef typename M::Store Store;
  constexpr int E = G::E, T = G::T;
  static_assert((UNEVEN_WG / T) * G::LDS_N <= UNEVEN_LDS, "item exceeds LDS");
  const int local = tid / T;
  const int t = tid & (T - 1);
  const bool active = local < d.y;
  long long off = 0;
  bool inv = false;
  if (active) {
    const long long w = a.xform[d.x + local];
    off = w >> 1;
    inv = (w & 1) != 0;
  }
  Comp v[E];
  if (active) {
    const Store *src = static_cast<const Store *>(a.in) + off;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      Comp z = M::load(src, t + T * e);
      v[e] = inv ? conj_pow2<LOG2N>(z) : z;  // BFP fold for inverse transforms
    }
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = Comp{};
  }
  EN::run(v, lds_all + local * G::LDS_N, static_cast<const typename M::Tw *>(a.tw[LOG2N - 8]), t);
  if (active) {
    Store *dst = static_cast<Store *>(a.out) + off;
    unsigned bad = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      Comp y = inv ? cconj(v[e]) : v[e];
      M::store(dst, t + T * e, y);
      if (a.flags & KF_CHECK_FINITE) bad += finite_c(to_c32(M::round_store(y))) ? 0u : 1u;
    }
    if (bad) atomicAdd(a.nonfinite, (unsigned long long)bad);
  }
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

template <class M>
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
      case 8: uneven_item<M, 8>(a, d, lds, tid); break;
      case 9: uneven_item<M, 9>(a, d, lds, tid); break;
      case 10: uneven_item<M, 10>(a, d, lds, tid); break;
      case 11: uneven_item<M, 11>(a, d, lds, tid); break;
      case 12: uneven_item<M, 12>(a, d, lds, tid); break;
      case 13: uneven_item<M, 13>(a, d, lds, tid); break;
      case 14: uneven_item<M, 14>(a, d, lds, tid); break;
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
  hipLaunchKernelGGL(uneven_kernel<MODE>, dim3(grid), dim3(UNEVEN_WG), 0, s, a);
  return hipGetLastError();
}

int BFP_CAT(uneven_blocks_per_cu_mode, BFP_MODE_ID)() {
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, uneven_kernel<MODE>, UNEVEN_WG, 0) !=
      hipSuccess)
    return 1;
  return blocks < 1 ? 1 : blocks;
}

}  // namespace bfp
