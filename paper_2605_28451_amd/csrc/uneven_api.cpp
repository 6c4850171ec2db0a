// Uneven persistent batch: plan construction (packing, grouping into work
// items, longest-first ordering) and execution.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <complex>
#include <new>
#include <numeric>
#include <vector>

#include "bfpfft.h"
#include "host_tables.hpp"
#include "internal.hpp"
#include "plan.hpp"

namespace {

int hip_err(hipError_t e, const char *what) {
  return bfp::set_error(BFP_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

template <class T>
int upload(const std::vector<T> &v, T **out) {
  const size_t bytes = std::max<size_t>(sizeof(T), v.size() * sizeof(T));
  if (hipMalloc((void **)out, bytes) != hipSuccess)
    return bfp::set_error(BFP_ENOMEM, "hipMalloc failed");
  if (!v.empty()) {
    hipError_t e = hipMemcpy(*out, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_err(e, "hipMemcpy");
  }
  return BFP_OK;
}

int table_for(int log2n, int prec, void **out) {
  int rad[4];
  const int passes = bfp::pass_count(log2n, 0);
  for (int p = 0; p < 4; ++p) rad[p] = bfp::pass_radix(log2n, 0, p);
  std::vector<std::complex<double>> t = bfp::twiddle_table(log2n, rad, passes);
  const int fmt = (prec == BFP_FP16 || prec == BFP_FP16_MUL_FP32_ACC) ? BFP_FMT_F16 : BFP_FMT_F32;
  const size_t bytes = std::max<size_t>(16, t.size() * bfp_format_bytes(fmt));
  std::vector<unsigned char> host(bytes, 0);
  bfp::encode_complex(t.data(), t.size(), fmt, host.data());
  if (hipMalloc(out, bytes) != hipSuccess) return bfp::set_error(BFP_ENOMEM, "hipMalloc failed");
  hipError_t e = hipMemcpy(*out, host.data(), bytes, hipMemcpyHostToDevice);
  return e == hipSuccess ? BFP_OK : hip_err(e, "hipMemcpy twiddles");
}

}  // namespace

extern "C" {

int fft_plan_uneven(bfp_plan *out, int count, const int *log2n, const unsigned char *inverse,
                    int prec, unsigned flags) {
  if (!out) return bfp::set_error(BFP_EINVAL, "out is NULL");
  *out = nullptr;
  if (count < 0) return bfp::set_error(BFP_EINVAL, "count < 0");
  if (count > 0 && (!log2n || !inverse)) return bfp::set_error(BFP_EINVAL, "NULL descriptor array");
  if (prec < BFP_FP32 || prec > BFP_FP8_E5M2_STORE)
    return bfp::set_error(BFP_EINVAL, "unknown precision mode");
  if (flags & ~(unsigned)BFP_FLAG_CHECK_FINITE)
    return bfp::set_error(BFP_EINVAL, "uneven plans accept only BFP_FLAG_CHECK_FINITE");
  for (int i = 0; i < count; ++i)
    if (log2n[i] < 8 || log2n[i] > 14)
      return bfp::set_error(BFP_EINVAL, "log2n must be in [8, 14]");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
    return bfp::set_error(BFP_ENODEV, "no HIP device visible");

  bfp_plan p = new (std::nothrow) bfp_plan_s;
  if (!p) return bfp::set_error(BFP_ENOMEM, "host allocation failed");
  p->kind = 1;
  p->prec = prec;
  p->flags = flags;
  p->count = count;
  (void)hipGetDevice(&p->device);

  // packing in the given order
  p->offsets.resize(count);
  long long off = 0;
  for (int i = 0; i < count; ++i) {
    p->offsets[i] = off;
    off += 1ll << log2n[i];
  }
  p->total = off;

  // group by length, longest first, then by direction (stable within a
  // group): every item holds transforms of one length and one direction
  std::vector<int> order(count);
  std::iota(order.begin(), order.end(), 0);
  auto dir = [&](int i) { return inverse[i] ? 1 : 0; };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return log2n[a] != log2n[b] ? log2n[a] > log2n[b] : dir(a) < dir(b);
  });
  std::vector<int4> items;
  for (int s = 0; s < count;) {
    const int l = log2n[order[s]], w = dir(order[s]);
    int e = s;
    while (e < count && log2n[order[e]] == l && dir(order[e]) == w) ++e;
    const int per = bfp::kUnevenWG / bfp::threads_per_transform(l);
    for (int i = s; i < e; i += per) items.push_back(make_int4(i, std::min(per, e - i), l, w));
    s = e;
  }
  p->n_items = (int)items.size();
  // each transform's offset and direction in one word, in item order, so a
  // workgroup reaches its data after a single dependent load
  std::vector<long long> xform(count);
  for (int s = 0; s < count; ++s)
    xform[s] = (p->offsets[order[s]] << 1) | (inverse[order[s]] ? 1 : 0);

  int st = BFP_OK;
  if (!st) st = upload(items, &p->items);
  if (!st) st = upload(xform, &p->xform_d);
  std::vector<void *> ptrs(7, nullptr);
  for (int l = 8; l <= 14 && !st; ++l) {
    st = table_for(l, prec, &p->tw_sizes[l - 8]);
    ptrs[l - 8] = p->tw_sizes[l - 8];
  }
  if (!st) {
    void **d = nullptr;
    st = upload(ptrs, &d);
    p->tw_ptrs_d = d;
  }
  if (!st && (hipMalloc((void **)&p->queue, sizeof(unsigned)) != hipSuccess ||
              hipMalloc((void **)&p->nonfinite, sizeof(unsigned long long)) != hipSuccess))
    st = bfp::set_error(BFP_ENOMEM, "hipMalloc failed");
  if (!st && hipMemset(p->nonfinite, 0, sizeof(unsigned long long)) != hipSuccess)
    st = bfp::set_error(BFP_EHIP, "hipMemset failed");
  if (!st) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, p->device) != hipSuccess)
      st = bfp::set_error(BFP_EHIP, "hipGetDeviceProperties failed");
    else {
      p->cu_count = prop.multiProcessorCount;
      p->uneven_max_bpc = bfp::uneven_blocks_per_cu(prec);
      p->grid = p->cu_count * p->uneven_max_bpc;
    }
  }
  if (st) {
    fft_destroy(p);
    return st;
  }
  *out = p;
  return BFP_OK;
}

int fft_uneven_offsets(bfp_plan p, long long *offsets) {
  if (!p || !offsets) return bfp::set_error(BFP_EINVAL, "NULL argument");
  if (p->kind != 1) return bfp::set_error(BFP_EINVAL, "not an uneven plan");
  std::copy(p->offsets.begin(), p->offsets.end(), offsets);
  return BFP_OK;
}

int fft_uneven_total(bfp_plan p, long long *total) {
  if (!p || !total) return bfp::set_error(BFP_EINVAL, "NULL argument");
  if (p->kind != 1) return bfp::set_error(BFP_EINVAL, "not an uneven plan");
  *total = p->total;
  return BFP_OK;
}

int fft_exec_uneven(bfp_plan p, const void *in, void *out, void *stream) {
  if (!p) return bfp::set_error(BFP_EINVAL, "plan is NULL");
  if (p->kind != 1) return bfp::set_error(BFP_EINVAL, "not an uneven plan");
  if (p->count == 0) return BFP_OK;
  if (!in || !out) return bfp::set_error(BFP_EINVAL, "NULL data pointer");
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != p->device) return bfp::set_error(BFP_EINVAL, "plan belongs to another device");
  bfp::UnevenArgs a;
  a.in = in;
  a.out = out;
  a.items = p->items;
  a.xform = p->xform_d;
  a.n_items = p->n_items;
  a.queue = p->queue;
  a.tw = p->tw_ptrs_d;
  a.flags = (p->flags & BFP_FLAG_CHECK_FINITE) ? bfp::KF_CHECK_FINITE : 0u;
  a.nonfinite = p->nonfinite;
  a.off32 = p->total * (long long)bfp_storage_bytes(p->prec) < (1ll << 32) ? 1 : 0;
  // no more workgroups than tiles (the extra ones would only exit)
  const int grid = std::min(p->grid, p->n_items);
  hipError_t e = bfp::launch_uneven(p->prec, a, grid, (hipStream_t)stream);
  return e == hipSuccess ? BFP_OK : hip_err(e, "uneven launch");
}

}  // extern "C"
