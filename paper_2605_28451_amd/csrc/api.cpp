// C ABI of libbfpfft: plans, argument validation, error reporting and the
// host side of every entry point declared in include/bfpfft.h.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <complex>
#include <new>
#include <string>
#include <vector>

#include "bfpfft.h"
#include "host_tables.hpp"
#include "internal.hpp"
#include "plan.hpp"

using bfp::RowArgs;

namespace {

// blocks_per_cu = kAutoBpc: the fused compression of pure FP16 up to n = 4096
// runs the pipelined kernel on a grid of 3 workgroups per CU (4 fit, by
// LDS; at 2048 rows of 4096, 3, 5 and 8 measure alike and 4 and 6 slower),
// and of 8 per CU from 4096 rows of 4096 on (31.5 against 33.5 us at 4096
// rows: the grid then outlasts one resident wave of workgroups), except for
// the transposed store, whose XCD-aware row order wants the persistent grid
// (a 4096 x 4096 frame with the fused corner turn: 156 us at 3, 166 us at
// 8); the FP32-output image with its entropy sums one round of its kernel's
// resident workgroups (sized in the launcher); every other operation one
// workgroup per row group (the single transforms are faster at full
// occupancy).
constexpr int kAutoBpc = -1;
constexpr int kPipelinedBpc = 3;
constexpr int kPipelinedBpcLarge = 8;

int effective_bpc(const bfp_plan_s *p, int op, int rows, unsigned flags) {
  if (p->tune_bpc != kAutoBpc) return p->tune_bpc;
  if (op != bfp::OP_COMPRESS || p->prec != BFP_FP16 || p->log2n > 12 || p->log2n < 8) return 0;
  const bool transposed = ((flags | p->flags) & BFP_FLAG_TRANSPOSED_STORE) != 0;
  return (p->log2n == 12 && rows >= 4096 && !transposed) ? kPipelinedBpcLarge : kPipelinedBpc;
}


// Rows per thread of a new plan: two in the modes with FP32 arithmetic,
// where sharing twiddles and barriers between two rows is ~20% faster at
// 2048 x 4096 (compression: FP16 storage 41.5 -> 33.5 us, FP32 48.8 -> 38.3,
// E4M3 40.5 -> 31.4); one in pure FP16 and FP16-multiply, whose two-row
// kernel is slower (17.8 -> 21.5 us, 26.3 -> 28.6: the 68 KiB of LDS of two
// rows halves the workgroups per CU).
int default_rows_per_thread(int prec) {
  return (prec == BFP_FP16 || prec == BFP_FP16_MUL_FP32_ACC) ? 1 : 2;
}

thread_local std::string g_last_error;

int fail(int status, const std::string &msg) {
  g_last_error = msg;
  return status;
}

}  // namespace

int bfp::set_error(int status, const std::string &msg) { return fail(status, msg); }

namespace {

int hip_fail(hipError_t e, const char *what) {
  return fail(BFP_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

bool valid_prec(int prec) { return prec >= BFP_FP32 && prec <= BFP_FP8_E5M2_STORE; }

// twiddle table format of a mode
int tw_format(int prec) {
  return (prec == BFP_FP16 || prec == BFP_FP16_MUL_FP32_ACC) ? BFP_FMT_F16 : BFP_FMT_F32;
}

int log2_exact(long long n) {
  if (n <= 0 || (n & (n - 1))) return -1;
  int k = 0;
  while ((1ll << k) < n) ++k;
  return k;
}

}  // namespace

namespace {

// The twiddle table of radix plan `plan` (the matrix-core operands first
// where the mode and size have that engine, plan 0 only).
int upload_twiddles(int log2n, int prec, int plan, void **out) {
  int rad[4];
  const int passes = bfp::pass_count(log2n, plan);
  for (int p = 0; p < 4; ++p) rad[p] = bfp::pass_radix(log2n, plan, p);
  std::vector<std::complex<double>> t = bfp::twiddle_table(log2n, rad, passes);
  if ((int)t.size() != bfp::twiddle_entries(log2n, plan))
    return fail(BFP_EINVAL, "internal: twiddle table size mismatch");
  const int fmt = tw_format(prec);
  size_t bytes = std::max<size_t>(16, t.size() * bfp_format_bytes(fmt));
  std::vector<unsigned char> host(bytes, 0);
  bfp::encode_complex(t.data(), t.size(), fmt, host.data());
  if (plan == 0 && bfp::has_mfma_engine(prec, log2n)) {
    // matrix-core table (DFT16 operands + dot2-form twiddles) first, the
    // vector-ALU engine's table after it at kMfmaTableBytes
    std::vector<uint16_t> m = bfp::mfma4096_table();
    std::vector<unsigned char> both((const unsigned char *)m.data(),
                                    (const unsigned char *)m.data() + m.size() * sizeof(uint16_t));
    if (both.size() != (size_t)bfp::kMfmaTableBytes)
      return fail(BFP_EINVAL, "internal: matrix-core table size mismatch");
    both.insert(both.end(), host.begin(), host.end());
    host.swap(both);
    bytes = host.size();
  }
  void *d = nullptr;
  hipError_t e = hipMalloc(&d, bytes);
  if (e != hipSuccess) return fail(BFP_ENOMEM, "hipMalloc twiddles failed");
  e = hipMemcpy(d, host.data(), bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d);
    return hip_fail(e, "hipMemcpy twiddles");
  }
  *out = d;
  return BFP_OK;
}

int check_device() {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0)
    return fail(BFP_ENODEV, "no HIP device visible");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(BFP_ENODEV, "hipGetDevice failed");
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return fail(BFP_ENODEV, "hipGetDeviceProperties failed");
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(BFP_ENODEV, std::string("device is ") + prop.gcnArchName + ", not gfx950");
  return BFP_OK;
}

void free_plan(bfp_plan p) {
  if (!p) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(p->device);
  (void)hipFree(p->tw);
  (void)hipFree(p->tw_alt);
  (void)hipFree(p->nonfinite);
  (void)hipFree(p->phasor);
  (void)hipFree(p->items);
  (void)hipFree(p->xform_d);
  (void)hipFree(p->queue);
  if (p->tw32 != p->tw) (void)hipFree(p->tw32);
  (void)hipFree(p->ent_partial);
  (void)hipFree(p->pg_partial);
  for (void *t : p->tw_sizes) (void)hipFree(t);
  (void)hipFree(p->tw_ptrs_d);
  (void)hipSetDevice(cur);
  delete p;
}

int check_rows_plan(bfp_plan p) {
  if (!p) return fail(BFP_EINVAL, "plan is NULL");
  if (p->kind != 0) return fail(BFP_EINVAL, "plan is not a batched-rows plan");
  return BFP_OK;
}

// Private bits of run_rows' flags (outside the public bfp_flags): kExactConj
// makes the call's BFP_FLAG_CONJ_FILTER bit authoritative (the plan's is not
// ORed in: the adjoint of a conjugate-filter plan uses the filter itself);
// kPostPhasor applies the phasor to the output (adjoint chains).
constexpr unsigned kExactConj = 1u << 31;
constexpr unsigned kPostPhasor = 1u << 30;

unsigned kflags(unsigned f) {
  unsigned k = 0;
  if (f & BFP_FLAG_NAIVE_POSTSCALE) k |= bfp::KF_NAIVE;
  if (f & BFP_FLAG_CHECK_FINITE) k |= bfp::KF_CHECK_FINITE;
  if (f & BFP_FLAG_CONJ_FILTER) k |= bfp::KF_CONJ_FILTER;
  if (f & BFP_FLAG_TRANSPOSED_STORE) k |= bfp::KF_TRANSPOSED;
  if (f & kPostPhasor) k |= bfp::KF_POST_PHASOR;
  return k;
}

int run_rows(bfp_plan p, int op, const void *in, void *out, const void *filter,
             const void *phasor, int rows, unsigned flags, void *stream,
             double *ent_partial = nullptr, int *grid_used = nullptr, int *row_exp = nullptr,
             const float *shift = nullptr) {
  if (rows < 0 || rows > p->batch) return fail(BFP_EINVAL, "row count outside [0, plan batch]");
  if (rows == 0) return BFP_OK;
  if (!in || !out) return fail(BFP_EINVAL, "NULL data pointer");
  RowArgs a;
  a.in = in;
  a.out = out;
  a.rows = rows;
  a.tw = p->tw;  // the launcher picks the engine's part of a two-engine table
  a.tw_alt = p->tw_alt;
  a.radix_plan = p->tune_plan;
  a.filter = filter;
  a.phasor = phasor;
  unsigned eff = flags | p->flags;
  if (flags & kExactConj) eff = (eff & ~(unsigned)BFP_FLAG_CONJ_FILTER) | (flags & BFP_FLAG_CONJ_FILTER);
  a.flags = kflags(eff);
  a.nonfinite = p->nonfinite;
  const int bpc = effective_bpc(p, op, rows, flags);
  a.grid_limit = bpc > 0 ? bpc * p->cu_count : 0;
  // the image with its entropy sums, under automatic tuning: one round of
  // resident workgroups (the launcher sizes it for the kernel it launches)
  a.resident_cus = (ent_partial && p->tune_bpc == kAutoBpc) ? p->cu_count : 0;
  a.engine = p->tune_engine;
  a.rows_per_thread = p->tune_rr;
  a.ent_partial = ent_partial;
  a.row_exp = row_exp;
  if (row_exp) a.flags |= bfp::KF_ADAPT;
  a.shift = shift;
  if (shift) a.flags |= bfp::KF_RAMP;
  a.grid_out = grid_used;
  const bool out32 = (eff & BFP_FLAG_OUT_FP32) != 0;
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != p->device) return fail(BFP_EINVAL, "plan belongs to another device");
  hipError_t e = bfp::launch_rows(p->prec, p->log2n, op, out32, a, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return BFP_OK;
}

}  // namespace

extern "C" {

int bfp_storage_bytes(int prec) {
  switch (prec) {
    case BFP_FP32: return 8;
    case BFP_FP16:
    case BFP_FP16_STORE_FP32_COMPUTE:
    case BFP_FP16_MUL_FP32_ACC: return 4;
    case BFP_FP8_E4M3_STORE:
    case BFP_FP8_E5M2_STORE: return 2;
  }
  return -1;
}

int bfp_filter_format(int prec) {
  if (!valid_prec(prec)) return -1;
  return (prec == BFP_FP16 || prec == BFP_FP16_STORE_FP32_COMPUTE || prec == BFP_FP16_MUL_FP32_ACC)
             ? BFP_FMT_F16
             : BFP_FMT_F32;
}

int bfp_format_bytes(int fmt) {
  switch (fmt) {
    case BFP_FMT_F32: return 8;
    case BFP_FMT_F16: return 4;
    case BFP_FMT_E4M3:
    case BFP_FMT_E5M2: return 2;
  }
  return -1;
}

const char *bfp_status_string(int status) {
  switch (status) {
    case BFP_OK: return "ok";
    case BFP_EINVAL: return "invalid argument";
    case BFP_EUNSUPPORTED: return "unsupported";
    case BFP_ENOMEM: return "out of memory";
    case BFP_EHIP: return "HIP runtime error";
    case BFP_ENODEV: return "no gfx950 device";
  }
  return "unknown status";
}

const char *bfp_last_error(void) { return g_last_error.c_str(); }

int bfp_device_count(void) {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess) return 0;
  int n = 0;
  for (int d = 0; d < count; ++d) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, d) == hipSuccess && strncmp(prop.gcnArchName, "gfx950", 6) == 0)
      ++n;
  }
  return n;
}

int fft_plan(bfp_plan *out, int n, int batch, int prec, unsigned flags) {
  if (!out) return fail(BFP_EINVAL, "out is NULL");
  *out = nullptr;
  const int l = log2_exact(n);
  if (l < 3 || l > 14) return fail(BFP_EINVAL, "n must be a power of two in [8, 16384]");
  if (batch < 0) return fail(BFP_EINVAL, "batch must be >= 0");
  if (!valid_prec(prec)) return fail(BFP_EINVAL, "unknown precision mode");
  if (flags & ~(unsigned)(BFP_FLAG_NAIVE_POSTSCALE | BFP_FLAG_CHECK_FINITE | BFP_FLAG_OUT_FP32 |
                          BFP_FLAG_CONJ_FILTER | BFP_FLAG_AUTOFOCUS))
    return fail(BFP_EINVAL, "unknown plan flag");
  if ((flags & BFP_FLAG_AUTOFOCUS) && prec != BFP_FP32 && prec != BFP_FP16_STORE_FP32_COMPUTE)
    return fail(BFP_EINVAL, "autofocus plans need BFP_FP32 or BFP_FP16_STORE_FP32_COMPUTE");
  if ((flags & BFP_FLAG_AUTOFOCUS) && l < 8)
    return fail(BFP_EINVAL, "autofocus plans need n >= 256");
  int st = check_device();
  if (st) return st;
  bfp_plan p = new (std::nothrow) bfp_plan_s;
  if (!p) return fail(BFP_ENOMEM, "host allocation failed");
  p->kind = 0;
  p->n = n;
  p->log2n = l;
  p->batch = batch;
  p->prec = prec;
  p->flags = flags;
  (void)hipGetDevice(&p->device);
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) p->cu_count = prop.multiProcessorCount;
    if (p->cu_count <= 0) p->cu_count = 1;
  }
  // default tuning: the vector engine, grid chosen per operation
  p->tune_engine = 1;
  p->tune_bpc = kAutoBpc;
  p->tune_rr = default_rows_per_thread(prec);
  // autofocus plans: the second radix plan, whose phase gradient runs twice
  // the wavefronts per row in the same LDS (82 against 98 us at 4096 x 4096)
  if ((flags & BFP_FLAG_AUTOFOCUS) && bfp::second_plan(l)) p->tune_plan = 1;
  st = upload_twiddles(l, prec, 0, &p->tw);
  if (!st && bfp::second_plan(l)) st = upload_twiddles(l, prec, 1, &p->tw_alt);
  if (st) {
    free_plan(p);
    return st;
  }
  if (hipMalloc((void **)&p->nonfinite, sizeof(unsigned long long)) != hipSuccess ||
      hipMalloc(&p->phasor, (size_t)n * 8) != hipSuccess) {
    free_plan(p);
    return fail(BFP_ENOMEM, "hipMalloc plan buffers failed");
  }
  hipError_t e = hipMemset(p->nonfinite, 0, sizeof(unsigned long long));
  if (e != hipSuccess) {
    free_plan(p);
    return hip_fail(e, "hipMemset");
  }
  // entropy partials: the grid-stride reduction (kEntropyBlocks) or one
  // per workgroup of a fused image launch (at most one per row)
  if (hipMalloc((void **)&p->ent_partial,
                sizeof(double) * 2 * (size_t)std::max(bfp::kEntropyBlocks, batch)) != hipSuccess) {
    free_plan(p);
    return fail(BFP_ENOMEM, "hipMalloc entropy workspace failed");
  }
  if (flags & BFP_FLAG_AUTOFOCUS) {
    p->tw32 = p->tw;  // both admitted modes keep FP32 twiddles
    const size_t bytes = sizeof(float) * (size_t)bfp::phase_grad_scratch_floats(l);
    if (hipMalloc((void **)&p->pg_partial, bytes) != hipSuccess) {
      free_plan(p);
      return fail(BFP_ENOMEM, "hipMalloc autofocus workspace failed");
    }
  }
  *out = p;
  return BFP_OK;
}

int fft_destroy(bfp_plan p) {
  if (!p) return fail(BFP_EINVAL, "plan is NULL");
  free_plan(p);
  return BFP_OK;
}

int fft_plan_info(bfp_plan p, int *n, int *batch, int *prec, unsigned *flags) {
  if (!p) return fail(BFP_EINVAL, "plan is NULL");
  if (n) *n = p->n;
  if (batch) *batch = p->kind == 0 ? p->batch : p->count;
  if (prec) *prec = p->prec;
  if (flags) *flags = p->flags;
  return BFP_OK;
}

int fft_exec_fwd(bfp_plan p, const void *in, void *out, void *stream) {
  int st = check_rows_plan(p);
  if (st) return st;
  return run_rows(p, bfp::OP_FWD, in, out, nullptr, nullptr, p->batch, 0, stream);
}

int fft_exec_inv_bfp_flags(bfp_plan p, const void *in, void *out, const void *filter,
                           unsigned flags, void *stream) {
  int st = check_rows_plan(p);
  if (st) return st;
  if (flags & ~(unsigned)(BFP_FLAG_NAIVE_POSTSCALE | BFP_FLAG_CHECK_FINITE | BFP_FLAG_CONJ_FILTER))
    return fail(BFP_EINVAL, "unknown flag for fft_exec_inv_bfp");
  return run_rows(p, bfp::OP_INV, in, out, filter, nullptr, p->batch, flags, stream);
}

int fft_exec_inv_bfp(bfp_plan p, const void *in, void *out, const void *filter, void *stream) {
  return fft_exec_inv_bfp_flags(p, in, out, filter, 0u, stream);
}

namespace {
// the adaptive shift exists for the modes with FP16 storage between passes
int check_adaptive(bfp_plan p, const int *row_exp) {
  if (!row_exp) return fail(BFP_EINVAL, "row_exp is NULL");
  if (p->prec != BFP_FP16 && p->prec != BFP_FP16_STORE_FP32_COMPUTE && p->prec != BFP_FP16_MUL_FP32_ACC)
    return fail(BFP_EUNSUPPORTED, "the adaptive shift is for the FP16-storage modes");
  if (p->flags & (BFP_FLAG_NAIVE_POSTSCALE | BFP_FLAG_CONJ_FILTER | BFP_FLAG_OUT_FP32))
    return fail(BFP_EUNSUPPORTED, "the adaptive shift combines with BFP_FLAG_CHECK_FINITE only");
  return BFP_OK;
}
}  // namespace

int fft_exec_inv_bfp_adaptive(bfp_plan p, const void *in, void *out, const void *filter,
                              int *row_exp, unsigned flags, void *stream) {
  int st = check_rows_plan(p);
  if (st) return st;
  if (flags & ~(unsigned)BFP_FLAG_CHECK_FINITE)
    return fail(BFP_EINVAL, "the adaptive inverse takes BFP_FLAG_CHECK_FINITE only");
  st = check_adaptive(p, row_exp);
  if (st) return st;
  return run_rows(p, bfp::OP_INV, in, out, filter, nullptr, p->batch, flags, stream, nullptr,
                  nullptr, row_exp);
}

int fft_plan_nonfinite(bfp_plan p, void *stream, unsigned long long *count) {
  if (!p || !count) return fail(BFP_EINVAL, "NULL argument");
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  e = hipMemcpy(count, p->nonfinite, sizeof(unsigned long long), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy counter");
  e = hipMemset(p->nonfinite, 0, sizeof(unsigned long long));
  if (e != hipSuccess) return hip_fail(e, "hipMemset counter");
  return BFP_OK;
}

int bfp_make_filter(const double *h, int len, int n, int fmt, void *out_host) {
  if (!h || !out_host) return fail(BFP_EINVAL, "NULL argument");
  if (log2_exact(n) < 0) return fail(BFP_EINVAL, "n must be a power of two");
  if (len < 1 || len > n) return fail(BFP_EINVAL, "replica length must be in [1, n]");
  if (bfp_format_bytes(fmt) < 0) return fail(BFP_EINVAL, "unknown format");
  std::vector<std::complex<double>> a((size_t)n, std::complex<double>(0.0, 0.0));
  for (int i = 0; i < len; ++i) a[i] = std::complex<double>(h[2 * i], h[2 * i + 1]);
  bfp::host_fft(a);
  double m = 0.0;
  for (auto &v : a) m = std::max(m, std::abs(v));
  if (!(m > 0.0)) return fail(BFP_EINVAL, "replica has an all-zero spectrum");
  for (auto &v : a) v = std::conj(v) / m;
  bfp::encode_complex(a.data(), a.size(), fmt, out_host);
  return BFP_OK;
}

int bfp_window(int kind, int len, int nbar, double sll_db, double *out_host) {
  if (!out_host) return fail(BFP_EINVAL, "NULL argument");
  if (len < 1) return fail(BFP_EINVAL, "window length must be >= 1");
  if (kind < BFP_WINDOW_RECT || kind > BFP_WINDOW_TAYLOR) return fail(BFP_EINVAL, "unknown window kind");
  if (kind == BFP_WINDOW_TAYLOR && (nbar < 1 || !(sll_db > 0.0) || sll_db > 300.0))
    return fail(BFP_EINVAL, "Taylor window needs nbar >= 1 and 0 < sll_db <= 300");
  if (!bfp::taper(kind, len, nbar, sll_db, out_host)) return fail(BFP_EINVAL, "bad window arguments");
  return BFP_OK;
}

int bfp_convert(const void *in, int in_fmt, void *out, int out_fmt, long long count, void *stream) {
  if (count < 0) return fail(BFP_EINVAL, "count < 0");
  if (count == 0) return BFP_OK;
  if (!in || !out) return fail(BFP_EINVAL, "NULL data pointer");
  if (in == out) return fail(BFP_EINVAL, "in and out must differ");
  if (bfp_format_bytes(in_fmt) < 0 || bfp_format_bytes(out_fmt) < 0)
    return fail(BFP_EINVAL, "unknown format");
  hipError_t e = bfp::launch_convert(in, in_fmt, out, out_fmt, count, (hipStream_t)stream);
  return e == hipSuccess ? BFP_OK : hip_fail(e, "convert launch");
}

int sar_range_compress(bfp_plan range_plan, const void *echo, void *rc, const void *h_range,
                       int n_pulses, unsigned flags, void *stream) {
  int st = check_rows_plan(range_plan);
  if (st) return st;
  if (!h_range) return fail(BFP_EINVAL, "range filter is NULL");
  if (flags & ~(unsigned)(BFP_FLAG_NAIVE_POSTSCALE | BFP_FLAG_CHECK_FINITE | BFP_FLAG_CONJ_FILTER |
                          BFP_FLAG_OUT_FP32 | BFP_FLAG_TRANSPOSED_STORE))
    return fail(BFP_EINVAL, "unknown flag for sar_range_compress");
  if ((flags & BFP_FLAG_TRANSPOSED_STORE) &&
      ((flags | range_plan->flags) &
       (BFP_FLAG_NAIVE_POSTSCALE | BFP_FLAG_CONJ_FILTER | BFP_FLAG_OUT_FP32)))
    return fail(BFP_EUNSUPPORTED, "BFP_FLAG_TRANSPOSED_STORE combines with BFP_FLAG_CHECK_FINITE only");
  if (echo == rc) return fail(BFP_EINVAL, "echo and rc must differ");
  return run_rows(range_plan, bfp::OP_COMPRESS, echo, rc, h_range, nullptr, n_pulses, flags,
                  stream);
}

int sar_range_compress_adaptive(bfp_plan range_plan, const void *echo, void *rc,
                                const void *h_range, int n_pulses, int *row_exp, unsigned flags,
                                void *stream) {
  int st = check_rows_plan(range_plan);
  if (st) return st;
  if (!h_range) return fail(BFP_EINVAL, "range filter is NULL");
  if (flags & ~(unsigned)BFP_FLAG_CHECK_FINITE)
    return fail(BFP_EINVAL, "the adaptive compression takes BFP_FLAG_CHECK_FINITE only");
  st = check_adaptive(range_plan, row_exp);
  if (st) return st;
  if (echo == rc) return fail(BFP_EINVAL, "echo and rc must differ");
  return run_rows(range_plan, bfp::OP_COMPRESS, echo, rc, h_range, nullptr, n_pulses, flags,
                  stream, nullptr, nullptr, row_exp);
}

int sar_range_compress_rcmc(bfp_plan range_plan, const void *in, void *out, const void *h_range,
                            const float *shift, int n_rows, unsigned flags, void *stream) {
  int st = check_rows_plan(range_plan);
  if (st) return st;
  if (!h_range) return fail(BFP_EINVAL, "range filter is NULL");
  if (!shift) return fail(BFP_EINVAL, "shift is NULL");
  if (flags & ~(unsigned)BFP_FLAG_CHECK_FINITE)
    return fail(BFP_EINVAL, "the migration-corrected compression takes BFP_FLAG_CHECK_FINITE only");
  if (range_plan->flags & (BFP_FLAG_NAIVE_POSTSCALE | BFP_FLAG_CONJ_FILTER | BFP_FLAG_OUT_FP32))
    return fail(BFP_EUNSUPPORTED, "the migration-corrected compression combines with BFP_FLAG_CHECK_FINITE only");
  if (in == out) return fail(BFP_EINVAL, "in and out must differ");
  return run_rows(range_plan, bfp::OP_COMPRESS, in, out, h_range, nullptr, n_rows, flags, stream,
                  nullptr, nullptr, nullptr, shift);
}

int bfp_device_copy(const void *in, void *out, long long bytes, void *stream) {
  if (bytes < 0 || (bytes % 16) != 0) return fail(BFP_EINVAL, "bytes must be a non-negative multiple of 16");
  if (bytes == 0) return BFP_OK;
  if (!in || !out) return fail(BFP_EINVAL, "NULL data pointer");
  if (((uintptr_t)in | (uintptr_t)out) & 15) return fail(BFP_EINVAL, "pointers must be 16-byte aligned");
  hipError_t e = bfp::launch_copy(in, out, bytes, (hipStream_t)stream);
  return e == hipSuccess ? BFP_OK : hip_fail(e, "copy launch");
}

int sar_corner_turn(const void *in, void *out, int rows, int cols, int fmt, void *stream) {
  if (rows < 0 || cols < 0) return fail(BFP_EINVAL, "negative size");
  if (rows == 0 || cols == 0) return BFP_OK;
  if (!in || !out) return fail(BFP_EINVAL, "NULL data pointer");
  if (in == out) return fail(BFP_EINVAL, "in and out must differ");
  const int b = bfp_format_bytes(fmt);
  if (b < 0) return fail(BFP_EINVAL, "unknown format");
  hipError_t e = bfp::launch_transpose(in, out, rows, cols, b, (hipStream_t)stream);
  return e == hipSuccess ? BFP_OK : hip_fail(e, "corner turn launch");
}

int sar_azimuth_compress(bfp_plan az_plan, const void *rc_t, void *image, const void *h_az,
                         const float *phase, int n_range, int adjoint, unsigned flags,
                         void *stream) {
  int st = check_rows_plan(az_plan);
  if (st) return st;
  if (!h_az) return fail(BFP_EINVAL, "azimuth filter is NULL");
  if (flags & ~(unsigned)(BFP_FLAG_NAIVE_POSTSCALE | BFP_FLAG_CHECK_FINITE | BFP_FLAG_CONJ_FILTER |
                          BFP_FLAG_OUT_FP32))
    return fail(BFP_EINVAL, "unknown flag for sar_azimuth_compress");
  if (rc_t == image) return fail(BFP_EINVAL, "rc_t and image must differ");
  // the filter is conjugated when exactly one of (the call's or the plan's
  // BFP_FLAG_CONJ_FILTER, adjoint) asks for it: the adjoint of the chain with
  // conj(H) is the chain with H
  const bool conj = (((flags | az_plan->flags) & BFP_FLAG_CONJ_FILTER) != 0) != (adjoint != 0);
  if ((flags | az_plan->flags) & BFP_FLAG_NAIVE_POSTSCALE) {
    if (conj || phase) return fail(BFP_EUNSUPPORTED, "BFP_FLAG_NAIVE_POSTSCALE combines with neither a phase nor the conjugated filter");
  }
  if (phase && ((flags | az_plan->flags) & BFP_FLAG_OUT_FP32) && (conj || adjoint))
    return fail(BFP_EUNSUPPORTED, "FP32 output with a phase vector is the forward chain with H only");
  flags = (flags & ~(unsigned)BFP_FLAG_CONJ_FILTER) | (conj ? BFP_FLAG_CONJ_FILTER : 0u) | kExactConj;
  const void *ph = nullptr;
  if (phase) {
    // forward: exp(+i phase) on the input; adjoint: exp(-i phase) on the output
    az_plan->phasor_sign = 0;
    hipError_t e = bfp::launch_phasor(phase, az_plan->phasor, az_plan->n, adjoint ? 1 : 0,
                                      (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "phasor launch");
    az_plan->phasor_sign = adjoint ? -1 : 1;
    ph = az_plan->phasor;
    if (adjoint) flags |= kPostPhasor;
  }
  return run_rows(az_plan, bfp::OP_COMPRESS, rc_t, image, h_az, ph, n_range, flags, stream);
}

int sar_image_entropy(bfp_plan plan, const void *image, long long count, double *stats,
                      void *stream) {
  if (!plan) return fail(BFP_EINVAL, "plan is NULL");
  if (!plan->ent_partial) return fail(BFP_EINVAL, "plan has no entropy workspace");
  if (count < 1) return fail(BFP_EINVAL, "count must be >= 1");
  if (!image || !stats) return fail(BFP_EINVAL, "NULL pointer");
  hipError_t e = bfp::launch_entropy(image, count, plan->ent_partial, stats, (hipStream_t)stream);
  return e == hipSuccess ? BFP_OK : hip_fail(e, "entropy launch");
}

int sar_image_entropy_noalloc(const void *image, long long count, double *stats, void *stream) {
  if (count < 1 || count > bfp::kEntropyNoAllocMaxCount)
    return fail(BFP_EINVAL, "count must lie in [1, 2^40]: the no-allocation entropy reduces at most "
                            "2^40 values through its fixed 1024-workgroup scratch");
  if (!image || !stats) return fail(BFP_EINVAL, "NULL pointer");
  hipError_t e = bfp::launch_entropy_noalloc(image, count, stats, (hipStream_t)stream);
  return e == hipSuccess ? BFP_OK : hip_fail(e, "no-allocation entropy launch");
}

int sar_azimuth_image_entropy(bfp_plan az_plan, const void *rc_t, void *image, const void *h_az,
                              const float *phase, int n_range, double *stats, void *stream) {
  int st = check_rows_plan(az_plan);
  if (st) return st;
  if (az_plan->prec != BFP_FP32 && az_plan->prec != BFP_FP16_STORE_FP32_COMPUTE)
    return fail(BFP_EUNSUPPORTED, "the fused image entropy runs in BFP_FP32 or BFP_FP16_STORE_FP32_COMPUTE");
  if (!h_az || !stats) return fail(BFP_EINVAL, "NULL pointer");
  if (n_range < 1 || n_range > az_plan->batch)
    return fail(BFP_EINVAL, "n_range outside [1, plan batch]");
  if (rc_t == image) return fail(BFP_EINVAL, "rc_t and image must differ");
  const void *ph = nullptr;
  if (phase) {
    az_plan->phasor_sign = 0;
    hipError_t e = bfp::launch_phasor(phase, az_plan->phasor, az_plan->n, 0, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "phasor launch");
    az_plan->phasor_sign = 1;
    ph = az_plan->phasor;
  }
  int grid = 0;
  st = run_rows(az_plan, bfp::OP_COMPRESS, rc_t, image, h_az, ph, n_range, BFP_FLAG_OUT_FP32,
                stream, az_plan->ent_partial, &grid);
  if (st) return st;
  hipError_t e = bfp::launch_entropy_final(az_plan->ent_partial, grid, stats, (hipStream_t)stream);
  return e == hipSuccess ? BFP_OK : hip_fail(e, "entropy launch");
}

int sar_entropy_grad(const void *image, const double *stats, const float *scale, void *grad,
                     long long count, void *stream) {
  if (count < 0) return fail(BFP_EINVAL, "count < 0");
  if (count == 0) return BFP_OK;
  if (!image || !stats || !grad) return fail(BFP_EINVAL, "NULL pointer");
  hipError_t e = bfp::launch_entropy_grad(image, stats, scale, grad, count, (hipStream_t)stream);
  return e == hipSuccess ? BFP_OK : hip_fail(e, "entropy gradient launch");
}

int sar_autofocus_adam(float *phase, const float *grad, float *m, float *v, unsigned *step, int n,
                       float lr, float beta1, float beta2, float eps, void *stream) {
  if (n < 1 || n > (1 << 20)) return fail(BFP_EINVAL, "n outside [1, 2^20]");
  if (!phase || !grad || !m || !v || !step) return fail(BFP_EINVAL, "NULL pointer");
  if (!(lr >= 0.0f && lr < 1e30f)) return fail(BFP_EINVAL, "lr must be finite and >= 0");
  if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f))
    return fail(BFP_EINVAL, "beta1 and beta2 must lie in [0, 1)");
  if (!(eps > 0.0f && eps < 1e30f)) return fail(BFP_EINVAL, "eps must be finite and > 0");
  hipError_t e = bfp::launch_adam(phase, grad, m, v, step, n, lr, beta1, beta2, eps, nullptr, 0,
                                  (hipStream_t)stream);
  return e == hipSuccess ? BFP_OK : hip_fail(e, "Adam launch");
}

int sar_autofocus_adam_schedule(float *phase, const float *grad, float *m, float *v, unsigned *step,
                                int n, const float *lr_schedule, int schedule_len, float beta1,
                                float beta2, float eps, void *stream) {
  if (n < 1 || n > (1 << 20)) return fail(BFP_EINVAL, "n outside [1, 2^20]");
  if (!phase || !grad || !m || !v || !step || !lr_schedule) return fail(BFP_EINVAL, "NULL pointer");
  if (schedule_len < 1 || schedule_len > (1 << 20))
    return fail(BFP_EINVAL, "schedule_len outside [1, 2^20]");
  if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f))
    return fail(BFP_EINVAL, "beta1 and beta2 must lie in [0, 1)");
  if (!(eps > 0.0f && eps < 1e30f)) return fail(BFP_EINVAL, "eps must be finite and > 0");
  hipError_t e = bfp::launch_adam(phase, grad, m, v, step, n, 0.0f, beta1, beta2, eps, lr_schedule,
                                  schedule_len, (hipStream_t)stream);
  return e == hipSuccess ? BFP_OK : hip_fail(e, "Adam launch");
}

int sar_azimuth_phase_grad(bfp_plan az_plan, const void *rc_t, const void *g, const double *stats,
                           const void *h_az, const float *phase, float *grad_phase, int n_range,
                           void *stream) {
  int st = check_rows_plan(az_plan);
  if (st) return st;
  if (!az_plan->pg_partial) return fail(BFP_EINVAL, "plan was not created with BFP_FLAG_AUTOFOCUS");
  if (n_range < 1 || n_range > az_plan->batch)
    return fail(BFP_EINVAL, "n_range outside [1, plan batch]");
  if (!rc_t || !g || !h_az || !grad_phase) return fail(BFP_EINVAL, "NULL pointer");
  if (!phase && az_plan->phasor_sign != 1)
    return fail(BFP_EINVAL, "phase is NULL and no earlier call on this plan left exp(+i phase) in its table");
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != az_plan->device) return fail(BFP_EINVAL, "plan belongs to another device");
  hipError_t e = hipSuccess;
  if (phase) {
    az_plan->phasor_sign = 0;
    e = bfp::launch_phasor(phase, az_plan->phasor, az_plan->n, 0, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "phasor launch");
    az_plan->phasor_sign = 1;
  }
  bfp::PhaseGradArgs a;
  a.gimg = g;
  a.stats = stats;
  a.rc_t = rc_t;
  a.filter = h_az;
  a.phasor = az_plan->phasor;
  a.tw32 = az_plan->tw32;
  a.tw32_alt = az_plan->tw_alt;  // FP32 as well in both admitted modes
  a.partial = az_plan->pg_partial;
  a.grad = grad_phase;
  a.rows = n_range;
  a.rows_per_thread = az_plan->tune_rr;
  a.radix_plan = az_plan->tune_plan;
  e = bfp::launch_phase_grad(az_plan->prec == BFP_FP16_STORE_FP32_COMPUTE, az_plan->log2n, a,
                             stats != nullptr, (hipStream_t)stream);
  return e == hipSuccess ? BFP_OK : hip_fail(e, "phase gradient launch");
}

int fft_plan_set_tuning(bfp_plan p, int engine, int blocks_per_cu) {
  if (!p) return fail(BFP_EINVAL, "plan is NULL");
  if (engine < 0 || engine > 1) return fail(BFP_EINVAL, "engine must be 0 or 1");
  if (blocks_per_cu < -1 || blocks_per_cu > 64)
    return fail(BFP_EINVAL, "blocks_per_cu must be -1 (automatic) or in [0, 64]");
  if (p->kind == 1 && blocks_per_cu < 0) return fail(BFP_EINVAL, "uneven plans take blocks_per_cu >= 0");
  if (p->kind == 1) {
    // above the resident maximum the hardware queues the extra workgroups
    const int b = blocks_per_cu == 0 ? p->uneven_max_bpc : blocks_per_cu;
    p->grid = b * p->cu_count;
  }
  p->tune_engine = engine;
  p->tune_bpc = blocks_per_cu;
  return BFP_OK;
}

int fft_plan_set_tuning_ex(bfp_plan p, const bfp_tuning *t) {
  if (!p || !t) return fail(BFP_EINVAL, "NULL argument");
  if (t->rows_per_thread < 1 || t->rows_per_thread > 2)
    return fail(BFP_EINVAL, "rows_per_thread must be 1 or 2");
  if (p->kind == 1 && t->rows_per_thread != 1)
    return fail(BFP_EINVAL, "uneven plans take rows_per_thread = 1");
  if (t->radix_plan < 0 || t->radix_plan > 1) return fail(BFP_EINVAL, "radix_plan must be 0 or 1");
  if (t->radix_plan == 1 && (p->kind != 0 || !bfp::second_plan(p->log2n)))
    return fail(BFP_EINVAL, "this plan's size has one radix plan (n <= 16, or an uneven plan)");
  int st = fft_plan_set_tuning(p, t->engine, t->blocks_per_cu);
  if (st) return st;
  p->tune_rr = t->rows_per_thread;
  p->tune_plan = t->radix_plan;
  return BFP_OK;
}

int fft_plan_get_tuning_ex(bfp_plan p, bfp_tuning *t) {
  if (!p || !t) return fail(BFP_EINVAL, "NULL argument");
  t->engine = p->tune_engine;
  t->blocks_per_cu = p->tune_bpc;
  t->rows_per_thread = p->tune_rr;
  t->radix_plan = p->tune_plan;
  return BFP_OK;
}

int fft_plan_get_tuning(bfp_plan p, int *engine, int *blocks_per_cu) {
  if (!p) return fail(BFP_EINVAL, "plan is NULL");
  if (engine) *engine = p->tune_engine;
  if (blocks_per_cu) *blocks_per_cu = p->tune_bpc;
  return BFP_OK;
}

int fft_autotune_sets(bfp_plan p, int op, const void *const *ins, void *const *outs, int n_sets,
                      const void *filter, int reps, float *best_ms, void *stream) {
  if (!p) return fail(BFP_EINVAL, "plan is NULL");
  if (reps < 1 || reps > 10000) return fail(BFP_EINVAL, "reps must be in [1, 10000]");
  if (n_sets < 1 || n_sets > 4096) return fail(BFP_EINVAL, "n_sets must be in [1, 4096]");
  if (!ins || !outs) return fail(BFP_EINVAL, "NULL buffer array");
  for (int i = 0; i < n_sets; ++i)
    if (!ins[i] || !outs[i]) return fail(BFP_EINVAL, "NULL buffer in the sets");
  if (p->kind == 0 && (op < 0 || op > 2)) return fail(BFP_EINVAL, "op must be 0, 1 or 2");
  if (p->kind == 0 && op == 2 && !filter) return fail(BFP_EINVAL, "compression needs a filter");
  std::vector<bfp_tuning> cands;
  if (p->kind == 1) {
    // resident grids (the persistent loop over the work queue), then larger
    // ones, up to one workgroup per tile, whose extra workgroups the
    // hardware dispatches as resident ones finish
    for (int b = 1; b <= p->uneven_max_bpc; ++b) cands.push_back({0, b, 1, 0});
    for (int b : {4, 8, 16, 32, 64})
      if (b > p->uneven_max_bpc) cands.push_back({0, b, 1, 0});
  } else {
    // engine x persistent grid x rows per thread x radix plan (the
    // matrix-core kernels take one row per workgroup and plan 0)
    const bool mf = bfp::has_mfma_engine(p->prec, p->log2n);
    const int plans = bfp::second_plan(p->log2n) ? 2 : 1;
    for (int e = 0; e <= (mf ? 1 : 0); ++e)
      for (int b : {kAutoBpc, 0, 1, 2, 3, 4, 5, 6, 8})
        for (int rr = 1; rr <= ((mf && e == 0) ? 1 : 2); ++rr)
          for (int pl = 0; pl < ((mf && e == 0) ? 1 : plans); ++pl) cands.push_back({mf ? e : 1, b, rr, pl});
  }
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(BFP_EHIP, "hipEventCreate failed");
  auto call = [&](int k) -> int {
    const void *in = ins[k % n_sets];
    void *out = outs[k % n_sets];
    if (p->kind == 1) return fft_exec_uneven(p, in, out, stream);
    if (op == 0) return fft_exec_fwd(p, in, out, stream);
    if (op == 1) return fft_exec_inv_bfp(p, in, out, filter, stream);
    return sar_range_compress(p, in, out, filter, p->batch, 0u, stream);
  };
  float best = 1e30f;
  bfp_tuning pick = cands.front();
  int st = BFP_OK;
  for (auto &c : cands) {
    if ((st = fft_plan_set_tuning_ex(p, &c))) break;
    // the rotation runs on from the warm-up calls, so the timed calls do not
    // start on the sets the warm-up just left in the last-level cache
    int k = 0;
    for (int w = 0; w < 2 && !st; ++w) st = call(k++);
    if (st) break;
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps && !st; ++r) st = call(k++);
    (void)hipEventRecord(e1, s);
    if (st) break;
    if (hipEventSynchronize(e1) != hipSuccess) { st = fail(BFP_EHIP, "hipEventSynchronize"); break; }
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    ms /= (float)reps;
    if (ms < best) { best = ms; pick = c; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) return st;
  if (best_ms) *best_ms = best;
  return fft_plan_set_tuning_ex(p, &pick);
}

int fft_autotune(bfp_plan p, int op, const void *in, void *out, const void *filter, int reps,
                 float *best_ms, void *stream) {
  const void *ins[1] = {in};
  void *outs[1] = {out};
  if (!in || !out) return fail(BFP_EINVAL, "NULL data pointer");
  return fft_autotune_sets(p, op, ins, outs, 1, filter, reps, best_ms, stream);
}

/* uneven entry points are defined in uneven_api.cpp */

}  // extern "C"
