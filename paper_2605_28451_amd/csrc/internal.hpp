// Host-side internal interfaces shared by the C-ABI layer and the kernel
// translation units.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace bfp {

enum Op { OP_FWD = 0, OP_INV = 1, OP_COMPRESS = 2 };

// runtime flags understood by the row kernels
enum KFlags : unsigned {
  KF_NAIVE = 1u,         // conventional post-scaling instead of the BFP fold
  KF_CHECK_FINITE = 2u,  // count non-finite outputs
  KF_TRANSPOSED = 4u,    // compression: store out[k][row] (n x rows)
  KF_CONJ_FILTER = 16u,  // multiply by conj(filter)
  KF_ADAPT = 32u,        // per-row adaptive block shift (row_exp)
  KF_RAMP = 64u,         // compression: per-row range shift (shift)
  KF_POST_PHASOR = 128u, // compression: multiply the output (not the input) by the phasor
};

struct RowArgs {
  const void *in;
  void *out;
  int rows;
  const void *tw;        // plan twiddle table (mode's twiddle type; with a matrix-core
                         // engine its operands first, the vector table at kMfmaTableBytes)
  const void *tw_alt;    // the second radix plan's table, or NULL
  const void *filter;    // n elements or NULL
  const void *phasor;    // n FP32 pairs exp(+-i phi_m) or NULL (compress only): applied
                         // to the input, or to the output with KF_POST_PHASOR
  unsigned flags;        // KFlags
  unsigned long long *nonfinite;  // device counter
  int grid_limit;        // > 0: persistent grid of at most this many workgroups
  int resident_cus;      // > 0 with grid_limit == 0 (image entropy variants): a persistent
                         // grid of the launched kernel's resident workgroups on this many CUs
  int engine;            // 0: matrix cores where available, 1: vector ALU only
  int rows_per_thread;   // 1, or 2: the multi-row kernel where it covers the variant
  int radix_plan;        // 0, or 1: the second radix plan (tw_alt) where the multi-row
                         // kernel covers the variant
  int *grid_out;         // host: set to the launch's workgroup count, or NULL
  double *ent_partial;   // compression to FP32 with phasor: per-workgroup (S, Q) of the
                         // output's entropy sums (one per workgroup: grid_out), or NULL
  int *row_exp;          // KF_ADAPT: per-row block exponent of the output, or NULL
  const float *shift;    // KF_RAMP: per-row range shift in bins (RCMC), or NULL
};


// whether (mode, size) has a matrix-core engine
inline bool has_mfma_engine(int mode, int log2n) { return mode == 3 && log2n == 12; }
// bytes of the matrix-core table (operand slices + dot2-form twiddles)
constexpr int kMfmaTableBytes = 2 * (2048 + 4 * (256 + 4096));

// Launch a row kernel; returns hipSuccess or the launch error.
hipError_t launch_rows(int mode, int log2n, int op, bool out32, const RowArgs &a,
                       hipStream_t stream);

// Number of twiddle-table entries of a size (all passes), and the
// (pass span, radix) sequence used to fill it on the host.
// (plan: 0 or 1, the radix plans of fft_engine.hpp)
int twiddle_entries(int log2n, int plan = 0);
int pass_count(int log2n, int plan = 0);
int pass_radix(int log2n, int plan, int p);
bool second_plan(int log2n);

// Uneven persistent batch.
struct UnevenArgs {
  const void *in;
  void *out;
  const int4 *items;          // (first position in xform[], count, log2n, inverse) per item
  // one word per transform, grouped by length, longest first:
  // (element offset << 1) | inverse
  const long long *xform;
  int n_items;
  unsigned *queue;            // work counter (items claimed after the first
                              // gridDim.x), zeroed by the launcher's reset kernel
  const void *const *tw;      // per-size twiddle tables, index log2n - 8
  unsigned flags;
  unsigned long long *nonfinite;
  int off32;                  // packed batch below 4 GiB: 32-bit byte offsets
};
hipError_t launch_uneven(int mode, const UnevenArgs &a, int grid, hipStream_t stream);
int uneven_blocks_per_cu(int mode);
int threads_per_transform(int log2n);
constexpr int kUnevenWG = 1024;

// Element-wise storage conversion.
hipError_t launch_convert(const void *in, int in_fmt, void *out, int out_fmt, long long count,
                          hipStream_t stream);

// Corner turn (transpose) of a rows x cols matrix of elements of `bytes`.
hipError_t launch_transpose(const void *in, void *out, int rows, int cols, int bytes,
                            hipStream_t stream);

// 16-byte-per-lane device copy of `bytes` (a multiple of 16).
hipError_t launch_copy(const void *in, void *out, long long bytes, hipStream_t stream);

// exp(i phi) table (FP32 pairs) from FP32 radians.
hipError_t launch_phasor(const float *phase, void *phasor, int n, int negate,
                         hipStream_t stream);

// Autofocus: entropy statistics (S, Q, E), entropy gradient and the fused
// adjoint + per-pulse phase-gradient reduction.
constexpr int kEntropyBlocks = 1024;
// grid of the phase-gradient kernel: one round of resident workgroups on
// MI355X (their ~66 KiB of LDS allow two per CU on 256 CUs), each workgroup
// writing one partial row per transform slot; 1024 (two rounds, twice the
// partial rows) measured 82.5 against 78.8 us at 4096 x 4096 (radix plan 1)
constexpr int kPhaseGradBlocks = 512;
struct PhaseGradArgs {
  const void *gimg;      // FP32 pairs: dL/dI, or the image itself when fused
  const double *stats;   // (S, Q, E) when fused, else unused
  const void *rc_t;      // range-compressed data, plan storage (FP16 or FP32)
  const void *filter;    // azimuth filter, plan filter format
  const void *phasor;    // FP32 pairs exp(i phi_m)
  const void *tw32;      // FP32 twiddle table of the size (radix plan 0)
  const void *tw32_alt;  // FP32 twiddle table of radix plan 1 (sizes with two plans)
  float *partial;        // kPhaseGradBlocks * transforms-per-workgroup rows of n floats
  float *grad;           // n floats out
  int rows;
  int rows_per_thread;   // 1, or 2 where the kernel fits (n <= 4096)
  int radix_plan;        // 0, or 1 where that plan fits the partials (see launch_pg)
};
// (S, Q, E) from `blocks` partial (S, Q) pairs, summed in a fixed order.
hipError_t launch_entropy_final(const double *partial, int blocks, double *stats, hipStream_t s);
hipError_t launch_entropy(const void *img, long long count, double *partial, double *stats,
                          hipStream_t s);
// launch_entropy with its partials in a file-scope device array (no
// allocation); kEntropyNoAllocPartials (S, Q) pairs = 16 KiB per device
constexpr int kEntropyNoAllocPartials = 1024;
constexpr int kMaxDevices = 64;
constexpr long long kEntropyNoAllocMaxCount = 1ll << 40;
hipError_t launch_entropy_noalloc(const void *img, long long count, double *stats, hipStream_t s);
hipError_t launch_entropy_grad(const void *img, const double *stats, const float *scale, void *grad,
                               long long count, hipStream_t s);
hipError_t launch_phase_grad(bool fp16_storage, int log2n, const PhaseGradArgs &a, bool fused,
                             hipStream_t s);
hipError_t launch_adam(float *phase, const float *grad, float *m, float *v, unsigned *step, int n,
                       float lr, float b1, float b2, float eps, const float *lr_sched, int sched_len,
                       hipStream_t s);
long long phase_grad_scratch_floats(int log2n);

}  // namespace bfp
