// Plan object shared by the C-ABI translation units (host only).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "bfpfft.h"

struct bfp_plan_s {
  int kind = 0;  // 0: rows, 1: uneven
  int n = 0, log2n = 0, batch = 0, prec = 0;
  unsigned flags = 0;
  int device = 0;
  void *tw = nullptr;                         // rows: this size's table
  void *tw_alt = nullptr;                     // rows: the second radix plan's table
  unsigned long long *nonfinite = nullptr;    // device counter
  void *phasor = nullptr;                     // n FP32 pairs (rows plans)
  int phasor_sign = 0;  // what the last call left in phasor: 0 nothing, +1 exp(+i phi)
                        // (forward), -1 exp(-i phi) (adjoint)
  // uneven plans
  int count = 0;
  long long total = 0;
  std::vector<long long> offsets;
  int4 *items = nullptr;
  long long *xform_d = nullptr;               // (offset << 1) | inverse, item order
  int n_items = 0;
  unsigned *queue = nullptr;
  int grid = 0;
  // tuning knobs (fft_plan_set_tuning / fft_autotune)
  int tune_engine = 1;     // 0: matrix cores where available, 1: vector ALU (default)
  int tune_bpc = 0;        // workgroups per CU of a persistent grid, 0 = default
  int tune_rr = 1;         // rows per thread (1, or 2: the multi-row kernel)
  int tune_plan = 0;       // radix plan (0, or 1 where the size has a second)
  int cu_count = 0;
  int uneven_max_bpc = 1;
  // autofocus workspace
  void *tw32 = nullptr;          // FP32 twiddles (owned only when tw is FP16)
  double *ent_partial = nullptr; // kEntropyBlocks x 2 doubles
  float *pg_partial = nullptr;   // phase-gradient partial rows
  void *tw_sizes[7] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  void **tw_ptrs_d = nullptr;
};

namespace bfp {
// Records msg as the calling thread's last error and returns status.
int set_error(int status, const std::string &msg);
}  // namespace bfp
