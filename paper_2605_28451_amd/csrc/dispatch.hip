// Dispatch from (mode, size, op) to the per-mode row-kernel objects, and the
// size geometry the host needs to build twiddle tables.
#include "fft_engine.hpp"
#include "internal.hpp"

namespace bfp {

hipError_t launch_rows_mode0(int, int, bool, const RowArgs &, hipStream_t);
hipError_t launch_rows_mode1(int, int, bool, const RowArgs &, hipStream_t);
hipError_t launch_rows_mode2(int, int, bool, const RowArgs &, hipStream_t);
hipError_t launch_rows_mode3(int, int, bool, const RowArgs &, hipStream_t);
hipError_t launch_rows_mode4(int, int, bool, const RowArgs &, hipStream_t);
hipError_t launch_rows_mode5(int, int, bool, const RowArgs &, hipStream_t);

hipError_t launch_rows(int mode, int log2n, int op, bool out32, const RowArgs &a,
                       hipStream_t s) {
  switch (mode) {
    case 0: return launch_rows_mode0(log2n, op, out32, a, s);
    case 1: return launch_rows_mode1(log2n, op, out32, a, s);
    case 2: return launch_rows_mode2(log2n, op, out32, a, s);
    case 3: return launch_rows_mode3(log2n, op, out32, a, s);
    case 4: return launch_rows_mode4(log2n, op, out32, a, s);
    case 5: return launch_rows_mode5(log2n, op, out32, a, s);
  }
  return hipErrorInvalidValue;
}

#define BFP_DECL_UNEVEN(m)                                                  \
  hipError_t launch_uneven_mode##m(const UnevenArgs &, int, hipStream_t); \
  int uneven_blocks_per_cu_mode##m();
BFP_DECL_UNEVEN(0)
BFP_DECL_UNEVEN(1)
BFP_DECL_UNEVEN(2)
BFP_DECL_UNEVEN(3)
BFP_DECL_UNEVEN(4)
BFP_DECL_UNEVEN(5)

hipError_t launch_uneven(int mode, const UnevenArgs &a, int grid, hipStream_t s) {
  switch (mode) {
    case 0: return launch_uneven_mode0(a, grid, s);
    case 1: return launch_uneven_mode1(a, grid, s);
    case 2: return launch_uneven_mode2(a, grid, s);
    case 3: return launch_uneven_mode3(a, grid, s);
    case 4: return launch_uneven_mode4(a, grid, s);
    case 5: return launch_uneven_mode5(a, grid, s);
  }
  return hipErrorInvalidValue;
}

int uneven_blocks_per_cu(int mode) {
  switch (mode) {
    case 0: return uneven_blocks_per_cu_mode0();
    case 1: return uneven_blocks_per_cu_mode1();
    case 2: return uneven_blocks_per_cu_mode2();
    case 3: return uneven_blocks_per_cu_mode3();
    case 4: return uneven_blocks_per_cu_mode4();
    case 5: return uneven_blocks_per_cu_mode5();
  }
  return 1;
}

template <int L, int PLAN>
static void geo(int &entries, int &passes, int *rad) {
  typedef Geometry<L, PLAN> G;
  entries = G::tw_entries();
  passes = G::S::P;
  for (int p = 0; p < 4; ++p) rad[p] = G::radix(p);
}

template <int PLAN>
static void geometry_plan(int log2n, int &entries, int &passes, int *rad) {
  switch (log2n) {
    case 3: geo<3, PLAN>(entries, passes, rad); return;
    case 4: geo<4, PLAN>(entries, passes, rad); return;
    case 5: geo<5, PLAN>(entries, passes, rad); return;
    case 6: geo<6, PLAN>(entries, passes, rad); return;
    case 7: geo<7, PLAN>(entries, passes, rad); return;
    case 8: geo<8, PLAN>(entries, passes, rad); return;
    case 9: geo<9, PLAN>(entries, passes, rad); return;
    case 10: geo<10, PLAN>(entries, passes, rad); return;
    case 11: geo<11, PLAN>(entries, passes, rad); return;
    case 12: geo<12, PLAN>(entries, passes, rad); return;
    case 13: geo<13, PLAN>(entries, passes, rad); return;
    case 14: geo<14, PLAN>(entries, passes, rad); return;
  }
  entries = passes = 0;
}

static void geometry(int log2n, int plan, int &entries, int &passes, int *rad) {
  if (plan == 1) geometry_plan<1>(log2n, entries, passes, rad);
  else geometry_plan<0>(log2n, entries, passes, rad);
}

int twiddle_entries(int log2n, int plan) {
  int e, p, r[4];
  geometry(log2n, plan, e, p, r);
  return e;
}
int pass_count(int log2n, int plan) {
  int e, p, r[4];
  geometry(log2n, plan, e, p, r);
  return p;
}
bool second_plan(int log2n) { return has_second_plan(log2n); }

int threads_per_transform(int log2n) {
  switch (log2n) {
    case 3: return Geometry<3>::T;
    case 4: return Geometry<4>::T;
    case 5: return Geometry<5>::T;
    case 6: return Geometry<6>::T;
    case 7: return Geometry<7>::T;
    case 8: return Geometry<8>::T;
    case 9: return Geometry<9>::T;
    case 10: return Geometry<10>::T;
    case 11: return Geometry<11>::T;
    case 12: return Geometry<12>::T;
    case 13: return Geometry<13>::T;
    case 14: return Geometry<14>::T;
  }
  return 0;
}

int pass_radix(int log2n, int plan, int q) {
  int e, p, r[4];
  geometry(log2n, plan, e, p, r);
  return (q >= 0 && q < 4) ? r[q] : 0;
}

}  // namespace bfp
