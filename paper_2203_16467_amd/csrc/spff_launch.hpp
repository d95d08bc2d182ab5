// Host-visible declarations of the kernel launchers defined in
// spff_kernels.hip (explicitly instantiated there for float and double).
#pragma once
#include <hip/hip_runtime.h>

#include "spff_engine.hpp"

namespace spff {

template <typename real> struct HostCplx;
template <> struct HostCplx<float> { using type = float2; };
template <> struct HostCplx<double> { using type = double2; };

struct LaunchGeom {
  int nx, ny, S;
  int R, ngr;  // rows per row work-group, row groups per slot
  int W, ngc;  // columns per column work-group, column groups per slot
  int threads;      // threads per row work-group
  int threads_col;  // threads per column work-group
  int col_reg;      // column kernel with register-resident transforms
  int col_pts;      // its points per lane: 8, or 16 (1024- and 2048-point columns)
  int row_reg;      // row kernels with register-resident transforms: 1 = 8, 2 = 4 points per lane
  int nyq_free;     // even grids: Nyquist modes of the strain fluctuation unconstrained
  size_t lds_row, lds_col;
};

// Device buffers of a handle's ticks.
template <typename real>
struct TickBufs {
  const int* list;            // listed slots (G.S entries, < 0: padding)
  const SlotPtr<real>* ptrs;  // per slot
  const SlotParam* prms;
  SlotCtl* ctl[2];            // control blocks; the host reads and writes ctl[0]
  const typename HostCplx<real>::type* twx;
  const typename HostCplx<real>::type* twy;
  double* prow[2];            // row-forward partials, alternating by tick
  double* pcol;
  double* pinv;
  double* prof;               // per-slot byte counters, or null
  SlotSeq* seqs;              // device load-step queues, or null
  StepRec* recs;
  KTime* kt;                  // six kernel timers (two ticks x three kernels), or null
  unsigned long long* ktsum;  // folded kernel times
};

// Tick i (0-based) of a block of ticks over the listed slots.  Tick 0 reads
// ctl[0], whose blocks must have no controller step pending (as the host
// and launch_close leave them).
template <typename real>
hipError_t launch_tick(const LaunchGeom& G, const TickBufs<real>& B, int i, hipStream_t st);

// Closes a block of k ticks: the controller step of tick k - 1, leaving
// every listed slot's control block in ctl[0].
template <typename real>
hipError_t launch_close(const LaunchGeom& G, const TickBufs<real>& B, int k, hipStream_t st);

template <typename real>
hipError_t launch_validate(const real* a, size_t n, double lo_excl, double lo_incl, double hi_incl,
                           unsigned int* bad, hipStream_t st);

template <typename real>
hipError_t launch_fields(const SlotPtr<real>* ptrs, const SlotParam* prms, const SlotCtl* ctls, int slot, int n,
                         real* strain, real* stress_out, real* psi, hipStream_t st);

// Address of the current device's copy of the library-owned scratch array
// (SPFF_STATIC_SCRATCH_BYTES bytes, 256-byte aligned).
hipError_t static_scratch(void** out);

}  // namespace spff
