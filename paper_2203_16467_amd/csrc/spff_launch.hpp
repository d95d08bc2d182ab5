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
  int row_reg;      // row kernels with register-resident transforms: 1 = 8, 2 = 4 points per lane
  int nyq_free;     // even grids: Nyquist modes of the strain fluctuation unconstrained
  size_t lds_row, lds_col;
};

// One solver tick over the slots list[0..G.S) (entries < 0 are padding).
template <typename real>
hipError_t launch_tick(const LaunchGeom& G, const int* list, const SlotPtr<real>* ptrs, const SlotParam* prms,
                       SlotCtl* ctls, const typename HostCplx<real>::type* twx,
                       const typename HostCplx<real>::type* twy, double* prow, double* pcol, double* pinv,
                       double* prof, SlotSeq* seqs, StepRec* recs, KTime* kt, unsigned long long* ktsum,
                       hipStream_t st);

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
