// Solver kernels for gfx950.  One tick = k_rowfwd -> k_col -> k_rowinv over
// all listed slots of a handle; the row-forward kernel first advances each
// slot's control block by the controller step of the previous tick, and a
// block of ticks ends with k_close (the controller step of its last tick).
// Every kernel looks up the phase of its slot and does that phase's share of
// the work (or returns).
//
// Data layout (per slot, real = float or double):
//   real planes [ny][nx]; tensors as 3 planes (xx, yy, xy)
//   spectrum: complex [C][nx/2][ny] -- the half spectrum of each plane,
//             stored transposed (one contiguous run of ny per kx) so the
//             column kernel reads and writes whole columns; kx = 0 holds
//             X[0] + i X[nx/2] (both columns of a real row transform are
//             real-valued per row, so they share one complex column).
//
// Row kernels: a work-group owns R consecutive rows of one slot and all C
// components; a column kernel work-group owns W consecutive kx columns.
#include <hip/hip_runtime.h>

#include <mutex>
#include <type_traits>

#include "spff.h"
#include "spff_device.hpp"
#include "spff_engine.hpp"
#include "spff_launch.hpp"

namespace spff {

constexpr int THREADS = 256;
constexpr int MAXE = 8;   // FFT elements per thread per chunk: M <= 2048
constexpr int PAD = 1;    // complex padding per LDS row (bank spread)
constexpr double TWO_PI = 6.283185307179586476925286766559;

__device__ __forceinline__ int phase_comps_row(int phase) {
  switch (phase) {
    case PH_M_RES:
    case PH_M_CG:
    case PH_X_PROJ:
    case PH_X_DISP:
      return 3;
    case PH_PF_ASM:
    case PH_PF_PQ:
    case PH_PF_R:
    case PH_STATS:
    case PH_X_LAP:
      return 1;
    default:
      return 0;
  }
}

// Number of FP64 partial sums a kernel's phase produces for the controller
// (the leading entries of its accumulator array).
__device__ __forceinline__ int nacc_rowfwd(int phase) {
  switch (phase) {
    case PH_M_RES:
    case PH_PF_PQ:
    case PH_PF_ASM:
      return 2;
    case PH_M_CG:
    case PH_AM_CHK:
      return 1;
    case PH_STATS:
      return NP_ROW;
    default:
      return 0;
  }
}
__device__ __forceinline__ int nacc_rowinv(int phase) {
  switch (phase) {
    case PH_M_RES:
    case PH_M_CG:
      return 1;
    case PH_PF_ASM:
    case PH_PF_R:
      return NP_INV;
    default:
      return 0;
  }
}

// Row-kernel coordinates (row group g, list index si) of this work-group.
// Work-groups are dispatched to the 8 XCDs round-robin by linear id; the
// remap gives consecutive row groups of a slot to one XCD, so the short
// transposed spectrum segments of neighbouring groups (R rows each) meet in
// the same L2 and leave it as whole lines.
__device__ __forceinline__ void row_coords(int ngr, int& g, int& si) {
  const int N = gridDim.x * gridDim.y;
  int L = blockIdx.x + blockIdx.y * gridDim.x;
  if ((N & 7) == 0) L = (L & 7) * (N >> 3) + (L >> 3);
  const int lg = ilog2(ngr);  // ngr is a power of two
  si = L >> lg;
  g = L & (ngr - 1);
}

// Field and spectrum accesses go through global-address-space pointers: the
// slot's field pointers are read from the pointer table, so the compiler
// cannot tell they address device memory and would use flat instructions,
// whose completion it can only wait for all at once (a flat access may be an
// LDS access).  Global loads complete in order and are waited for one by
// one, so the loads of a prologue overlap the arithmetic on the first ones.
#define SPFF_GLOBAL __attribute__((address_space(1)))

template <typename real>
struct V2 {
  real a, b;
};

template <typename real>
struct Pair;
template <>
struct Pair<float> {
  typedef float type __attribute__((ext_vector_type(2)));
};
template <>
struct Pair<double> {
  typedef double type __attribute__((ext_vector_type(2)));
};
template <typename real>
__device__ __forceinline__ V2<real> ld2(const real* p) {
  using T = typename Pair<real>::type;
  const T v = *(const SPFF_GLOBAL T*)(p);
  return {v.x, v.y};
}
template <typename real>
__device__ __forceinline__ void st2(real* p, real a, real b) {
  using T = typename Pair<real>::type;
  T v;
  v.x = a;
  v.y = b;
  *(SPFF_GLOBAL T*)(p) = v;
}
// one complex value of a spectrum
template <typename real>
__device__ __forceinline__ cplx<real> ldc(const cplx<real>* p) {
  using T = typename Pair<real>::type;
  const T v = *(const SPFF_GLOBAL T*)(p);
  return mk<cplx<real>>(v.x, v.y);
}
template <typename real>
__device__ __forceinline__ void stc(cplx<real>* p, const cplx<real>& c) {
  using T = typename Pair<real>::type;
  T v;
  v.x = c.x;
  v.y = c.y;
  *(SPFF_GLOBAL T*)(p) = v;
}
__device__ __forceinline__ unsigned char ldb(const unsigned char* p) { return *(const SPFF_GLOBAL unsigned char*)(p); }
__device__ __forceinline__ void stb(unsigned char* p, unsigned char v) { *(SPFF_GLOBAL unsigned char*)(p) = v; }

template <typename real>
__device__ __forceinline__ real lower_bound(real pref, const SlotParam& P) {
  if (P.irr == 1) return pref;
  return pref >= real(P.threshold) ? pref : real(0);
}

// Per-slot scalars of a tick shared by the row prologue and epilogue.
template <typename real>
struct RowCtx {
  int phase, flags, split, contact, n, ncomp;  // split: driving-force model, contact: stress model
  real lt, mt, kres, eb0, eb1, eb2, beta_m, beta_pf, alpha_pf;
  real ne_gamma;  // near-equilibrium strain scaling (FL_NE_SCALE)
  double eta_dt;
};

template <typename real>
__device__ __forceinline__ RowCtx<real> row_ctx(const SlotCtl& ctl, const SlotParam& P, int phase, int ncomp, int n) {
  RowCtx<real> X;
  X.phase = phase;
  X.flags = ctl.flags;
  X.split = P.split;
  X.contact = P.contact;
  X.n = n;
  X.ncomp = ncomp;
  X.lt = real(P.lam_t);
  X.mt = real(P.mu_t);
  X.kres = real(P.k_res);
  X.eb0 = real(ctl.eps_bar[0]);
  X.eb1 = real(ctl.eps_bar[1]);
  X.eb2 = real(ctl.eps_bar[2]);
  X.beta_m = real(ctl.beta_m);
  X.beta_pf = real(ctl.beta_pf);
  X.alpha_pf = real(ctl.alpha_pf);
  X.eta_dt = ctl.eta_dt;
  X.ne_gamma = real(ctl.gamma);
  return X;
}

// Row-forward prologue for the pixel pair (o, o + 1): the phase's pointwise
// work, the values entering the transforms (val[c][0..1]) and the FP64
// partial sums.
// Inputs of the row prologue for one pixel pair, loaded ahead of the
// arithmetic (see row_prologue_n); the slots each phase uses are listed
// with pro_load_chunk.
template <typename real>
struct ProIn {
  V2<real> a[11];
  unsigned char m[2];
};

template <typename real, int PH = -1, bool PRE = false>
__device__ __forceinline__ void row_prologue(const RowCtx<real>& X, const SlotParam& P, const real* __restrict__ Ep,
                                             real* __restrict__ phip, real* __restrict__ prefp,
                                             real* __restrict__ epsp, real* __restrict__ thp,
                                             real* __restrict__ rmp, real* __restrict__ pmp, int o,
                                             real (&val)[3][2], double (&acc)[NP_ROW],
                                             const ProIn<real>& in = ProIn<real>{}) {
  // PH >= 0: the phase is known at compile time (the other cases fold away).
  // PRE: the inputs of this pair were loaded into `in` (PH one of M_RES,
  // M_CG, PF_ASM, PF_PQ, PF_R)
  const int phase = PH >= 0 ? PH : X.phase;
  const int flags = X.flags, split = X.split, contact = X.contact, n = X.n, ncomp = X.ncomp;
  const real lt = X.lt, mt = X.mt, kres = X.kres, eb0 = X.eb0, eb1 = X.eb1, eb2 = X.eb2;
#pragma unroll
  for (int q = 0; q < 2; ++q) val[0][q] = val[1][q] = val[2][q] = real(0);
  switch (phase) {
    case PH_M_RES: {
      const V2<real> E = PRE ? in.a[0] : ld2(Ep + o), ph = PRE ? in.a[1] : ld2(phip + o);
      if (flags & FL_FIRST_OF_STEP) st2(prefp + o, ph.a, ph.b);
      V2<real> ex = PRE ? in.a[2] : ld2(epsp + o), ey = PRE ? in.a[3] : ld2(epsp + n + o),
               exy = PRE ? in.a[4] : ld2(epsp + 2 * n + o);
      if (flags & FL_THETA_PENDING) {
        const V2<real> tx = PRE ? in.a[5] : ld2(thp + o), ty = PRE ? in.a[6] : ld2(thp + n + o),
                       txy = PRE ? in.a[7] : ld2(thp + 2 * n + o);
        ex = {ex.a + tx.a, ex.b + tx.b};
        ey = {ey.a + ty.a, ey.b + ty.b};
        exy = {exy.a + txy.a, exy.b + txy.b};
        st2(epsp + o, ex.a, ex.b);
        st2(epsp + n + o, ey.a, ey.b);
        st2(epsp + 2 * n + o, exy.a, exy.b);
      }
      const real Ev[2] = {E.a, E.b}, pv[2] = {ph.a, ph.b};
      const real xv[2] = {ex.a, ex.b}, yv[2] = {ey.a, ey.b}, sv[2] = {exy.a, exy.b};
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const real lam = lt * Ev[q], mu = mt * Ev[q];
        const real hk = (real(1) - pv[q]) * (real(1) - pv[q]) + kres;
        const Sym<real> e = {eb0 + xv[q], eb1 + yv[q], eb2 + sv[q]};
        const Sym<real> sg = stress(e, lam, mu, hk, contact);
        const Sym<real> eh = {eb0, eb1, eb2};
        const Sym<real> sh = stress(eh, lam, mu, hk, contact);
        acc[0] += double(ddot(sh, sh));
        acc[1] += double(ddot(sg, sg));
        val[0][q] = sg.xx;
        val[1][q] = sg.yy;
        val[2][q] = sg.xy;
      }
      break;
    }
    case PH_M_CG: {
      const V2<real> E = PRE ? in.a[0] : ld2(Ep + o), ph = PRE ? in.a[1] : ld2(phip + o);
      V2<real> px = PRE ? in.a[2] : ld2(rmp + o), py = PRE ? in.a[3] : ld2(rmp + n + o),
               pxy = PRE ? in.a[4] : ld2(rmp + 2 * n + o);
      if (!(flags & FL_CG_FIRST)) {
        const real bt = real(X.beta_m);
        const V2<real> qx = PRE ? in.a[5] : ld2(pmp + o), qy = PRE ? in.a[6] : ld2(pmp + n + o),
                       qxy = PRE ? in.a[7] : ld2(pmp + 2 * n + o);
        px = {px.a + bt * qx.a, px.b + bt * qx.b};
        py = {py.a + bt * qy.a, py.b + bt * qy.b};
        pxy = {pxy.a + bt * qxy.a, pxy.b + bt * qxy.b};
      }
      st2(pmp + o, px.a, px.b);
      st2(pmp + n + o, py.a, py.b);
      st2(pmp + 2 * n + o, pxy.a, pxy.b);
      V2<real> ex = {0, 0}, ey = {0, 0}, exy = {0, 0};
      if (contact != 0) {
        ex = PRE ? in.a[8] : ld2(epsp + o);
        ey = PRE ? in.a[9] : ld2(epsp + n + o);
        exy = PRE ? in.a[10] : ld2(epsp + 2 * n + o);
      }
      const real Ev[2] = {E.a, E.b}, pv[2] = {ph.a, ph.b};
      const real xv[2] = {ex.a, ex.b}, yv[2] = {ey.a, ey.b}, sv[2] = {exy.a, exy.b};
      const real pxv[2] = {px.a, px.b}, pyv[2] = {py.a, py.b}, psv[2] = {pxy.a, pxy.b};
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const real lam = lt * Ev[q], mu = mt * Ev[q];
        const real hk = (real(1) - pv[q]) * (real(1) - pv[q]) + kres;
        const Sym<real> e = {eb0 + xv[q], eb1 + yv[q], eb2 + sv[q]};
        const Sym<real> p = {pxv[q], pyv[q], psv[q]};
        const Sym<real> cp = tangent(e, p, lam, mu, hk, contact);
        acc[0] += double(ddot(p, cp));
        val[0][q] = cp.xx;
        val[1][q] = cp.yy;
        val[2][q] = cp.xy;
      }
      break;
    }
    case PH_PF_ASM: {
      const V2<real> E = PRE ? in.a[0] : ld2(Ep + o), ph = PRE ? in.a[1] : ld2(phip + o),
                     pr = PRE ? in.a[2] : ld2(prefp + o);
      V2<real> ex = PRE ? in.a[3] : ld2(epsp + o), ey = PRE ? in.a[4] : ld2(epsp + n + o),
               exy = PRE ? in.a[5] : ld2(epsp + 2 * n + o);
      if (flags & FL_NE_SCALE) {
        // near-equilibrium evolution: eps* <- gamma eps* (eps_bar was scaled
        // by the controller)
        const real g = X.ne_gamma;
        ex = {g * ex.a, g * ex.b};
        ey = {g * ey.a, g * ey.b};
        exy = {g * exy.a, g * exy.b};
        st2(epsp + o, ex.a, ex.b);
        st2(epsp + n + o, ey.a, ey.b);
        st2(epsp + 2 * n + o, exy.a, exy.b);
      }
      const real Ev[2] = {E.a, E.b}, pv[2] = {ph.a, ph.b}, rv[2] = {pr.a, pr.b};
      const real xv[2] = {ex.a, ex.b}, yv[2] = {ey.a, ey.b}, sv[2] = {exy.a, exy.b};
      real dv[2], bv[2], cv[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const real lam = lt * Ev[q], mu = mt * Ev[q];
        const Sym<real> e = {eb0 + xv[q], eb1 + yv[q], eb2 + sv[q]};
        real pp, pm;
        energies(e, lam, mu, split, &pp, &pm);
        dv[q] = real(2) * pp + real(P.cwl * P.wpp + X.eta_dt);
        // crack driving force -h'(phi_n) psi0+ (near-equilibrium trigger)
        if (flags & FL_NE_CHECK) acc[1] = fmax(acc[1], double(real(2) * (real(1) - rv[q]) * pp));
        bv[q] = real(2) * pp - real(P.cwl * P.dw0) + real(X.eta_dt) * rv[q];
        const real lo = lower_bound(rv[q], P);
        cv[q] = fmin(fmax(pv[q], lo), real(1));
        acc[0] += double(bv[q]) * double(bv[q]);
        val[0][q] = cv[q];
      }
      st2(thp + o, dv[0], dv[1]);
      st2(thp + n + o, bv[0], bv[1]);
      st2(thp + 2 * n + o, ph.a, ph.b);  // phi at the start of this PF solve
      st2(phip + o, cv[0], cv[1]);
      break;
    }
    case PH_PF_PQ: {
      const V2<real> r = PRE ? in.a[0] : ld2(rmp + o), d = PRE ? in.a[1] : ld2(thp + o);
      V2<real> p;
      if (flags & FL_PF_FIRST) {
        p = {-r.a, -r.b};
      } else {
        const V2<real> po = PRE ? in.a[2] : ld2(pmp + o);
        const real bt = real(X.beta_pf);
        p = {-r.a + bt * po.a, -r.b + bt * po.b};
      }
      const unsigned char* mask = reinterpret_cast<const unsigned char*>(pmp + n);
      if (PRE ? in.m[0] : ldb(mask + o)) p.a = real(0);
      if (PRE ? in.m[1] : ldb(mask + o + 1)) p.b = real(0);
      st2(pmp + o, p.a, p.b);
      acc[0] += double(d.a) * double(p.a) * double(p.a) + double(d.b) * double(p.b) * double(p.b);
      acc[1] += double(r.a) * double(p.a) + double(r.b) * double(p.b);
      val[0][0] = p.a;
      val[0][1] = p.b;
      break;
    }
    case PH_PF_R: {
      const V2<real> ph = PRE ? in.a[0] : ld2(phip + o), p = PRE ? in.a[1] : ld2(pmp + o),
                     pr = PRE ? in.a[2] : ld2(prefp + o);
      const real al = real(X.alpha_pf);
      const real a0 = fmin(fmax(ph.a + al * p.a, lower_bound(pr.a, P)), real(1));
      const real a1 = fmin(fmax(ph.b + al * p.b, lower_bound(pr.b, P)), real(1));
      st2(phip + o, a0, a1);
      val[0][0] = a0;
      val[0][1] = a1;
      break;
    }
    case PH_TD_RESTORE: {
      const V2<real> pr = ld2(prefp + o);
      st2(phip + o, pr.a, pr.b);
      break;
    }
    case PH_AM_CHK: {
      const V2<real> ph = ld2(phip + o), pa = ld2(thp + 2 * n + o);
      acc[0] += fabs(double(ph.a) - double(pa.a)) + fabs(double(ph.b) - double(pa.b));
      break;
    }
    case PH_STATS: {
      const V2<real> E = ld2(Ep + o), ph = ld2(phip + o);
      const V2<real> ex = ld2(epsp + o), ey = ld2(epsp + n + o), exy = ld2(epsp + 2 * n + o);
      const real Ev[2] = {E.a, E.b}, pv[2] = {ph.a, ph.b};
      const real xv[2] = {ex.a, ex.b}, yv[2] = {ey.a, ey.b}, sv[2] = {exy.a, exy.b};
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const real lam = lt * Ev[q], mu = mt * Ev[q];
        const real hk = (real(1) - pv[q]) * (real(1) - pv[q]) + kres;
        const Sym<real> e = {eb0 + xv[q], eb1 + yv[q], eb2 + sv[q]};
        real pp, pm;
        energies(e, lam, mu, contact, &pp, &pm);  // elastic energy of the stress model
        const Sym<real> sg = stress(e, lam, mu, hk, contact);
        acc[0] += double(hk) * double(pp) + double(pm);
        acc[1] += P.at == 1 ? double(pv[q]) : double(pv[q]) * double(pv[q]);
        acc[2] += double(pv[q]);
        acc[3] = fmax(acc[3], double(pv[q]));
        acc[4] += pv[q] > real(0.9) ? 1.0 : 0.0;
        acc[5] += double(sg.xx);
        acc[6] += double(sg.yy);
        acc[7] += double(sg.xy);
        val[0][q] = pv[q];
      }
      break;
    }
    case PH_X_PROJ:
    case PH_X_DISP:
    case PH_X_LAP: {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (c < ncomp) {
          const V2<real> t = ld2(thp + c * n + o);
          val[c][0] = t.a;
          val[c][1] = t.b;
        }
      }
      break;
    }
    default:
      break;
  }
}

// The prologue for NQ pixel pairs o0 + q OSTEP of one lane.  The field
// pointers are restrict-qualified here so that the loads of later pairs may
// be issued before the stores of earlier ones (the pairs never overlap).
// Loads the prologue inputs of CH pixel pairs o0 + c OSTEP of phase PH, all
// before any of them is used: the arithmetic of a pair branches (the
// spectral split), which keeps the compiler from issuing the next pair's
// loads early, so without this every pair cost a memory round trip.  Loads
// that depend on the phase's flags are grouped under one test per chunk.
template <typename real, int PH, int CH, int OSTEP>
__device__ __forceinline__ void pro_load_chunk(const RowCtx<real>& X, const real* __restrict__ Ep,
                                               const real* __restrict__ phip, const real* __restrict__ prefp,
                                               const real* __restrict__ epsp, const real* __restrict__ thp,
                                               const real* __restrict__ rmp, const real* __restrict__ pmp, int o0,
                                               ProIn<real> (&in)[CH]) {
  const int n = X.n, flags = X.flags;
  if constexpr (PH == PH_M_RES) {
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int o = o0 + c * OSTEP;
      in[c].a[0] = ld2(Ep + o);
      in[c].a[1] = ld2(phip + o);
#pragma unroll
      for (int k = 0; k < 3; ++k) in[c].a[2 + k] = ld2(epsp + k * n + o);
    }
    if (flags & FL_THETA_PENDING) {
#pragma unroll
      for (int c = 0; c < CH; ++c)
#pragma unroll
        for (int k = 0; k < 3; ++k) in[c].a[5 + k] = ld2(thp + k * n + o0 + c * OSTEP);
    }
  } else if constexpr (PH == PH_M_CG) {
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int o = o0 + c * OSTEP;
      in[c].a[0] = ld2(Ep + o);
      in[c].a[1] = ld2(phip + o);
#pragma unroll
      for (int k = 0; k < 3; ++k) in[c].a[2 + k] = ld2(rmp + k * n + o);
    }
    if (!(flags & FL_CG_FIRST)) {
#pragma unroll
      for (int c = 0; c < CH; ++c)
#pragma unroll
        for (int k = 0; k < 3; ++k) in[c].a[5 + k] = ld2(pmp + k * n + o0 + c * OSTEP);
    }
    if (X.contact != 0) {
#pragma unroll
      for (int c = 0; c < CH; ++c)
#pragma unroll
        for (int k = 0; k < 3; ++k) in[c].a[8 + k] = ld2(epsp + k * n + o0 + c * OSTEP);
    }
  } else if constexpr (PH == PH_PF_ASM) {
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int o = o0 + c * OSTEP;
      in[c].a[0] = ld2(Ep + o);
      in[c].a[1] = ld2(phip + o);
      in[c].a[2] = ld2(prefp + o);
#pragma unroll
      for (int k = 0; k < 3; ++k) in[c].a[3 + k] = ld2(epsp + k * n + o);
    }
  } else if constexpr (PH == PH_PF_PQ) {
    const unsigned char* mask = reinterpret_cast<const unsigned char*>(pmp + n);
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int o = o0 + c * OSTEP;
      in[c].a[0] = ld2(rmp + o);
      in[c].a[1] = ld2(thp + o);
      in[c].m[0] = ldb(mask + o);
      in[c].m[1] = ldb(mask + o + 1);
    }
    if (!(flags & FL_PF_FIRST)) {
#pragma unroll
      for (int c = 0; c < CH; ++c) in[c].a[2] = ld2(pmp + o0 + c * OSTEP);
    }
  } else if constexpr (PH == PH_PF_R) {
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int o = o0 + c * OSTEP;
      in[c].a[0] = ld2(phip + o);
      in[c].a[1] = ld2(pmp + o);
      in[c].a[2] = ld2(prefp + o);
    }
  }
}

template <typename real, int NQ, int OSTEP>
__device__ __forceinline__ void row_prologue_n(const RowCtx<real>& X, const SlotParam& P, const real* __restrict__ Ep,
                                               real* __restrict__ phip, real* __restrict__ prefp,
                                               real* __restrict__ epsp, real* __restrict__ thp,
                                               real* __restrict__ rmp, real* __restrict__ pmp, int o0,
                                               real (&val)[NQ][3][2], double (&acc)[NP_ROW]) {
#define SPFF_PRO_CASE(PHC)                                                                                 \
  case PHC:                                                                                               \
    _Pragma("unroll") for (int q = 0; q < NQ; ++q)                                                        \
        row_prologue<real, PHC>(X, P, Ep, phip, prefp, epsp, thp, rmp, pmp, o0 + q * OSTEP, val[q], acc); \
    break;
  // the phases a solve iterates on: chunks of up to four pairs, each loaded
  // in full before its arithmetic (with sixteen pairs per lane, 2048-point
  // rows, the registers are spent and the per-pair path is faster)
  constexpr bool CHUNK = NQ <= 8;
  constexpr int CH = NQ < 4 ? NQ : 4;
  static_assert(NQ % CH == 0, "pairs per lane in whole chunks");
#define SPFF_PRO_HOT(PHC)                                                                                    \
  case PHC:                                                                                                 \
    if constexpr (CHUNK) {                                                                                  \
      _Pragma("unroll") for (int q0 = 0; q0 < NQ; q0 += CH) {                                               \
        ProIn<real> in[CH];                                                                                 \
        pro_load_chunk<real, PHC, CH, OSTEP>(X, Ep, phip, prefp, epsp, thp, rmp, pmp, o0 + q0 * OSTEP, in); \
        _Pragma("unroll") for (int c = 0; c < CH; ++c)                                                      \
            row_prologue<real, PHC, true>(X, P, Ep, phip, prefp, epsp, thp, rmp, pmp,                       \
                                          o0 + (q0 + c) * OSTEP, val[q0 + c], acc, in[c]);                  \
      }                                                                                                     \
    } else {                                                                                                \
      _Pragma("unroll") for (int q = 0; q < NQ; ++q)                                                        \
          row_prologue<real, PHC>(X, P, Ep, phip, prefp, epsp, thp, rmp, pmp, o0 + q * OSTEP, val[q], acc); \
    }                                                                                                       \
    break;
  switch (X.phase) {
    SPFF_PRO_HOT(PH_M_RES)
    SPFF_PRO_HOT(PH_M_CG)
    SPFF_PRO_HOT(PH_PF_ASM)
    SPFF_PRO_HOT(PH_PF_PQ)
    SPFF_PRO_HOT(PH_PF_R)
    SPFF_PRO_CASE(PH_AM_CHK)
    SPFF_PRO_CASE(PH_TD_RESTORE)
    SPFF_PRO_CASE(PH_STATS)
    SPFF_PRO_CASE(PH_X_PROJ)
    SPFF_PRO_CASE(PH_X_DISP)
    SPFF_PRO_CASE(PH_X_LAP)
    default:
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        val[q][0][0] = val[q][0][1] = val[q][1][0] = val[q][1][1] = val[q][2][0] = val[q][2][1] = real(0);
      break;
  }
#undef SPFF_PRO_CASE
#undef SPFF_PRO_HOT
}

// Inputs of the controller step that a row-forward kernel runs for the
// previous tick (and the closing kernel for the last tick of a block).
struct CtrlArgs {
  const SlotCtl* ctl_in;  // control blocks as the previous tick left them
  SlotCtl* ctl_out;       // advanced blocks, read by this tick's other kernels
  const double* prow;     // partial sums of the previous tick
  const double* pcol;
  const double* pinv;
  double* prof;
  SlotSeq* seqs;
  StepRec* recs;
  int ngc;
};

template <typename real>
__device__ __forceinline__ void ctrl_slot(int s, const SlotPtr<real>* __restrict__ ptrs,
                                          const SlotParam* __restrict__ prms, SlotCtl& C, bool writer,
                                          const double* __restrict__ prow, const double* __restrict__ pcol,
                                          const double* __restrict__ pinv, double* __restrict__ prof,
                                          SlotSeq* __restrict__ seqs, StepRec* __restrict__ recs, int nx, int ny,
                                          int ngr, int ngc);

// Control block of slot s for this tick, in `lc` (LDS): a copy of the input
// block, advanced by the controller step of the previous tick if that is
// still pending.  Every work-group of the slot computes the same block (the
// same inputs reduced in the same order); the one that owns row block 0
// (`writer`) publishes it to ctl_out and records the step.  The input block
// is not written, so groups that start late read what the early ones read.
// Every thread of the group calls this (it synchronises the group).
template <typename real>
__device__ __forceinline__ void tick_control(int s, bool writer, const CtrlArgs& A,
                                             const SlotPtr<real>* __restrict__ ptrs,
                                             const SlotParam* __restrict__ prms, int nx, int ny, int ngr,
                                             SlotCtl& lc) {
  constexpr int NW = (int)(sizeof(SlotCtl) / sizeof(int));
  static_assert(sizeof(SlotCtl) % sizeof(int) == 0, "the control block is copied as words");
  const int* src = reinterpret_cast<const int*>(A.ctl_in + s);
  int* dst = reinterpret_cast<int*>(&lc);
  for (int i = threadIdx.x; i < NW; i += blockDim.x) dst[i] = src[i];
  __syncthreads();
  if (threadIdx.x < 64) {
    if (lc.pending)
      ctrl_slot<real>(s, ptrs, prms, lc, writer, A.prow, A.pcol, A.pinv, A.prof, A.seqs, A.recs, nx, ny, ngr,
                      A.ngc);
    // the slot's controller step after this tick is pending if it works
    if (threadIdx.x == 0) lc.pending = lc.phase != PH_IDLE ? 1 : 0;
  }
  __syncthreads();
  if (writer) {
    int* out = reinterpret_cast<int*>(A.ctl_out + s);
    for (int i = threadIdx.x; i < NW; i += blockDim.x) out[i] = dst[i];
  }
}

// ===========================================================================
// Row-forward kernel: prologue (per phase) -> R2C row FFTs -> transposed
// store of the half spectra; FP64 partial sums per work-group.
// ===========================================================================
template <typename real>
__device__ __forceinline__ void k_rowfwd_body(const int* __restrict__ list,
                                                    const SlotPtr<real>* __restrict__ ptrs,
                                                    const SlotParam* __restrict__ prms, const CtrlArgs A,
                                                    const cplx<real>* __restrict__ twx, double* __restrict__ part,
                                                    int nx, int ny, int R, int ngr) {
  using C = cplx<real>;
  extern __shared__ unsigned char smem_raw[];
  __shared__ double red[(THREADS / 64) * NP_ROW];
  __shared__ SlotCtl lctl;
  int g, si;
  row_coords(ngr, g, si);
  const int s = list[si];
  if (s < 0) return;
  tick_control<real>(s, g == 0, A, ptrs, prms, nx, ny, ngr, lctl);
  const SlotCtl& ctl = lctl;
  const int phase = ctl.phase;
  const int ncomp = phase_comps_row(phase);
  if (phase != PH_AM_CHK && phase != PH_TD_RESTORE && ncomp == 0) return;
  const SlotParam& P = prms[s];
  const SlotPtr<real> F = ptrs[s];
  const int flags = ctl.flags;
  const int M = nx >> 1, stride = M + PAD;
  const int y0 = g * R;
  const int n = nx * ny;
  C* buf = reinterpret_cast<C*>(smem_raw);
  double acc[NP_ROW];
#pragma unroll
  for (int i = 0; i < NP_ROW; ++i) acc[i] = 0.0;
  if (phase == PH_STATS) acc[3] = -1.0e300;

  const RowCtx<real> X = row_ctx<real>(ctl, P, phase, ncomp, n);

  const int logM = ilog2(M), logR = ilog2(R);
  for (int idx = threadIdx.x; idx < R * M; idx += blockDim.x) {
    const int r = idx >> logM, h = idx & (M - 1);
    const int o = (y0 + r) * nx + 2 * h;
    const int li = r * stride + h;  // LDS index of component 0
    real val[3][2];
    row_prologue<real>(X, P, F.E, F.phi, F.phi_ref, F.eps, F.theta, F.rm, F.pm, o, val, acc);
    if (ncomp > 0) {
#pragma unroll
      for (int c = 0; c < 3; ++c)
        if (c < ncomp) buf[c * R * stride + li] = mk<C>(val[c][0], val[c][1]);
    }
  }
  if (ncomp > 0) {
    __syncthreads();
    fft_lds<real, false, MAXE>(buf, M, ncomp * R, stride, twx, 2);
    r2c_post<real>(buf, M, ncomp * R, stride, twx);
    // transposed store: spec[c][kx][y0 + r]
    C* spec = reinterpret_cast<C*>(F.spec);
    const int tot = ncomp * M * R;
    for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
      const int r = idx & (R - 1);
      const int rest = idx >> logR;
      const int kx = rest & (M - 1), c = rest >> logM;
      stc<real>(spec + (size_t)(rest) * ny + y0 + r, buf[(c * R + r) * stride + kx]);
    }
  }
  block_reduce_store<NP_ROW>(acc, red, part + (size_t)s * NP_ROW * ngr + g, ngr, nacc_rowfwd(phase),
                             phase == PH_STATS ? 3 : (phase == PH_PF_ASM ? 1 : -1));
}

// ===========================================================================
// Column kernel: forward column FFTs -> per-mode operator -> inverse column
// FFTs (or a Parseval reduction only).  Normalisation 1/(nx ny) is applied
// with the operator.
// ===========================================================================
template <typename real>
__device__ __forceinline__ void project3(real* a, real fx, real fy) {
  // G^:A = A - (t.A.t) t(x)t, t = (-fy, fx)/|f|; G^ = 0 at f = 0.
  const real n2 = fx * fx + fy * fy;
  if (n2 == real(0)) {
    a[0] = a[1] = a[2] = real(0);
    return;
  }
  const real inv = real(1) / n2;
  const real txx = fy * fy * inv, tyy = fx * fx * inv, txy = -fx * fy * inv;
  const real sdot = txx * a[0] + tyy * a[1] + real(2) * txy * a[2];
  a[0] -= sdot * txx;
  a[1] -= sdot * tyy;
  a[2] -= sdot * txy;
}

// Projection at one mode of an even grid.  nyq: the mode has a Nyquist
// index (ky = ny/2, or the kx = nx/2 column); its gradient component along
// that direction is already zero in (fx, fy).  With the free Nyquist
// treatment such a mode is left unconstrained (identity).
template <typename real>
__device__ __forceinline__ void project3_mode(real* a, real fx, real fy, bool nyq, int nyq_free) {
  if (nyq && nyq_free) return;
  project3(a, fx, fy);
}

// Displacement at one mode.  The strain is the unknown of the mechanics
// problem (Sec. 3.1.1); the periodic displacement u* is recovered from the
// compatible eps* by inverting eps^ = sym(i u^ (x) xi) at each mode:
//   u^ = -i [ 2 eps^ xi / |xi|^2 - xi (xi . eps^ . xi) / |xi|^4 ],
// xi = 2 pi (fx, fy) the gradient wavevector (Nyquist components zero), and
// u^ = 0 where xi = 0 (the mean, and modes that are Nyquist in every
// direction).  v[0..2] = (xx, yy, xy) in; v[0..1] = (x, y) out, v[2] = 0;
// scale carries the 1/(nx ny) of the inverse transform.
template <typename real>
__device__ __forceinline__ void disp_part(const real* a, real gx, real gy, real* u) {
  const real n2 = gx * gx + gy * gy;
  if (n2 == real(0)) {
    u[0] = u[1] = real(0);
    return;
  }
  const real inv = real(1) / n2;
  const real ex = a[0] * gx + a[2] * gy, ey = a[2] * gx + a[1] * gy;
  const real s = (gx * ex + gy * ey) * inv;
  u[0] = (real(2) * ex - gx * s) * inv;
  u[1] = (real(2) * ey - gy * s) * inv;
}

template <typename real>
__device__ __forceinline__ void disp3(cplx<real>* v, real fx, real fy, real scale) {
  using C = cplx<real>;
  const real gx = real(TWO_PI) * fx, gy = real(TWO_PI) * fy;
  const real re[3] = {v[0].x, v[1].x, v[2].x}, im[3] = {v[0].y, v[1].y, v[2].y};
  real ur[2], ui[2];
  disp_part(re, gx, gy, ur);
  disp_part(im, gx, gy, ui);
  // -i (ur + i ui) = ui - i ur
  v[0] = mk<C>(ui[0] * scale, -ur[0] * scale);
  v[1] = mk<C>(ui[1] * scale, -ur[1] * scale);
  v[2] = mk<C>(real(0), real(0));
}

template <typename real>
__device__ __forceinline__ void k_col_body(const int* __restrict__ list, const SlotPtr<real>* __restrict__ ptrs,
                                                 const SlotParam* __restrict__ prms,
                                                 const SlotCtl* __restrict__ ctls,
                                                 const cplx<real>* __restrict__ twy, double* __restrict__ part,
                                                 int nx, int ny, int W, int ngc, int nyq_free) {
  using C = cplx<real>;
  extern __shared__ unsigned char smem_raw[];
  __shared__ double red[(THREADS / 64) * NP_COL];
  const int s = list[blockIdx.y], g = blockIdx.x;
  if (s < 0) return;
  const int phase = ctls[s].phase;
  int ncomp, mode;  // mode 0: projection, 1: Laplacian, 2: Parseval reduction, 3: displacement
  switch (phase) {
    case PH_M_RES:
    case PH_M_CG:
    case PH_X_PROJ:
      ncomp = 3;
      mode = 0;
      break;
    case PH_X_DISP:
      ncomp = 3;
      mode = 3;
      break;
    case PH_X_LAP:
      ncomp = 1;
      mode = 1;
      break;
    case PH_PF_ASM:
    case PH_PF_R:
      ncomp = 1;
      mode = 1;
      break;
    case PH_PF_PQ:
    case PH_STATS:
      ncomp = 1;
      mode = 2;
      break;
    default:
      return;
  }
  const SlotParam& P = prms[s];
  const SlotPtr<real> F = ptrs[s];
  const int M = nx >> 1, stride = ny + PAD;
  const int kx0 = g * W;
  C* buf = reinterpret_cast<C*>(smem_raw);
  C* spec = reinterpret_cast<C*>(F.spec);
  const real inv_n = real(1.0 / (double(nx) * double(ny)));
  const real two_pi = real(TWO_PI);

  // load W columns of each component
  const int tot = ncomp * W * ny;
  const int logny = ilog2(ny), logW = ilog2(W);
  for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
    const int y = idx & (ny - 1), rest = idx >> logny;
    const int w = rest & (W - 1), c = rest >> logW;
    buf[rest * stride + y] = ldc<real>(spec + (size_t)(c * M + kx0 + w) * ny + y);
  }
  __syncthreads();
  fft_lds<real, false, MAXE>(buf, ny, ncomp * W, stride, twy, 1);

  double acc[NP_COL] = {0.0, 0.0};
  const real lap_scale = (phase == PH_X_LAP ? real(1) : real(P.kappa)) * inv_n;
  // per-mode operator; thread owns mode (w, ky); for the packed column kx = 0
  // threads with ky <= ny/2 own the pair (ky, ny - ky)
  for (int idx = threadIdx.x; idx < W * ny; idx += blockDim.x) {
    const int w = idx >> logny, ky = idx & (ny - 1);
    const int kx = kx0 + w;
    const int kys = ky < ny / 2 ? ky : ky - ny;
    const real fy_true = real(kys) / real(ny);
    const real fy_grad = (2 * ky == ny) ? real(0) : fy_true;
    if (kx > 0) {
      const real fx = real(kx) / real(nx);
      if (mode == 3) {
        C a[3] = {buf[(0 * W + w) * stride + ky], buf[(1 * W + w) * stride + ky], buf[(2 * W + w) * stride + ky]};
        disp3(a, fx, fy_grad, inv_n);
#pragma unroll
        for (int c = 0; c < 3; ++c) buf[(c * W + w) * stride + ky] = a[c];
      } else if (mode == 0) {
        C* a0 = buf + (0 * W + w) * stride + ky;
        C* a1 = buf + (1 * W + w) * stride + ky;
        C* a2 = buf + (2 * W + w) * stride + ky;
        real re[3] = {a0->x, a1->x, a2->x}, im[3] = {a0->y, a1->y, a2->y};
        project3_mode(re, fx, fy_grad, 2 * ky == ny, nyq_free);
        project3_mode(im, fx, fy_grad, 2 * ky == ny, nyq_free);
        *a0 = mk<C>(re[0] * inv_n, im[0] * inv_n);
        *a1 = mk<C>(re[1] * inv_n, im[1] * inv_n);
        *a2 = mk<C>(re[2] * inv_n, im[2] * inv_n);
      } else {
        const real L = two_pi * two_pi * (fx * fx + fy_true * fy_true);
        C* a = buf + w * stride + ky;
        if (mode == 1) {
          *a = cscale(*a, L * lap_scale);
        } else {
          const C v = *a;
          acc[0] += 2.0 * double(L) * (double(v.x) * double(v.x) + double(v.y) * double(v.y));
        }
      }
    } else {
      if (2 * ky > ny) continue;  // partner handled by ky' = ny - ky
      const int km = (ny - ky) & (ny - 1);
      const bool self = (km == ky);
      // split packed column into A (kx = 0 column) and B (kx = nx/2 column)
      const real fxN_true = real(0.5);
      if (mode == 3) {
        C Aa[3], Bb[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const C cp = buf[(c * W + w) * stride + ky];
          const C cm = cconj(buf[(c * W + w) * stride + km]);
          Aa[c] = cscale(cadd(cp, cm), real(0.5));
          Bb[c] = cscale(cmulni(csub(cp, cm)), real(0.5));
        }
        // kx = 0 and kx = nx/2 (x-component of the gradient wavevector zero)
        disp3(Aa, real(0), fy_grad, inv_n);
        disp3(Bb, real(0), fy_grad, inv_n);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          buf[(c * W + w) * stride + ky] = cadd(Aa[c], cmuli(Bb[c]));
          if (!self) buf[(c * W + w) * stride + km] = cadd(cconj(Aa[c]), cmuli(cconj(Bb[c])));
        }
      } else if (mode == 0) {
        C Aa[3], Bb[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const C cp = buf[(c * W + w) * stride + ky];
          const C cm = cconj(buf[(c * W + w) * stride + km]);
          Aa[c] = cscale(cadd(cp, cm), real(0.5));
          Bb[c] = cscale(cmulni(csub(cp, cm)), real(0.5));
        }
        real ar[3] = {Aa[0].x, Aa[1].x, Aa[2].x}, ai[3] = {Aa[0].y, Aa[1].y, Aa[2].y};
        real br[3] = {Bb[0].x, Bb[1].x, Bb[2].x}, bi[3] = {Bb[0].y, Bb[1].y, Bb[2].y};
        project3_mode(ar, real(0), fy_grad, 2 * ky == ny, nyq_free);
        project3_mode(ai, real(0), fy_grad, 2 * ky == ny, nyq_free);
        // kx = nx/2: gradient wavevector x-component is zero (Nyquist)
        project3_mode(br, real(0), fy_grad, true, nyq_free);
        project3_mode(bi, real(0), fy_grad, true, nyq_free);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const C A = mk<C>(ar[c] * inv_n, ai[c] * inv_n), B = mk<C>(br[c] * inv_n, bi[c] * inv_n);
          buf[(c * W + w) * stride + ky] = cadd(A, cmuli(B));
          if (!self) buf[(c * W + w) * stride + km] = cadd(cconj(A), cmuli(cconj(B)));
        }
      } else {
        const C cp = buf[w * stride + ky];
        const C cm = cconj(buf[w * stride + km]);
        const C A = cscale(cadd(cp, cm), real(0.5));
        const C B = cscale(cmulni(csub(cp, cm)), real(0.5));
        const real L0 = two_pi * two_pi * (fy_true * fy_true);
        const real LN = two_pi * two_pi * (fxN_true * fxN_true + fy_true * fy_true);
        if (mode == 1) {
          const C A2 = cscale(A, L0 * lap_scale), B2 = cscale(B, LN * lap_scale);
          buf[w * stride + ky] = cadd(A2, cmuli(B2));
          if (!self) buf[w * stride + km] = cadd(cconj(A2), cmuli(cconj(B2)));
        } else {
          const double wgt = self ? 1.0 : 2.0;
          acc[0] += wgt * (double(L0) * (double(A.x) * double(A.x) + double(A.y) * double(A.y)) +
                           double(LN) * (double(B.x) * double(B.x) + double(B.y) * double(B.y)));
        }
      }
    }
  }
  __syncthreads();
  if (mode != 2) {
    fft_lds<real, true, MAXE>(buf, ny, ncomp * W, stride, twy, 1);
    for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
      const int y = idx & (ny - 1), rest = idx >> logny;
      const int w = rest & (W - 1), c = rest >> logW;
      stc<real>(spec + (size_t)(c * M + kx0 + w) * ny + y, buf[rest * stride + y]);
    }
  }
  block_reduce_store<NP_COL>(acc, red, part + (size_t)s * NP_COL * ngc + g, ngc, mode == 2 ? 1 : 0);
}

// Column kernel with register-resident transforms (ny = N in {128, ...,
// 2048}, FP32): a group of L = N/E lanes owns one kx column of every
// component, E modes per lane per component (lane l: ky = l + m L).
// Forward FFTs, the per-mode operator and the inverse FFTs run on the lane's
// registers; only the Stockham exchanges between radix-8 passes go through
// LDS, inside the group.  The packed column kx = 0 (X[0] + i X[nx/2]) takes
// the partner mode -ky from lane (L - l) mod L by a cross-lane shuffle
// (through LDS where the group spans several wavefronts).
template <typename real, int N, int E>
__device__ __forceinline__ void k_colr_body(const int* __restrict__ list, const SlotPtr<real>* __restrict__ ptrs,
                                            const SlotParam* __restrict__ prms, const SlotCtl* __restrict__ ctls,
                                            const cplx<real>* __restrict__ twy, double* __restrict__ part, int nx,
                                            int ngc, int nyq_free) {
  using C = cplx<real>;
  // E = 8 points per lane up to 512-point columns; 1024 and 2048 points
  // take 16 (one or two wavefronts per column) or 8 (two or four: twice
  // the wavefronts in flight for launches with one or two problems).  A
  // group wider than a wavefront is the work-group's only column, so every
  // barrier below is reached by all its threads.
  constexpr int L = N / E;
  static_assert(E == 8 || E == 16, "8 or 16 points per lane");
  static_assert(L <= 64 || N >= 1024, "groups wider than a wavefront are 1024- or 2048-point columns");
  extern __shared__ unsigned char smem_raw[];
  __shared__ double red[(THREADS / 64) * NP_COL];
  const int s = list[blockIdx.y], g = blockIdx.x;
  if (s < 0) return;
  const int phase = ctls[s].phase;
  int ncomp, mode;  // mode 0: projection, 1: Laplacian, 2: Parseval reduction, 3: displacement
  switch (phase) {
    case PH_M_RES:
    case PH_M_CG:
    case PH_X_PROJ:
      ncomp = 3;
      mode = 0;
      break;
    case PH_X_DISP:
      ncomp = 3;
      mode = 3;
      break;
    case PH_X_LAP:
    case PH_PF_ASM:
    case PH_PF_R:
      ncomp = 1;
      mode = 1;
      break;
    case PH_PF_PQ:
    case PH_STATS:
      ncomp = 1;
      mode = 2;
      break;
    default:
      return;
  }
  const SlotParam& P = prms[s];
  const SlotPtr<real> F = ptrs[s];
  const int M = nx >> 1;
  const int W = blockDim.x / L;
  const int col = threadIdx.x / L, lane = threadIdx.x & (L - 1);
  const int kx = g * W + col;
  C* x = reinterpret_cast<C*>(smem_raw) + col * XArea<N>::size;
  C* spec = reinterpret_cast<C*>(F.spec);
  const real inv_n = real(1.0 / (double(nx) * double(N)));
  const real two_pi = real(TWO_PI);
  const real lap_scale = (phase == PH_X_LAP ? real(1) : real(P.kappa)) * inv_n;

  C v[3][E];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (c < ncomp) {
      const C* src = spec + (size_t)(c * M + kx) * N + lane;
#pragma unroll
      for (int m = 0; m < E; ++m) v[c][m] = ldc<real>(src + m * L);
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c)
    if (c < ncomp) reg_fft<real, false, N, E>(v[c], x, lane, twy, 1);

  double acc[NP_COL] = {0.0, 0.0};
  if (kx > 0) {
    const real fx = real(kx) / real(nx);
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int ky = lane + m * L;
      const int kys = ky < N / 2 ? ky : ky - N;
      const real fy_true = real(kys) / real(N);
      const real fy_grad = (2 * ky == N) ? real(0) : fy_true;
      if (mode == 3) {
        C a[3] = {v[0][m], v[1][m], v[2][m]};
        disp3(a, fx, fy_grad, inv_n);
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c][m] = a[c];
      } else if (mode == 0) {
        real re[3] = {v[0][m].x, v[1][m].x, v[2][m].x}, im[3] = {v[0][m].y, v[1][m].y, v[2][m].y};
        project3_mode(re, fx, fy_grad, 2 * ky == N, nyq_free);
        project3_mode(im, fx, fy_grad, 2 * ky == N, nyq_free);
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c][m] = mk<C>(re[c] * inv_n, im[c] * inv_n);
      } else {
        const real Lk = two_pi * two_pi * (fx * fx + fy_true * fy_true);
        if (mode == 1) {
          v[0][m] = cscale(v[0][m], Lk * lap_scale);
        } else {
          acc[0] += 2.0 * double(Lk) * (double(v[0][m].x) * double(v[0][m].x) + double(v[0][m].y) * double(v[0][m].y));
        }
      }
    }
  } else {
    // packed column: A = X(kx = 0), B = X(kx = nx/2) at ky, from Z(ky) and
    // conj Z(-ky); the partner of slot m of lane l is slot E-1-m of lane
    // L-l (l > 0), or slot (E-m) mod E of lane 0 itself
    C Pn[3][E];
    const int src = (L - lane) & (L - 1);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (c < ncomp) {
        if constexpr (L <= 64) {
#pragma unroll
          for (int i = 0; i < E; ++i) {
            const real px = __shfl(v[c][i].x, src, L), py = __shfl(v[c][i].y, src, L);
            Pn[c][E - 1 - i] = mk<C>(px, py);
          }
        } else {
          // the partner lane may sit in the other wavefront: exchange
          // through the column's LDS area (free between transforms)
#pragma unroll
          for (int i = 0; i < E; ++i) x[xpad(lane + i * L)] = v[c][i];
          group_sync<L>();
#pragma unroll
          for (int i = 0; i < E; ++i) Pn[c][E - 1 - i] = x[xpad(src + i * L)];
          group_sync<L>();
        }
        if (lane == 0) {
#pragma unroll
          for (int m = 0; m < E; ++m) Pn[c][m] = v[c][(E - m) & (E - 1)];
        }
      }
    }
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int ky = lane + m * L;
      const int kys = ky < N / 2 ? ky : ky - N;
      const real fy_true = real(kys) / real(N);
      const real fy_grad = (2 * ky == N) ? real(0) : fy_true;
      if (mode == 3) {
        C Aa[3], Bb[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const C cp = v[c][m], cm = cconj(Pn[c][m]);
          Aa[c] = cscale(cadd(cp, cm), real(0.5));
          Bb[c] = cscale(cmulni(csub(cp, cm)), real(0.5));
        }
        disp3(Aa, real(0), fy_grad, inv_n);
        disp3(Bb, real(0), fy_grad, inv_n);
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c][m] = cadd(Aa[c], cmuli(Bb[c]));
      } else if (mode == 0) {
        real ar[3], ai[3], br[3], bi[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const C cp = v[c][m], cm = cconj(Pn[c][m]);
          const C A = cscale(cadd(cp, cm), real(0.5));
          const C Bq = cscale(cmulni(csub(cp, cm)), real(0.5));
          ar[c] = A.x;
          ai[c] = A.y;
          br[c] = Bq.x;
          bi[c] = Bq.y;
        }
        project3_mode(ar, real(0), fy_grad, 2 * ky == N, nyq_free);
        project3_mode(ai, real(0), fy_grad, 2 * ky == N, nyq_free);
        // kx = nx/2: gradient wavevector x-component is zero (Nyquist)
        project3_mode(br, real(0), fy_grad, true, nyq_free);
        project3_mode(bi, real(0), fy_grad, true, nyq_free);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const C A = mk<C>(ar[c] * inv_n, ai[c] * inv_n), Bq = mk<C>(br[c] * inv_n, bi[c] * inv_n);
          v[c][m] = cadd(A, cmuli(Bq));
        }
      } else {
        const C cp = v[0][m], cm = cconj(Pn[0][m]);
        const C A = cscale(cadd(cp, cm), real(0.5));
        const C Bq = cscale(cmulni(csub(cp, cm)), real(0.5));
        const real L0 = two_pi * two_pi * (fy_true * fy_true);
        const real LN = two_pi * two_pi * (real(0.25) + fy_true * fy_true);
        if (mode == 1) {
          v[0][m] = cadd(cscale(A, L0 * lap_scale), cmuli(cscale(Bq, LN * lap_scale)));
        } else {
          acc[0] += double(L0) * (double(A.x) * double(A.x) + double(A.y) * double(A.y)) +
                    double(LN) * (double(Bq.x) * double(Bq.x) + double(Bq.y) * double(Bq.y));
        }
      }
    }
  }
  if (mode != 2) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (c < ncomp) {
        reg_fft<real, true, N, E>(v[c], x, lane, twy, 1);
        C* dst = spec + (size_t)(c * M + kx) * N + lane;
#pragma unroll
        for (int m = 0; m < E; ++m) stc<real>(dst + m * L, v[c][m]);
      }
    }
  }
  block_reduce_store<NP_COL>(acc, red, part + (size_t)s * NP_COL * ngc + g, ngc, mode == 2 ? 1 : 0);
}

// Row-inverse epilogue for the pixel pair (o, o + 1): q[c] holds the
// transformed values of component c at the pair (x: o, y: o + 1).
// Inputs of the row epilogue for one pixel pair, loaded ahead of the
// arithmetic (see epi_load_chunk for the slots of each phase).
template <typename real>
struct EpiIn {
  V2<real> a[9];
};

template <typename real, int PH = -1, bool PRE = false>
__device__ __forceinline__ void row_epilogue(const RowCtx<real>& X, const SlotParam& P, real* __restrict__ phip,
                                             real* __restrict__ prefp, real* __restrict__ thp,
                                             real* __restrict__ rmp, real* __restrict__ pmp, int o,
                                             const cplx<real> (&q)[3], real alpha, double (&acc)[NP_INV],
                                             const EpiIn<real>& in = EpiIn<real>{}) {
  // PRE: the inputs of this pair were loaded into `in` (PH one of M_CG,
  // PF_ASM, PF_R; see row_epilogue_n)
  using C = cplx<real>;
  const int phase = PH >= 0 ? PH : X.phase;
  const int n = X.n, ncomp = X.ncomp;
  switch (phase) {
    case PH_M_RES: {
      const C q0 = q[0], q1 = q[1], q2 = q[2];
      st2(rmp + o, -q0.x, -q0.y);
      st2(rmp + n + o, -q1.x, -q1.y);
      st2(rmp + 2 * n + o, -q2.x, -q2.y);
      acc[0] += double(q0.x) * q0.x + double(q0.y) * q0.y + double(q1.x) * q1.x + double(q1.y) * q1.y +
                2.0 * (double(q2.x) * q2.x + double(q2.y) * q2.y);
      break;
    }
    case PH_M_CG: {
      const bool first = X.flags & FL_CG_FIRST;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const V2<real> p = PRE ? in.a[c] : ld2(pmp + c * n + o);
        V2<real> r2 = PRE ? in.a[3 + c] : ld2(rmp + c * n + o);
        V2<real> th = first ? V2<real>{0, 0} : (PRE ? in.a[6 + c] : ld2(thp + c * n + o));
        th = {th.a + alpha * p.a, th.b + alpha * p.b};
        r2 = {r2.a - alpha * q[c].x, r2.b - alpha * q[c].y};
        st2(thp + c * n + o, th.a, th.b);
        st2(rmp + c * n + o, r2.a, r2.b);
        const double wc = c == 2 ? 2.0 : 1.0;
        acc[0] += wc * (double(r2.a) * r2.a + double(r2.b) * r2.b);
      }
      break;
    }
    case PH_PF_ASM:
    case PH_PF_R: {
      const C lap = q[0];
      const V2<real> ph = PRE ? in.a[0] : ld2(phip + o), d = PRE ? in.a[1] : ld2(thp + o),
                     b = PRE ? in.a[2] : ld2(thp + n + o);
      const V2<real> pr = PRE ? in.a[3] : ld2(prefp + o);
      const real rr0 = d.a * ph.a + lap.x - b.a;
      const real rr1 = d.b * ph.b + lap.y - b.b;
      const real lo0 = lower_bound(pr.a, P), lo1 = lower_bound(pr.b, P);
      const bool a0 = (ph.a <= lo0 && rr0 > real(0)) || (ph.a >= real(1) && rr0 < real(0));
      const bool a1 = (ph.b <= lo1 && rr1 > real(0)) || (ph.b >= real(1) && rr1 < real(0));
      const real r0 = a0 ? real(0) : rr0, r1 = a1 ? real(0) : rr1;
      if (phase == PH_PF_ASM && (X.flags & FL_NE_CHECK)) {
        // near-equilibrium evolution: phi = phi_n here, so the unmasked
        // residual is F_phi(phi_n, eps_n); keep it for the search of x*
        st2(rmp + n + o, rr0, rr1);
        acc[1] = fmax(acc[1], fmax(-double(rr0), -double(rr1)));
      }
      if (phase == PH_PF_R) {
        const V2<real> ro = PRE ? in.a[4] : ld2(rmp + o);
        acc[1] += double(r0) * ro.a + double(r1) * ro.b;
      }
      st2(rmp + o, r0, r1);
      unsigned char* mask = reinterpret_cast<unsigned char*>(pmp + n);
      stb(mask + o, a0 ? 1 : 0);
      stb(mask + o + 1, a1 ? 1 : 0);
      acc[0] += double(r0) * r0 + double(r1) * r1;
      acc[2] += double(ph.a) * ph.a + double(ph.b) * ph.b;
      acc[3] += double(d.a * ph.a) * double(d.a * ph.a) + double(d.b * ph.b) * double(d.b * ph.b);
      break;
    }
    case PH_X_PROJ:
    case PH_X_DISP:
    case PH_X_LAP: {
#pragma unroll
      for (int c = 0; c < 3; ++c)
        if (c < ncomp) st2(rmp + c * n + o, q[c].x, q[c].y);
      break;
    }
    default:
      break;
  }
}

// Loads the epilogue inputs of CH pixel pairs o0 + c OSTEP of phase PH
// before any store of the chunk: on this GPU a wait for a load also waits
// for the stores issued before it, so interleaved per-pair loads and stores
// cost a round trip per pair.
template <typename real, int PH, int CH, int OSTEP>
__device__ __forceinline__ void epi_load_chunk(const RowCtx<real>& X, const real* __restrict__ phip,
                                               const real* __restrict__ prefp, const real* __restrict__ thp,
                                               const real* __restrict__ rmp, const real* __restrict__ pmp, int o0,
                                               EpiIn<real> (&in)[CH]) {
  const int n = X.n;
  if constexpr (PH == PH_M_CG) {
#pragma unroll
    for (int c = 0; c < CH; ++c)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        in[c].a[k] = ld2(pmp + k * n + o0 + c * OSTEP);
        in[c].a[3 + k] = ld2(rmp + k * n + o0 + c * OSTEP);
      }
    if (!(X.flags & FL_CG_FIRST)) {
#pragma unroll
      for (int c = 0; c < CH; ++c)
#pragma unroll
        for (int k = 0; k < 3; ++k) in[c].a[6 + k] = ld2(thp + k * n + o0 + c * OSTEP);
    }
  } else if constexpr (PH == PH_PF_ASM || PH == PH_PF_R) {
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int o = o0 + c * OSTEP;
      in[c].a[0] = ld2(phip + o);
      in[c].a[1] = ld2(thp + o);
      in[c].a[2] = ld2(thp + n + o);
      in[c].a[3] = ld2(prefp + o);
      if constexpr (PH == PH_PF_R) in[c].a[4] = ld2(rmp + o);
    }
  }
}

// The epilogue for NQ pixel pairs o0 + q OSTEP of one lane (restrict
// pointers: see row_prologue_n).
template <typename real, int NQ, int OSTEP>
__device__ __forceinline__ void row_epilogue_n(const RowCtx<real>& X, const SlotParam& P, real* __restrict__ phip,
                                               real* __restrict__ prefp, real* __restrict__ thp,
                                               real* __restrict__ rmp, real* __restrict__ pmp, int o0,
                                               const cplx<real> (&q)[NQ][3], real alpha, double (&acc)[NP_INV]) {
#define SPFF_EPI_CASE(PHC)                                                                             \
  case PHC:                                                                                           \
    _Pragma("unroll") for (int i = 0; i < NQ; ++i)                                                    \
        row_epilogue<real, PHC>(X, P, phip, prefp, thp, rmp, pmp, o0 + i * OSTEP, q[i], alpha, acc); \
    break;
  // up to four pairs per lane (launches with few problems): all loaded
  // before their stores; with more pairs the registers this takes would
  // cost occupancy, and the per-pair path stays
  constexpr bool CHUNK = NQ <= 4;
#define SPFF_EPI_HOT(PHC)                                                                                    \
  case PHC:                                                                                                   \
    if constexpr (CHUNK) {                                                                                    \
      EpiIn<real> in[NQ];                                                                                     \
      epi_load_chunk<real, PHC, NQ, OSTEP>(X, phip, prefp, thp, rmp, pmp, o0, in);                            \
      _Pragma("unroll") for (int c = 0; c < NQ; ++c)                                                          \
          row_epilogue<real, PHC, true>(X, P, phip, prefp, thp, rmp, pmp, o0 + c * OSTEP, q[c], alpha, acc,   \
                                        in[c]);                                                               \
    } else {                                                                                                  \
      _Pragma("unroll") for (int i = 0; i < NQ; ++i)                                                          \
          row_epilogue<real, PHC>(X, P, phip, prefp, thp, rmp, pmp, o0 + i * OSTEP, q[i], alpha, acc);       \
    }                                                                                                         \
    break;
  switch (X.phase) {
    SPFF_EPI_CASE(PH_M_RES)
    SPFF_EPI_HOT(PH_M_CG)
    SPFF_EPI_HOT(PH_PF_ASM)
    SPFF_EPI_HOT(PH_PF_R)
    SPFF_EPI_CASE(PH_X_PROJ)
    SPFF_EPI_CASE(PH_X_DISP)
    SPFF_EPI_CASE(PH_X_LAP)
    default:
      break;
  }
#undef SPFF_EPI_CASE
#undef SPFF_EPI_HOT
}

// ---------------------------------------------------------------------------
// Row kernels with register-resident transforms (M = nx/2 in {64 .. 1024},
// FP32): a group of L = M/E lanes (E = 4, 8, or 16 for M = 1024) owns one row
// (R = blockDim/L rows per work-group); lane l holds z[h] = x[2h] + i x[2h+1]
// for h = l + m L.  The
// prologue / epilogue run per pixel pair on the registers; the real <->
// half-spectrum step pairs bin k with M - k by a cross-lane shuffle (same
// pattern as the packed column); the transposed spectrum store / load goes
// through an LDS tile [kx][row] so that R consecutive y of one kx move as
// one run.
// ---------------------------------------------------------------------------
template <int M>
struct RowLds {
  // exchange areas of the R row groups, then the [kx][row] tile
  static __device__ __forceinline__ int tile_index(int k, int r, int R) { return k * (R + 1) + r; }
  static size_t bytes(int R, size_t csize) {
    return ((size_t)R * XArea<M>::size + (size_t)M * (R + 1)) * csize;
  }
};

// partner slots for bin k = l + m L and M - k: slot E-1-m of lane L-l, or
// for lane 0 its own slot (E-m) mod E
template <typename real, int E, int L>
__device__ __forceinline__ void partner_bins(const cplx<real> (&v)[E], cplx<real> (&pn)[E], int lane) {
  const int src = (L - lane) & (L - 1);
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const real px = __shfl(v[i].x, src, L), py = __shfl(v[i].y, src, L);
    pn[E - 1 - i] = mk<cplx<real>>(px, py);
  }
  if (lane == 0) {
#pragma unroll
    for (int m = 0; m < E; ++m) pn[m] = v[(E - m) & (E - 1)];
  }
}

template <typename real, int M, int E>
__device__ __forceinline__ void k_rowfwdr_body(const int* __restrict__ list, const SlotPtr<real>* __restrict__ ptrs,
                                               const SlotParam* __restrict__ prms, const CtrlArgs A,
                                               const cplx<real>* __restrict__ twx, double* __restrict__ part,
                                               int ny, int ngr) {
  using C = cplx<real>;
  constexpr int L = M / E, nx = 2 * M;
  extern __shared__ unsigned char smem_raw[];
  __shared__ double red[(THREADS / 64) * NP_ROW];
  __shared__ SlotCtl lctl;
  int g, si;
  row_coords(ngr, g, si);
  const int s = list[si];
  if (s < 0) return;
  tick_control<real>(s, g == 0, A, ptrs, prms, nx, ny, ngr, lctl);
  const SlotCtl& ctl = lctl;
  const int phase = ctl.phase;
  const int ncomp = phase_comps_row(phase);
  if (phase != PH_AM_CHK && phase != PH_TD_RESTORE && ncomp == 0) return;
  const SlotParam& P = prms[s];
  const SlotPtr<real> F = ptrs[s];
  const int R = blockDim.x / L;
  const int row = threadIdx.x / L, lane = threadIdx.x & (L - 1);
  const int y0 = g * R;
  const int n = nx * ny;
  C* xa = reinterpret_cast<C*>(smem_raw) + row * XArea<M>::size;
  C* tile = reinterpret_cast<C*>(smem_raw) + R * XArea<M>::size;
  double acc[NP_ROW];
#pragma unroll
  for (int i = 0; i < NP_ROW; ++i) acc[i] = 0.0;
  if (phase == PH_STATS) acc[3] = -1.0e300;
  const RowCtx<real> X = row_ctx<real>(ctl, P, phase, ncomp, n);

  C v[3][E];
  {
    real val[E][3][2];
    row_prologue_n<real, E, 2 * L>(X, P, F.E, F.phi, F.phi_ref, F.eps, F.theta, F.rm, F.pm,
                                   (y0 + row) * nx + 2 * lane, val, acc);
#pragma unroll
    for (int m = 0; m < E; ++m)
#pragma unroll
      for (int c = 0; c < 3; ++c) v[c][m] = mk<C>(val[m][c][0], val[m][c][1]);
  }
  if (ncomp > 0) {
    C* spec = reinterpret_cast<C*>(F.spec);
    const int logR = ilog2(R);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (c < ncomp) {
        reg_fft<real, false, M, E>(v[c], xa, lane, twx, 2);
        // half spectrum of the real row: X[k] = e + w^k o (k > 0), bin 0
        // packs X[0] + i X[M]
        C pn[E];
        partner_bins<real, E, L>(v[c], pn, lane);
        __syncthreads();  // the tile is free
#pragma unroll
        for (int m = 0; m < E; ++m) {
          const int k = lane + m * L;
          C out;
          if (k == 0) {
            out = mk<C>(v[c][m].x + v[c][m].y, v[c][m].x - v[c][m].y);
          } else {
            const C zk = v[c][m], zm = cconj(pn[m]);
            const C e = cscale(cadd(zk, zm), real(0.5));
            const C od = cscale(cmulni(csub(zk, zm)), real(0.5));
            out = cadd(e, cmul(twx[k], od));
          }
          tile[RowLds<M>::tile_index(k, row, R)] = out;
        }
        __syncthreads();
        // transposed store: spec[c][kx][y0 + r], r fastest
        for (int idx = threadIdx.x; idx < M * R; idx += blockDim.x) {
          const int r = idx & (R - 1), k = idx >> logR;
          stc<real>(spec + (size_t)(c * M + k) * ny + y0 + r, tile[RowLds<M>::tile_index(k, r, R)]);
        }
      }
    }
  }
  block_reduce_store<NP_ROW>(acc, red, part + (size_t)s * NP_ROW * ngr + g, ngr, nacc_rowfwd(phase),
                             phase == PH_STATS ? 3 : (phase == PH_PF_ASM ? 1 : -1));
}

template <typename real, int M, int E>
__device__ __forceinline__ void k_rowinvr_body(const int* __restrict__ list, const SlotPtr<real>* __restrict__ ptrs,
                                               const SlotParam* __restrict__ prms, const SlotCtl* __restrict__ ctls,
                                               const cplx<real>* __restrict__ twx,
                                               const double* __restrict__ part_row, double* __restrict__ part,
                                               int ny, int ngr) {
  using C = cplx<real>;
  constexpr int L = M / E, nx = 2 * M;
  extern __shared__ unsigned char smem_raw[];
  __shared__ double red[(THREADS / 64) * NP_INV];
  int g, si;
  row_coords(ngr, g, si);
  const int s = list[si];
  if (s < 0) return;
  const SlotCtl& ctl = ctls[s];
  const int phase = ctl.phase;
  int ncomp;
  switch (phase) {
    case PH_M_RES:
    case PH_M_CG:
    case PH_X_PROJ:
    case PH_X_DISP:
      ncomp = 3;
      break;
    case PH_PF_ASM:
    case PH_PF_R:
    case PH_X_LAP:
      ncomp = 1;
      break;
    default:
      return;
  }
  const SlotParam& P = prms[s];
  const SlotPtr<real> F = ptrs[s];
  const int R = blockDim.x / L;
  const int row = threadIdx.x / L, lane = threadIdx.x & (L - 1);
  const int y0 = g * R;
  const int n = nx * ny;
  const RowCtx<real> X = row_ctx<real>(ctl, P, phase, ncomp, n);
  C* xa = reinterpret_cast<C*>(smem_raw) + row * XArea<M>::size;
  C* tile = reinterpret_cast<C*>(smem_raw) + R * XArea<M>::size;
  const C* spec = reinterpret_cast<const C*>(F.spec);
  const int logR = ilog2(R);

  // Few problems per launch (four points per lane): the group's tile entries
  // of every component (E per thread and component: R rows x M bins over
  // R L threads) are loaded up front, so that the components cost one
  // memory round trip instead of one each
  C pre[3][E];
  if constexpr (E == 4) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (c < ncomp) {
#pragma unroll
        for (int i = 0; i < E; ++i) {
          const int idx = threadIdx.x + i * blockDim.x;
          const int r = idx & (R - 1), k = idx >> logR;
          pre[c][i] = ldc<real>(spec + (size_t)(c * M + k) * ny + y0 + r);
        }
      }
    }
  }

  // CG step length from this tick's row-forward partials (same fixed-order
  // reduction as the controller)
  __shared__ double scal[1];
  real alpha = 0;
  if (phase == PH_M_CG) {
    if (threadIdx.x < 64) {
      const double pcp = wave_reduce_partials(part_row + (size_t)s * NP_ROW * ngr, ngr);
      if (threadIdx.x == 0) scal[0] = (pcp > 0.0 && isfinite(pcp)) ? ctl.rr / pcp : 0.0;
    }
    __syncthreads();
    alpha = real(scal[0]);
  }

  C v[3][E];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (c < ncomp) {
      if (c > 0) __syncthreads();  // the previous component's tile reads are done
      if constexpr (E == 4) {
#pragma unroll
        for (int i = 0; i < E; ++i) {
          const int idx = threadIdx.x + i * blockDim.x;
          const int r = idx & (R - 1), k = idx >> logR;
          tile[RowLds<M>::tile_index(k, r, R)] = pre[c][i];
        }
      } else {
        for (int idx = threadIdx.x; idx < M * R; idx += blockDim.x) {
          const int r = idx & (R - 1), k = idx >> logR;
          tile[RowLds<M>::tile_index(k, r, R)] = ldc<real>(spec + (size_t)(c * M + k) * ny + y0 + r);
        }
      }
      __syncthreads();
#pragma unroll
      for (int m = 0; m < E; ++m) v[c][m] = tile[RowLds<M>::tile_index(lane + m * L, row, R)];
      // from the packed half spectrum to Z whose unnormalised inverse FFT
      // gives nx (x[2h] + i x[2h+1])
      C pn[E];
      partner_bins<real, E, L>(v[c], pn, lane);
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int k = lane + m * L;
        if (k == 0) {
          v[c][m] = mk<C>(v[c][m].x + v[c][m].y, v[c][m].x - v[c][m].y);
        } else {
          const C xk = v[c][m], xm = cconj(pn[m]);
          const C a = cadd(xk, xm), b = csub(xk, xm);
          v[c][m] = cadd(a, cmuli(cmul(cconj(twx[k]), b)));
        }
      }
      reg_fft<real, true, M, E>(v[c], xa, lane, twx, 2);
    }
  }
  double acc[NP_INV] = {0.0, 0.0, 0.0, 0.0};
  if (phase == PH_PF_ASM) acc[1] = -1.0e300;  // max of -F_phi (near-equilibrium)
  {
    C q[E][3];
#pragma unroll
    for (int m = 0; m < E; ++m)
#pragma unroll
      for (int c = 0; c < 3; ++c) q[m][c] = c < ncomp ? v[c][m] : mk<C>(real(0), real(0));
    row_epilogue_n<real, E, 2 * L>(X, P, F.phi, F.phi_ref, F.theta, F.rm, F.pm, (y0 + row) * nx + 2 * lane, q,
                                   alpha, acc);
  }
  block_reduce_store<NP_INV>(acc, red, part + (size_t)s * NP_INV * ngr + g, ngr, nacc_rowinv(phase),
                             phase == PH_PF_ASM ? 1 : -1);
}

// ===========================================================================
// Row-inverse kernel: transposed load -> C2R row FFTs -> epilogue (per
// phase); FP64 partial sums per work-group.
// ===========================================================================
template <typename real>
__device__ __forceinline__ void k_rowinv_body(const int* __restrict__ list,
                                                    const SlotPtr<real>* __restrict__ ptrs,
                                                    const SlotParam* __restrict__ prms,
                                                    const SlotCtl* __restrict__ ctls,
                                                    const cplx<real>* __restrict__ twx,
                                                    const double* __restrict__ part_row,
                                                    double* __restrict__ part, int nx, int ny, int R, int ngr) {
  using C = cplx<real>;
  extern __shared__ unsigned char smem_raw[];
  __shared__ double red[(THREADS / 64) * NP_INV];
  int g, si;
  row_coords(ngr, g, si);
  const int s = list[si];
  if (s < 0) return;
  const SlotCtl& ctl = ctls[s];
  const int phase = ctl.phase;
  int ncomp;
  switch (phase) {
    case PH_M_RES:
    case PH_M_CG:
    case PH_X_PROJ:
    case PH_X_DISP:
      ncomp = 3;
      break;
    case PH_PF_ASM:
    case PH_PF_R:
    case PH_X_LAP:
      ncomp = 1;
      break;
    default:
      return;
  }
  const SlotParam& P = prms[s];
  const SlotPtr<real> F = ptrs[s];
  const int M = nx >> 1, stride = M + PAD;
  const int y0 = g * R;
  const int n = nx * ny;
  const RowCtx<real> X = row_ctx<real>(ctl, P, phase, ncomp, n);
  C* buf = reinterpret_cast<C*>(smem_raw);
  const C* spec = reinterpret_cast<const C*>(F.spec);

  // CG step length from this tick's row-forward partials (same fixed-order
  // reduction as the controller)
  __shared__ double scal[1];
  real alpha = 0;
  if (phase == PH_M_CG) {
    if (threadIdx.x < 64) {
      const double pcp = wave_reduce_partials(part_row + (size_t)s * NP_ROW * ngr, ngr);
      if (threadIdx.x == 0) scal[0] = (pcp > 0.0 && isfinite(pcp)) ? ctl.rr / pcp : 0.0;
    }
    __syncthreads();
    alpha = real(scal[0]);
  }

  const int tot = ncomp * M * R;
  const int logM = ilog2(M), logR = ilog2(R);
  for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
    const int r = idx & (R - 1);
    const int rest = idx >> logR;
    const int kx = rest & (M - 1), c = rest >> logM;
    buf[(c * R + r) * stride + kx] = ldc<real>(spec + (size_t)rest * ny + y0 + r);
  }
  __syncthreads();
  c2r_pre<real>(buf, M, ncomp * R, stride, twx);
  fft_lds<real, true, MAXE>(buf, M, ncomp * R, stride, twx, 2);

  double acc[NP_INV] = {0.0, 0.0, 0.0, 0.0};
  if (phase == PH_PF_ASM) acc[1] = -1.0e300;  // max of -F_phi (near-equilibrium)
  for (int idx = threadIdx.x; idx < R * M; idx += blockDim.x) {
    const int r = idx >> logM, h = idx & (M - 1);
    const int o = (y0 + r) * nx + 2 * h;
    const int li = r * stride + h;
    C q[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) q[c] = c < ncomp ? buf[c * R * stride + li] : mk<C>(real(0), real(0));
    row_epilogue<real>(X, P, F.phi, F.phi_ref, F.theta, F.rm, F.pm, o, q, alpha, acc);
  }
  block_reduce_store<NP_INV>(acc, red, part + (size_t)s * NP_INV * ngr + g, ngr, nacc_rowinv(phase),
                             phase == PH_PF_ASM ? 1 : -1);
}

// Algorithmic HBM bytes per pixel moved by the row-forward, column and
// row-inverse kernels for the phase a slot executed (r = sizeof(real)):
// every input plane read once, every output plane written once, half spectra
// (nx/2 * ny complex values = r bytes per pixel per component) written by the
// row-forward kernel, read and written by the column kernel, read by the
// row-inverse kernel.
__device__ inline void phase_bytes(int phase, int flags, int split, double r, double* b) {
  const double sp = r;  // half spectrum, per pixel per component
  b[0] = b[1] = b[2] = 0.0;
  switch (phase) {
    case PH_M_RES:
      b[0] = r * 5 + 3 * sp + ((flags & FL_THETA_PENDING) ? 6 * r : 0) + ((flags & FL_FIRST_OF_STEP) ? r : 0);
      b[1] = 6 * sp;
      b[2] = 3 * sp + 3 * r;
      break;
    case PH_M_CG:
      b[0] = r * (2 + 3 + ((flags & FL_CG_FIRST) ? 0 : 3) + (split ? 3 : 0) + 3) + 3 * sp;
      b[1] = 6 * sp;
      b[2] = 3 * sp + r * (3 + 3 + ((flags & FL_CG_FIRST) ? 0 : 3) + 6);
      break;
    case PH_PF_ASM:
      b[0] = r * (6 + 4) + sp + ((flags & FL_NE_SCALE) ? 3 * r : 0);
      b[1] = 2 * sp;
      b[2] = sp + r * (4 + 1) + 1 + ((flags & FL_NE_CHECK) ? r : 0);
      break;
    case PH_PF_PQ:
      b[0] = r * (2 + ((flags & FL_PF_FIRST) ? 0 : 1) + 1) + 1 + sp;
      b[1] = sp;
      break;
    case PH_PF_R:
      b[0] = r * (3 + 1) + sp;
      b[1] = 2 * sp;
      b[2] = sp + r * (5 + 1) + 1;
      break;
    case PH_AM_CHK:
    case PH_TD_RESTORE:
      b[0] = 2 * r;
      break;
    case PH_STATS:
      b[0] = r * 5 + sp;
      b[1] = sp;
      break;
    default:
      break;
  }
}

// ===========================================================================
// Controller of one slot, run by one wavefront.  Reduces the tick's partials
// in a fixed order, updates FP64 scalars and moves the slot's state machine.
// ===========================================================================
__device__ __forceinline__ int wave_min_int(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
  return v;
}

// Near-equilibrium strain scaling (Sec. 3.2.2, Algorithm 4).  fm is the
// largest -F_phi(phi_n, eps_n); the row-inverse kernel of the assembly kept
// the unmasked residual F_phi in rm[1] and its per-row-group maxima in
// gmax[0 .. ngr).  x* is the first pixel (row-major) where -F_phi equals fm:
// the first row group holding the maximum, then the first pixel of that
// group's rows.  With d = -h'(phi_n) psi0+ at x*, gamma^2 =
// (fphi_max - (fm - d)) / d (psi0+ is degree-two homogeneous in the strain),
// clamped at 0 and capped at 1 + deps_max / max|eps_bar|.  Returns false
// (no scaling) when x* is not found or d is not positive.  One wavefront.
template <typename real>
__device__ bool ne_gamma(const SlotPtr<real>& F, const SlotParam& P, const SlotCtl& C, double fm,
                         const double* __restrict__ gmax, int nx, int ny, int ngr, double* gamma) {
  const int lane = threadIdx.x & 63;
  int gs = ngr;
  for (int i = lane; i < ngr; i += 64)
    if (gmax[i] == fm) {
      gs = i;
      break;
    }
  gs = wave_min_int(gs);
  if (gs >= ngr) return false;
  const int n = nx * ny, rows = ny / ngr;
  const int base = gs * rows * nx, cnt = rows * nx;
  const real* fr = F.rm + n;
  int xi = n;
  for (int i = lane; i < cnt; i += 64)
    if (-double(fr[base + i]) == fm) {
      xi = base + i;
      break;
    }
  xi = wave_min_int(xi);
  if (xi >= n) return false;
  const real E = F.E[xi], ph = F.phi_ref[xi];
  const real lam = real(P.lam_t) * E, mu = real(P.mu_t) * E;
  const Sym<real> e = {real(C.eps_bar[0]) + F.eps[xi], real(C.eps_bar[1]) + F.eps[n + xi],
                       real(C.eps_bar[2]) + F.eps[2 * n + xi]};
  real pp, pm;
  energies(e, lam, mu, P.split, &pp, &pm);
  const double d = double(real(2) * (real(1) - ph) * pp);
  if (!(d > 0.0)) return false;
  double g = sqrt(fmax((P.fphi_max - (fm - d)) / d, 0.0));
  const double eb = fmax(fabs(C.eps_bar[0]), fmax(fabs(C.eps_bar[1]), fabs(C.eps_bar[2])));
  if (eb > 0.0) g = fmin(g, 1.0 + P.deps_max / eb);
  *gamma = g;
  return true;
}

// The controller step of slot s after a tick: one wavefront reads the
// tick's partial sums and the control block C, lane 0 writes the advanced
// block back into C.  `writer`: this wavefront also records the step's
// statistics (byte counters, finished load steps, the queue position); the
// other wavefronts that run the same step on their own copy of C (every
// row-forward work-group of the slot) only advance their copy.
template <typename real>
__device__ __forceinline__ void ctrl_slot(int s, const SlotPtr<real>* __restrict__ ptrs,
                                          const SlotParam* __restrict__ prms, SlotCtl& C, bool writer,
                                          const double* __restrict__ prow, const double* __restrict__ pcol,
                                          const double* __restrict__ pinv, double* __restrict__ prof,
                                          SlotSeq* __restrict__ seqs, StepRec* __restrict__ recs, int nx, int ny,
                                          int ngr, int ngc) {
  const double* pr = prow + (size_t)s * NP_ROW * ngr;
  const double* pc = pcol + (size_t)s * NP_COL * ngc;
  const double* pi = pinv + (size_t)s * NP_INV * ngr;
  const int phase = C.phase;
  if (phase == PH_IDLE) return;
  if (threadIdx.x == 0 && C.ticks == 0 && C.t_start == 0) C.t_start = wall_clock64();
  const SlotParam& P = prms[s];
  if (prof && writer && threadIdx.x == 0) {
    double b[3];
    phase_bytes(phase, C.flags, P.contact, double(sizeof(real)), b);
    const double npx = double(nx) * double(ny);
    prof[3 * s + 0] += b[0] * npx;
    prof[3 * s + 1] += b[1] * npx;
    prof[3 * s + 2] += b[2] * npx;
  }
  const double inv_n = 1.0 / (double(nx) * double(ny));
  // all lanes compute the same values; lane 0 writes
  double v[8];
  int nphase = phase;
  int flags = C.flags;
  int cg = C.cg, cg_newton = C.cg_newton, newton = C.newton, bccg = C.bccg, pf_it = C.pf_it, am = C.am;
  int newton_solve = C.newton_solve;
  int status = C.status;
  double mech_ref = C.mech_ref, mech_target = C.mech_target, mech_res = C.mech_res, rr = C.rr;
  double inner_tol = C.inner_tol, alpha_m = C.alpha_m, beta_m = C.beta_m;
  double pf_ref = C.pf_ref, pf_target = C.pf_target, pf_res = C.pf_res, rr_pf = C.rr_pf;
  double alpha_pf = C.alpha_pf, beta_pf = C.beta_pf, pq = C.pq, rp = C.rp, dphi = C.dphi;
  double pf_bnorm = C.pf_bnorm, pf_best = C.pf_best, mech_floor = C.mech_floor, pf_floor = C.pf_floor;
  int pf_best_it = C.pf_best_it;
  double eta_dt = C.eta_dt, dt = C.dt;
  int halvings = C.halvings, advance = C.advance;
  double gamma = C.gamma, fmax_ne = C.fmax_ne;
  int ne_flag = C.ne_flag;
  bool scaled = false;
  bool bad = false;
  auto pf_done = [&]() {
    if (flags & FL_INIT_SOLVE) {
      flags &= ~FL_INIT_SOLVE;
      nphase = PH_IDLE;
    } else {
      nphase = PH_AM_CHK;
    }
  };
  switch (phase) {
    case PH_M_RES: {
      double o[3];
      wave_reduce_partials_n<3>({pr, pr + 1 * ngr, pi}, {ngr, ngr, ngr}, o);
      const double sh2 = o[0], sg2 = o[1], r2 = o[2];
      bad = !isfinite(sh2) || !isfinite(r2) || !isfinite(sg2);
      mech_res = sqrt(r2);
      // G[sigma] cannot be evaluated more accurately than the rounding of
      // sigma and of the transforms: below that floor the solve is done
      mech_floor = P.floor_coef * sqrt(sg2);
      if (!(flags & FL_MECH_STARTED)) {
        // first residual of this mechanics solve fixes the reference norm
        mech_ref = fmax(sqrt(sh2), mech_res);
        mech_target = P.tol_mech * mech_ref + P.tol_abs_mech;
        flags |= FL_MECH_STARTED;
        newton_solve = 0;
      }
      flags &= ~(FL_FIRST_OF_STEP | FL_THETA_PENDING);
      if (mech_res <= fmax(mech_target, mech_floor)) {
        nphase = PH_PF_ASM;
      } else if (newton_solve >= P.max_newton) {
        flags |= FL_NOT_CONVERGED;
        nphase = PH_PF_ASM;
      } else {
        rr = r2;
        inner_tol = (P.contact == 0) ? fmax(mech_target, mech_floor)
                                   : fmax(0.1 * mech_res, fmax(mech_target, mech_floor));
        cg_newton = 0;
        flags |= FL_CG_FIRST;
        nphase = PH_M_CG;
      }
      if (nphase == PH_PF_ASM) flags &= ~FL_MECH_STARTED;
      break;
    }
    case PH_M_CG: {
      double o[2];
      wave_reduce_partials_n<2>({pr, pi}, {ngr, ngr}, o);
      const double pcp = o[0], r2 = o[1];
      bad = !isfinite(pcp) || !isfinite(r2);
      alpha_m = (pcp > 0.0) ? rr / pcp : 0.0;
      ++cg;
      ++cg_newton;
      flags &= ~FL_CG_FIRST;
      beta_m = (rr > 0.0) ? r2 / rr : 0.0;
      rr = r2;
      if (sqrt(r2) <= inner_tol || cg_newton >= P.max_cg || pcp <= 0.0) {
        if (sqrt(r2) > inner_tol) flags |= FL_NOT_CONVERGED;
        ++newton;
        ++newton_solve;
        flags |= FL_THETA_PENDING;
        nphase = PH_M_RES;
      }
      break;
    }
    case PH_PF_ASM: {
      flags &= ~FL_NE_SCALE;
      if (flags & FL_NE_CHECK) {
        // Algorithm 4: -F_phi(phi_n, eps_n) and the crack driving force
        // -h'(phi_n) psi0+ were evaluated by this assembly
        flags &= ~FL_NE_CHECK;
        double o[2];
        wave_reduce_partials_n<2>({pi + 1 * ngr, pr + 1 * ngr}, {ngr, ngr}, o, 3u);
        fmax_ne = o[0];
        const double dmax = o[1];
        if (fmax_ne > P.fphi_max && dmax > P.drive_thr) ne_flag = 1;
        if (fmax_ne > P.fphi_max && ne_flag &&
            ne_gamma<real>(ptrs[s], P, C, fmax_ne, pi + 1 * ngr, nx, ny, ngr, &gamma)) {
          scaled = true;
          flags |= FL_NE_SCALE;
          nphase = PH_PF_ASM;  // assemble again at the scaled strain
          break;
        }
      }
      double o[4];
      wave_reduce_partials_n<4>({pr, pi, pi + 2 * ngr, pi + 3 * ngr}, {ngr, ngr, ngr, ngr}, o);
      const double b2 = o[0], r2 = o[1], x2 = o[2], dx2 = o[3];
      bad = !isfinite(b2) || !isfinite(r2);
      pf_res = sqrt(r2);
      pf_bnorm = sqrt(b2);
      pf_ref = fmax(pf_bnorm, pf_res);
      pf_target = P.tol_pf * pf_ref + P.tol_abs_pf;
      // attainable accuracy of r = J phi - b in the working precision
      pf_floor = P.floor_coef * (sqrt(dx2) + P.kappa * P.lap_rms * sqrt(x2) + pf_bnorm);
      rr_pf = r2;
      pf_it = 0;
      pf_best = pf_res;
      pf_best_it = 0;
      if (pf_res <= fmax(pf_target, pf_floor)) {
        pf_done();
      } else {
        flags |= FL_PF_FIRST;
        nphase = PH_PF_PQ;
      }
      break;
    }
    case PH_PF_PQ: {
      // sum d p^2, sum r p, sum L |p^|^2
      double o[3];
      wave_reduce_partials_n<3>({pr, pr + 1 * ngr, pc}, {ngr, ngr, ngc}, o);
      v[0] = o[0];
      v[1] = o[1];
      v[2] = o[2];
      bad = !isfinite(v[0]) || !isfinite(v[1]) || !isfinite(v[2]);
      pq = v[0] + P.kappa * inv_n * v[2];
      rp = v[1];
      flags &= ~FL_PF_FIRST;
      if (!(pq > 0.0)) {
        flags |= FL_NOT_CONVERGED;
        pf_done();
      } else {
        alpha_pf = -rp / pq;
        nphase = PH_PF_R;
      }
      break;
    }
    case PH_PF_R: {
      double o[4];
      wave_reduce_partials_n<4>({pi, pi + 1 * ngr, pi + 2 * ngr, pi + 3 * ngr}, {ngr, ngr, ngr, ngr}, o);
      const double r2 = o[0], rro = o[1], x2 = o[2], dx2 = o[3];
      bad = !isfinite(r2) || !isfinite(rro);
      beta_pf = (r2 - rro) / (alpha_pf * pq);
      rr_pf = r2;
      pf_res = sqrt(r2);
      pf_floor = P.floor_coef * (sqrt(dx2) + P.kappa * P.lap_rms * sqrt(x2) + pf_bnorm);
      ++pf_it;
      ++bccg;
      if (pf_res < pf_best) {
        pf_best = pf_res;
        pf_best_it = pf_it;
      }
      if (pf_res <= fmax(pf_target, pf_floor)) {
        pf_done();
      } else if (P.stall_iters > 0 && pf_it - pf_best_it >= P.stall_iters) {
        flags |= FL_STALLED;
        pf_done();
      } else if (pf_it >= P.max_bccg) {
        flags |= FL_NOT_CONVERGED;
        pf_done();
      } else {
        nphase = PH_PF_PQ;
      }
      break;
    }
    case PH_AM_CHK: {
      dphi = wave_reduce_partials(pr, ngr);
      bad = !isfinite(dphi);
      ++am;
      if (P.evolution == 2) {
        advance = dphi < P.dphi_min ? 1 : 0;
        nphase = PH_STATS;
        break;
      }
      if (P.evolution == 1) {
        // Algorithm 3: accept the phase field if its change is small enough
        // or dt has reached its floor, else retry from phi_n with dt / 2
        if (dphi < P.dphi_max || dt <= P.dt_min) {
          if (dphi < 0.5 * P.dphi_max) dt = fmin(2.0 * dt, P.dt_max);
          advance = (dphi < P.dphi_min && dt >= P.dt_max) ? 1 : 0;
          nphase = PH_STATS;
        } else {
          dt *= 0.5;
          ++halvings;
          eta_dt = P.eta / dt;
          nphase = PH_TD_RESTORE;
        }
        break;
      }
      if (dphi <= P.tol_am) {
        nphase = PH_STATS;
      } else if (am >= P.max_am) {
        flags |= FL_NOT_CONVERGED;
        nphase = PH_STATS;
      } else {
        nphase = PH_M_RES;
      }
      break;
    }
    case PH_TD_RESTORE:
      nphase = PH_PF_ASM;
      break;
    case PH_X_PROJ:
    case PH_X_DISP:
    case PH_X_LAP:
      nphase = PH_IDLE;
      break;
    case PH_STATS: {
      double o[4];
      wave_reduce_partials_n<4>({pr, pr + 1 * ngr, pr + 2 * ngr, pr + 3 * ngr}, {ngr, ngr, ngr, ngr}, o, 8u);
      for (int i = 0; i < 4; ++i) v[i] = o[i];
      wave_reduce_partials_n<4>({pr + 4 * ngr, pr + 5 * ngr, pr + 6 * ngr, pr + 7 * ngr}, {ngr, ngr, ngr, ngr}, o);
      for (int i = 0; i < 4; ++i) v[4 + i] = o[i];
      const double lg = wave_reduce_partials(pc, ngc);
      bad = false;
      for (int i = 0; i < 8; ++i) bad |= !isfinite(v[i]);
      if (threadIdx.x == 0) {
        C.F_e = v[0];
        C.F_f = P.cwl * (v[1] + P.ell * P.ell * inv_n * lg);
        C.phi_sum = v[2];
        C.phi_max = v[3];
        C.crack_px = v[4];
        C.sbar[0] = v[5] * inv_n;
        C.sbar[1] = v[6] * inv_n;
        C.sbar[2] = v[7] * inv_n;
      }
      nphase = PH_IDLE;
      break;
    }
    default:
      break;
  }
  if (bad) {
    flags |= FL_NONFINITE;
    status = -4;
    nphase = PH_IDLE;
  }
  // a load step just ended: record it and start the next one of the queue
  bool restart = false;
  if (seqs && nphase == PH_IDLE && (phase == PH_STATS || bad) && !(flags & FL_INIT_SOLVE) && threadIdx.x == 0 &&
      C.seq_pos < seqs[s].len) {
    const int pos = C.seq_pos;
    if (writer) {
      StepRec& r = recs[(size_t)s * SEQ_MAX + pos];
      r.status = status;
      r.flags = flags;
      r.am = am;
      r.newton = newton;
      r.cg = cg;
      r.bccg = bccg;
      r.ticks = C.ticks + 1;
      r.dt = dt;
      r.halvings = halvings;
      r.advance = advance;
      r.gamma = gamma;
      r.fmax_ne = fmax_ne;
      r.ne_flag = ne_flag;
      r.t_start = C.t_start;
      r.t_end = wall_clock64();
      r.dphi = dphi;
      r.mech_res = mech_res;
      r.pf_res = pf_res;
      r.F_e = C.F_e;
      r.F_f = C.F_f;
      for (int k = 0; k < 3; ++k) {
        r.sbar[k] = C.sbar[k];
        r.eps_bar[k] = C.eps_bar[k];
      }
      r.phi_sum = C.phi_sum;
      r.phi_max = C.phi_max;
      r.crack_px = C.crack_px;
      seqs[s].pos = pos + 1;
    }
    C.seq_pos = pos + 1;
    if (pos + 1 < seqs[s].len && status >= 0) restart = true;
  }
  if (restart) {
    // fresh control block for the next load step of the queue
    const SlotSeq& q = seqs[s];
    const int pos = C.seq_pos;
    if (q.incr) {
      // evolution queue: the next step continues from this step's final
      // macroscopic strain, plus the increment if the algorithm advances
      const double a = advance ? 1.0 : 0.0;
      C.eps_bar[0] += a * q.eps_bar[pos][0];
      C.eps_bar[1] += a * q.eps_bar[pos][1];
      C.eps_bar[2] += a * q.eps_bar[pos][2];
    } else {
      C.eps_bar[0] = q.eps_bar[pos][0];
      C.eps_bar[1] = q.eps_bar[pos][1];
      C.eps_bar[2] = q.eps_bar[pos][2];
    }
    C.phase = PH_M_RES;
    C.flags = FL_FIRST_OF_STEP | (P.evolution == 2 ? FL_NE_CHECK : 0);
    C.am = C.newton = C.cg = C.bccg = C.cg_newton = C.pf_it = C.newton_solve = 0;
    C.ticks = 0;
    C.status = 0;
    C.dphi = 0.0;
    C.dt = dt;
    C.halvings = 0;
    C.advance = 0;
    C.eta_dt = P.evolution == 1 ? P.eta / dt : (P.evolution == 2 ? P.eta / P.dt_max : P.eta_dt);
    C.gamma = 1.0;
    C.fmax_ne = 0.0;
    C.ne_flag = ne_flag;
    C.t_start = wall_clock64();
    return;
  }
  if (threadIdx.x == 0) {
    C.phase = nphase;
    C.flags = flags;
    C.cg = cg;
    C.cg_newton = cg_newton;
    C.newton = newton;
    C.bccg = bccg;
    C.pf_it = pf_it;
    C.newton_solve = newton_solve;
    C.am = am;
    C.status = status;
    C.mech_ref = mech_ref;
    C.mech_target = mech_target;
    C.mech_res = mech_res;
    C.rr = rr;
    C.inner_tol = inner_tol;
    C.alpha_m = alpha_m;
    C.beta_m = beta_m;
    C.pf_ref = pf_ref;
    C.pf_target = pf_target;
    C.pf_res = pf_res;
    C.rr_pf = rr_pf;
    C.alpha_pf = alpha_pf;
    C.beta_pf = beta_pf;
    C.pq = pq;
    C.rp = rp;
    C.dphi = dphi;
    C.pf_bnorm = pf_bnorm;
    C.pf_best = pf_best;
    C.pf_best_it = pf_best_it;
    C.mech_floor = mech_floor;
    C.pf_floor = pf_floor;
    C.eta_dt = eta_dt;
    C.dt = dt;
    C.halvings = halvings;
    C.advance = advance;
    C.gamma = gamma;
    C.fmax_ne = fmax_ne;
    C.ne_flag = ne_flag;
    if (scaled) {
      C.eps_bar[0] *= gamma;
      C.eps_bar[1] *= gamma;
      C.eps_bar[2] *= gamma;
    }
    C.ticks = C.ticks + 1;
  }
}

// ===========================================================================
// Kernel entry points: the bodies above, stamped with the device clock when
// profiling (kt != nullptr).
// ===========================================================================
__device__ __forceinline__ int kt_line() {
  return (blockIdx.x + blockIdx.y * 29) & (KT_LINES - 1);
}
__device__ __forceinline__ void kt_begin(KTime* kt) {
  if (kt && threadIdx.x == 0)
    atomicMin(&kt->start[kt_line() * KT_STRIDE], (unsigned long long)wall_clock64());
}
__device__ __forceinline__ void kt_end(KTime* kt) {
  if (kt) {
    __syncthreads();
    if (threadIdx.x == 0) atomicMax(&kt->end[kt_line() * KT_STRIDE], (unsigned long long)wall_clock64());
  }
}

// Folds the kernel times of one tick (kt[0..2]: row-forward, column,
// row-inverse) into ktsum and resets the words for the tick after next; one
// wavefront, lane l takes line l.  ktsum[j]: activity of kernel j (first
// start to last end); ktsum[4 + j]: its span (first start to the first
// start of the kernel after it; t_next for the row-inverse kernel).
__device__ __forceinline__ void kt_fold(KTime* kt, unsigned long long t_next, unsigned long long* ktsum) {
  const int l = threadIdx.x & 63;
  unsigned long long st[3], en[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    unsigned long long a = kt[j].start[l * KT_STRIDE], b = kt[j].end[l * KT_STRIDE];
    kt[j].start[l * KT_STRIDE] = ~0ull;
    kt[j].end[l * KT_STRIDE] = 0ull;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const unsigned long long a2 = __shfl_xor(a, off, 64), b2 = __shfl_xor(b, off, 64);
      a = a2 < a ? a2 : a;
      b = b2 > b ? b2 : b;
    }
    st[j] = a;
    en[j] = b;
  }
  if (l == 0) {
    const unsigned long long nxt[3] = {st[1], st[2], t_next};
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      if (en[j] > st[j]) ktsum[j] += en[j] - st[j];
      if (nxt[j] > st[j] && st[j] != ~0ull) ktsum[4 + j] += nxt[j] - st[j];
    }
  }
}
// First start stamped in kt (one wavefront).
__device__ __forceinline__ unsigned long long kt_first_start(const KTime* kt) {
  unsigned long long a = kt->start[(threadIdx.x & 63) * KT_STRIDE];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long a2 = __shfl_xor(a, off, 64);
    a = a2 < a ? a2 : a;
  }
  return a;
}

// Timer bookkeeping of the column kernel: with timers on, the launch has one
// extra row of work-groups; its group 0 folds the previous tick's times
// (kt_prev, null for the first tick of a block) -- the previous tick ended
// before this tick's row-forward kernel, whose first start (kt_row) closes
// the previous row-inverse span -- and the other extra groups return.
struct ColTimers {
  KTime* kt;             // this column kernel's stamps
  KTime* kt_prev;        // the previous tick's three kernels
  const KTime* kt_row;   // this tick's row-forward kernel
  unsigned long long* ktsum;
};
__device__ __forceinline__ bool col_timer_group(const ColTimers& T) {
  if (!T.kt || blockIdx.y != gridDim.y - 1) return false;
  if (T.kt_prev && blockIdx.x == 0 && threadIdx.x < 64) kt_fold(T.kt_prev, kt_first_start(T.kt_row), T.ktsum);
  return true;
}

template <typename real>
__global__ __launch_bounds__(THREADS) void k_rowfwd(const int* __restrict__ list, const SlotPtr<real>* __restrict__ ptrs,
                                                    const SlotParam* __restrict__ prms, const CtrlArgs A,
                                                    const cplx<real>* __restrict__ twx, double* __restrict__ part,
                                                    int nx, int ny, int R, int ngr, KTime* kt) {
  kt_begin(kt);
  k_rowfwd_body<real>(list, ptrs, prms, A, twx, part, nx, ny, R, ngr);
  kt_end(kt);
}

template <typename real>
__global__ __launch_bounds__(THREADS) void k_col(const int* __restrict__ list, const SlotPtr<real>* __restrict__ ptrs,
                                                 const SlotParam* __restrict__ prms,
                                                 const SlotCtl* __restrict__ ctls,
                                                 const cplx<real>* __restrict__ twy, double* __restrict__ part,
                                                 int nx, int ny, int W, int ngc, int nyq_free, const ColTimers T) {
  if (col_timer_group(T)) return;
  kt_begin(T.kt);
  k_col_body<real>(list, ptrs, prms, ctls, twy, part, nx, ny, W, ngc, nyq_free);
  kt_end(T.kt);
}

template <typename real, int N, int E>
__global__ __launch_bounds__(THREADS) void k_colr(const int* __restrict__ list, const SlotPtr<real>* __restrict__ ptrs,
                                                  const SlotParam* __restrict__ prms,
                                                  const SlotCtl* __restrict__ ctls,
                                                  const cplx<real>* __restrict__ twy, double* __restrict__ part,
                                                  int nx, int ngc, int nyq_free, const ColTimers T) {
  if (col_timer_group(T)) return;
  kt_begin(T.kt);
  k_colr_body<real, N, E>(list, ptrs, prms, ctls, twy, part, nx, ngc, nyq_free);
  kt_end(T.kt);
}

template <typename real, int M, int E>
__global__ __launch_bounds__(THREADS) void k_rowfwdr(const int* __restrict__ list,
                                                     const SlotPtr<real>* __restrict__ ptrs,
                                                     const SlotParam* __restrict__ prms, const CtrlArgs A,
                                                     const cplx<real>* __restrict__ twx, double* __restrict__ part,
                                                     int ny, int ngr, KTime* kt) {
  kt_begin(kt);
  k_rowfwdr_body<real, M, E>(list, ptrs, prms, A, twx, part, ny, ngr);
  kt_end(kt);
}

template <typename real, int M, int E>
__global__ __launch_bounds__(THREADS) void k_rowinvr(const int* __restrict__ list,
                                                     const SlotPtr<real>* __restrict__ ptrs,
                                                     const SlotParam* __restrict__ prms,
                                                     const SlotCtl* __restrict__ ctls,
                                                     const cplx<real>* __restrict__ twx,
                                                     const double* __restrict__ part_row, double* __restrict__ part,
                                                     int ny, int ngr, KTime* kt) {
  kt_begin(kt);
  k_rowinvr_body<real, M, E>(list, ptrs, prms, ctls, twx, part_row, part, ny, ngr);
  kt_end(kt);
}

template <typename real>
__global__ __launch_bounds__(THREADS) void k_rowinv(const int* __restrict__ list, const SlotPtr<real>* __restrict__ ptrs,
                                                    const SlotParam* __restrict__ prms,
                                                    const SlotCtl* __restrict__ ctls,
                                                    const cplx<real>* __restrict__ twx,
                                                    const double* __restrict__ part_row,
                                                    double* __restrict__ part, int nx, int ny, int R, int ngr,
                                                    KTime* kt) {
  kt_begin(kt);
  k_rowinv_body<real>(list, ptrs, prms, ctls, twx, part_row, part, nx, ny, R, ngr);
  kt_end(kt);
}

// Closing kernel of a block of ticks: the controller step of the last tick,
// one work-group per listed slot, from A.ctl_in into A.ctl_out (buffer 0,
// possibly the same block), so that the host reads every slot's current
// block in buffer 0.  With timers on, the second wavefront of group 0 folds
// the last tick's kernel times meanwhile.
template <typename real>
__global__ __launch_bounds__(128) void k_close(const int* __restrict__ list, const SlotPtr<real>* __restrict__ ptrs,
                                              const SlotParam* __restrict__ prms, const CtrlArgs A, int nx, int ny,
                                              int ngr, KTime* kt_last, unsigned long long* __restrict__ ktsum) {
  constexpr int NW = (int)(sizeof(SlotCtl) / sizeof(int));
  __shared__ SlotCtl lc;
  const unsigned long long t_close = wall_clock64();
  const int s = list[blockIdx.x];
  int* w = reinterpret_cast<int*>(&lc);
  if (s >= 0) {
    const int* src = reinterpret_cast<const int*>(A.ctl_in + s);
    for (int i = threadIdx.x; i < NW; i += blockDim.x) w[i] = src[i];
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    if (s >= 0) {
      if (lc.pending)
        ctrl_slot<real>(s, ptrs, prms, lc, true, A.prow, A.pcol, A.pinv, A.prof, A.seqs, A.recs, nx, ny, ngr,
                        A.ngc);
      if (threadIdx.x == 0) lc.pending = 0;
    }
  } else if (kt_last && blockIdx.x == 0) {
    kt_fold(kt_last, t_close, ktsum);
  }
  __syncthreads();
  if (s >= 0) {
    int* out = reinterpret_cast<int*>(A.ctl_out + s);
    for (int i = threadIdx.x; i < NW; i += blockDim.x) out[i] = w[i];
  }
}

// ===========================================================================
// Small utility kernels
// ===========================================================================
// Count non-finite or non-positive entries (E validation).
template <typename real>
__global__ void k_validate(const real* __restrict__ a, size_t n, real lo_excl, real lo_incl, real hi_incl,
                           unsigned int* __restrict__ bad) {
  unsigned int cnt = 0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const real v = a[i];
    const bool ok = isfinite(v) && v > lo_excl && v >= lo_incl && v <= hi_incl;
    cnt += ok ? 0u : 1u;
  }
  if (cnt) atomicAdd(bad, cnt);
}

// Pointwise output fields of one slot (see SPFF_FIELD_*).
template <typename real>
__global__ void k_fields(const SlotPtr<real>* __restrict__ ptrs, const SlotParam* __restrict__ prms,
                         const SlotCtl* __restrict__ ctls, int slot, int n, real* __restrict__ strain,
                         real* __restrict__ stress_out, real* __restrict__ psi_out) {
  const SlotPtr<real> F = ptrs[slot];
  const SlotParam& P = prms[slot];
  const SlotCtl& C = ctls[slot];
  const real lt = real(P.lam_t), mt = real(P.mu_t), kres = real(P.k_res);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const Sym<real> e = {real(C.eps_bar[0]) + F.eps[i], real(C.eps_bar[1]) + F.eps[n + i],
                         real(C.eps_bar[2]) + F.eps[2 * n + i]};
    const real E = F.E[i], ph = F.phi[i];
    const real lam = lt * E, mu = mt * E, hk = (real(1) - ph) * (real(1) - ph) + kres;
    if (strain) {
      strain[i] = e.xx;
      strain[n + i] = e.yy;
      strain[2 * n + i] = e.xy;
    }
    if (stress_out) {
      const Sym<real> sg = stress(e, lam, mu, hk, P.contact);
      stress_out[i] = sg.xx;
      stress_out[n + i] = sg.yy;
      stress_out[2 * n + i] = sg.xy;
    }
    if (psi_out) {
      real pp, pm;
      energies(e, lam, mu, P.split, &pp, &pm);
      psi_out[i] = pp;
    }
  }
}

// ===========================================================================
// Host-side launchers (called from the C-ABI implementation).
// ===========================================================================

template <typename real>
hipError_t launch_tick(const LaunchGeom& G, const TickBufs<real>& B, int i, hipStream_t st) {
  // tick i reads control block (i & 1) and the partials of tick i - 1
  // (row partials double-buffered: this tick's row-forward kernel writes the
  // other half while its groups reduce the previous one)
  const int cur = i & 1, nxt = cur ^ 1;
  CtrlArgs A;
  A.ctl_in = B.ctl[cur];
  A.ctl_out = B.ctl[nxt];
  A.prow = B.prow[nxt];
  A.pcol = B.pcol;
  A.pinv = B.pinv;
  A.prof = B.prof;
  A.seqs = B.seqs;
  A.recs = B.recs;
  A.ngc = G.ngc;
  const int* list = B.list;
  const SlotPtr<real>* ptrs = B.ptrs;
  const SlotParam* prms = B.prms;
  const SlotCtl* ctls = B.ctl[nxt];
  const auto* twx = B.twx;
  const auto* twy = B.twy;
  double* prow = B.prow[cur];
  double* pcol = B.pcol;
  double* pinv = B.pinv;
  KTime* ktset = B.kt ? B.kt + 3 * cur : nullptr;
  KTime* ktf = ktset;
  KTime* kti = ktset ? ktset + 2 : nullptr;
  ColTimers T;
  T.kt = ktset ? ktset + 1 : nullptr;
  T.kt_prev = (B.kt && i > 0) ? B.kt + 3 * nxt : nullptr;
  T.kt_row = ktf;
  T.ktsum = B.ktsum;
  dim3 grow(G.ngr, G.S), gcol(G.ngc, G.S + (B.kt ? 1 : 0));
  bool row_done = false;
  if constexpr (std::is_same<real, float>::value) {
    if (G.row_reg) {
      row_done = true;
#define SPFF_ROWS_FWD(MM, EE)                                                                                   \
  hipLaunchKernelGGL((k_rowfwdr<real, MM, EE>), grow, dim3(G.threads), G.lds_row, st, list, ptrs, prms, A, twx, \
                     prow, G.ny, G.ngr, ktf)
      if (G.row_reg == 2) {
        switch (G.nx) {
          case 128: SPFF_ROWS_FWD(64, 4); break;
          case 256: SPFF_ROWS_FWD(128, 4); break;
          default: SPFF_ROWS_FWD(256, 4); break;
        }
      } else {
        switch (G.nx) {
          case 128: SPFF_ROWS_FWD(64, 8); break;
          case 256: SPFF_ROWS_FWD(128, 8); break;
          case 512: SPFF_ROWS_FWD(256, 8); break;
          case 1024: SPFF_ROWS_FWD(512, 8); break;
          default: SPFF_ROWS_FWD(1024, 16); break;
        }
      }
#undef SPFF_ROWS_FWD
    }
  }
  if (!row_done)
    hipLaunchKernelGGL(k_rowfwd<real>, grow, dim3(G.threads), G.lds_row, st, list, ptrs, prms, A, twx, prow,
                       G.nx, G.ny, G.R, G.ngr, ktf);
  bool col_done = false;
  if constexpr (std::is_same<real, float>::value) {
    if (G.col_reg) {
      col_done = true;
#define SPFF_COLS(NN, EE)                                                                                           \
  hipLaunchKernelGGL((k_colr<real, NN, EE>), gcol, dim3(G.threads_col), G.lds_col, st, list, ptrs, prms, ctls, twy, \
                     pcol, G.nx, G.ngc, G.nyq_free, T)
      switch (G.ny) {
        case 128: SPFF_COLS(128, 8); break;
        case 256: SPFF_COLS(256, 8); break;
        case 512: SPFF_COLS(512, 8); break;
        case 1024:
          if (G.col_pts == 8) {
            SPFF_COLS(1024, 8);
          } else {
            SPFF_COLS(1024, 16);
          }
          break;
        default:
          if (G.col_pts == 8) {
            SPFF_COLS(2048, 8);
          } else {
            SPFF_COLS(2048, 16);
          }
          break;
      }
#undef SPFF_COLS
    }
  }
  if (!col_done)
    hipLaunchKernelGGL(k_col<real>, gcol, dim3(G.threads_col), G.lds_col, st, list, ptrs, prms, ctls, twy, pcol,
                       G.nx, G.ny, G.W, G.ngc, G.nyq_free, T);
  if (row_done) {
    if constexpr (std::is_same<real, float>::value) {
#define SPFF_ROWS_INV(MM, EE)                                                                                   \
  hipLaunchKernelGGL((k_rowinvr<real, MM, EE>), grow, dim3(G.threads), G.lds_row, st, list, ptrs, prms, ctls, twx, \
                     prow, pinv, G.ny, G.ngr, kti)
      if (G.row_reg == 2) {
        switch (G.nx) {
          case 128: SPFF_ROWS_INV(64, 4); break;
          case 256: SPFF_ROWS_INV(128, 4); break;
          default: SPFF_ROWS_INV(256, 4); break;
        }
      } else {
        switch (G.nx) {
          case 128: SPFF_ROWS_INV(64, 8); break;
          case 256: SPFF_ROWS_INV(128, 8); break;
          case 512: SPFF_ROWS_INV(256, 8); break;
          case 1024: SPFF_ROWS_INV(512, 8); break;
          default: SPFF_ROWS_INV(1024, 16); break;
        }
      }
#undef SPFF_ROWS_INV
    }
  } else {
    hipLaunchKernelGGL(k_rowinv<real>, grow, dim3(G.threads), G.lds_row, st, list, ptrs, prms, ctls, twx, prow,
                       pinv, G.nx, G.ny, G.R, G.ngr, kti);
  }
  return hipGetLastError();
}

template <typename real>
hipError_t launch_close(const LaunchGeom& G, const TickBufs<real>& B, int k, hipStream_t st) {
  // after ticks 0..k-1 the latest control blocks are in buffer (k & 1)
  const int last = (k - 1) & 1;
  CtrlArgs A;
  A.ctl_in = B.ctl[k & 1];
  A.ctl_out = B.ctl[0];
  A.prow = B.prow[last];
  A.pcol = B.pcol;
  A.pinv = B.pinv;
  A.prof = B.prof;
  A.seqs = B.seqs;
  A.recs = B.recs;
  A.ngc = G.ngc;
  hipLaunchKernelGGL(k_close<real>, dim3(G.S), dim3(128), 0, st, B.list, B.ptrs, B.prms, A, G.nx, G.ny, G.ngr,
                     B.kt ? B.kt + 3 * last : nullptr, B.ktsum);
  return hipGetLastError();
}

template <typename real>
hipError_t launch_validate(const real* a, size_t n, double lo_excl, double lo_incl, double hi_incl,
                           unsigned int* bad, hipStream_t st) {
  int blocks = (int)((n + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_validate<real>, dim3(blocks), dim3(256), 0, st, a, n, real(lo_excl), real(lo_incl),
                     real(hi_incl), bad);
  return hipGetLastError();
}

template <typename real>
hipError_t launch_fields(const SlotPtr<real>* ptrs, const SlotParam* prms, const SlotCtl* ctls, int slot, int n,
                         real* strain, real* stress_out, real* psi, hipStream_t st) {
  int blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fields<real>, dim3(blocks), dim3(256), 0, st, ptrs, prms, ctls, slot, n, strain,
                     stress_out, psi);
  return hipGetLastError();
}

template hipError_t launch_tick<float>(const LaunchGeom&, const TickBufs<float>&, int, hipStream_t);
template hipError_t launch_tick<double>(const LaunchGeom&, const TickBufs<double>&, int, hipStream_t);
template hipError_t launch_close<float>(const LaunchGeom&, const TickBufs<float>&, int, hipStream_t);
template hipError_t launch_close<double>(const LaunchGeom&, const TickBufs<double>&, int, hipStream_t);
template hipError_t launch_validate<float>(const float*, size_t, double, double, double, unsigned int*,
                                           hipStream_t);
template hipError_t launch_validate<double>(const double*, size_t, double, double, double, unsigned int*,
                                            hipStream_t);
template hipError_t launch_fields<float>(const SlotPtr<float>*, const SlotParam*, const SlotCtl*, int, int,
                                         float*, float*, float*, hipStream_t);
template hipError_t launch_fields<double>(const SlotPtr<double>*, const SlotParam*, const SlotCtl*, int, int,
                                          double*, double*, double*, hipStream_t);


// ===========================================================================
// Library-owned scratch of the allocation-free entry point
// (spff_load_step_static): one array per device, held until the process
// ends, shared by every call on that device.  In host code the array's name
// is not a device address; static_scratch() returns the address of the
// current device's copy, taken once per device with that device current.
// ===========================================================================
static __device__ __align__(256) unsigned char scratch[SPFF_STATIC_SCRATCH_BYTES];

hipError_t static_scratch(void** out) {
  constexpr int MAX_DEVICES = 64;
  static std::mutex mu;
  static void* addr[MAX_DEVICES] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = ptr;
  }
  *out = addr[dev];
  return hipSuccess;
}

}  // namespace spff
