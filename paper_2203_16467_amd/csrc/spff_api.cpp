// C-ABI implementation: validation, workspace layout, FFT tables, the tick
// loop and result readback.  See include/spff.h for the contract.
#include "spff.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <unordered_map>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "spff_engine.hpp"
#include "spff_launch.hpp"

using namespace spff;

namespace {

thread_local std::string g_last_error;

spff_status fail(spff_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(SPFF_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));       \
  } while (0)

constexpr size_t ALIGN = 256;
constexpr int THREADS = 256;
constexpr int MAXE = 8;
constexpr int PAD = 1;
constexpr size_t LDS_TARGET = 60 * 1024;
constexpr size_t LDS_MAX = 150 * 1024;

inline size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }
inline bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

struct Layout {
  // ctl: two control blocks per slot (ticks alternate; the host uses the
  // first); prow: two halves of row-forward partials (ticks alternate)
  size_t ctl, prm, ptr, twx, twy, prow, prow1, pcol, pinv, list, bad, prof, seq, rec, kt, ktsum;
  size_t slot0, slot_bytes;
  // offsets inside a slot
  size_t E, phi, phi_ref, eps, theta, rm, pm, spec;
  size_t total;
};

spff_status check_config(const spff_config* c) {
  if (!c) return fail(SPFF_E_INVALID, "config is NULL");
  if (!pow2(c->nx) || !pow2(c->ny) || c->nx < 8 || c->ny < 8 || c->nx > 2048 || c->ny > 2048)
    return fail(SPFF_E_INVALID, "nx, ny must be powers of two in [8, 2048] (got %d x %d)", c->nx, c->ny);
  if (!(c->nu > -1.0 && c->nu < 0.5)) return fail(SPFF_E_INVALID, "nu must lie in (-1, 0.5)");
  if (!(c->ell > 0.0) || !std::isfinite(c->ell)) return fail(SPFF_E_INVALID, "ell must be > 0");
  if (!(c->gc > 0.0) || !std::isfinite(c->gc)) return fail(SPFF_E_INVALID, "gc must be > 0");
  if (c->at != SPFF_AT1 && c->at != SPFF_AT2) return fail(SPFF_E_INVALID, "at must be 1 or 2");
  if (c->split != SPFF_SPLIT_NONE && c->split != SPFF_SPLIT_SPECTRAL && c->split != SPFF_SPLIT_VOLDEV)
    return fail(SPFF_E_INVALID, "bad split");
  if (c->contact != SPFF_CONTACT_SAME && c->contact != SPFF_SPLIT_NONE && c->contact != SPFF_SPLIT_SPECTRAL &&
      c->contact != SPFF_SPLIT_VOLDEV)
    return fail(SPFF_E_INVALID, "bad contact model");
  if (c->nyquist != SPFF_NYQ_ZERO && c->nyquist != SPFF_NYQ_FREE) return fail(SPFF_E_INVALID, "bad nyquist");
  if (c->evolution != SPFF_EVOL_AM && c->evolution != SPFF_EVOL_TIME && c->evolution != SPFF_EVOL_NEAR_EQ)
    return fail(SPFF_E_INVALID, "bad evolution");
  if (c->evolution == SPFF_EVOL_NEAR_EQ &&
      (!(c->eta >= 0.0) || !(c->dt_max > 0.0) || !std::isfinite(c->dt_max) || !(c->dphi_min >= 0.0) ||
       !(c->fphi_max > 0.0) || !std::isfinite(c->fphi_max) || !(c->drive_threshold >= 0.0) ||
       !(c->deps_max >= 0.0)))
    return fail(SPFF_E_INVALID, "near-equilibrium evolution needs eta >= 0, dt_max > 0, dphi_min >= 0, "
                                "fphi_max > 0, drive_threshold >= 0, deps_max >= 0");
  if (c->evolution == SPFF_EVOL_TIME &&
      (!(c->eta >= 0.0) || !(c->dt_min > 0.0) || !(c->dt_max >= c->dt_min) || !std::isfinite(c->dt_max) ||
       !(c->dphi_max > 0.0) || !(c->dphi_min >= 0.0)))
    return fail(SPFF_E_INVALID, "time-discretized evolution needs eta >= 0, 0 < dt_min <= dt_max, dphi_max > 0, "
                                "dphi_min >= 0");
  if (c->irreversibility != SPFF_IRR_CRACK_SET && c->irreversibility != SPFF_IRR_DAMAGE)
    return fail(SPFF_E_INVALID, "bad irreversibility");
  if (c->precision != SPFF_FP32 && c->precision != SPFF_FP64) return fail(SPFF_E_INVALID, "bad precision");
  if (!(c->k_res >= 0.0) || !(c->eta_over_dt >= 0.0)) return fail(SPFF_E_INVALID, "k_res, eta_over_dt >= 0");
  if (!(c->tol_mech >= 0.0) || !(c->tol_pf >= 0.0) || !(c->tol_abs_mech >= 0.0) || !(c->tol_abs_pf >= 0.0))
    return fail(SPFF_E_INVALID, "tolerances must be >= 0");
  if (c->max_cg < 1 || c->max_newton < 1 || c->max_bccg < 1 || c->max_am < 1)
    return fail(SPFF_E_INVALID, "iteration caps must be >= 1");
  if (c->ticks_per_sync < 1 || c->ticks_per_sync > 4096) return fail(SPFF_E_INVALID, "ticks_per_sync in [1, 4096]");
  if (!(c->floor_factor >= 0.0) || c->stall_iters < 0) return fail(SPFF_E_INVALID, "floor_factor, stall_iters >= 0");
  if (c->plan_rows < 0 || (c->plan_rows > 0 && (!pow2(c->plan_rows) || c->plan_rows > c->ny)))
    return fail(SPFF_E_INVALID, "plan_rows must be 0 or a power of two <= ny");
  if (c->plan_cols < 0 || (c->plan_cols > 0 && (!pow2(c->plan_cols) || c->plan_cols > c->nx / 2)))
    return fail(SPFF_E_INVALID, "plan_cols must be 0 or a power of two <= nx/2");
  if (c->plan_threads != 0 && c->plan_threads != 64 && c->plan_threads != 128 && c->plan_threads != 256)
    return fail(SPFF_E_INVALID, "plan_threads must be 0, 64, 128 or 256");
  {
    const int T = c->plan_threads > 0 ? c->plan_threads : THREADS;
    if (T * MAXE < c->nx / 2 || T * MAXE < c->ny)
      return fail(SPFF_E_INVALID, "plan_threads * 8 must cover nx/2 and ny");
  }
  return SPFF_OK;
}

// ---------------------------------------------------------------------------
// Launch plans.  A plan fixes, for one bucket of active problems, the kind
// of FFT kernel for rows and for columns (LDS Stockham radix-4/2 with one
// point pair per thread, or register-resident radix-8 with 8 points per
// lane), the rows / columns per work-group and the threads per work-group.
// auto_plan() is the built-in heuristic; the autotuner replaces it per
// bucket through spff_set_plan().
// ---------------------------------------------------------------------------
bool reg_rows_ok(const spff_config* c, int kind = SPFF_FFT_REG) {
  const int M = c->nx / 2;
  return c->precision == SPFF_FP32 && M >= 64 && M <= (kind == SPFF_FFT_REG4 ? 256 : 1024);
}
bool reg_cols_ok(const spff_config* c) {
  return c->precision == SPFF_FP32 &&
         (c->ny == 128 || c->ny == 256 || c->ny == 512 || c->ny == 1024 || c->ny == 2048);
}
// points per lane of the register kinds: 8 up to 512-point transforms, 16
// for 1024 and 2048 (a 2048-point row is 1024 complex points: 64 lanes);
// REG4 rows: 4
int reg_points(int n) { return n > 512 ? 16 : 8; }
// Register columns of 1024 or 2048 points take 8 points per lane (ny/8
// lanes: two or four wavefronts, one column per work-group) when a plan has
// cols = 1 and col_threads = ny/8 (the built-in plans); otherwise 16.
int reg_col_lanes(const spff_config* c, const spff_plan& pl) {
  if (c->ny >= 1024 && pl.cols == 1 && pl.col_threads == c->ny / 8) return c->ny / 8;
  return c->ny / reg_points(c->ny);
}
// columns per work-group of the register column kind: at least one
// wavefront, at most THREADS lanes; a column wider than a wavefront alone
int reg_cols_min(int Lc) { return Lc >= 64 ? 1 : 64 / Lc; }
int reg_cols_max(int Lc) { return Lc > 64 ? 1 : THREADS / Lc; }

spff_plan auto_plan(const spff_config* c, int S, size_t csize) {
  spff_plan pl{};
  const int M = c->nx / 2;
  // at least ~TARGET_WG work-groups per launch when the batch allows it
  const long TARGET_WG = 1024;
  int R = 1;
  while (R * 2 <= c->ny && 3 * (size_t)(2 * R) * (M + PAD) * csize <= LDS_TARGET &&
         (long)(c->ny / (2 * R)) * S >= TARGET_WG)
    R *= 2;
  int W = 1;
  while (W * 2 <= M && 3 * (size_t)(2 * W) * (c->ny + PAD) * csize <= LDS_TARGET &&
         (long)(M / (2 * W)) * S >= TARGET_WG)
    W *= 2;
  if (c->plan_rows > 0) R = c->plan_rows;
  if (c->plan_cols > 0) W = c->plan_cols;
  const int T = c->plan_threads > 0 ? c->plan_threads : THREADS;
  pl.row_kind = SPFF_FFT_LDS;
  pl.rows = R;
  pl.row_threads = T;
  pl.col_kind = SPFF_FFT_LDS;
  pl.cols = W;
  pl.col_threads = T;
  // FP32 columns of 128..2048 points: register-resident transforms, a group
  // of ny/8 lanes per column (8 points per lane), W columns per work-group
  // (at least one wavefront, at most THREADS lanes); W is fixed by plan_cols
  // if given so that the partial sums (hence the results) do not depend on
  // the batch.  1024- and 2048-point columns take one column per group (the
  // 16-point form of their lanes holds one wavefront per SIMD in registers);
  // plan_cols > 1 asks a 1024-point column for that form, 16 points per lane
  // with up to four columns per group.
  if (reg_cols_ok(c)) {
    const bool wide = c->ny == 2048 || (c->ny == 1024 && c->plan_cols <= 1);
    const int Lc = wide ? c->ny / 8 : c->ny / reg_points(c->ny);
    const int wmin = reg_cols_min(Lc), wmax = reg_cols_max(Lc);
    if (wmin <= M) {
      int Wr = wmin;
      if (c->plan_cols > 0) {
        Wr = std::max(wmin, std::min(wmax, c->plan_cols));
      } else {
        while (Wr * 2 <= wmax && Wr * 2 <= M && (long)(M / (2 * Wr)) * S >= TARGET_WG) Wr *= 2;
      }
      if (Wr <= M) {
        pl.col_kind = SPFF_FFT_REG;
        pl.cols = Wr;
        pl.col_threads = Wr * Lc;
      }
    }
  }
  // FP32 rows of 64..1024 complex points (nx = 128..2048): register-resident
  // transforms, a group of nx/16 (nx/32 for 2048) lanes per row, R rows per work-group (at
  // least one wavefront, at most THREADS lanes); R fixed by plan_rows if
  // given.  A lane walks 8 pixel pairs of its row one after the other, so
  // the path needs enough wavefronts in flight to hide that: below ~8 per
  // CU (a few problems of a small grid) the LDS row kernels, whose threads
  // take one pixel pair each, finish sooner.
  const bool many_waves = (long)S * c->ny * (M / 8) / 64 >= 2048;
  if (reg_rows_ok(c) && (many_waves || c->plan_rows > 0)) {
    const int Lr = M / reg_points(M);
    const int rmin = std::max(1, 64 / Lr), rmax = THREADS / Lr;
    if (rmin <= c->ny) {
      int Rr = rmin;
      if (c->plan_rows > 0) {
        Rr = std::max(rmin, std::min(rmax, c->plan_rows));
      } else {
        while (Rr * 2 <= rmax && Rr * 2 <= c->ny && (long)(c->ny / (2 * Rr)) * S >= TARGET_WG) Rr *= 2;
      }
      if (Rr <= c->ny) {
        pl.row_kind = SPFF_FFT_REG;
        pl.rows = Rr;
        pl.row_threads = Rr * Lr;
      }
    }
  } else if (reg_rows_ok(c, SPFF_FFT_REG4) && c->plan_rows == 0) {
    // few wavefronts: 4 points per lane (twice the lanes per row) hides the
    // per-lane latency better than either 8 points per lane or the LDS path
    const int Lr = M / 4;
    const int Rr = std::max(1, 64 / Lr);
    if (Rr <= c->ny) {
      pl.row_kind = SPFF_FFT_REG4;
      pl.rows = Rr;
      pl.row_threads = Rr * Lr;
    }
  }
  return pl;
}

// Validate a plan for a configuration; fills the derived thread counts of
// the register kinds.
spff_status check_plan(const spff_config* c, spff_plan* pl, size_t csize) {
  const int M = c->nx / 2;
  if (pl->row_kind == SPFF_FFT_REG || pl->row_kind == SPFF_FFT_REG4) {
    if (!reg_rows_ok(c, pl->row_kind))
      return fail(SPFF_E_INVALID, "register row FFT needs FP32 and 128 <= nx <= 2048 (512 with 4 points per lane)");
    const int Lr = M / (pl->row_kind == SPFF_FFT_REG4 ? 4 : reg_points(M));
    if (!pow2(pl->rows) || pl->rows * Lr < 64 || pl->rows * Lr > THREADS || pl->rows > c->ny)
      return fail(SPFF_E_INVALID, "register row FFT: rows * lanes per row must be a power of two in [64, %d]",
                  THREADS);
    pl->row_threads = pl->rows * Lr;
  } else if (pl->row_kind == SPFF_FFT_LDS) {
    if (!pow2(pl->rows) || pl->rows > c->ny) return fail(SPFF_E_INVALID, "rows must be a power of two <= ny");
    if (pl->row_threads != 64 && pl->row_threads != 128 && pl->row_threads != 256)
      return fail(SPFF_E_INVALID, "row_threads must be 64, 128 or 256");
    if (pl->row_threads * MAXE < M) return fail(SPFF_E_INVALID, "row_threads * 8 must cover nx/2");
    if (3 * (size_t)pl->rows * (M + PAD) * csize > LDS_MAX) return fail(SPFF_E_INVALID, "row tile exceeds LDS");
  } else {
    return fail(SPFF_E_INVALID, "bad row_kind");
  }
  if (pl->col_kind == SPFF_FFT_REG) {
    if (!reg_cols_ok(c))
      return fail(SPFF_E_INVALID, "register column FFT needs FP32 and ny in {128, ..., 2048}");
    const int Lc = reg_col_lanes(c, *pl);
    if (!pow2(pl->cols) || pl->cols < reg_cols_min(Lc) || pl->cols > reg_cols_max(Lc) || pl->cols > M)
      return fail(SPFF_E_INVALID, "register column FFT: cols * lanes per column must be a power of two in [64, %d] "
                                  "(one column per work-group where a column spans several wavefronts)", THREADS);
    pl->col_threads = pl->cols * Lc;
  } else if (pl->col_kind == SPFF_FFT_LDS) {
    if (!pow2(pl->cols) || pl->cols > M) return fail(SPFF_E_INVALID, "cols must be a power of two <= nx/2");
    if (pl->col_threads != 64 && pl->col_threads != 128 && pl->col_threads != 256)
      return fail(SPFF_E_INVALID, "col_threads must be 64, 128 or 256");
    if (pl->col_threads * MAXE < c->ny) return fail(SPFF_E_INVALID, "col_threads * 8 must cover ny");
    if (3 * (size_t)pl->cols * (c->ny + PAD) * csize > LDS_MAX)
      return fail(SPFF_E_INVALID, "column tile exceeds LDS");
  } else {
    return fail(SPFF_E_INVALID, "bad col_kind");
  }
  return SPFF_OK;
}

LaunchGeom geom_from_plan(const spff_config* c, int S, size_t csize, const spff_plan& pl) {
  LaunchGeom G{};
  G.nx = c->nx;
  G.ny = c->ny;
  G.S = S;
  const int M = c->nx / 2;
  G.R = pl.rows;
  G.ngr = c->ny / pl.rows;
  G.threads = pl.row_threads;
  G.row_reg = pl.row_kind == SPFF_FFT_REG ? 1 : (pl.row_kind == SPFF_FFT_REG4 ? 2 : 0);
  G.lds_row = G.row_reg ? ((size_t)pl.rows * (M + M / 8) + (size_t)M * (pl.rows + 1)) * csize
                        : 3 * (size_t)pl.rows * (M + PAD) * csize;
  G.W = pl.cols;
  G.ngc = M / pl.cols;
  G.threads_col = pl.col_threads;
  G.col_reg = pl.col_kind == SPFF_FFT_REG;
  G.col_pts = G.col_reg ? c->ny / reg_col_lanes(c, pl) : 0;
  G.nyq_free = c->nyquist == SPFF_NYQ_FREE ? 1 : 0;
  G.lds_col = G.col_reg ? (size_t)pl.cols * (c->ny + c->ny / 8) * csize
                        : 3 * (size_t)pl.cols * (c->ny + PAD) * csize;
  return G;
}

// scratch_only: slots hold solver scratch only; the resident planes
// (E, phi, phi_ref, eps*) of the problem bound to a slot live elsewhere.
Layout layout(const spff_config* c, int S, size_t rsize, bool scratch_only = false) {
  Layout L{};
  const size_t n = (size_t)c->nx * c->ny;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  L.ctl = take(2 * sizeof(SlotCtl) * S);
  L.prm = take(sizeof(SlotParam) * S);
  L.ptr = take(sizeof(SlotPtr<double>) * S);
  L.twx = take(2 * rsize * c->nx);
  L.twy = take(2 * rsize * c->ny);
  // partial sums sized for the finest launch plan (one row / column per group)
  L.prow = take(sizeof(double) * S * c->ny * NP_ROW);
  L.prow1 = take(sizeof(double) * S * c->ny * NP_ROW);
  L.pcol = take(sizeof(double) * S * (c->nx / 2) * NP_COL);
  L.pinv = take(sizeof(double) * S * c->ny * NP_INV);
  L.list = take(sizeof(int32_t) * S);
  L.bad = take(64);
  L.prof = take(sizeof(double) * 3 * S);
  L.seq = take(sizeof(SlotSeq) * S);
  L.kt = take(sizeof(KTime) * 6);
  L.ktsum = take(sizeof(unsigned long long) * 8);
  L.rec = take(sizeof(StepRec) * SEQ_MAX * S);
  L.slot0 = off;
  size_t so = 0;
  auto stake = [&](size_t bytes) {
    size_t o = so;
    so = align_up(so + bytes);
    return o;
  };
  if (!scratch_only) {
    L.E = stake(rsize * n);
    L.phi = stake(rsize * n);
    L.phi_ref = stake(rsize * n);
    L.eps = stake(3 * rsize * n);
  }
  L.theta = stake(3 * rsize * n);
  L.rm = stake(3 * rsize * n);
  L.pm = stake(3 * rsize * n);
  L.spec = stake(3 * 2 * rsize * (size_t)(c->nx / 2) * c->ny);
  L.slot_bytes = so;
  L.total = L.slot0 + (size_t)S * so;
  return L;
}

}  // namespace

struct spff_problem {
  spff_config cfg;
  int S;
  size_t rsize;
  Layout L;
  unsigned char* ws;
  hipStream_t stream;
  hipStream_t cap_stream;
  // launch plans by number of active slots: bucket b covers up to
  // bucket_size[b] slots (powers of two, the last one = S)
  std::vector<int> bucket_size;
  std::vector<LaunchGeom> geoms;
  std::vector<spff_plan> plans;  // per bucket, geoms[i] derived from plans[i]
  std::vector<hipGraphExec_t> graphs;  // one captured tick block per bucket (lazy)
  int cur_bucket = -1;
  int32_t* host_list = nullptr;  // pinned staging of the device slot list
  std::vector<int32_t> cur_list;
  SlotCtl* host_ctl;  // pinned mirror
  std::vector<SlotParam> prm;
  std::vector<double> last_eps_bar;
  std::vector<int> last_advance;  // advance flag of each problem's last step (1 before the first)
  bool scratch_only = false;
  std::vector<SlotPtr<double>> host_ptrs;  // layout-identical for float and double
  // profiling
  bool prof_on = false;
  int64_t launches[4] = {0, 0, 0, 0};
  int64_t prof_ticks = 0;

  SlotCtl* d_ctl() const { return reinterpret_cast<SlotCtl*>(ws + L.ctl); }
  SlotParam* d_prm() const { return reinterpret_cast<SlotParam*>(ws + L.prm); }
  void* d_ptr() const { return ws + L.ptr; }
  double* d_prof() const { return reinterpret_cast<double*>(ws + L.prof); }
  int32_t* d_list() const { return reinterpret_cast<int32_t*>(ws + L.list); }
  SlotSeq* d_seq() const { return reinterpret_cast<SlotSeq*>(ws + L.seq); }
  StepRec* d_rec() const { return reinterpret_cast<StepRec*>(ws + L.rec); }
  KTime* d_kt() const { return reinterpret_cast<KTime*>(ws + L.kt); }
  unsigned long long* d_ktsum() const { return reinterpret_cast<unsigned long long*>(ws + L.ktsum); }
  double clock_khz = 0.0;
  unsigned char* slot(int s) const { return ws + L.slot0 + (size_t)s * L.slot_bytes; }
  size_t n() const { return (size_t)cfg.nx * cfg.ny; }
};

namespace {

template <typename real>
TickBufs<real> tick_bufs(const spff_problem* p) {
  using C = typename HostCplx<real>::type;
  TickBufs<real> B;
  B.list = p->d_list();
  B.ptrs = reinterpret_cast<const SlotPtr<real>*>(p->d_ptr());
  B.prms = p->d_prm();
  B.ctl[0] = p->d_ctl();
  B.ctl[1] = p->d_ctl() + p->S;
  B.twx = reinterpret_cast<const C*>(p->ws + p->L.twx);
  B.twy = reinterpret_cast<const C*>(p->ws + p->L.twy);
  B.prow[0] = reinterpret_cast<double*>(p->ws + p->L.prow);
  B.prow[1] = reinterpret_cast<double*>(p->ws + p->L.prow1);
  B.pcol = reinterpret_cast<double*>(p->ws + p->L.pcol);
  B.pinv = reinterpret_cast<double*>(p->ws + p->L.pinv);
  B.prof = p->prof_on ? p->d_prof() : nullptr;
  B.seqs = p->d_seq();
  B.recs = p->d_rec();
  B.kt = p->prof_on ? p->d_kt() : nullptr;
  B.ktsum = p->prof_on ? p->d_ktsum() : nullptr;
  return B;
}

// k ticks and the closing controller step (leaves the control blocks in
// the host-visible buffer)
template <typename real>
hipError_t enqueue_block(spff_problem* p, int k, hipStream_t st, int b) {
  const TickBufs<real> B = tick_bufs<real>(p);
  for (int i = 0; i < k; ++i) {
    hipError_t e = launch_tick<real>(p->geoms[b], B, i, st);
    if (e != hipSuccess) return e;
  }
  return launch_close<real>(p->geoms[b], B, k, st);
}

hipError_t enqueue_ticks(spff_problem* p, int k, hipStream_t st, int b) {
  return p->cfg.precision == SPFF_FP64 ? enqueue_block<double>(p, k, st, b) : enqueue_block<float>(p, k, st, b);
}

// After a synchronised block of k ticks: count the launches (the kernel
// times are accumulated on the device): k of each FFT kernel, one closing
// controller launch.
void collect_profile(spff_problem* p, int k) {
  if (!p->prof_on) return;
  for (int j = 0; j < 3; ++j) p->launches[j] += k;
  p->launches[3] += 1;
  p->prof_ticks += k;
}

spff_status build_graph(spff_problem* p, int b) {
  const int K = p->cfg.ticks_per_sync;
  if (p->graphs[b]) {
    HIP_TRY(hipGraphExecDestroy(p->graphs[b]));
    p->graphs[b] = nullptr;
  }
  if (!p->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
  HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = enqueue_ticks(p, K, p->cap_stream, b);
  hipGraph_t graph = nullptr;
  hipError_t e2 = hipStreamEndCapture(p->cap_stream, &graph);
  if (e != hipSuccess) return fail(SPFF_E_DEVICE, "tick capture failed: %s", hipGetErrorString(e));
  if (e2 != hipSuccess) return fail(SPFF_E_DEVICE, "end capture failed: %s", hipGetErrorString(e2));
  HIP_TRY(hipGraphInstantiate(&p->graphs[b], graph, nullptr, nullptr, 0));
  HIP_TRY(hipGraphDestroy(graph));
  return SPFF_OK;
}

void drop_graphs(spff_problem* p) {
  for (auto& g : p->graphs)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
}

// Upload the slot list for `b` (active slots, padded with -1) if it changed.
spff_status set_list(spff_problem* p, const std::vector<int32_t>& active, int b) {
  std::vector<int32_t> lst(active);
  lst.resize(p->bucket_size[b], -1);
  if (lst == p->cur_list) return SPFF_OK;
  // the previous upload was followed by a synchronisation, so the pinned
  // staging buffer is free
  std::copy(lst.begin(), lst.end(), p->host_list);
  HIP_TRY(hipMemcpyAsync(p->d_list(), p->host_list, sizeof(int32_t) * lst.size(), hipMemcpyHostToDevice,
                         p->stream));
  p->cur_list.swap(lst);
  return SPFF_OK;
}

int bucket_for(const spff_problem* p, int nactive) {
  int b = 0;
  while (p->bucket_size[b] < nactive) ++b;
  return b;
}

// Enqueue one block of ticks over the slots that are not idle (host mirror)
// with the launch plan of their count.  Returns SPFF_OK without launching
// when no slot is active.
spff_status launch_block(spff_problem* p, bool* launched, int* nticks) {
  std::vector<int32_t> active;
  for (int s = 0; s < p->S; ++s)
    if (p->host_ctl[s].phase != PH_IDLE) active.push_back(s);
  *launched = false;
  *nticks = 0;
  if (active.empty()) return SPFF_OK;
  const int b = bucket_for(p, (int)active.size());
  spff_status st = set_list(p, active, b);
  if (st != SPFF_OK) return st;
  const int K = p->cfg.ticks_per_sync;
  if (p->cfg.use_graph) {
    if (!p->graphs[b]) {
      st = build_graph(p, b);
      if (st != SPFF_OK) return st;
    }
    HIP_TRY(hipGraphLaunch(p->graphs[b], p->stream));
  } else {
    hipError_t e = enqueue_ticks(p, K, p->stream, b);
    if (e != hipSuccess) return fail(SPFF_E_DEVICE, "tick launch failed: %s", hipGetErrorString(e));
  }
  *launched = true;
  *nticks = K;
  return SPFF_OK;
}

// Run ticks until every slot is idle.
spff_status run_until_idle(spff_problem* p) {
  const size_t cbytes = sizeof(SlotCtl) * p->S;
  for (;;) {
    bool launched;
    int k;
    spff_status st = launch_block(p, &launched, &k);
    if (st != SPFF_OK) return st;
    if (!launched) break;
    HIP_TRY(hipMemcpyAsync(p->host_ctl, p->d_ctl(), cbytes, hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    collect_profile(p, k);
  }
  return SPFF_OK;
}

template <typename real>
void fill_twiddles(std::vector<unsigned char>& out, int n) {
  using C = typename HostCplx<real>::type;
  out.resize(sizeof(C) * n);
  C* t = reinterpret_cast<C*>(out.data());
  const double two_pi = 6.283185307179586476925286766559;
  for (int k = 0; k < n; ++k) {
    const double a = -two_pi * (double)k / (double)n;
    t[k].x = (real)std::cos(a);
    t[k].y = (real)std::sin(a);
  }
}

SlotParam make_param(const spff_config* c) {
  SlotParam P{};
  const double nu = c->nu;
  P.lam_t = nu / (1.0 - nu - 2.0 * nu * nu);  // Sec. 2.1, per unit E
  P.mu_t = 1.0 / (2.0 + 2.0 * nu);
  P.ell = c->ell;
  P.gc = c->gc;
  const double cw = c->at == SPFF_AT1 ? 8.0 / 3.0 : 2.0;
  P.cwl = c->gc / (cw * c->ell);
  P.kappa = 2.0 * c->gc * c->ell / cw;
  P.wpp = c->at == SPFF_AT1 ? 0.0 : 2.0;
  P.dw0 = c->at == SPFF_AT1 ? 1.0 : 0.0;
  P.eta_dt = c->eta_over_dt;
  P.k_res = c->k_res;
  P.threshold = c->crack_set_threshold;
  P.tol_mech = c->tol_mech;
  P.tol_abs_mech = c->tol_abs_mech;
  P.tol_pf = c->tol_pf;
  P.tol_abs_pf = c->tol_abs_pf;
  P.tol_am = c->tol_am < 0.0 ? 1e-3 * c->ell * c->ell : c->tol_am;
  const double u = c->precision == SPFF_FP64 ? 0x1p-53 : 0x1p-24;
  P.floor_coef = c->floor_factor * u * std::sqrt(std::log2((double)c->nx * (double)c->ny));
  // mean of |2 pi q|^2 over the grid's modes: rounding noise of the
  // transforms is spread evenly over the spectrum
  P.lap_rms = 4.0 * M_PI * M_PI / 6.0;
  P.stall_iters = c->stall_iters;
  P.at = c->at;
  P.split = c->split;
  P.contact = c->contact == SPFF_CONTACT_SAME ? c->split : c->contact;
  P.evolution = c->evolution;
  P.eta = c->eta;
  P.dt_max = c->dt_max;
  P.dt_min = c->dt_min;
  P.dphi_max = c->dphi_max;
  P.dphi_min = c->dphi_min;
  P.fphi_max = c->fphi_max;
  P.drive_thr = c->drive_threshold;
  P.deps_max = c->deps_max;
  P.irr = c->irreversibility;
  P.max_cg = c->max_cg;
  P.max_newton = c->max_newton;
  P.max_bccg = c->max_bccg;
  P.max_am = c->max_am;
  return P;
}

template <typename real>
spff_status init_device(spff_problem* p, const void* E_dev, const void* phi_init_dev) {
  const size_t n = p->n();
  const size_t rb = sizeof(real) * n;
  static_assert(sizeof(SlotPtr<real>) == sizeof(SlotPtr<double>), "pointer tables differ");
  p->host_ptrs.assign(p->S, SlotPtr<double>{});
  for (int s = 0; s < p->S; ++s) {
    unsigned char* b = p->slot(s);
    SlotPtr<real> e{};
    if (!p->scratch_only) {
      e.E = reinterpret_cast<const real*>(b + p->L.E);
      e.phi = reinterpret_cast<real*>(b + p->L.phi);
      e.phi_ref = reinterpret_cast<real*>(b + p->L.phi_ref);
      e.eps = reinterpret_cast<real*>(b + p->L.eps);
    }
    e.theta = reinterpret_cast<real*>(b + p->L.theta);
    e.rm = reinterpret_cast<real*>(b + p->L.rm);
    e.pm = reinterpret_cast<real*>(b + p->L.pm);
    e.spec = reinterpret_cast<void*>(b + p->L.spec);
    std::memcpy(&p->host_ptrs[s], &e, sizeof(e));
  }
  HIP_TRY(hipMemcpyAsync(p->d_ptr(), p->host_ptrs.data(), sizeof(SlotPtr<real>) * p->S, hipMemcpyHostToDevice,
                         p->stream));
  HIP_TRY(hipMemcpyAsync(p->d_prm(), p->prm.data(), sizeof(SlotParam) * p->S, hipMemcpyHostToDevice, p->stream));
  std::vector<unsigned char> tw;
  fill_twiddles<real>(tw, p->cfg.nx);
  HIP_TRY(hipMemcpyAsync(p->ws + p->L.twx, tw.data(), tw.size(), hipMemcpyHostToDevice, p->stream));
  fill_twiddles<real>(tw, p->cfg.ny);
  HIP_TRY(hipMemcpyAsync(p->ws + p->L.twy, tw.data(), tw.size(), hipMemcpyHostToDevice, p->stream));
  // the synchronous twiddle staging buffer is reused: wait for the copies
  HIP_TRY(hipStreamSynchronize(p->stream));

  HIP_TRY(hipMemsetAsync(p->d_seq(), 0, sizeof(SlotSeq) * p->S, p->stream));
  if (p->scratch_only) {
    for (int s = 0; s < p->S; ++s) {
      unsigned char* b = p->slot(s);
      HIP_TRY(hipMemsetAsync(b + p->L.theta, 0, 9 * rb, p->stream));
    }
    HIP_TRY(hipStreamSynchronize(p->stream));
    return SPFF_OK;
  }
  // inputs and zeroed state
  unsigned int* bad = reinterpret_cast<unsigned int*>(p->ws + p->L.bad);
  HIP_TRY(hipMemsetAsync(bad, 0, 2 * sizeof(unsigned int), p->stream));
  for (int s = 0; s < p->S; ++s) {
    unsigned char* b = p->slot(s);
    HIP_TRY(hipMemcpyAsync(b + p->L.E, static_cast<const unsigned char*>(E_dev) + s * rb, rb,
                           hipMemcpyDeviceToDevice, p->stream));
    HIP_TRY(hipMemsetAsync(b + p->L.eps, 0, 3 * rb, p->stream));
    HIP_TRY(hipMemsetAsync(b + p->L.theta, 0, 3 * rb, p->stream));
    HIP_TRY(hipMemsetAsync(b + p->L.rm, 0, 3 * rb, p->stream));
    HIP_TRY(hipMemsetAsync(b + p->L.pm, 0, 3 * rb, p->stream));
    if (phi_init_dev) {
      const unsigned char* src = static_cast<const unsigned char*>(phi_init_dev) + s * rb;
      HIP_TRY(hipMemcpyAsync(b + p->L.phi, src, rb, hipMemcpyDeviceToDevice, p->stream));
      HIP_TRY(hipMemcpyAsync(b + p->L.phi_ref, src, rb, hipMemcpyDeviceToDevice, p->stream));
    } else {
      HIP_TRY(hipMemsetAsync(b + p->L.phi, 0, rb, p->stream));
      HIP_TRY(hipMemsetAsync(b + p->L.phi_ref, 0, rb, p->stream));
    }
    HIP_TRY(launch_validate<real>(reinterpret_cast<const real*>(b + p->L.E), n, 0.0, -1e300, 1e300, bad,
                                  p->stream));
    if (phi_init_dev)
      HIP_TRY(launch_validate<real>(reinterpret_cast<const real*>(b + p->L.phi), n, -1e300, 0.0, 1.0, bad + 1,
                                    p->stream));
  }
  unsigned int hbad[2] = {0, 0};
  HIP_TRY(hipMemcpyAsync(hbad, bad, sizeof(hbad), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  if (hbad[0]) return fail(SPFF_E_INVALID, "E has %u non-positive or non-finite entries", hbad[0]);
  if (hbad[1]) return fail(SPFF_E_INVALID, "phi_init has %u entries outside [0, 1]", hbad[1]);
  return SPFF_OK;
}

void reset_ctl(spff_problem* p, int s) {
  SlotCtl& c = p->host_ctl[s];
  std::memset(&c, 0, sizeof(SlotCtl));
}

spff_status slot_status(const SlotCtl& c) {
  if (c.status < 0) return (spff_status)c.status;
  if (c.flags & FL_NOT_CONVERGED) return SPFF_WARN_NOT_CONVERGED;
  return SPFF_OK;
}

void fill_stats(size_t npx, const SlotCtl& c, spff_step_stats& o, double wall_ms) {
  std::memset(&o, 0, sizeof(o));
  o.status = slot_status(c);
  o.am_iters = c.am;
  o.newton_iters = c.newton;
  o.cg_iters = c.cg;
  o.bccg_iters = c.bccg;
  o.ticks = c.ticks;
  o.dphi_l1 = c.dphi;
  o.mech_residual = c.mech_res;
  o.pf_residual = c.pf_res;
  o.F_e = c.F_e;
  o.F_f = c.F_f;
  o.dt = c.dt;
  o.halvings = c.halvings;
  o.advance = c.advance;
  o.gamma = c.gamma;
  o.fphi_max = c.fmax_ne;
  for (int k = 0; k < 3; ++k) o.eps_bar[k] = c.eps_bar[k];
  o.ne_flag = c.ne_flag;
  for (int k = 0; k < 3; ++k) o.sigma_bar[k] = c.sbar[k];
  int kmax = 0;
  for (int k = 1; k < 3; ++k)
    if (std::fabs(c.eps_bar[k]) > std::fabs(c.eps_bar[kmax])) kmax = k;
  o.C_bar = c.eps_bar[kmax] != 0.0 ? c.sbar[kmax] / c.eps_bar[kmax] : NAN;
  o.phi_max = c.phi_max;
  o.phi_mean = c.phi_sum / (double)npx;
  o.crack_px = (int64_t)std::llround(c.crack_px);
  o.wall_ms = wall_ms;
}

// Start a load step of slot s under configuration cfg (the handle's, or a
// served problem's).  The time step of the time-discretized evolution and
// the trigger flag of the near-equilibrium evolution carry over from the
// slot's control block (the server stores them per problem and restores
// them before each request).
void start_step(spff_problem* p, int s, const double* eb, const spff_config& cfg) {
  const double dt = p->host_ctl[s].dt > 0.0 ? p->host_ctl[s].dt : cfg.dt_max;
  const int ne_flag = p->host_ctl[s].ne_flag;
  reset_ctl(p, s);
  SlotCtl& c = p->host_ctl[s];
  for (int k = 0; k < 3; ++k) c.eps_bar[k] = eb[k];
  const int evol = cfg.evolution;
  c.phase = PH_M_RES;
  c.flags = FL_FIRST_OF_STEP | (evol == SPFF_EVOL_NEAR_EQ ? FL_NE_CHECK : 0);
  c.dt = dt;
  c.eta_dt = evol == SPFF_EVOL_TIME      ? cfg.eta / dt
             : evol == SPFF_EVOL_NEAR_EQ ? cfg.eta / cfg.dt_max
                                         : cfg.eta_over_dt;
  c.gamma = 1.0;
  c.ne_flag = ne_flag;
}

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// One diagnostic tick (PH_X_PROJ, PH_X_LAP or PH_X_DISP) over the slots
// `slots`: copies pin planes from src(s) into the slot's theta planes, runs
// the tick with the plan of the slot count's bucket, copies pout planes of
// rm to dst(s), and restores the control blocks (step statistics stay
// readable).  Every listed slot must be idle.
template <typename Src, typename Dst>
spff_status run_diag(spff_problem* p, int phase, const std::vector<int32_t>& slots, int pin, int pout, Src src,
                     Dst dst) {
  const size_t rb = p->rsize * p->n();
  for (int s : slots)
    if (p->host_ctl[s].phase != PH_IDLE) return fail(SPFF_E_BUSY, "slot %d is not idle", s);
  if (slots.empty()) return SPFF_OK;
  for (int s : slots)
    HIP_TRY(hipMemcpyAsync(p->slot(s) + p->L.theta, src(s), pin * rb, hipMemcpyDeviceToDevice, p->stream));
  std::vector<SlotCtl> saved(p->host_ctl, p->host_ctl + p->S);
  for (int s : slots) p->host_ctl[s].phase = phase;
  HIP_TRY(hipMemcpyAsync(p->d_ctl(), p->host_ctl, sizeof(SlotCtl) * p->S, hipMemcpyHostToDevice, p->stream));
  const int b = bucket_for(p, (int)slots.size());
  spff_status lst = set_list(p, slots, b);
  if (lst != SPFF_OK) return lst;
  const bool prof = p->prof_on;
  p->prof_on = false;
  hipError_t e = enqueue_ticks(p, 1, p->stream, b);
  p->prof_on = prof;
  if (e != hipSuccess) return fail(SPFF_E_DEVICE, "operator launch failed: %s", hipGetErrorString(e));
  for (int s : slots)
    HIP_TRY(hipMemcpyAsync(dst(s), p->slot(s) + p->L.rm, pout * rb, hipMemcpyDeviceToDevice, p->stream));
  // the pinned mirror is the source of the pending upload above: wait before
  // reusing it, then restore the control blocks
  HIP_TRY(hipStreamSynchronize(p->stream));
  std::copy(saved.begin(), saved.end(), p->host_ctl);
  HIP_TRY(hipMemcpyAsync(p->d_ctl(), p->host_ctl, sizeof(SlotCtl) * p->S, hipMemcpyHostToDevice, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  return SPFF_OK;
}

}  // namespace

extern "C" {

void spff_default_config(spff_config* c) {
  if (!c) return;
  std::memset(c, 0, sizeof(*c));
  c->nx = c->ny = 64;
  c->at = SPFF_AT1;
  c->split = SPFF_SPLIT_SPECTRAL;
  c->contact = SPFF_CONTACT_SAME;
  c->evolution = SPFF_EVOL_AM;
  c->eta = 0.0;
  c->dt_max = 1.0;
  c->dt_min = 1e-3;
  c->dphi_max = 1.0;
  c->dphi_min = 0.0;
  c->fphi_max = 0.35;        // 0.7 G_c / l at the default G_c = 1, l = 2
  c->drive_threshold = 0.5;  // 1 G_c / l
  c->deps_max = 0.0;
  c->nyquist = SPFF_NYQ_ZERO;
  c->irreversibility = SPFF_IRR_CRACK_SET;
  c->precision = SPFF_FP32;
  c->nu = 0.2;
  c->ell = 2.0;
  c->gc = 1.0;
  c->crack_set_threshold = 0.9;
  c->k_res = 0.0;
  c->eta_over_dt = 0.0;
  c->tol_mech = 1e-6;
  c->tol_abs_mech = 0.0;
  c->tol_pf = 1e-6;
  c->tol_abs_pf = 0.0;
  c->tol_am = -1.0;
  c->max_cg = 20000;
  c->max_newton = 50;
  c->max_bccg = 20000;
  c->max_am = 1000;
  c->ticks_per_sync = 1;
  c->use_graph = 0;
  c->floor_factor = 2.0;
  c->stall_iters = 200;
}

spff_status spff_workspace_bytes(const spff_config* cfg, int32_t nbatch, size_t* bytes) {
  spff_status st = check_config(cfg);
  if (st != SPFF_OK) return st;
  if (nbatch < 1) return fail(SPFF_E_INVALID, "nbatch must be >= 1");
  if (!bytes) return fail(SPFF_E_INVALID, "bytes is NULL");
  const size_t rsize = cfg->precision == SPFF_FP64 ? 8 : 4;
  *bytes = layout(cfg, nbatch, rsize).total;
  return SPFF_OK;
}

}  // extern "C"

namespace {

spff_status engine_create(const spff_config* cfg, int32_t nbatch, const void* E_dev, const void* phi_init_dev,
                          void* workspace, size_t workspace_bytes, void* stream, bool scratch_only,
                          spff_problem** out) {
  spff_status st = check_config(cfg);
  if (st != SPFF_OK) return st;
  if (!out) return fail(SPFF_E_INVALID, "out is NULL");
  *out = nullptr;
  if (nbatch < 1) return fail(SPFF_E_INVALID, "nbatch must be >= 1");
  if (!E_dev && !scratch_only) return fail(SPFF_E_INVALID, "E_dev is NULL");
  if (!workspace) return fail(SPFF_E_INVALID, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % ALIGN) return fail(SPFF_E_INVALID, "workspace must be 256-byte aligned");
  const size_t rsize = cfg->precision == SPFF_FP64 ? 8 : 4;
  std::vector<int> bsize;
  for (int v = 1;; v *= 2) {
    bsize.push_back(std::min(v, (int)nbatch));
    if (v >= nbatch) break;
  }
  std::vector<LaunchGeom> geoms;
  std::vector<spff_plan> plans;
  for (int v : bsize) {
    spff_plan pl = auto_plan(cfg, v, 2 * rsize);
    LaunchGeom G = geom_from_plan(cfg, v, 2 * rsize, pl);
    if (G.lds_row > LDS_MAX || G.lds_col > LDS_MAX) return fail(SPFF_E_INVALID, "grid too large for LDS tiles");
    geoms.push_back(G);
    plans.push_back(pl);
  }
  Layout L = layout(cfg, nbatch, rsize, scratch_only);
  if (workspace_bytes < L.total)
    return fail(SPFF_E_NOMEM, "workspace too small: %zu < %zu bytes", workspace_bytes, L.total);

  spff_problem* p = new spff_problem();
  p->scratch_only = scratch_only;
  p->cfg = *cfg;
  p->S = nbatch;
  p->rsize = rsize;
  p->L = L;
  p->ws = static_cast<unsigned char*>(workspace);
  p->stream = static_cast<hipStream_t>(stream);
  p->cap_stream = nullptr;
  p->bucket_size = bsize;
  p->geoms = geoms;
  p->plans = plans;
  p->graphs.assign(bsize.size(), nullptr);
  p->host_ctl = nullptr;
  p->prm.assign(nbatch, make_param(cfg));
  p->last_eps_bar.assign(3 * (size_t)nbatch, 0.0);
  p->last_advance.assign((size_t)nbatch, 1);
  auto cleanup = [&](spff_status s) {
    spff_destroy_problem(p);
    return s;
  };
  if (hipHostMalloc(reinterpret_cast<void**>(&p->host_ctl), sizeof(SlotCtl) * nbatch, hipHostMallocDefault) !=
          hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&p->host_list), sizeof(int32_t) * nbatch, hipHostMallocDefault) !=
          hipSuccess)
    return cleanup(fail(SPFF_E_DEVICE, "pinned host allocation failed"));
  for (int s = 0; s < nbatch; ++s) reset_ctl(p, s);
  st = cfg->precision == SPFF_FP64 ? init_device<double>(p, E_dev, phi_init_dev)
                                   : init_device<float>(p, E_dev, phi_init_dev);
  if (st != SPFF_OK) return cleanup(st);
  // control blocks: idle, or the zero-strain phase-field solve for phi_init
  for (int s = 0; s < nbatch; ++s) {
    reset_ctl(p, s);
    if (phi_init_dev) {
      p->host_ctl[s].phase = PH_PF_ASM;
      p->host_ctl[s].flags = FL_INIT_SOLVE;
    }
  }
  if (hipMemcpyAsync(p->d_ctl(), p->host_ctl, sizeof(SlotCtl) * nbatch, hipMemcpyHostToDevice, p->stream) !=
      hipSuccess)
    return cleanup(fail(SPFF_E_DEVICE, "control upload failed"));
  if (phi_init_dev) {
    st = run_until_idle(p);
    if (st != SPFF_OK) return cleanup(st);
  }
  if (hipStreamSynchronize(p->stream) != hipSuccess) return cleanup(fail(SPFF_E_DEVICE, "stream sync failed"));
  *out = p;
  return SPFF_OK;
}

}  // namespace

extern "C" {

spff_status spff_create_batch(const spff_config* cfg, int32_t nbatch, const void* E_dev, const void* phi_init_dev,
                              void* workspace, size_t workspace_bytes, void* stream, spff_problem** out) {
  return engine_create(cfg, nbatch, E_dev, phi_init_dev, workspace, workspace_bytes, stream, false, out);
}

spff_status spff_create_problem(const spff_config* cfg, const void* E_dev, const void* phi_init_dev,
                                void* workspace, size_t workspace_bytes, void* stream, spff_problem** out) {
  return spff_create_batch(cfg, 1, E_dev, phi_init_dev, workspace, workspace_bytes, stream, out);
}

static spff_status run_queue(spff_problem* p, int32_t nsteps, const double* eps_bar, spff_step_stats* stats,
                             bool incr);

spff_status spff_run_sequence(spff_problem* p, int32_t nsteps, const double* eps_bar, spff_step_stats* stats) {
  return run_queue(p, nsteps, eps_bar, stats, false);
}

spff_status spff_run_evolution(spff_problem* p, int32_t nsteps, const double* deps, spff_step_stats* stats) {
  if (p && p->cfg.evolution == SPFF_EVOL_AM)
    return fail(SPFF_E_INVALID, "spff_run_evolution needs SPFF_EVOL_TIME or SPFF_EVOL_NEAR_EQ; use spff_run_sequence");
  return run_queue(p, nsteps, deps, stats, true);
}

// Device step queues: per problem, steps at the given macroscopic strains
// (incr = false) or, for the time-discretized / near-equilibrium evolution,
// steps that continue from the previous step's final strain plus the given
// increment when that step advanced the load (incr = true).
static spff_status run_queue(spff_problem* p, int32_t nsteps, const double* eps_bar, spff_step_stats* stats,
                             bool incr) {
  if (!p) return fail(SPFF_E_INVALID, "problem is NULL");
  if (nsteps < 1) return fail(SPFF_E_INVALID, "nsteps must be >= 1");
  if (!eps_bar) return fail(SPFF_E_INVALID, "eps_bar is NULL");
  for (size_t i = 0; i < (size_t)3 * p->S * nsteps; ++i)
    if (!std::isfinite(eps_bar[i])) return fail(SPFF_E_INVALID, "eps_bar must be finite");
  const int S = p->S;
  if (p->clock_khz <= 0.0) {
    int dev = 0, khz = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    p->clock_khz = khz > 0 ? (double)khz : 1e5;
  }
  // Steps are handed to the device in chunks of at most SEQ_MAX per slot; the
  // controller chains the steps of a chunk on the device.
  std::vector<int> next(S, 0);      // first step of the slot's current chunk
  std::vector<int> clen(S, 0);      // length of the slot's current chunk
  std::vector<SlotSeq> q(1);
  std::vector<StepRec> rec(SEQ_MAX);
  auto upload_chunk = [&](int s) -> spff_status {
    const int len = std::min(SEQ_MAX, nsteps - next[s]);
    SlotSeq& h = q[0];
    h.len = len;
    h.pos = 0;
    h.incr = incr ? 1 : 0;
    for (int k = 0; k < len; ++k)
      for (int c = 0; c < 3; ++c) h.eps_bar[k][c] = eps_bar[3 * ((size_t)s * nsteps + next[s] + k) + c];
    HIP_TRY(hipMemcpyAsync(p->d_seq() + s, &h, sizeof(SlotSeq), hipMemcpyHostToDevice, p->stream));
    // the staging struct is reused for the next slot: wait for this copy
    HIP_TRY(hipStreamSynchronize(p->stream));
    clen[s] = len;
    double eb[3];
    for (int c = 0; c < 3; ++c)
      eb[c] = incr ? p->last_eps_bar[3 * s + c] + (p->last_advance[s] ? h.eps_bar[0][c] : 0.0) : h.eps_bar[0][c];
    start_step(p, s, eb, p->cfg);
    return SPFF_OK;
  };
  for (int s = 0; s < S; ++s) {
    spff_status st = upload_chunk(s);
    if (st != SPFF_OK) return st;
  }
  HIP_TRY(hipMemcpyAsync(p->d_ctl(), p->host_ctl, sizeof(SlotCtl) * S, hipMemcpyHostToDevice, p->stream));
  spff_status worst = SPFF_OK;
  int remaining = S;
  const size_t cbytes = sizeof(SlotCtl) * S;
  while (remaining > 0) {
    bool launched;
    int k;
    spff_status bst = launch_block(p, &launched, &k);
    if (bst != SPFF_OK) return bst;
    HIP_TRY(hipMemcpyAsync(p->host_ctl, p->d_ctl(), cbytes, hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    collect_profile(p, k);
    bool dirty = false;
    for (int s = 0; s < S; ++s) {
      if (clen[s] == 0 || p->host_ctl[s].phase != PH_IDLE) continue;
      // the slot's chunk has ended (all steps done, or a step failed)
      HIP_TRY(hipMemcpyAsync(rec.data(), p->d_rec() + (size_t)s * SEQ_MAX, sizeof(StepRec) * clen[s],
                             hipMemcpyDeviceToHost, p->stream));
      HIP_TRY(hipMemcpyAsync(&q[0], p->d_seq() + s, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, p->stream));
      HIP_TRY(hipStreamSynchronize(p->stream));
      const int done = q[0].pos;
      bool failed = done < clen[s];
      for (int j = 0; j < done; ++j) {
        const StepRec& r = rec[j];
        SlotCtl c{};
        c.am = r.am;
        c.newton = r.newton;
        c.cg = r.cg;
        c.bccg = r.bccg;
        c.ticks = r.ticks;
        c.status = r.status;
        c.dt = r.dt;
        c.halvings = r.halvings;
        c.advance = r.advance;
        c.gamma = r.gamma;
        c.fmax_ne = r.fmax_ne;
        c.ne_flag = r.ne_flag;
        c.flags = r.flags;
        c.dphi = r.dphi;
        c.mech_res = r.mech_res;
        c.pf_res = r.pf_res;
        c.F_e = r.F_e;
        c.F_f = r.F_f;
        for (int m = 0; m < 3; ++m) {
          c.sbar[m] = r.sbar[m];
          c.eps_bar[m] = r.eps_bar[m];
        }
        c.phi_sum = r.phi_sum;
        c.phi_max = r.phi_max;
        c.crack_px = r.crack_px;
        const spff_status ss = slot_status(c);
        if (ss < 0 && (worst >= 0 || ss < worst)) worst = ss;
        if (ss > 0 && worst == SPFF_OK) worst = ss;
        if (ss < 0) failed = true;
        const double ms = (double)(r.t_end - r.t_start) / p->clock_khz;
        if (stats) fill_stats(p->n(), c, stats[(size_t)s * nsteps + next[s] + j], ms);
        for (int m = 0; m < 3; ++m) p->last_eps_bar[3 * s + m] = r.eps_bar[m];
        p->last_advance[s] = r.advance;
      }
      if (done == 0 && p->host_ctl[s].status < 0) {
        // failed before its record was written
        const spff_status ss = (spff_status)p->host_ctl[s].status;
        if (worst >= 0 || ss < worst) worst = ss;
        failed = true;
      }
      next[s] += clen[s];
      clen[s] = 0;
      if (!failed && next[s] < nsteps) {
        spff_status st = upload_chunk(s);
        if (st != SPFF_OK) return st;
        dirty = true;
      } else {
        --remaining;
      }
    }
    // the device is idle here (synchronised), so the whole mirror is current
    if (dirty) HIP_TRY(hipMemcpyAsync(p->d_ctl(), p->host_ctl, cbytes, hipMemcpyHostToDevice, p->stream));
  }
  if (worst < 0) g_last_error = "a problem of the batch failed (see per-problem status)";
  return worst;
}

spff_status spff_load_step_batch(spff_problem* p, const double* eps_bar, spff_step_stats* stats) {
  return spff_run_sequence(p, 1, eps_bar, stats);
}

spff_status spff_load_step(spff_problem* p, const double eps_bar[3], spff_step_stats* stats) {
  if (!p) return fail(SPFF_E_INVALID, "problem is NULL");
  if (p->S != 1) return fail(SPFF_E_INVALID, "spff_load_step needs nbatch == 1; use spff_load_step_batch");
  return spff_load_step_batch(p, eps_bar, stats);
}

spff_status spff_get_fields(spff_problem* p, int32_t index, uint32_t mask, void* const* dst) {
  if (!p) return fail(SPFF_E_INVALID, "problem is NULL");
  if (index < -1 || index >= p->S) return fail(SPFF_E_INVALID, "index out of range");
  if (mask & ~0x7Fu) return fail(SPFF_E_INVALID, "unknown field bits");
  if (mask && !dst) return fail(SPFF_E_INVALID, "dst is NULL");
  const size_t n = p->n(), rb = p->rsize * n;
  const int s0 = index < 0 ? 0 : index, s1 = index < 0 ? p->S : index + 1;
  int k = 0;
  void* out[7] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  for (int b = 0; b < 7; ++b)
    if (mask & (1u << b)) {
      if (!dst[k]) return fail(SPFF_E_INVALID, "dst[%d] is NULL", k);
      out[b] = dst[k++];
    }
  const size_t planes[7] = {1, 1, 3, 3, 1, 3, 2};
  if (out[6]) {
    // displacement u* of eps*: one diagnostic tick over the selected slots
    std::vector<int32_t> sl;
    for (int s = s0; s < s1; ++s) sl.push_back(s);
    spff_status st = run_diag(
        p, PH_X_DISP, sl, 3, 2, [&](int s) { return static_cast<const unsigned char*>(p->slot(s) + p->L.eps); },
        [&](int s) { return static_cast<unsigned char*>(out[6]) + (size_t)(s - s0) * 2 * rb; });
    if (st != SPFF_OK) return st;
  }
  for (int s = s0; s < s1; ++s) {
    const int j = s - s0;
    unsigned char* b = p->slot(s);
    auto at = [&](int f) { return static_cast<unsigned char*>(out[f]) + (size_t)j * planes[f] * rb; };
    if (out[0]) HIP_TRY(hipMemcpyAsync(at(0), b + p->L.phi, rb, hipMemcpyDeviceToDevice, p->stream));
    if (out[1]) HIP_TRY(hipMemcpyAsync(at(1), b + p->L.phi_ref, rb, hipMemcpyDeviceToDevice, p->stream));
    if (out[5]) HIP_TRY(hipMemcpyAsync(at(5), b + p->L.eps, 3 * rb, hipMemcpyDeviceToDevice, p->stream));
    if (out[2] || out[3] || out[4]) {
      hipError_t e;
      if (p->cfg.precision == SPFF_FP64)
        e = launch_fields<double>(reinterpret_cast<const SlotPtr<double>*>(p->d_ptr()), p->d_prm(), p->d_ctl(), s,
                                  (int)n, reinterpret_cast<double*>(out[2] ? at(2) : nullptr),
                                  reinterpret_cast<double*>(out[3] ? at(3) : nullptr),
                                  reinterpret_cast<double*>(out[4] ? at(4) : nullptr), p->stream);
      else
        e = launch_fields<float>(reinterpret_cast<const SlotPtr<float>*>(p->d_ptr()), p->d_prm(), p->d_ctl(), s,
                                 (int)n, reinterpret_cast<float*>(out[2] ? at(2) : nullptr),
                                 reinterpret_cast<float*>(out[3] ? at(3) : nullptr),
                                 reinterpret_cast<float*>(out[4] ? at(4) : nullptr), p->stream);
      if (e != hipSuccess) return fail(SPFF_E_DEVICE, "field kernel failed: %s", hipGetErrorString(e));
    }
  }
  HIP_TRY(hipStreamSynchronize(p->stream));
  return SPFF_OK;
}

size_t spff_state_bytes(const spff_problem* p) { return p ? (size_t)p->S * 5 * p->rsize * p->n() : 0; }

spff_status spff_get_state(spff_problem* p, void* dst_dev, double* eps_bar_host) {
  if (!p) return fail(SPFF_E_INVALID, "problem is NULL");
  if (!dst_dev) return fail(SPFF_E_INVALID, "dst is NULL");
  const size_t rb = p->rsize * p->n();
  for (int s = 0; s < p->S; ++s) {
    unsigned char* d = static_cast<unsigned char*>(dst_dev) + (size_t)s * 5 * rb;
    unsigned char* b = p->slot(s);
    HIP_TRY(hipMemcpyAsync(d, b + p->L.eps, 3 * rb, hipMemcpyDeviceToDevice, p->stream));
    HIP_TRY(hipMemcpyAsync(d + 3 * rb, b + p->L.phi, rb, hipMemcpyDeviceToDevice, p->stream));
    HIP_TRY(hipMemcpyAsync(d + 4 * rb, b + p->L.phi_ref, rb, hipMemcpyDeviceToDevice, p->stream));
  }
  HIP_TRY(hipStreamSynchronize(p->stream));
  if (eps_bar_host) std::copy(p->last_eps_bar.begin(), p->last_eps_bar.end(), eps_bar_host);
  return SPFF_OK;
}

spff_status spff_set_state(spff_problem* p, const void* src_dev, const double* eps_bar_host) {
  if (!p) return fail(SPFF_E_INVALID, "problem is NULL");
  if (!src_dev) return fail(SPFF_E_INVALID, "src is NULL");
  if (eps_bar_host)
    for (int k = 0; k < 3 * p->S; ++k)
      if (!std::isfinite(eps_bar_host[k])) return fail(SPFF_E_INVALID, "eps_bar must be finite");
  const size_t rb = p->rsize * p->n();
  // every value finite (checked before anything is copied: an error leaves
  // the state unchanged)
  {
    unsigned int* bad = reinterpret_cast<unsigned int*>(p->ws + p->L.bad);
    const size_t cnt = (size_t)p->S * 5 * p->n();
    HIP_TRY(hipMemsetAsync(bad, 0, sizeof(unsigned int), p->stream));
    hipError_t e = p->cfg.precision == SPFF_FP64
                       ? launch_validate<double>(static_cast<const double*>(src_dev), cnt, -1e300, -1e300, 1e300,
                                                 bad, p->stream)
                       : launch_validate<float>(static_cast<const float*>(src_dev), cnt, -1e300, -1e300, 1e300, bad,
                                                p->stream);
    if (e != hipSuccess) return fail(SPFF_E_DEVICE, "validation launch failed: %s", hipGetErrorString(e));
    unsigned int hbad = 0;
    HIP_TRY(hipMemcpyAsync(&hbad, bad, sizeof(hbad), hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    if (hbad) return fail(SPFF_E_INVALID, "state has %u non-finite entries", hbad);
  }
  for (int s = 0; s < p->S; ++s) {
    const unsigned char* d = static_cast<const unsigned char*>(src_dev) + (size_t)s * 5 * rb;
    unsigned char* b = p->slot(s);
    HIP_TRY(hipMemcpyAsync(b + p->L.eps, d, 3 * rb, hipMemcpyDeviceToDevice, p->stream));
    HIP_TRY(hipMemcpyAsync(b + p->L.phi, d + 3 * rb, rb, hipMemcpyDeviceToDevice, p->stream));
    HIP_TRY(hipMemcpyAsync(b + p->L.phi_ref, d + 4 * rb, rb, hipMemcpyDeviceToDevice, p->stream));
  }
  if (eps_bar_host) {
    std::copy(eps_bar_host, eps_bar_host + 3 * p->S, p->last_eps_bar.begin());
  std::fill(p->last_advance.begin(), p->last_advance.end(), 1);
    for (int s = 0; s < p->S; ++s)
      for (int k = 0; k < 3; ++k) p->host_ctl[s].eps_bar[k] = eps_bar_host[3 * s + k];
    HIP_TRY(hipMemcpyAsync(p->d_ctl(), p->host_ctl, sizeof(SlotCtl) * p->S, hipMemcpyHostToDevice, p->stream));
  }
  HIP_TRY(hipStreamSynchronize(p->stream));
  return SPFF_OK;
}

spff_status spff_apply_operator(spff_problem* p, int32_t op, const void* in_dev, void* out_dev) {
  if (!p) return fail(SPFF_E_INVALID, "problem is NULL");
  if (op != SPFF_OP_PROJECT && op != SPFF_OP_NEG_LAPLACIAN && op != SPFF_OP_DISPLACEMENT)
    return fail(SPFF_E_INVALID, "unknown operator");
  if (!in_dev || !out_dev) return fail(SPFF_E_INVALID, "in/out is NULL");
  const int pin = op == SPFF_OP_NEG_LAPLACIAN ? 1 : 3;
  const int pout = op == SPFF_OP_NEG_LAPLACIAN ? 1 : (op == SPFF_OP_DISPLACEMENT ? 2 : 3);
  const int phase = op == SPFF_OP_PROJECT ? PH_X_PROJ : (op == SPFF_OP_DISPLACEMENT ? PH_X_DISP : PH_X_LAP);
  std::vector<int32_t> all(p->S);
  for (int s = 0; s < p->S; ++s) all[s] = s;
  return run_diag(p, phase, all, pin, pout, [&](int s) { return static_cast<const unsigned char*>(in_dev) + (size_t)s * pin * p->rsize * p->n(); },
                  [&](int s) { return static_cast<unsigned char*>(out_dev) + (size_t)s * pout * p->rsize * p->n(); });
}

spff_status spff_profile_enable(spff_problem* p, int32_t enable) {
  if (!p) return fail(SPFF_E_INVALID, "problem is NULL");
  HIP_TRY(hipStreamSynchronize(p->stream));
  if (p->clock_khz <= 0.0) {
    int dev = 0, khz = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    p->clock_khz = khz > 0 ? (double)khz : 1e5;
  }
  p->prof_on = enable != 0;
  for (int j = 0; j < 4; ++j) p->launches[j] = 0;
  p->prof_ticks = 0;
  std::vector<KTime> init(6);
  for (KTime& k : init) {
    std::fill(std::begin(k.start), std::end(k.start), ~0ull);
    std::fill(std::begin(k.end), std::end(k.end), 0ull);
  }
  HIP_TRY(hipMemcpyAsync(p->d_kt(), init.data(), sizeof(KTime) * 6, hipMemcpyHostToDevice, p->stream));
  HIP_TRY(hipMemsetAsync(p->d_ktsum(), 0, sizeof(unsigned long long) * 8, p->stream));
  HIP_TRY(hipMemsetAsync(p->d_prof(), 0, sizeof(double) * 3 * p->S, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  // the profiling buffers are compiled into the captured blocks: recapture lazily
  drop_graphs(p);
  return SPFF_OK;
}

spff_status spff_profile_read(spff_problem* p, spff_profile* out) {
  if (!p || !out) return fail(SPFF_E_INVALID, "NULL argument");
  std::vector<double> b(3 * (size_t)p->S);
  unsigned long long ks[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  HIP_TRY(hipMemcpyAsync(b.data(), p->d_prof(), sizeof(double) * b.size(), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipMemcpyAsync(ks, p->d_ktsum(), sizeof(ks), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  std::memset(out, 0, sizeof(*out));
  for (int s = 0; s < p->S; ++s)
    for (int j = 0; j < 3; ++j) out->alg_bytes[j] += b[3 * s + j];
  for (int j = 0; j < 4; ++j) {
    out->kernel_ms[j] = p->clock_khz > 0.0 ? (double)ks[j] / p->clock_khz : 0.0;
    out->kernel_span_ms[j] = p->clock_khz > 0.0 ? (double)ks[4 + j] / p->clock_khz : 0.0;
    out->launches[j] = p->launches[j];
  }
  out->ticks = p->prof_ticks;
  return SPFF_OK;
}

spff_status spff_plan_buckets(const spff_problem* p, int32_t* count, int32_t* sizes) {
  if (!p || !count) return fail(SPFF_E_INVALID, "NULL argument");
  *count = (int32_t)p->bucket_size.size();
  if (sizes)
    for (size_t i = 0; i < p->bucket_size.size(); ++i) sizes[i] = p->bucket_size[i];
  return SPFF_OK;
}

spff_status spff_get_plan(const spff_problem* p, int32_t bucket, spff_plan* out) {
  if (!p || !out) return fail(SPFF_E_INVALID, "NULL argument");
  if (bucket < 0 || bucket >= (int32_t)p->plans.size()) return fail(SPFF_E_INVALID, "bucket out of range");
  *out = p->plans[bucket];
  return SPFF_OK;
}

spff_status spff_set_plan(spff_problem* p, int32_t bucket, spff_plan* plan) {
  if (!p) return fail(SPFF_E_INVALID, "problem is NULL");
  if (bucket < 0 || bucket >= (int32_t)p->plans.size()) return fail(SPFF_E_INVALID, "bucket out of range");
  const size_t csize = 2 * p->rsize;
  const int v = p->bucket_size[bucket];
  spff_plan pl = plan ? *plan : auto_plan(&p->cfg, v, csize);
  const spff_status st = check_plan(&p->cfg, &pl, csize);
  if (st != SPFF_OK) return st;
  HIP_TRY(hipStreamSynchronize(p->stream));
  p->plans[bucket] = pl;
  p->geoms[bucket] = geom_from_plan(&p->cfg, v, csize, pl);
  if (p->graphs[bucket]) {
    HIP_TRY(hipGraphExecDestroy(p->graphs[bucket]));
    p->graphs[bucket] = nullptr;
  }
  if (plan) *plan = pl;
  return SPFF_OK;
}

spff_status spff_problem_info(const spff_problem* p, int32_t* nbatch, int32_t* nx, int32_t* ny,
                              int32_t* precision) {
  if (!p) return fail(SPFF_E_INVALID, "problem is NULL");
  if (nbatch) *nbatch = p->S;
  if (nx) *nx = p->cfg.nx;
  if (ny) *ny = p->cfg.ny;
  if (precision) *precision = p->cfg.precision;
  return SPFF_OK;
}

spff_status spff_destroy_problem(spff_problem* p) {
  if (!p) return SPFF_OK;
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  drop_graphs(p);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  if (p->host_ctl) (void)hipHostFree(p->host_ctl);
  if (p->host_list) (void)hipHostFree(p->host_list);
  delete p;
  return SPFF_OK;
}

}  // extern "C"

namespace {

// One load step of one problem for spff_load_step_static: the state planes
// are the caller's, every other array is carved out of the static scratch
// with the single-slot scratch-only layout.  Host staging lives on this
// stack frame and is consumed before the function returns (the stream is
// synchronised after each group of uploads).
template <typename real>
spff_status static_step(const spff_config* cfg, const Layout& L, const LaunchGeom& G, unsigned char* ws,
                        const void* E_dev, void* state_dev, const double* eb, spff_step_stats* stats,
                        hipStream_t st) {
  using C = typename HostCplx<real>::type;
  const double t0 = now_ms();
  const size_t n = (size_t)cfg->nx * cfg->ny;
  SlotPtr<real> F{};
  F.E = static_cast<const real*>(E_dev);
  F.eps = static_cast<real*>(state_dev);
  F.phi = F.eps + 3 * n;
  F.phi_ref = F.eps + 4 * n;
  unsigned char* slot = ws + L.slot0;
  F.theta = reinterpret_cast<real*>(slot + L.theta);
  F.rm = reinterpret_cast<real*>(slot + L.rm);
  F.pm = reinterpret_cast<real*>(slot + L.pm);
  F.spec = slot + L.spec;
  const SlotParam P = make_param(cfg);
  SlotCtl ctl;
  std::memset(&ctl, 0, sizeof(ctl));
  for (int k = 0; k < 3; ++k) ctl.eps_bar[k] = eb[k];
  ctl.phase = PH_M_RES;
  ctl.flags = FL_FIRST_OF_STEP;
  ctl.dt = cfg->dt_max;
  ctl.eta_dt = cfg->eta_over_dt;
  ctl.gamma = 1.0;
  const int32_t list0 = 0;
  C tw[2048];
  auto twiddles = [&](int m) {
    const double two_pi = 6.283185307179586476925286766559;
    for (int k = 0; k < m; ++k) {
      const double a = -two_pi * (double)k / (double)m;
      tw[k].x = (real)std::cos(a);
      tw[k].y = (real)std::sin(a);
    }
  };
  SlotCtl* d_ctl = reinterpret_cast<SlotCtl*>(ws + L.ctl);
  SlotParam* d_prm = reinterpret_cast<SlotParam*>(ws + L.prm);
  SlotPtr<real>* d_ptr = reinterpret_cast<SlotPtr<real>*>(ws + L.ptr);
  int32_t* d_list = reinterpret_cast<int32_t*>(ws + L.list);
  unsigned int* d_bad = reinterpret_cast<unsigned int*>(ws + L.bad);
  C* twx = reinterpret_cast<C*>(ws + L.twx);
  C* twy = reinterpret_cast<C*>(ws + L.twy);
  HIP_TRY(hipMemcpyAsync(d_ptr, &F, sizeof(F), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(d_prm, &P, sizeof(P), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(d_ctl, &ctl, sizeof(ctl), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(d_list, &list0, sizeof(list0), hipMemcpyHostToDevice, st));
  twiddles(cfg->nx);
  HIP_TRY(hipMemcpyAsync(twx, tw, sizeof(C) * cfg->nx, hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  twiddles(cfg->ny);
  HIP_TRY(hipMemcpyAsync(twy, tw, sizeof(C) * cfg->ny, hipMemcpyHostToDevice, st));
  // inputs: E > 0 and finite, phi and phi_ref in [0, 1]
  HIP_TRY(hipMemsetAsync(d_bad, 0, 2 * sizeof(unsigned int), st));
  HIP_TRY(launch_validate<real>(F.E, n, 0.0, -1e300, 1e300, d_bad, st));
  HIP_TRY(launch_validate<real>(F.phi, 2 * n, -1e300, 0.0, 1.0, d_bad + 1, st));
  unsigned int bad[2] = {0, 0};
  HIP_TRY(hipMemcpyAsync(bad, d_bad, sizeof(bad), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (bad[0]) return fail(SPFF_E_INVALID, "E has %u non-positive or non-finite entries", bad[0]);
  if (bad[1]) return fail(SPFF_E_INVALID, "phi / phi_ref have %u entries outside [0, 1]", bad[1]);
  TickBufs<real> B{};
  B.list = d_list;
  B.ptrs = d_ptr;
  B.prms = d_prm;
  B.ctl[0] = d_ctl;
  B.ctl[1] = d_ctl + 1;
  B.twx = twx;
  B.twy = twy;
  B.prow[0] = reinterpret_cast<double*>(ws + L.prow);
  B.prow[1] = reinterpret_cast<double*>(ws + L.prow1);
  B.pcol = reinterpret_cast<double*>(ws + L.pcol);
  B.pinv = reinterpret_cast<double*>(ws + L.pinv);
  const int K = cfg->ticks_per_sync;
  for (;;) {
    for (int i = 0; i < K; ++i) {
      hipError_t e = launch_tick<real>(G, B, i, st);
      if (e != hipSuccess) return fail(SPFF_E_DEVICE, "tick launch failed: %s", hipGetErrorString(e));
    }
    hipError_t e = launch_close<real>(G, B, K, st);
    if (e != hipSuccess) return fail(SPFF_E_DEVICE, "tick launch failed: %s", hipGetErrorString(e));
    HIP_TRY(hipMemcpyAsync(&ctl, d_ctl, sizeof(ctl), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (ctl.phase == PH_IDLE) break;
  }
  if (stats) fill_stats(n, ctl, *stats, now_ms() - t0);
  const spff_status ss = slot_status(ctl);
  if (ss < 0) g_last_error = "a reduction produced NaN or Inf";
  return ss;
}

}  // namespace

extern "C" {

spff_status spff_load_step_static(const spff_config* cfg, const void* E_dev, void* state_dev,
                                  const double eps_bar[3], spff_step_stats* stats, void* stream) {
  spff_status st = check_config(cfg);
  if (st != SPFF_OK) return st;
  if (!E_dev || !state_dev || !eps_bar) return fail(SPFF_E_INVALID, "E_dev, state_dev and eps_bar must not be NULL");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(eps_bar[k])) return fail(SPFF_E_INVALID, "eps_bar must be finite");
  if (cfg->evolution != SPFF_EVOL_AM)
    return fail(SPFF_E_INVALID, "spff_load_step_static runs alternating minimisation (SPFF_EVOL_AM) only");
  const size_t rsize = cfg->precision == SPFF_FP64 ? 8 : 4;
  const Layout L = layout(cfg, 1, rsize, true);
  if (L.total > SPFF_STATIC_SCRATCH_BYTES)
    return fail(SPFF_E_INVALID, "a %d x %d %s problem needs %zu bytes of scratch; the static scratch holds %zu",
                cfg->nx, cfg->ny, rsize == 8 ? "FP64" : "FP32", L.total, (size_t)SPFF_STATIC_SCRATCH_BYTES);
  const spff_plan pl = auto_plan(cfg, 1, 2 * rsize);
  const LaunchGeom G = geom_from_plan(cfg, 1, 2 * rsize, pl);
  if (G.lds_row > LDS_MAX || G.lds_col > LDS_MAX) return fail(SPFF_E_INVALID, "grid too large for LDS tiles");
  void* ws = nullptr;
  hipError_t e = static_scratch(&ws);
  if (e != hipSuccess) return fail(SPFF_E_DEVICE, "static scratch address: %s", hipGetErrorString(e));
  hipStream_t hs = static_cast<hipStream_t>(stream);
  unsigned char* w = static_cast<unsigned char*>(ws);
  return cfg->precision == SPFF_FP64 ? static_step<double>(cfg, L, G, w, E_dev, state_dev, eps_bar, stats, hs)
                                     : static_step<float>(cfg, L, G, w, E_dev, state_dev, eps_bar, stats, hs);
}

const char* spff_last_error(void) { return g_last_error.c_str(); }

const char* spff_version(void) { return "spff 0.1 (gfx950)"; }

}  // extern "C"

// ===========================================================================
// Serving: continuous batching over resident problems (see include/spff.h).
// ===========================================================================
namespace {

struct SrvRequest {
  uint64_t ticket;
  double eb[3];
  double t_submit;
};

struct SrvProblem {
  int cls;
  spff_config cfg;
  unsigned char *E, *phi, *phi_ref, *eps;  // resident planes in the arena
  std::deque<SrvRequest> queue;            // submitted, not yet admitted
  bool running = false;
  double t_submit = 0.0;
  uint64_t ticket = 0;
  double dt = 0.0;  // time-discretized evolution: the problem's dt (0: dt_max)
  int ne_flag = 0;  // near-equilibrium evolution: the problem's trigger flag
};

struct SrvClass {
  int nx, ny, precision, nyquist;
  spff_problem* eng = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t done_ev = nullptr;
  std::vector<int> owner;  // problem id per slot, -1 free
  std::deque<int> ready;   // problems with a request waiting for a slot
  bool inflight = false;
  std::vector<int> members;
};

}  // namespace

struct spff_server {
  unsigned char* arena;
  size_t arena_bytes, used;
  size_t scratch_budget, scratch_used;
  int ticks_per_sync, use_graph;
  hipStream_t setup;
  std::vector<SrvProblem> probs;
  std::vector<SrvClass> classes;
  std::unordered_map<uint64_t, spff_step_stats> done;
  std::unordered_map<uint64_t, int> live;  // ticket -> problem (queued or running)
  uint64_t next_ticket = 1;
};

namespace {

unsigned char* arena_take(spff_server* sv, size_t bytes) {
  const size_t off = align_up(sv->used);
  if (off + bytes > sv->arena_bytes) return nullptr;
  sv->used = off + bytes;
  return sv->arena + off;
}

// Create the engine of a class: as many scratch slots as the budget share of
// the class allows (at least one, at most its number of problems).
spff_status class_start(spff_server* sv, int c) {
  SrvClass& C = sv->classes[c];
  const spff_config& cfg0 = sv->probs[C.members[0]].cfg;
  spff_config ec = cfg0;
  ec.ticks_per_sync = sv->ticks_per_sync;
  ec.use_graph = sv->use_graph;
  const size_t rsize = ec.precision == SPFF_FP64 ? 8 : 4;
  const size_t one = layout(&ec, 1, rsize, true).total;
  const size_t two = layout(&ec, 2, rsize, true).total;
  const size_t per_slot = two - one;
  // budget share proportional to the class's pixels over all classes
  double px_all = 0.0, px_c = 0.0;
  for (const SrvClass& K : sv->classes) px_all += (double)K.nx * K.ny * K.members.size();
  px_c = (double)C.nx * C.ny * C.members.size();
  size_t budget = sv->scratch_budget ? (size_t)(sv->scratch_budget * (px_c / px_all)) : sv->arena_bytes;
  int S = (int)std::min<size_t>(C.members.size(), budget > one ? 1 + (budget - one) / per_slot : 1);
  S = std::max(1, std::min(S, 1024));
  for (;;) {
    const size_t bytes = layout(&ec, S, rsize, true).total;
    const size_t off = align_up(sv->used);
    if (off + bytes <= sv->arena_bytes) break;
    if (S == 1) return fail(SPFF_E_NOMEM, "arena too small for a class engine");
    S = S / 2;
  }
  const size_t bytes = layout(&ec, S, rsize, true).total;
  unsigned char* ws = arena_take(sv, bytes);
  HIP_TRY(hipStreamCreateWithFlags(&C.stream, hipStreamNonBlocking));
  HIP_TRY(hipEventCreateWithFlags(&C.done_ev, hipEventDisableTiming));
  spff_status st = engine_create(&ec, S, nullptr, nullptr, ws, bytes, C.stream, true, &C.eng);
  if (st != SPFF_OK) return st;
  sv->scratch_used += bytes;
  C.owner.assign(S, -1);
  return SPFF_OK;
}

// Bind problem `id` to slot s of its class engine and start its next request.
spff_status class_admit(spff_server* sv, SrvClass& C, int s, int id) {
  SrvProblem& P = sv->probs[id];
  spff_problem* e = C.eng;
  SrvRequest rq = P.queue.front();
  P.queue.pop_front();
  P.running = true;
  P.ticket = rq.ticket;
  P.t_submit = rq.t_submit;
  C.owner[s] = id;
  SlotPtr<double>& ptr = e->host_ptrs[s];
  ptr.E = reinterpret_cast<const double*>(P.E);
  ptr.phi = reinterpret_cast<double*>(P.phi);
  ptr.phi_ref = reinterpret_cast<double*>(P.phi_ref);
  ptr.eps = reinterpret_cast<double*>(P.eps);
  e->prm[s] = make_param(&P.cfg);
  HIP_TRY(hipMemcpyAsync(static_cast<unsigned char*>(e->d_ptr()) + s * sizeof(SlotPtr<double>), &ptr,
                         sizeof(SlotPtr<double>), hipMemcpyHostToDevice, C.stream));
  HIP_TRY(hipMemcpyAsync(e->d_prm() + s, &e->prm[s], sizeof(SlotParam), hipMemcpyHostToDevice, C.stream));
  e->host_ctl[s].dt = P.dt;
  e->host_ctl[s].ne_flag = P.ne_flag;
  start_step(e, s, rq.eb, P.cfg);
  return SPFF_OK;
}

}  // namespace

extern "C" {

spff_status spff_server_create(void* arena_dev, size_t arena_bytes, size_t scratch_budget_bytes,
                               int32_t ticks_per_sync, int32_t use_graph, spff_server** out) {
  if (!out) return fail(SPFF_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!arena_dev || reinterpret_cast<uintptr_t>(arena_dev) % ALIGN)
    return fail(SPFF_E_INVALID, "arena must be a 256-byte aligned device pointer");
  if (ticks_per_sync < 1 || ticks_per_sync > 4096) return fail(SPFF_E_INVALID, "ticks_per_sync in [1, 4096]");
  spff_server* sv = new spff_server();
  sv->arena = static_cast<unsigned char*>(arena_dev);
  sv->arena_bytes = arena_bytes;
  sv->used = 0;
  sv->scratch_budget = scratch_budget_bytes;
  sv->scratch_used = 0;
  sv->ticks_per_sync = ticks_per_sync;
  sv->use_graph = use_graph;
  if (hipStreamCreateWithFlags(&sv->setup, hipStreamNonBlocking) != hipSuccess) {
    delete sv;
    return fail(SPFF_E_DEVICE, "stream creation failed");
  }
  *out = sv;
  return SPFF_OK;
}

spff_status spff_server_register(spff_server* sv, const spff_config* cfg, const void* E_dev, int32_t* id) {
  if (!sv || !cfg || !E_dev || !id) return fail(SPFF_E_INVALID, "NULL argument");
  spff_status st = check_config(cfg);
  if (st != SPFF_OK) return st;
  const size_t rsize = cfg->precision == SPFF_FP64 ? 8 : 4;
  const size_t rb = rsize * (size_t)cfg->nx * cfg->ny;
  int c = -1;
  for (size_t k = 0; k < sv->classes.size(); ++k)
    if (sv->classes[k].nx == cfg->nx && sv->classes[k].ny == cfg->ny && sv->classes[k].precision == cfg->precision &&
        sv->classes[k].nyquist == cfg->nyquist)
      c = (int)k;
  const size_t used0 = sv->used;
  SrvProblem P;
  P.cfg = *cfg;
  P.E = arena_take(sv, rb);
  P.phi = arena_take(sv, rb);
  P.phi_ref = arena_take(sv, rb);
  P.eps = arena_take(sv, 3 * rb);
  unsigned char* bad = arena_take(sv, 64);
  if (!P.E || !P.phi || !P.phi_ref || !P.eps || !bad) {
    sv->used = used0;
    return fail(SPFF_E_NOMEM, "arena full");
  }
  HIP_TRY(hipMemcpyAsync(P.E, E_dev, rb, hipMemcpyDeviceToDevice, sv->setup));
  HIP_TRY(hipMemsetAsync(P.phi, 0, rb, sv->setup));
  HIP_TRY(hipMemsetAsync(P.phi_ref, 0, rb, sv->setup));
  HIP_TRY(hipMemsetAsync(P.eps, 0, 3 * rb, sv->setup));
  HIP_TRY(hipMemsetAsync(bad, 0, 64, sv->setup));
  const size_t n = (size_t)cfg->nx * cfg->ny;
  hipError_t e = cfg->precision == SPFF_FP64
                     ? launch_validate<double>(reinterpret_cast<const double*>(P.E), n, 0.0, -1e300, 1e300,
                                               reinterpret_cast<unsigned int*>(bad), sv->setup)
                     : launch_validate<float>(reinterpret_cast<const float*>(P.E), n, 0.0, -1e300, 1e300,
                                              reinterpret_cast<unsigned int*>(bad), sv->setup);
  if (e != hipSuccess) return fail(SPFF_E_DEVICE, "validation launch failed: %s", hipGetErrorString(e));
  unsigned int hbad = 0;
  HIP_TRY(hipMemcpyAsync(&hbad, bad, sizeof(hbad), hipMemcpyDeviceToHost, sv->setup));
  HIP_TRY(hipStreamSynchronize(sv->setup));
  if (hbad) {
    sv->used = used0;
    return fail(SPFF_E_INVALID, "E has %u non-positive or non-finite entries", hbad);
  }
  if (c < 0) {
    SrvClass C;
    C.nx = cfg->nx;
    C.ny = cfg->ny;
    C.precision = cfg->precision;
    C.nyquist = cfg->nyquist;
    sv->classes.push_back(C);
    c = (int)sv->classes.size() - 1;
  }
  P.cls = c;
  sv->probs.push_back(P);
  *id = (int32_t)sv->probs.size() - 1;
  sv->classes[c].members.push_back(*id);
  return SPFF_OK;
}

spff_status spff_server_submit(spff_server* sv, int32_t id, const double eps_bar[3], uint64_t* ticket) {
  if (!sv || !eps_bar || !ticket) return fail(SPFF_E_INVALID, "NULL argument");
  if (id < 0 || id >= (int32_t)sv->probs.size()) return fail(SPFF_E_INVALID, "unknown problem id");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(eps_bar[k])) return fail(SPFF_E_INVALID, "eps_bar must be finite");
  SrvProblem& P = sv->probs[id];
  SrvRequest rq;
  rq.ticket = sv->next_ticket++;
  for (int k = 0; k < 3; ++k) rq.eb[k] = eps_bar[k];
  rq.t_submit = now_ms();
  const bool was_idle = !P.running && P.queue.empty();
  P.queue.push_back(rq);
  if (was_idle) sv->classes[P.cls].ready.push_back(id);
  sv->live[rq.ticket] = id;
  *ticket = rq.ticket;
  return SPFF_OK;
}

spff_status spff_server_progress(spff_server* sv, int32_t max_rounds, int32_t* completed, int32_t* pending) {
  if (!sv) return fail(SPFF_E_INVALID, "server is NULL");
  int done_count = 0;
  for (int round = 0; round < max_rounds; ++round) {
    bool any = false;
    // 1. admit and launch, class by class (each on its own stream)
    for (size_t c = 0; c < sv->classes.size(); ++c) {
      SrvClass& C = sv->classes[c];
      if (C.ready.empty() && (!C.eng || std::all_of(C.owner.begin(), C.owner.end(), [](int o) { return o < 0; })))
        continue;
      if (!C.eng) {
        spff_status st = class_start(sv, (int)c);
        if (st != SPFF_OK) return st;
      }
      spff_problem* e = C.eng;
      bool dirty = false;
      for (int s = 0; s < e->S && !C.ready.empty(); ++s) {
        if (C.owner[s] >= 0) continue;
        const int id = C.ready.front();
        C.ready.pop_front();
        spff_status st = class_admit(sv, C, s, id);
        if (st != SPFF_OK) return st;
        dirty = true;
      }
      if (dirty)
        HIP_TRY(hipMemcpyAsync(e->d_ctl(), e->host_ctl, sizeof(SlotCtl) * e->S, hipMemcpyHostToDevice, C.stream));
      bool launched;
      int k;
      spff_status st = launch_block(e, &launched, &k);
      if (st != SPFF_OK) return st;
      if (!launched) continue;
      HIP_TRY(hipMemcpyAsync(e->host_ctl, e->d_ctl(), sizeof(SlotCtl) * e->S, hipMemcpyDeviceToHost, C.stream));
      HIP_TRY(hipEventRecord(C.done_ev, C.stream));
      C.inflight = true;
      any = true;
    }
    if (!any) break;
    // 2. collect finished requests; a request completes when the host has
    // seen the end of its class's tick block
    for (SrvClass& C : sv->classes) {
      if (!C.inflight) continue;
      HIP_TRY(hipEventSynchronize(C.done_ev));
      const double t = now_ms();
      C.inflight = false;
      spff_problem* e = C.eng;
      for (int s = 0; s < e->S; ++s) {
        const int id = C.owner[s];
        if (id < 0 || e->host_ctl[s].phase != PH_IDLE) continue;
        SrvProblem& P = sv->probs[id];
        spff_step_stats o;
        fill_stats(e->n(), e->host_ctl[s], o, t - P.t_submit);
        P.dt = e->host_ctl[s].dt;
        P.ne_flag = e->host_ctl[s].ne_flag;
        sv->done[P.ticket] = o;
        sv->live.erase(P.ticket);
        P.running = false;
        C.owner[s] = -1;
        ++done_count;
        if (!P.queue.empty()) C.ready.push_back(id);
      }
    }
  }
  if (completed) *completed = done_count;
  if (pending) *pending = (int32_t)sv->live.size();
  return SPFF_OK;
}

spff_status spff_server_poll(spff_server* sv, uint64_t ticket, spff_step_stats* out) {
  if (!sv) return fail(SPFF_E_INVALID, "server is NULL");
  auto it = sv->done.find(ticket);
  if (it == sv->done.end()) {
    if (sv->live.count(ticket)) return SPFF_E_BUSY;
    return fail(SPFF_E_INVALID, "unknown ticket");
  }
  if (out) *out = it->second;
  sv->done.erase(it);
  return SPFF_OK;
}

spff_status spff_server_get_fields(spff_server* sv, int32_t id, uint32_t mask, void* const* dst) {
  if (!sv) return fail(SPFF_E_INVALID, "server is NULL");
  if (id < 0 || id >= (int32_t)sv->probs.size()) return fail(SPFF_E_INVALID, "unknown problem id");
  if (mask & ~(uint32_t)(SPFF_FIELD_PHI | SPFF_FIELD_PHI_REF | SPFF_FIELD_EPS_STAR))
    return fail(SPFF_E_INVALID, "only phi, phi_ref and eps* are resident fields");
  SrvProblem& P = sv->probs[id];
  if (P.running || !P.queue.empty()) return fail(SPFF_E_BUSY, "problem has pending requests");
  const size_t rb = (P.cfg.precision == SPFF_FP64 ? 8 : 4) * (size_t)P.cfg.nx * P.cfg.ny;
  int k = 0;
  if (mask && !dst) return fail(SPFF_E_INVALID, "dst is NULL");
  if (mask & SPFF_FIELD_PHI) HIP_TRY(hipMemcpyAsync(dst[k++], P.phi, rb, hipMemcpyDeviceToDevice, sv->setup));
  if (mask & SPFF_FIELD_PHI_REF)
    HIP_TRY(hipMemcpyAsync(dst[k++], P.phi_ref, rb, hipMemcpyDeviceToDevice, sv->setup));
  if (mask & SPFF_FIELD_EPS_STAR)
    HIP_TRY(hipMemcpyAsync(dst[k++], P.eps, 3 * rb, hipMemcpyDeviceToDevice, sv->setup));
  HIP_TRY(hipStreamSynchronize(sv->setup));
  return SPFF_OK;
}

spff_status spff_server_info(const spff_server* sv, int32_t* nclasses, int32_t* total_slots, size_t* arena_used) {
  if (!sv) return fail(SPFF_E_INVALID, "server is NULL");
  int slots = 0;
  for (const SrvClass& C : sv->classes) slots += C.eng ? C.eng->S : 0;
  if (nclasses) *nclasses = (int32_t)sv->classes.size();
  if (total_slots) *total_slots = slots;
  if (arena_used) *arena_used = sv->used;
  return SPFF_OK;
}

spff_status spff_server_destroy(spff_server* sv) {
  if (!sv) return SPFF_OK;
  for (SrvClass& C : sv->classes) {
    if (C.stream) (void)hipStreamSynchronize(C.stream);
    if (C.eng) spff_destroy_problem(C.eng);
    if (C.done_ev) (void)hipEventDestroy(C.done_ev);
    if (C.stream) (void)hipStreamDestroy(C.stream);
  }
  if (sv->setup) (void)hipStreamDestroy(sv->setup);
  delete sv;
  return SPFF_OK;
}

}  // extern "C"
