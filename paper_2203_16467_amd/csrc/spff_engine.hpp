// Engine structures shared by the device kernels and the host driver.
//
// Execution model.  A handle owns S "slots"; a slot holds one problem (its
// resident state and its solver scratch).  Every slot runs its own state
// machine for one load step of alternating minimisation (Algorithm 2):
//
//   M_RES   mechanics residual R = G[sigma(eps_bar + eps*)] (Newton start)
//   M_CG    one CG iteration on G[C_m : theta] = -R (Sec. 3.1.1)
//   PF_ASM  phase-field assembly (d, b) and BCCG initial residual
//   PF_PQ   BCCG step length: p update, p.Jp via Parseval (Alg. 1)
//   PF_R    BCCG update phi <- clip(phi + alpha p), new residual (Alg. 1)
//   AM_CHK  ||phi_n+1 - phi_n||_1 (Sec. 3.2.1)
//   STATS   energies, mean stress, phi statistics
//
// The host advances all slots together in "ticks": one tick launches the
// row-forward, column and row-inverse FFT kernels (each does the part of the
// current phase that belongs to it, or nothing).  The controller step of a
// tick -- reduce the tick's partial sums in a fixed order, compute the FP64
// scalars (alpha, beta, norms) and move the slot to its next phase -- runs
// at the start of the next tick's row-forward kernel, redundantly in every
// work-group of the slot (same inputs, same order: same result), and for
// the last tick of a block in a closing kernel.  The control block is
// double-buffered across ticks: the row-forward kernel of tick i reads
// block (i & 1), the group of row block 0 writes the advanced one to block
// ((i + 1) & 1), which the column and row-inverse kernels of tick i read.
// Ticks contain no host round trip, so blocks of ticks can be replayed as a
// captured HIP graph; the host polls phases between blocks (the closing
// kernel leaves the current block in buffer 0).
#pragma once
#include <stdint.h>

namespace spff {

enum Phase : int32_t {
  PH_IDLE = 0,
  PH_M_RES = 1,
  PH_M_CG = 2,
  PH_PF_ASM = 3,
  PH_PF_PQ = 4,
  PH_PF_R = 5,
  PH_AM_CHK = 6,
  PH_STATS = 7,
  PH_X_PROJ = 8,  // diagnostic: rm = G[theta] (3 planes)
  PH_X_LAP = 9,   // diagnostic: rm[0] = -lap theta[0]
  PH_TD_RESTORE = 10,  // time-discretized evolution: phi <- phi_n before a retry with dt/2
  PH_X_DISP = 11,      // diagnostic: rm[0..1] = displacement u* of the strain field in theta (3 planes)
};

// ctl.flags bits
enum : int32_t {
  FL_FIRST_OF_STEP = 1,   // next M_RES copies phi -> phi_ref
  FL_THETA_PENDING = 2,   // next M_RES applies eps* += theta
  FL_CG_FIRST = 4,        // next M_CG is the first of a Newton step
  FL_INIT_SOLVE = 8,      // phase-field solve at zero strain (phi_init)
  FL_MECH_STARTED = 16,   // reference norm of the current mechanics solve set
  FL_NOT_CONVERGED = 32,  // an iteration cap was hit during the step
  FL_NONFINITE = 64,      // a reduction was NaN/Inf
  FL_PF_FIRST = 128,      // next PF_PQ is the first BCCG iteration (beta = 0)
  FL_STALLED = 256,       // BCCG residual stopped improving (stall guard)
  FL_NE_CHECK = 512,      // near-equilibrium: this PF_ASM evaluates -F_phi(phi_n, eps_n)
  FL_NE_SCALE = 1024,     // near-equilibrium: this PF_ASM first scales eps* by gamma
};

// Per-slot physical and solver parameters (read-only during a step).
struct SlotParam {
  double lam_t, mu_t;      // Lame constants per unit E (plane strain)
  double ell, gc;
  double cwl;              // G_c / (c_w ell)
  double kappa;            // 2 G_c ell / c_w   (coefficient of -lap in F_phi)
  double wpp;              // w'' (0 for AT1, 2 for AT2)
  double dw0;              // w'(0) (1 for AT1, 0 for AT2)
  double eta_dt, k_res, threshold;
  double tol_mech, tol_abs_mech, tol_pf, tol_abs_pf, tol_am;
  // attainable-accuracy floor of a residual computed in the working
  // precision: floor = floor_coef * (norm of the terms the residual is
  // computed from); floor_coef = floor_factor * u * sqrt(log2(nx ny))
  double floor_coef;
  double lap_rms;          // mean |2 pi q|^2 over the grid's modes (2 pi^2 / 3)
  int32_t at, split, irr, stall_iters;  // split: driving-force model
  int32_t contact, evolution;             // stress model; SPFF_EVOL_*
  double eta, dt_max, dt_min, dphi_max, dphi_min;  // time-discretized evolution
  double fphi_max, drive_thr, deps_max;            // near-equilibrium evolution
  int32_t max_cg, max_newton, max_bccg, max_am;
};

// Per-slot control block (advanced by the controller step on the device; the
// host writes it, in the buffer the closing kernel leaves it in, only while
// the slot is idle).
struct SlotCtl {
  int32_t phase, flags;
  int32_t am, newton, cg, bccg;     // counters of the current load step
  int32_t cg_newton, pf_it;         // CG iterations of the current Newton step, BCCG of the current solve
  int32_t newton_solve;             // Newton steps of the current mechanics solve
  int32_t pending;                  // the controller step of the last tick is still to run
  uint64_t t_start;                 // device wall clock at the start of the step
  int32_t ticks, status;
  double eps_bar[3];
  // mechanics
  double mech_ref, mech_target, mech_res, rr, inner_tol, alpha_m, beta_m;
  // phase field
  double pf_ref, pf_target, pf_res, rr_pf, alpha_pf, beta_pf, pq, rp;
  double pf_bnorm, pf_best, mech_floor, pf_floor;
  int32_t pf_best_it;
  int32_t seq_pos;                  // position in the device-side load-step queue
  // alternating minimisation
  double dphi;
  // viscous term of the running phase-field solve; time-discretized
  // evolution: time step (kept between load steps), halvings, load advance
  double eta_dt, dt;
  int32_t halvings, advance;
  // near-equilibrium evolution: strain scaling of the step, largest -F_phi
  // before it, trigger flag (kept between load steps)
  double gamma, fmax_ne;
  int32_t ne_flag, pad2;
  // statistics of the finished step
  double F_e, F_f, sbar[3], phi_sum, phi_max, crack_px;
};

// Per-slot device pointers (resident state + scratch).  Scratch planes are
// shared between the mechanics and phase-field phases, which never overlap:
//   theta[0..2] (mech update)      | d, b, phi_am   (phase field)
//   rm[0..2]    (mech residual)    | r_pf = rm[0]
//   pm[0..2]    (mech direction)   | p_pf = pm[0], mask = bytes of pm[1]
template <typename real>
struct SlotPtr {
  const real* E;
  real* phi;
  real* phi_ref;
  real* eps;     // eps* planes xx, yy, xy  ([3][n])
  real* theta;   // [3][n]
  real* rm;      // [3][n]
  real* pm;      // [3][n]
  void* spec;    // complex [3][nx/2][ny]  (half spectrum, transposed)
};

// Device-side load-step queue of a slot: the controller step starts step pos+1
// as soon as step pos has finished, without a host round trip, and records
// the finished step's statistics in the slot's StepRec array.
constexpr int SEQ_MAX = 256;

struct SlotSeq {
  int32_t len, pos;
  int32_t incr;  // 1: eps_bar[] are load increments, applied after steps that advance
  int32_t pad;
  double eps_bar[SEQ_MAX][3];
};

struct StepRec {
  int32_t status, flags, am, newton, cg, bccg, ticks, halvings;
  int32_t advance, ne_flag;
  double dt, gamma, fmax_ne;
  uint64_t t_start, t_end;  // device wall clock
  double dphi, mech_res, pf_res, F_e, F_f, sbar[3], phi_sum, phi_max, crack_px;
  double eps_bar[3];
};

// Device-side kernel timing (profiling) of one kernel: every work-group
// lowers one of KT_LINES `start` words to its first clock reading and raises
// one of KT_LINES `end` words to its last (hashed by work-group, one word per
// 128-byte line, so that thousands of groups do not contend on one address).
// Ticks alternate between two sets of three (one per FFT kernel).  An extra
// work-group of the next tick's column kernel (or the closing kernel, for
// the last tick of a block) folds, per FFT kernel, its activity (last end -
// first start) and its span (first start to the next kernel's first start:
// activity plus the dead time of its drain, write-back and the next
// dispatch), and resets the words.
constexpr int KT_LINES = 64;
constexpr int KT_STRIDE = 16;  // 64-bit words per line
struct KTime {
  unsigned long long start[KT_LINES * KT_STRIDE];
  unsigned long long end[KT_LINES * KT_STRIDE];
};

// Number of FP64 partials per work-group written by each kernel.
constexpr int NP_ROW = 8;
constexpr int NP_COL = 2;
constexpr int NP_INV = 4;

}  // namespace spff
