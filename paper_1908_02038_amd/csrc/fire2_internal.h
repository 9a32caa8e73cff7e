// fire2_internal.h -- device-side records shared by the HIP translation units
// of libfire2 (single-system path in fire2.hip, batched path in batched.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "fire2.h"

namespace fire {

constexpr int kBlock = 256;   // threads per block of the per-atom kernels
constexpr int kMaxTile = 512; // atoms (threads) per tile of the LDS-staged LJ pass; real-atom capacity is a multiple
constexpr int kRed = 8;       // doubles per reduction record
constexpr int kPartAtoms = 64; // reduction records exist for grids of up to ncap / kPartAtoms blocks
// reduction record layout (one per block of the force pass); the last two
// are the mass-weighted sums sum_i s_i v_i.F_i and sum_i s_i^2 |F_i|^2
// (s_i = 1 / m_i), kept only when the atoms carry masses
enum RedField { R_E = 0, R_P = 1, R_F2 = 2, R_V2 = 3, R_FMAX2 = 4, R_VMAX2 = 5, R_SVF = 6, R_SFF = 7 };
constexpr int kCtl = 8;       // reduced values the control reads (the record's fields)

// ctrl->status: 0 running, 10 paused for the host, FIRE_STOP_* when stopped,
// negative FIRE_E_* on a device-detected error.
constexpr int ST_RUNNING = 0;
constexpr int ST_PAUSED = 10;
// ctrl->pause bits
constexpr int PAUSE_REBUILD = 1;    // an atom moved more than skin/2 in the last update:
                                    // rebuild the list, then evaluate forces
constexpr int PAUSE_PRECISION = 4;  // mixed mode: continue with FP64 pair terms
// ctrl->error bits (set by kernels)
constexpr int ERR_OVERLAP = 1;
constexpr int ERR_NONFINITE = 2;

// Orthorhombic box, per-axis periodicity.
struct BoxDev {
  double L[3], invL[3], lo[3];
  int per[3];
};

// Potential constants prepared on the host.
struct PotDev {
  int kind, conv;
  double rc, rc2;      // cutoff (LJ rc, Gupta r_out) and its square
  double eps, sig2, shift;  // LJ: shift = 4 eps [(s/rc)^12 - (s/rc)^6]
  double A, pr0, qr0, xi, r0, r_in, inv_w;  // Gupta: pr0 = p / r0, qr0 = 2 q / r0
  double cpair, epair;  // Gupta force / energy weights of the pair term (RGL 2, 1; half 1, 1/2)
  double k[3];          // harmonic well
  // Stillinger-Weber: phi2 = Aeps [B (s/r)^p - (s/r)^q] exp(s / (r - as)),
  // h = leps (cos + 1/3)^2 g g, g = exp(gs / (r - as)); rc = as
  double sw_s, sw_as, sw_Aeps, sw_B, sw_p, sw_q, sw_leps, sw_gs;
};

// FIRE control record of one system, resident in device memory.  The first
// 32 bytes are what the host polls.
struct Ctrl {
  int status, pause, precision, error;  // precision: 0 FP64 pair terms, 1 FP32
  long long iter, evals;
  int viol;            // set by the update when an atom left its skin
  int eval_only;       // 1: the force pass only records E and the norms
  unsigned int ticket; // blocks of the current force pass that are done
  int pad0;
  // parameters
  double dt_start, dtmax, dtmin, dtgrow, dtshrink, alpha0, alphashrink, f2a;
  double tol, switch_tol, skin_half2, dmax;
  long long max_steps, trace_cap, iter_low;
  int delaystep, vdfmax, halfstepback, initialdelay;
  int integrator, criterion, variant, mode;
  double natoms;
  // FIRE state
  double dt, alpha;
  long long npos, nneg;
  int branch, neg, mix_first;
  int cur;             // which state buffer holds the current positions (0: the primary set)
  double P_used;
  // coefficients of the next update
  double hsb, kick1, kick2, kick3, cv, cf, dtx;
  // results of the last force evaluation
  double energy, fmax, f2norm, P, v2, F2, vmax;
};

}  // namespace fire
