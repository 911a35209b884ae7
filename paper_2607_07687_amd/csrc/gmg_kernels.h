// GMG kernels for gfx950 (CDNA4): residual, red-black half-sweeps, fused
// residual + restriction, prolongation + correction, hierarchy set-up,
// reductions and the device-side solve state.  All of them are memory-bound
// stencils (about 1 flop per byte); see the launch helpers in gmg_lib.hip.
#pragma once

#include "gmg_device.h"
#include "../../include/gmg.h"

namespace gmg {

// Device-resident solver state: adaptive relaxation factor, accepted-iterate
// selector and convergence flag, decided on the device after every V-cycle.
struct SolveState {
  double rho;      // ||r|| of the accepted iterate
  double rho0;     // ||r|| of the initial guess
  double snorm;    // ||sigma|| over active cells
  double omega;    // relaxation factor for the next cycle
  double rtol;
  double last;     // ||r|| of the most recent cycle's result
  int cur;         // 0: accepted iterate in buffer A, 1: in buffer B
  int done;        // 1 once converged or out of cycles
  int cycles, accepted, max_cycles, status;
  // deferred decision (gmg_solve): the norm of a cycle's result is taken by
  // the next cycle's first sweep, whose output is redone when the decision
  // changes omega; level-0 roles through map (0 accepted, 1 candidate,
  // 2 and 3 work)
  int map[4];
  int pending;     // a candidate awaits its decision
  int redo;        // the speculative first sweep must be redone
  int bad;         // set-up: a face coefficient given to gmg_setup is not finite
  int coarse_sweeps;  // sweeps of the coarsest level in the last V-cycle's tail
  double omega_spec;  // omega of the next cycle if the candidate is accepted
  double scr[4];   // scratch for one-off reductions (gmg_residual)
  double hist[GMG_MAX_HISTORY];
  double omegas[GMG_MAX_HISTORY];
  int acc[GMG_MAX_HISTORY];
};

// Device-resident state of the mixed-precision iterative refinement.
struct IRState {
  double snorm;    // ||sigma|| (FP64, active cells)
  double rnorm;    // latest ||sigma - A x|| (FP64)
  double beta;     // scale of the current correction problem
  double rtol;
  int outer;       // refinement steps applied
  int done;
  int status;
  int max_outer;
  int inner_total;
  int n_active;
  int pad0, pad1;
  double inner_base;  // inner tolerance asked for by the caller
  double target;      // ir_target of the parameters (0: inner_base alone)
  double inner_rtol;  // inner tolerance of the next outer step
  double hist[GMG_MAX_HISTORY];
  int inner[GMG_MAX_HISTORY];
};

// Inner tolerance of the outer step that starts from residual norm rn: the
// caller's inner tolerance, raised to target * rtol * ||sigma|| / rn when that
// is larger, so that the inner solve stops once the correction brings the
// outer residual within reach of the outer tolerance instead of always
// reducing its own residual by the full inner factor.
__device__ inline double ir_inner_tolerance(const IRState* ir, double rn) {
  if (ir->target > 0.0 && rn > 0.0)
    return fmax(ir->inner_base, ir->target * ir->rtol * ir->snorm / rn);
  return ir->inner_base;
}

// Status of a solve (or refinement) state that met a non-finite norm: NaN or
// Inf in sigma, in the initial guess or in the faces, or an overflow.  The
// solve stops at once; the host reports it as GMG_EINVAL.
constexpr int kStNonFinite = GMG_EINVAL;

// Adaptive-relaxation constants, passed by value.
struct OmegaRule {
  double omega_min, omega_max, theta_dec, theta_inc;
  int rollback;
};

constexpr int BX = 128, BY = 2, BT = BX * BY;  // cell-kernel block: two waves per row

// Uniform bricks: BX x BY x 2 cells of a level in which every face of
// direction d reads the same value u_d (bit for bit), the high faces of the
// brick's last column, row and plane included, except the faces of a low wall,
// which read +0.  (A high wall's face is never read: the stencil takes it as
// zero.)  The residual kernels take such a block's faces from u and the wall
// flags of each cell instead of loading them: the same values, the same
// arithmetic, bitwise the same result.  In immersed-boundary problems the faces
// are 1 (times the coarsening factors on coarse levels) away from the bodies,
// so most bricks qualify.
constexpr int kUBZ = 2;  // planes per brick
struct UBrick {
  double u[3];  // the faces of x, y, z (as read through ldL)
  int ok;       // 1: uniform
  int act;      // 1: every cell of the brick is active (D != 0)
};

}  // namespace gmg
