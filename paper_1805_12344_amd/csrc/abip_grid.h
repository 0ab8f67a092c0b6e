// Control block and arguments of the grid engine (shared by host and device code).
#pragma once
#include "abip_internal.h"

// rows per workgroup of k_grid_red (host and device)
#define GRID_RED_ROWS 8

// Host-visible control block of the grid engine (device memory).
struct GridCtl {
    // the state the next k_grid_col starts from
    double tau, kappa, theta, mu;
    double p0, p1;             // border solution of the pending update (mode OP_PROX)
    int32_t mode;              // OP_PROX / OP_RESTART / OP_REFRESH for the next column pass
    int32_t phase;             // 0: FP32-streamed data, 1: FP64
    int32_t status;            // 0 while running
    int32_t ybuf;              // which y buffer holds the current y
    int32_t first;             // 1 until the first decision
    int32_t exit_pend;         // 1: the next FP64 check measures the FP32 phase's exit (kfx)
    int64_t iters, iters64, ipm, cp32, cp64, passes;
    int64_t fixed_left;        // fixed mode: updates still to run
    int32_t fixed_mode;        // 1: run exactly fixed_left updates, no tests or restarts
    int32_t decide;            // 1: this block describes a pass whose decision is pending
    // last check
    double pres, dres, gap, pobj, dobj, by, cx;
    double kfx;                // relative KKT of the FP32 phase's last iterate with FP64 data
    // scalars of the state produced by the last column pass (for the decision)
    double tau_n, kappa_n, theta_n;
    StallTrack stall;          // FP32 precision-floor test of the current inner loop
    // adaptive beta (Section 4.3)
    double beta;               // the outer iteration's beta (settings.beta unless chosen)
    int32_t bbf;               // GBB_* bits
};

// GridCtl.bbf: adaptive beta on (a full solve), the outer iteration's choice
// pending, the stage of the choice (1 / 2: first / second probe, 3: start point
// restored), the paused pass was an update, and resume: the pass's decision was
// taken before a beta step paused the grid (status -2), so the next column pass
// takes the paused pass's sums without deciding again.
#define GBB_ON 1
#define GBB_PEND 2
#define GBB_STAGE_SHIFT 2      // two bits
#define GBB_WAS_UPDATE 16
#define GBB_RESUME 32

// The rest of the choice's state, touched only by k_grid_bb_step (one workgroup,
// while the grid is paused) and by the init / finish kernels.
struct GridBB {
    double bbs[6];             // tau, kappa, theta of the start point and of the first probe
    int64_t bbp;               // probe updates
    int32_t est, bbe;          // estimates of this choice (redos included) / of the solve
};

struct GridArgs {
    int32_t m, n, ld;
    int32_t NB, NR, NG;        // workgroups of the three kernels
    int32_t cw, gw;            // columns (column pairs when n2 > 0) per workgroup (k_grid_col, k_grid_ginv)
    int32_t n2;                // A = [A0, -A0]: n / 2, and k_grid_col reads A0 only; 0 otherwise
    const double* A64; const float* A32;
    const double* G64; const float* G32;
    const double *b, *bbar, *Ac, *Acb, *Zy0, *Zy1;
    const double *C, *CB, *Zx0, *Zx1;
    double *X, *S;
    double *X0, *S0, *X1, *S1, *Y0, *Y1;   // adaptive beta: start point and first probe
    double* Y2;                // 2 * ld: current / next y
    double* Pf;                // NB * ld partial A(x+s)
    double* Px;                // NB * ld partial A x
    double* pcol;              // 2 x pcol_stride column-side sums (NB * 8 used), by pass parity
    int32_t pcol_stride;
    double* prow;              // NR * 8 row-side sums
    double* pa;                // NG * 4 border dots of a
    double* t;                 // ld
    double* a;                 // ld
    GridCtl* ctl;              // the pass's state: written by k_grid_col (workgroup 0), read by
                               // k_grid_red / k_grid_ginv
    GridCtl* ctl_next;         // its copy for the next k_grid_col (written by k_grid_ginv's
                               // workgroup 0) and the host
    GridBB* bb;                // adaptive beta: the choice's state
    const LPCtrl* lc;          // K^{-1}, zbar, norms
    SolveParams prm;
};


int grid_nchw(int ld);
hipError_t grid_launch_iteration(int nchw, const GridArgs& g, hipStream_t st);
__global__ void k_grid_init(GridArgs g, double beta, int phase, int64_t fixed, int bb);
__global__ void k_grid_bb_step(GridArgs g);
__global__ void k_grid_pair_check(const double* A, int m, int ld, int n2, int* flag);
__global__ void k_grid_finish(GridArgs g, double* Ypool_slice, LPCtrl* lc);
__global__ void k_grid_from_state(GridArgs g, const double* Yslice, const LPCtrl* lc, int phase, int64_t fixed);
