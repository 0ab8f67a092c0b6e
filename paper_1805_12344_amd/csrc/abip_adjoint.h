// Adjoint of the converged fixed point for a handle that holds one large LP:
// the dense one-large-LP engine (A and G^{-1} in the pools) and the sparse
// engine (CSR A, CG on G).  Internal header.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include "abip_internal.h"
#include "abip_sparse.h"

// Everything one application of the transposed ADMM step needs.
struct BigAdj {
    int32_t m, n, ld;
    bool sparse;
    const double* A;             // dense: column-major ld x n (FP64 pool)
    const double* G;             // dense: G^{-1}, ld x m column-major (FP64 pool)
    SpArgs sp;                   // sparse: the engine's arguments (CSR(A), CSR(A^T), CG work vectors)
    int32_t sp_nb;               // sparse: workgroups of the cooperative CG launch
    double cg_tol;               // sparse: relative CG tolerance of each G solve
    int32_t cg_max;              // sparse: CG iteration cap of each G solve
    int64_t* cg_iters;           // sparse: device word for the CG iteration count
    const double *X, *S, *Y;     // the iterate (x, s: n; y: m)
    const double *b, *bbar, *C, *CB;               // HSD constants
    const double *zy0, *zy1, *zx0, *zx1;           // border of I - Q (Z_y: m, Z_x: n)
    LPCtrl cl;                   // host copy of the LP's control block (tau, kappa, theta, K_A^{-1})
    double alpha;                // relaxation of Algorithm 2
    double* ws;                  // device workspace of big_adj_ws_doubles(m, n, ld) doubles
};

int64_t big_adj_ws_doubles(int32_t m, int32_t n, int32_t ld);

// Solve (I - J^T) lam = dL/dz by BiCGSTAB and contract lam into dL/dc, dL/db
// and (dA non-null) dL/dA: row-major m x n for a dense LP, the nnz values in
// the CSR order of A (rp, ci) for a sparse one.  Host-driven: one host
// synchronisation per scalar of the recurrence.  *iters, *rel: host outputs.
// A sparse G solve that ends at a timed-out grid barrier sets *barrier_err.
hipError_t big_adjoint(const BigAdj& B, const double* win, double* dc, double* db, double* dA,
                       const int32_t* rp, const int32_t* ci, int64_t max_iters, double tol, int64_t* iters,
                       double* rel, int* barrier_err, hipStream_t st);

// x1^T y1 and (x2 non-null) x2^T y2 by partial sums added on the host in
// block order; part: 2 * 512 doubles of device scratch.
hipError_t big_dot2(const double* x1, const double* y1, const double* x2, const double* y2, int64_t N,
                    double* part, double* s0, double* s1, hipStream_t st);
