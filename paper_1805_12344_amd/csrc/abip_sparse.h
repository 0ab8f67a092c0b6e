// Sparse engine: one LP with A in CSR, the linear step by preconditioned CG
// on G = I + A A^T (Section 4.4, indirect variant).  Internal header.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include "abip_internal.h"

// per-workgroup partial sums (slots of SP_PS doubles per workgroup)
#define SP_PS 32
#define SP_COL 0       // 7 column-side sums of the check
#define SP_ROW 8       // 5 row-side sums of the check
#define SP_CG 13       // r^T z, r^T r, t^T t
#define SP_BD 16       // b^T a, bbar^T a, (A c)^T a, (A cbar)^T a
#define SP_PQ 20       // p^T G p

struct SpArgs {
    int32_t m, n;
    int64_t nnz;
    int32_t LA, LT;                      // lanes per row of CSR(A), of CSR(A^T)
    const int32_t* rp; const int32_t* ci; const double* va;     // CSR(A)
    const int32_t* rpt; const int32_t* cit; const double* vat;  // CSR(A^T)
    const double* dG;                    // 1 + ||A_{i,:}||^2 (Jacobi preconditioner of G)
    // constants (pools of the dense engine, one LP)
    const double *b, *bbar, *Ac, *Acb, *Zy0, *Zy1;              // m
    const double *C, *CB, *Zx0, *Zx1, *ATZy0, *ATZy1;          // n
    // state and work vectors (written during the solve)
    double *Y, *X, *S;                   // iterate (Y: m, X, S: n)
    double *ATY, *ATA;                   // n: A^T y of the current iterate, A^T a of the last solve
    double *a, *r, *z, *p, *q, *sv;      // m: CG solution (warm start) and work vectors
                                         //    (z = u, q = w = G u, sv = s = G p)
    double *q1;                          // n: A^T p
    double* part;                        // gridDim.x * SP_PS partial sums
    unsigned* bar;                       // grid barrier: counter, generation
    int* err;                            // set when a grid barrier times out
    LPCtrl* lc;                          // scalars in / out
    SolveParams prm;
    double cg_tol;                       // relative floor: stop CG when ||r|| <= cg_tol ||t||
    int32_t cg_max;
    int32_t cg_rule;                     // 0: also stop at 0.1 ||Q u - v|| / (1 + k); 1: floor only
    int64_t fixed_iters;                 // > 0: exactly this many updates, no tests or restarts
};

// setup helpers (abip_solve_sparse.hip)
hipError_t sp_validate_rows(const SpArgs& g, int* flag, hipStream_t st);
hipError_t sp_validate_entries(const SpArgs& g, int* flag, hipStream_t st);
hipError_t sp_check_finite(const double* v, int64_t len, int* flag, int bit, hipStream_t st);
hipError_t sp_affine(const double* x, double a, double c, int64_t len, double* out, hipStream_t st);
hipError_t sp_transpose(SpArgs& g, int32_t* rpt, int32_t* cit, double* vat, int32_t* cursor, hipStream_t st);
hipError_t sp_spmv(const int32_t* rp, const int32_t* ci, const double* va, int32_t rows, const double* v,
                   double alpha, const double* w, double beta, double* out, hipStream_t st);
hipError_t sp_rowsq(const SpArgs& g, double* dG, hipStream_t st);
hipError_t sp_dots(const double* x, const double* const* ys, int ny, int64_t len, double* partial, int nblk,
                   hipStream_t st);
hipError_t sp_cg_solve(SpArgs g, const double* rhs, double* out, double tol, int32_t maxit, int nb,
                       int64_t* iters, hipStream_t st);
hipError_t sp_solve(SpArgs g, int nb, hipStream_t st);
int sp_max_blocks(int cu_count);
