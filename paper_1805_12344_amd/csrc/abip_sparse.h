// Sparse engine: one LP with A in CSR, the linear step by preconditioned CG
// on G = I + A A^T (Section 4.4, indirect variant).  Internal header.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include "abip_internal.h"

// per-workgroup partial sums: slot k of workgroup b at part[k * nbp + b]
// (one value's partials are contiguous, so the reduction reads them coalesced)
#define SP_PS 32
#define SP_COL 0       // 7 column-side sums of the check
#define SP_ROW 7       // 12 row-side sums: 5 of the check, one unused, r^T r and t^T t of the CG start,
                       // 4 border dots of a
#define SP_BB 26       // the five sums of the adaptive beta's estimate (Section 4.3)
#define SP_CG 19       // per CG iteration: r^T u, w^T u, r^T r, then b^T a, bbar^T a, (A c)^T a, (A cbar)^T a

// CG state of one row i of G a = t, read together by the column pass of every
// workgroup (one 32-byte record instead of four scattered loads):
// r = residual, w = G u, s = G p, idg = 1 / diag(G)_i.
struct __align__(32) SpRow {
    double r, w, s, idg;
};

struct SpArgs {
    int32_t m, n;
    int64_t nnz;
    int32_t LA, LT;                      // lanes per row of CSR(A), of CSR(A^T) (global-memory passes)
    const int32_t* rp; const int32_t* ci; const double* va;     // CSR(A)
    const int32_t* rpt; const int32_t* cit; const double* vat;  // CSR(A^T)
    const double* dG;                    // 1 + ||A_{i,:}||^2 (Jacobi preconditioner of G)
    // constants (pools of the dense engine, one LP)
    const double *b, *bbar, *Ac, *Acb, *Zy0, *Zy1;              // m
    const double *C, *CB, *Zx0, *Zx1, *ATZy0, *ATZy1;          // n
    // state and work vectors (written during the solve)
    double *Y, *X, *S;                   // iterate (Y: m, X, S: n)
    double *Y0, *X0, *S0, *Y1, *X1, *S1; // adaptive beta: start point and first probe
    double *ATY, *ATA;                   // n: A^T y of the current iterate, A^T a of the last solve
    double *a, *z, *p;                   // m: CG solution (warm start), u = D^{-1} r, search direction
    SpRow* rw;                           // m: r, G u, G p, 1 / diag(G)
    SpRow* rw2;                          // m: the second record buffer of the explicit-G CG
    // explicit G~ = A A^T in CSR (null: the CG multiplies by A^T then A)
    const int32_t* grp; const int32_t* gci; const double* gva;
    int32_t LG;                          // lanes per row of G~
    double *q1;                          // n: A^T u of the next CG iterate
    double* part;                        // SP_PS * nbp partial sums
    int32_t nbp;                         // workgroup capacity of part (>= gridDim.x)
    int32_t lds_bytes;                   // dynamic LDS of the launch (0: no LDS-resident slices)
    unsigned* bar;                       // grid barrier: counter, generation
    int* err;                            // set when a grid barrier times out
    LPCtrl* lc;                          // scalars in / out
    SolveParams prm;
    double cg_tol;                       // relative floor: stop CG when ||r|| <= cg_tol ||t||
    int32_t cg_max;
    int32_t cg_rule;                     // 0: also stop at 0.1 ||Q u - v|| / (1 + k); 1: floor only
    int64_t fixed_iters;                 // > 0: exactly this many updates, no tests or restarts
};

// Contiguous share [lo, hi) of `total` items for workgroup `b` of `nb`
// (the same split on the host and on the device).
__host__ __device__ inline void sp_share(int total, int b, int nb, int* lo, int* hi) {
    const int per = (total + nb - 1) / nb;
    const int l = (int)((int64_t)b * per < total ? (int64_t)b * per : total);
    *lo = l;
    *hi = (l + per < total) ? l + per : total;
}

// LDS bytes of one workgroup's slices: CSR(A^T) rows of its columns (tnc rows,
// tne entries) and CSR(A) rows of its rows (anr rows, ane entries), with a
// product buffer for the larger of the two.
__host__ __device__ inline int64_t sp_slice_bytes(int tnc, int tne, int anr, int ane) {
    const int pe = tne > ane ? tne : ane;
    return 8 * ((int64_t)tne + ane + pe) + 4 * ((int64_t)tne + ane + tnc + 1 + anr + 1);
}

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
hipError_t sp_gram_count(const SpArgs& g, int32_t* cnt, hipStream_t st);
hipError_t sp_gram_fill(const SpArgs& g, const int32_t* grp, int32_t* gci, double* gva, hipStream_t st);
hipError_t sp_scan(const int32_t* cnt, int32_t n, int32_t* ptr, hipStream_t st);
hipError_t sp_set_lds_limit(int bytes);
int sp_max_blocks(int cu_count, int lds_bytes);
