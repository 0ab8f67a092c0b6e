// Adjoint of the converged fixed point for one large LP (dense one-large-LP
// engine, sparse engine).  The recurrence is the BiCGSTAB of the one-workgroup
// k_adjoint: (I - J^T) lam = dL/dz, J the linearised ADMM step of Algorithm 2
// at the final iterate, each product with J^T one transposed step through
// (I + Q)^{-T} = (I - Q)^{-1}.  Here every product is spread over the whole
// GPU and the host runs the scalar recurrence:
//   dense:  A wx and G^{-1} t by column-block partial sums (each workgroup a
//           256-row x cw-column tile of the column-major array, partials
//           summed in block order), A^T a by one wave per column;
//   sparse: A wx and A^T a by CSR products, G^{-1} t by the engine's
//           cooperative Jacobi-preconditioned CG.
// Dot products: one partial per workgroup, added on the host in block order
// (the same sum for the same inputs on every run).
#include <hip/hip_runtime.h>
#include <cmath>
#include <vector>
#include "abip_adjoint.h"

#define AB_T 256            // threads of every kernel here
#define AB_NB 512           // maximum workgroups of a partial-sum launch
#define AB_NCB 64           // maximum column blocks of the dense products

namespace {

inline int nblk(int64_t N) {
    const int64_t b = (N + AB_T - 1) / AB_T;
    return (int)(b < 1 ? 1 : (b > AB_NB ? AB_NB : b));
}

// scalars of one application that the elementwise tail needs
struct AbScal {
    double alpha, rt;            // rt = tau / (tau + kappa)
    double KA00, KA01, KA10, KA11;
};

// Workspace carve-up (doubles): seven Krylov vectors of N = m + 2n + 3, then
// wx, d (n each), wb (m + n + 2), t, a (m each), the dense partials
// (AB_NCB x ld), three partial-dot areas (2 x AB_NB each).
struct AbWs {
    double *LAM, *Rv, *R0, *Pv, *V, *Sv, *Tv;
    double *WX, *Dv, *WB, *t, *a, *part, *pv, *pa, *pd;
};

AbWs carve(double* ws, int m, int n, int ld) {
    const int64_t N = (int64_t)m + 2 * (int64_t)n + 3;
    AbWs w;
    double* p = ws;
    w.LAM = p; p += N; w.Rv = p; p += N; w.R0 = p; p += N; w.Pv = p; p += N;
    w.V = p; p += N; w.Sv = p; p += N; w.Tv = p; p += N;
    w.WX = p; p += n; w.Dv = p; p += n; w.WB = p; p += (int64_t)m + n + 2;
    w.t = p; p += m; w.a = p; p += m;
    w.part = p; p += (int64_t)AB_NCB * ld;
    w.pv = p; p += 2 * AB_NB; w.pa = p; p += 2 * AB_NB; w.pd = p; p += 2 * AB_NB;
    return w;
}

}  // namespace

int64_t big_adj_ws_doubles(int32_t m, int32_t n, int32_t ld) {
    const int64_t N = (int64_t)m + 2 * (int64_t)n + 3;
    return 7 * N + 2 * (int64_t)n + ((int64_t)m + n + 2) + 2 * (int64_t)m + (int64_t)AB_NCB * ld + 6 * AB_NB;
}

// ---- partial dot products -------------------------------------------------
// part[blk] = sum over the block's share of x1 . y1, part[nb + blk] of x2 . y2
// (x2 null: 0)
__global__ __launch_bounds__(AB_T) void k_ab_dot2(const double* __restrict__ x1, const double* __restrict__ y1,
                                                  const double* __restrict__ x2, const double* __restrict__ y2,
                                                  int64_t N, double* __restrict__ part) {
    __shared__ double sb[2 * (AB_T / 64)];
    double v[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * AB_T + threadIdx.x; i < N; i += (int64_t)gridDim.x * AB_T) {
        v[0] = fma(x1[i], y1[i], v[0]);
        if (x2) v[1] = fma(x2[i], y2[i], v[1]);
    }
    block_sum_n<2>(v, sb);
    if (threadIdx.x == 0) { part[blockIdx.x] = v[0]; part[gridDim.x + blockIdx.x] = v[1]; }
}

// ---- Krylov vector updates --------------------------------------------------
// g = dL/dz = (0, w / tau, -w^T x / tau^2, 0, 0, 0); r = r0 = g, p = v = 0;
// lam = g when no iteration is asked for (one contraction of dL/dz), else 0
__global__ __launch_bounds__(AB_T) void k_ab_init(const double* __restrict__ win, int m, int n, double tau,
                                                  double wx, int lam_g, double* LAM, double* Rv, double* R0,
                                                  double* Pv, double* V, int64_t N) {
    for (int64_t i = (int64_t)blockIdx.x * AB_T + threadIdx.x; i < N; i += (int64_t)gridDim.x * AB_T) {
        double g = 0.0;
        if (i >= m && i < (int64_t)m + n) g = win[i - m] / tau;
        else if (i == (int64_t)m + n) g = -wx / (tau * tau);
        LAM[i] = lam_g ? g : 0.0;
        Rv[i] = g; R0[i] = g; Pv[i] = 0.0; V[i] = 0.0;
    }
}

// restart with the current residual as the shadow: r0 = r, p = v = 0
__global__ __launch_bounds__(AB_T) void k_ab_restart(double* R0, double* Pv, double* V, const double* Rv,
                                                     int64_t N) {
    for (int64_t i = (int64_t)blockIdx.x * AB_T + threadIdx.x; i < N; i += (int64_t)gridDim.x * AB_T) {
        R0[i] = Rv[i]; Pv[i] = 0.0; V[i] = 0.0;
    }
}

// p = r + beta (p - om v)
__global__ __launch_bounds__(AB_T) void k_ab_p(double* Pv, const double* Rv, const double* V, double beta,
                                               double om, int64_t N) {
    for (int64_t i = (int64_t)blockIdx.x * AB_T + threadIdx.x; i < N; i += (int64_t)gridDim.x * AB_T)
        Pv[i] = Rv[i] + beta * (Pv[i] - om * V[i]);
}

// s = r - al v, with partials of s^T s
__global__ __launch_bounds__(AB_T) void k_ab_s(double* Sv, const double* Rv, const double* V, double al, int64_t N,
                                               double* part) {
    __shared__ double sb[AB_T / 64];
    double v[1] = {0.0};
    for (int64_t i = (int64_t)blockIdx.x * AB_T + threadIdx.x; i < N; i += (int64_t)gridDim.x * AB_T) {
        const double s = Rv[i] - al * V[i];
        Sv[i] = s;
        v[0] = fma(s, s, v[0]);
    }
    block_sum_n<1>(v, sb);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// lam += al p
__global__ __launch_bounds__(AB_T) void k_ab_axpy(double* LAM, const double* Pv, double al, int64_t N) {
    for (int64_t i = (int64_t)blockIdx.x * AB_T + threadIdx.x; i < N; i += (int64_t)gridDim.x * AB_T)
        LAM[i] += al * Pv[i];
}

// lam += al p + om s; r = s - om t; partials of r^T r and r0^T r
__global__ __launch_bounds__(AB_T) void k_ab_lr(double* LAM, double* Rv, const double* Pv, const double* Sv,
                                                const double* Tv, const double* R0, double al, double om, int64_t N,
                                                double* part) {
    __shared__ double sb[2 * (AB_T / 64)];
    double v[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * AB_T + threadIdx.x; i < N; i += (int64_t)gridDim.x * AB_T) {
        LAM[i] += al * Pv[i] + om * Sv[i];
        const double r = Sv[i] - om * Tv[i];
        Rv[i] = r;
        v[0] = fma(r, r, v[0]);
        v[1] = fma(R0[i], r, v[1]);
    }
    block_sum_n<2>(v, sb);
    if (threadIdx.x == 0) { part[blockIdx.x] = v[0]; part[gridDim.x + blockIdx.x] = v[1]; }
}

// ---- one transposed ADMM step ----------------------------------------------
// wx_j = rx_j in_x[j] + (rx_j - 1) in_s[j], rx_j = x_j / (x_j + s_j)
__global__ __launch_bounds__(AB_T) void k_ab_wx(const double* __restrict__ X, const double* __restrict__ S,
                                                const double* __restrict__ in, int m, int n, double* __restrict__ WX) {
    const int j = blockIdx.x * AB_T + threadIdx.x;
    if (j >= n) return;
    const double rx = X[j] / (X[j] + S[j]);
    WX[j] = rx * in[m + j] + (rx - 1.0) * in[m + n + 2 + j];
}

// Column-block partial products of a column-major array M (leading dimension
// ld): part[cb * ld + r] = sum_{j in block cb} M[j ld + r] v[j] for r < rows.
// Workgroup (rb, cb): rows rb*256 ..., columns cb*cw ...; every column read is
// 256 consecutive doubles.
__global__ __launch_bounds__(AB_T) void k_ab_gemv(const double* __restrict__ M, int ld, int rows, int cols, int cw,
                                                  const double* __restrict__ v, double* __restrict__ part) {
    const int r = blockIdx.x * AB_T + threadIdx.x;
    if (r >= rows) return;
    const int j0 = blockIdx.y * cw;
    const int j1 = min(cols, j0 + cw);
    const double* Mr = M + r;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int j = j0;
    for (; j + 3 < j1; j += 4) {
        s0 = fma(Mr[(int64_t)j * ld], v[j], s0);
        s1 = fma(Mr[(int64_t)(j + 1) * ld], v[j + 1], s1);
        s2 = fma(Mr[(int64_t)(j + 2) * ld], v[j + 2], s2);
        s3 = fma(Mr[(int64_t)(j + 3) * ld], v[j + 3], s3);
    }
    for (; j < j1; ++j) s0 = fma(Mr[(int64_t)j * ld], v[j], s0);
    part[(int64_t)blockIdx.y * ld + r] = (s0 + s1) + (s2 + s3);
}

// out[r] = sc (base[r] + sum_cb part[cb ld + r]) (base may be null); with u1
// non-null, partials of u1^T out and u2^T out per workgroup into pdot
__global__ __launch_bounds__(AB_T) void k_ab_red(const double* __restrict__ part, int ld, int rows, int ncb,
                                                 const double* __restrict__ base, double sc, double* __restrict__ out,
                                                 const double* __restrict__ u1, const double* __restrict__ u2,
                                                 double* __restrict__ pdot) {
    __shared__ double sb[2 * (AB_T / 64)];
    double v[2] = {0.0, 0.0};
    for (int r = blockIdx.x * AB_T + threadIdx.x; r < rows; r += gridDim.x * AB_T) {
        double s = 0.0;
        for (int cb = 0; cb < ncb; ++cb) s += part[(int64_t)cb * ld + r];
        const double o = sc * ((base ? base[r] : 0.0) + s);
        out[r] = o;
        if (u1) { v[0] = fma(u1[r], o, v[0]); v[1] = fma(u2[r], o, v[1]); }
    }
    if (u1) {
        block_sum_n<2>(v, sb);
        if (threadIdx.x == 0) { pdot[blockIdx.x] = v[0]; pdot[gridDim.x + blockIdx.x] = v[1]; }
    }
}

// d_j = alpha wx_j - A_{:,j}^T a, one wave per column; partials of c^T d, cbar^T d
__global__ __launch_bounds__(AB_T) void k_ab_atd(const double* __restrict__ A, int ld, int m, int n,
                                                 const double* __restrict__ a, const double* __restrict__ WX,
                                                 double alpha, const double* __restrict__ C,
                                                 const double* __restrict__ CB, double* __restrict__ Dv,
                                                 double* __restrict__ pdot) {
    __shared__ double sb[2 * (AB_T / 64)];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double v[2] = {0.0, 0.0};
    for (int j = blockIdx.x * (AB_T / 64) + wave; j < n; j += gridDim.x * (AB_T / 64)) {
        const double* col = A + (int64_t)j * ld;
        double s0 = 0.0, s1 = 0.0;
        int i = lane;
        for (; i + 64 < m; i += 128) { s0 = fma(col[i], a[i], s0); s1 = fma(col[i + 64], a[i + 64], s1); }
        if (i < m) s0 = fma(col[i], a[i], s0);
        const double tot = wave_sum(s0 + s1);
        if (lane == 0) {
            const double dj = alpha * WX[j] - tot;
            Dv[j] = dj;
            v[0] = fma(C[j], dj, v[0]);
            v[1] = fma(CB[j], dj, v[1]);
        }
    }
    block_sum_n<2>(v, sb);
    if (threadIdx.x == 0) { pdot[blockIdx.x] = v[0]; pdot[gridDim.x + blockIdx.x] = v[1]; }
}

// Sum of part[0 .. np) in a fixed order (lane-strided, then the wave's tree);
// called by one whole wave.
__device__ double ab_wave_total(const double* part, int np) {
    const int lane = threadIdx.x & 63;
    double s = 0.0;
    for (int k = lane; k < np; k += 64) s += part[k];
    return wave_sum(s);
}

// The rest of the step: with b^T a, bbar^T a (pa, npa partials each) and
// c^T d, cbar^T d (pd, npd), p = K_A^{-1} q for the border's rank-2 term,
// wb = the (I - Q)^{-1} solution, out = in - J^T in.
__global__ __launch_bounds__(AB_T) void k_ab_fin(const double* __restrict__ in, double* __restrict__ out,
                                                 const double* __restrict__ a, const double* __restrict__ Dv,
                                                 const double* __restrict__ WX, double* __restrict__ WB,
                                                 const double* __restrict__ zy0, const double* __restrict__ zy1,
                                                 const double* __restrict__ zx0, const double* __restrict__ zx1,
                                                 const double* __restrict__ pa, int npa,
                                                 const double* __restrict__ pd, int npd, AbScal sc, int m, int n) {
    __shared__ double sp[2];
    if (threadIdx.x < 64) {
        const double ba = ab_wave_total(pa, npa), bba = ab_wave_total(pa + npa, npa);
        const double cd = ab_wave_total(pd, npd), cbd = ab_wave_total(pd + npd, npd);
        if (threadIdx.x == 0) {
            const int OT = m + n, OH = m + n + 1, OK = m + 2 * n + 2;
            const double wt = sc.rt * in[OT] + (sc.rt - 1.0) * in[OK];
            const double q0 = sc.alpha * wt + (ba - cd);
            const double q1 = sc.alpha * in[OH] + (-bba + cbd);
            sp[0] = sc.KA00 * q0 + sc.KA01 * q1;
            sp[1] = sc.KA10 * q0 + sc.KA11 * q1;
        }
    }
    __syncthreads();
    const double p0 = sp[0], p1 = sp[1];
    const double alpha = sc.alpha;
    const int i = blockIdx.x * AB_T + threadIdx.x;
    if (i < m) {
        const double wby = a[i] - zy0[i] * p0 - zy1[i] * p1;
        WB[i] = wby;
        out[i] = in[i] - ((1.0 - alpha) * in[i] + wby);
    } else if (i < m + n) {
        const int j = i - m, OX = m, OS = m + n + 2;
        const double wbx = Dv[j] - zx0[j] * p0 - zx1[j] * p1;
        const double wx = WX[j];
        WB[m + j] = wbx;
        out[OX + j] = in[OX + j] - ((1.0 - alpha) * wx + wbx);
        out[OS + j] = in[OS + j] - (-wx + wbx);
    } else if (i == m + n) {
        const int OT = m + n, OH = m + n + 1, OK = m + 2 * n + 2;
        const double wt = sc.rt * in[OT] + (sc.rt - 1.0) * in[OK];
        WB[m + n] = p0;
        WB[m + n + 1] = p1;
        out[OT] = in[OT] - ((1.0 - alpha) * wt + p0);
        out[OH] = in[OH] - ((1.0 - alpha) * in[OH] + p1);
        out[OK] = in[OK] - (-wt + p0);
    }
}

// ---- contraction with d(Q u)/d(c, b, A) ----------------------------------
__global__ __launch_bounds__(AB_T) void k_ab_grad(const double* __restrict__ X, const double* __restrict__ Y,
                                                  const double* __restrict__ WB, int m, int n, double tau,
                                                  double theta, double* __restrict__ dc, double* __restrict__ db) {
    const int i = blockIdx.x * AB_T + threadIdx.x;
    const double zt = WB[m + n], zh = WB[m + n + 1];
    if (i < n) {
        const double xj = X[i];
        dc[i] = -(WB[m + i] * (tau - theta) + zt * (theta - xj) + zh * (xj - tau));
    } else if (i < n + m) {
        const int r = i - n;
        const double yi = Y[r];
        db[r] = -(WB[r] * (theta - tau) + zt * yi - zh * yi);
    }
}

// dL/dA row-major m x n: workgroup (jb, ib) writes 256 consecutive entries of row ib
__global__ __launch_bounds__(AB_T) void k_ab_grad_dense(const double* __restrict__ X, const double* __restrict__ Y,
                                                        const double* __restrict__ WB, int m, int n, double theta,
                                                        double* __restrict__ dA) {
    const int j = blockIdx.x * AB_T + threadIdx.x;
    if (j >= n) return;
    const double zh = WB[m + n + 1];
    const double xj = X[j], wbx = WB[m + j];
    for (int i = blockIdx.y; i < m; i += gridDim.y) {
        const double yi = Y[i];
        dA[(int64_t)i * n + j] = -(WB[i] * (xj - theta) - wbx * yi + zh * yi);
    }
}

// dL/dA on the pattern of CSR(A): the nnz values in its order, one thread per row
__global__ __launch_bounds__(AB_T) void k_ab_grad_csr(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                      const double* __restrict__ X, const double* __restrict__ Y,
                                                      const double* __restrict__ WB, int m, int n, double theta,
                                                      double* __restrict__ dA) {
    const int i = blockIdx.x * AB_T + threadIdx.x;
    if (i >= m) return;
    const double zh = WB[m + n + 1], yi = Y[i], wby = WB[i];
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
        const int j = ci[e];
        dA[e] = -(wby * (X[j] - theta) - WB[m + j] * yi + zh * yi);
    }
}

__global__ __launch_bounds__(AB_T) void k_ab_fill(double* p, int64_t len, double v) {
    for (int64_t i = (int64_t)blockIdx.x * AB_T + threadIdx.x; i < len; i += (int64_t)gridDim.x * AB_T) p[i] = v;
}

// ---- host side --------------------------------------------------------------
namespace {

#define ABCHK(call) do { hipError_t e_ = (call); if (e_ != hipSuccess) return e_; } while (0)

// the two partial sums of a launch of nb workgroups, added in block order
hipError_t host_sums(const double* dpart, int nb, double* s0, double* s1, hipStream_t st) {
    double h[2 * AB_NB];
    ABCHK(hipMemcpyAsync(h, dpart, sizeof(double) * 2 * nb, hipMemcpyDeviceToHost, st));
    ABCHK(hipStreamSynchronize(st));
    double a = 0.0, b = 0.0;
    for (int k = 0; k < nb; ++k) { a += h[k]; b += h[nb + k]; }
    *s0 = a;
    if (s1) *s1 = b;
    return hipSuccess;
}

hipError_t dot2(const double* x1, const double* y1, const double* x2, const double* y2, int64_t N, double* part,
                double* s0, double* s1, hipStream_t st) {
    const int nb = nblk(N);
    hipLaunchKernelGGL(k_ab_dot2, dim3(nb), dim3(AB_T), 0, st, x1, y1, x2, y2, N, part);
    ABCHK(hipGetLastError());
    return host_sums(part, nb, s0, s1, st);
}

// out = in - J^T in (wb left in W.WB)
hipError_t apply_op(const BigAdj& B, const AbWs& W, const double* in, double* out, int* barrier_err,
                    hipStream_t st) {
    const int m = B.m, n = B.n;
    hipLaunchKernelGGL(k_ab_wx, dim3((n + AB_T - 1) / AB_T), dim3(AB_T), 0, st, B.X, B.S, in, m, n, W.WX);
    ABCHK(hipGetLastError());
    int npa, npd;
    if (!B.sparse) {
        const int ld = B.ld, rb = (m + AB_T - 1) / AB_T;
        // t = alpha (in_y + A wx)
        int ncb = (n + 31) / 32;
        if (ncb > AB_NCB) ncb = AB_NCB;
        int cw = (n + ncb - 1) / ncb;
        ncb = (n + cw - 1) / cw;
        hipLaunchKernelGGL(k_ab_gemv, dim3(rb, ncb), dim3(AB_T), 0, st, B.A, ld, m, n, cw, W.WX, W.part);
        ABCHK(hipGetLastError());
        hipLaunchKernelGGL(k_ab_red, dim3(nblk(m)), dim3(AB_T), 0, st, W.part, ld, m, ncb, in, B.alpha, W.t,
                           nullptr, nullptr, nullptr);
        ABCHK(hipGetLastError());
        // a = G^{-1} t, with partials of b^T a, bbar^T a
        int ncg = (m + 31) / 32;
        if (ncg > AB_NCB) ncg = AB_NCB;
        int cg = (m + ncg - 1) / ncg;
        ncg = (m + cg - 1) / cg;
        hipLaunchKernelGGL(k_ab_gemv, dim3(rb, ncg), dim3(AB_T), 0, st, B.G, ld, m, m, cg, W.t, W.part);
        ABCHK(hipGetLastError());
        npa = nblk(m);
        hipLaunchKernelGGL(k_ab_red, dim3(npa), dim3(AB_T), 0, st, W.part, ld, m, ncg, nullptr, 1.0, W.a, B.b,
                           B.bbar, W.pa);
        ABCHK(hipGetLastError());
        // d = alpha wx - A^T a, with partials of c^T d, cbar^T d
        npd = (n + 3) / 4;
        if (npd > AB_NB) npd = AB_NB;
        hipLaunchKernelGGL(k_ab_atd, dim3(npd), dim3(AB_T), 0, st, B.A, ld, m, n, W.a, W.WX, B.alpha, B.C, B.CB,
                           W.Dv, W.pd);
        ABCHK(hipGetLastError());
    } else {
        const SpArgs& g = B.sp;
        ABCHK(sp_spmv(g.rp, g.ci, g.va, m, W.WX, B.alpha, in, B.alpha, W.t, st));        // alpha (A wx + in_y)
        ABCHK(sp_cg_solve(g, W.t, W.a, B.cg_tol, B.cg_max, B.sp_nb, B.cg_iters, st));   // a = G^{-1} t
        ABCHK(sp_spmv(g.rpt, g.cit, g.vat, n, W.a, -1.0, W.WX, B.alpha, W.Dv, st));      // alpha wx - A^T a
        npa = nblk(m);
        hipLaunchKernelGGL(k_ab_dot2, dim3(npa), dim3(AB_T), 0, st, B.b, W.a, B.bbar, W.a, (int64_t)m, W.pa);
        ABCHK(hipGetLastError());
        npd = nblk(n);
        hipLaunchKernelGGL(k_ab_dot2, dim3(npd), dim3(AB_T), 0, st, B.C, W.Dv, B.CB, W.Dv, (int64_t)n, W.pd);
        ABCHK(hipGetLastError());
        (void)barrier_err;
    }
    AbScal sc;
    sc.alpha = B.alpha;
    sc.rt = B.cl.tau / (B.cl.tau + B.cl.kappa);
    sc.KA00 = B.cl.KA00; sc.KA01 = B.cl.KA01; sc.KA10 = B.cl.KA10; sc.KA11 = B.cl.KA11;
    hipLaunchKernelGGL(k_ab_fin, dim3((m + n + 1 + AB_T - 1) / AB_T), dim3(AB_T), 0, st, in, out, W.a, W.Dv, W.WX,
                       W.WB, B.zy0, B.zy1, B.zx0, B.zx1, W.pa, npa, W.pd, npd, sc, m, n);
    return hipGetLastError();
}

}  // namespace

hipError_t big_dot2(const double* x1, const double* y1, const double* x2, const double* y2, int64_t N,
                    double* part, double* s0, double* s1, hipStream_t st) {
    return dot2(x1, y1, x2, y2, N, part, s0, s1, st);
}

hipError_t big_adjoint(const BigAdj& B, const double* win, double* dc, double* db, double* dA, const int32_t* rp,
                       const int32_t* ci, int64_t max_iters, double tol, int64_t* iters, double* rel_out,
                       int* barrier_err, hipStream_t st) {
    const int m = B.m, n = B.n;
    const int64_t N = (int64_t)m + 2 * (int64_t)n + 3;
    const AbWs W = carve(B.ws, m, n, B.ld);
    const LPCtrl& cl = B.cl;
    const double tau = cl.tau, theta = cl.theta;
    *barrier_err = 0;
    if ((cl.status != 1 && !(cl.flags & 4)) || !(tau > 0.0)) {      // nothing to differentiate
        hipLaunchKernelGGL(k_ab_fill, dim3(nblk(n)), dim3(AB_T), 0, st, dc, (int64_t)n, (double)NAN);
        hipLaunchKernelGGL(k_ab_fill, dim3(nblk(m)), dim3(AB_T), 0, st, db, (int64_t)m, (double)NAN);
        if (dA) {
            const int64_t len = B.sparse ? (int64_t)B.sp.nnz : (int64_t)m * n;
            hipLaunchKernelGGL(k_ab_fill, dim3(AB_NB), dim3(AB_T), 0, st, dA, len, (double)NAN);
        }
        ABCHK(hipGetLastError());
        *iters = 0;
        *rel_out = NAN;
        return hipStreamSynchronize(st);
    }
    const int nv = nblk(N);
    double wx;
    ABCHK(dot2(win, B.X, nullptr, nullptr, n, W.pv, &wx, nullptr, st));
    hipLaunchKernelGGL(k_ab_init, dim3(nv), dim3(AB_T), 0, st, win, m, n, tau, wx, max_iters == 0 ? 1 : 0, W.LAM,
                       W.Rv, W.R0, W.Pv, W.V, N);
    ABCHK(hipGetLastError());
    double g2;
    ABCHK(dot2(W.Rv, W.Rv, nullptr, nullptr, N, W.pv, &g2, nullptr, st));
    const double gnorm = std::sqrt(g2);
    double rho = 1.0, al = 1.0, om = 1.0, rel = 1.0;
    double rr = g2, rho1n = g2;          // r^T r; r0^T r for the next iteration
    int64_t it = 0;
    bool restart = false;
    if (gnorm > 0.0) {
        for (it = 1; it <= max_iters; ++it) {
            double rho1 = rho1n;
            // breakdown (r0 orthogonal to r, or a zero / non-finite step):
            // restart with the current residual as the shadow
            if (restart || !(std::fabs(rho1) > 0.0) || !std::isfinite(rho1)) {
                restart = false;
                hipLaunchKernelGGL(k_ab_restart, dim3(nv), dim3(AB_T), 0, st, W.R0, W.Pv, W.V, W.Rv, N);
                ABCHK(hipGetLastError());
                rho1 = rr;
                rho = 1.0; al = 1.0; om = 1.0;
            }
            const double beta = (rho1 / rho) * (al / om);
            hipLaunchKernelGGL(k_ab_p, dim3(nv), dim3(AB_T), 0, st, W.Pv, W.Rv, W.V, beta, om, N);
            ABCHK(hipGetLastError());
            ABCHK(apply_op(B, W, W.Pv, W.V, barrier_err, st));
            double rv;
            ABCHK(dot2(W.R0, W.V, nullptr, nullptr, N, W.pv, &rv, nullptr, st));
            if (!(std::fabs(rv) > 0.0) || !std::isfinite(rv)) { restart = true; continue; }
            al = rho1 / rv;
            if (!std::isfinite(al)) { restart = true; continue; }
            hipLaunchKernelGGL(k_ab_s, dim3(nv), dim3(AB_T), 0, st, W.Sv, W.Rv, W.V, al, N, W.pv);
            ABCHK(hipGetLastError());
            double sn2;
            ABCHK(host_sums(W.pv, nv, &sn2, nullptr, st));
            const double sn = std::sqrt(sn2);
            if (sn <= tol * gnorm) {
                hipLaunchKernelGGL(k_ab_axpy, dim3(nv), dim3(AB_T), 0, st, W.LAM, W.Pv, al, N);
                ABCHK(hipGetLastError());
                rel = sn / gnorm;
                break;
            }
            ABCHK(apply_op(B, W, W.Sv, W.Tv, barrier_err, st));
            double tt, ts;
            ABCHK(dot2(W.Tv, W.Tv, W.Tv, W.Sv, N, W.pv, &tt, &ts, st));
            om = (tt > 0.0 && std::isfinite(ts / tt)) ? ts / tt : 0.0;   // 0: half step, then restart
            hipLaunchKernelGGL(k_ab_lr, dim3(nv), dim3(AB_T), 0, st, W.LAM, W.Rv, W.Pv, W.Sv, W.Tv, W.R0, al, om, N,
                               W.pv);
            ABCHK(hipGetLastError());
            ABCHK(host_sums(W.pv, nv, &rr, &rho1n, st));
            rel = std::sqrt(rr) / gnorm;
            if (rel <= tol) break;
            rho = rho1;
            if (om == 0.0) restart = true;         // stagnation
        }
    }
    // zeta = wb(lam): one more application (its output is discarded into Tv)
    ABCHK(apply_op(B, W, W.LAM, W.Tv, barrier_err, st));
    hipLaunchKernelGGL(k_ab_grad, dim3((m + n + AB_T - 1) / AB_T), dim3(AB_T), 0, st, B.X, B.Y, W.WB, m, n, tau,
                       theta, dc, db);
    ABCHK(hipGetLastError());
    if (dA) {
        if (B.sparse) {
            hipLaunchKernelGGL(k_ab_grad_csr, dim3((m + AB_T - 1) / AB_T), dim3(AB_T), 0, st, rp, ci, B.X, B.Y, W.WB,
                               m, n, theta, dA);
        } else {
            const int gy = m < 65535 ? m : 65535;
            hipLaunchKernelGGL(k_ab_grad_dense, dim3((n + AB_T - 1) / AB_T, gy), dim3(AB_T), 0, st, B.X, B.Y, W.WB,
                               m, n, theta, dA);
        }
        ABCHK(hipGetLastError());
    }
    if (B.sparse) {
        ABCHK(hipMemcpyAsync(barrier_err, B.sp.err, sizeof(int), hipMemcpyDeviceToHost, st));
    }
    ABCHK(hipStreamSynchronize(st));
    *iters = it;
    *rel_out = rel;
    return hipSuccess;
}
