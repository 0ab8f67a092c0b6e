// FP64 recheck of a finished solve (Section 4.1 residuals of the returned point).
//
// The loop's own tests are evaluated from sums it carries along (the A^T y
// recurrence of the LDS-resident loop, the FP32-streamed products of the bulk
// phase).  After the solve, these kernels recompute the residuals of the point
// the caller receives from the FP64 copies of A, b and c, independently of the
// loop's sums:
//   SOLVED / MAX_ITERS:  max(pres, dres, gap) of (x/tau, y/tau, s/tau)
//   PRIMAL_INFEASIBLE:   ||A^T yc + sc|| ||b|| with (yc, sc) = (y, s)/(b^T y)
//                        (the certificate test of Section 4.1 passes when <= eps)
//   DUAL_INFEASIBLE:     ||A xc|| ||c|| with xc = -x/(c^T x)
// The result goes to LPCtrl.err64.  Partial sums are written per workgroup and
// added in a fixed order, so the value is reproducible.  A scaled LP (pools
// holding D A E, D b, E c and the iterate of that LP) is measured as the LP the
// caller gave: row residuals times 1/D_i, column residuals times 1/E_j, and the
// norms of the given b and c (c^T x and b^T y do not change under the scaling).
#include <hip/hip_runtime.h>
#include "abip_internal.h"

enum { RC_PR2 = 0, RC_DR2, RC_CX, RC_BY, RC_AX2, RC_ATS2, RC_B2, RC_C2, RC_N = 8 };

// Per-workgroup sums for LP blockIdx.y, share blockIdx.x of P: rows
// [r0, r1) (one thread per row, coalesced down the column-major columns) and
// columns [c0, c1) (one wave per column).
__global__ __launch_bounds__(256) void k_recheck_dense(const LPDesc* __restrict__ desc,
                                                        const LPCtrl* __restrict__ ctrl, const double* __restrict__ A64,
                                                        const double* __restrict__ Mv, const double* __restrict__ Nv,
                                                        int64_t Mtot, int64_t Ntot, double* __restrict__ part, int P) {
    __shared__ double sbuf[4 * RC_N];
    const int k = blockIdx.y, p = blockIdx.x;
    const LPDesc d = desc[k];
    const double tau = ctrl[k].tau;
    const int m = d.m, n = d.n, ld = d.ld;
    const double* A = A64 + d.oA;
    const double* b = Mv + MF_B * Mtot + d.om;
    const double* y = Mv + MF_Y * Mtot + d.om;
    const double* c = Nv + NF_C * Ntot + d.on;
    const double* x = Nv + NF_X * Ntot + d.on;
    const double* s = Nv + NF_S * Ntot + d.on;
    const double* Dv = Mv + MF_SD * Mtot + d.om;
    const double* Ev = Nv + NF_SE * Ntot + d.on;
    const double it = (tau > 0.0) ? 1.0 / tau : 0.0;
    double v[RC_N] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int rpb = (m + P - 1) / P, cpb = (n + P - 1) / P;
    const int r0 = p * rpb, r1 = min(m, r0 + rpb);
    for (int i = r0 + (int)threadIdx.x; i < r1; i += blockDim.x) {
        double ax = 0.0;
        for (int j = 0; j < n; ++j) ax = fma(A[(int64_t)j * ld + i], x[j], ax);
        const double wi = 1.0 / Dv[i];
        const double r = (ax * it - b[i]) * wi;
        const double axw = ax * wi, bw = b[i] * wi;
        v[RC_PR2] = fma(r, r, v[RC_PR2]);
        v[RC_AX2] = fma(axw, axw, v[RC_AX2]);
        v[RC_BY] = fma(b[i], y[i], v[RC_BY]);
        v[RC_B2] = fma(bw, bw, v[RC_B2]);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, W = blockDim.x >> 6;
    const int c0 = p * cpb, c1 = min(n, c0 + cpb);
    for (int j = c0 + wave; j < c1; j += W) {
        double aty = 0.0;
        for (int i = lane; i < m; i += 64) aty = fma(A[(int64_t)j * ld + i], y[i], aty);
        aty = wave_sum(aty);
        if (lane == 0) {
            const double wj = 1.0 / Ev[j];
            const double r = ((aty + s[j]) * it - c[j]) * wj;
            const double q = (aty + s[j]) * wj, cw = c[j] * wj;
            v[RC_DR2] = fma(r, r, v[RC_DR2]);
            v[RC_ATS2] = fma(q, q, v[RC_ATS2]);
            v[RC_CX] = fma(c[j], x[j], v[RC_CX]);
            v[RC_C2] = fma(cw, cw, v[RC_C2]);
        }
    }
    block_sum_n<RC_N>(v, sbuf);
    if (threadIdx.x == 0)
        for (int q = 0; q < RC_N; ++q) part[((int64_t)k * P + p) * RC_N + q] = v[q];
}

// The same sums for a CSR matrix (one LP): rows of CSR(A) for A x, rows of
// CSR(A^T) for A^T y.
__global__ __launch_bounds__(256) void k_recheck_csr(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                      const double* __restrict__ va, const int32_t* __restrict__ rpt,
                                                      const int32_t* __restrict__ cit, const double* __restrict__ vat,
                                                      int m, int n, const LPCtrl* __restrict__ ctrl,
                                                      const double* __restrict__ b, const double* __restrict__ y,
                                                      const double* __restrict__ c, const double* __restrict__ x,
                                                      const double* __restrict__ s, double* __restrict__ part, int P) {
    __shared__ double sbuf[4 * RC_N];
    const int p = blockIdx.x;
    const double tau = ctrl[0].tau;
    const double it = (tau > 0.0) ? 1.0 / tau : 0.0;
    double v[RC_N] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int rpb = (m + P - 1) / P, cpb = (n + P - 1) / P;
    const int r0 = p * rpb, r1 = min(m, r0 + rpb);
    for (int i = r0 + (int)threadIdx.x; i < r1; i += blockDim.x) {
        double ax = 0.0;
        for (int e = rp[i]; e < rp[i + 1]; ++e) ax = fma(va[e], x[ci[e]], ax);
        const double r = ax * it - b[i];
        v[RC_PR2] = fma(r, r, v[RC_PR2]);
        v[RC_AX2] = fma(ax, ax, v[RC_AX2]);
        v[RC_BY] = fma(b[i], y[i], v[RC_BY]);
        v[RC_B2] = fma(b[i], b[i], v[RC_B2]);
    }
    const int c0 = p * cpb, c1 = min(n, c0 + cpb);
    for (int j = c0 + (int)threadIdx.x; j < c1; j += blockDim.x) {
        double aty = 0.0;
        for (int e = rpt[j]; e < rpt[j + 1]; ++e) aty = fma(vat[e], y[cit[e]], aty);
        const double r = (aty + s[j]) * it - c[j];
        const double q = aty + s[j];
        v[RC_DR2] = fma(r, r, v[RC_DR2]);
        v[RC_ATS2] = fma(q, q, v[RC_ATS2]);
        v[RC_CX] = fma(c[j], x[j], v[RC_CX]);
        v[RC_C2] = fma(c[j], c[j], v[RC_C2]);
    }
    block_sum_n<RC_N>(v, sbuf);
    if (threadIdx.x == 0)
        for (int q = 0; q < RC_N; ++q) part[(int64_t)p * RC_N + q] = v[q];
}

// Totals in a fixed order and the status-dependent residual (one thread per LP).
__global__ void k_recheck_fin(LPCtrl* __restrict__ ctrl, const double* __restrict__ part, int B, int P) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= B) return;
    double t[RC_N] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int p = 0; p < P; ++p)
        for (int q = 0; q < RC_N; ++q) t[q] += part[((int64_t)k * P + p) * RC_N + q];
    LPCtrl& c = ctrl[k];
    const double tau = c.tau, nb = sqrt(t[RC_B2]), nc = sqrt(t[RC_C2]);
    double e = __builtin_nan("");
    if (c.status == 2) {
        const double by = t[RC_BY];
        if (by > 0.0) e = sqrt(t[RC_ATS2]) / by * nb;
    } else if (c.status == 3) {
        const double cx = t[RC_CX];
        if (cx < 0.0) e = sqrt(t[RC_AX2]) / (-cx) * nc;
    } else if (tau > 0.0) {
        const double pobj = t[RC_CX] / tau, dobj = t[RC_BY] / tau;
        const double pres = sqrt(t[RC_PR2]) / (1.0 + nb);
        const double dres = sqrt(t[RC_DR2]) / (1.0 + nc);
        const double gap = fabs(pobj - dobj) / (1.0 + fabs(pobj) + fabs(dobj));
        e = fmax(pres, fmax(dres, gap));
    }
    c.err64 = e;
}

hipError_t launch_recheck_dense(const LPDesc* desc, LPCtrl* ctrl, const double* A64, const double* Mv,
                                const double* Nv, int64_t Mtot, int64_t Ntot, double* part, int B, int P,
                                hipStream_t st) {
    hipLaunchKernelGGL(k_recheck_dense, dim3(P, B), dim3(256), 0, st, desc, ctrl, A64, Mv, Nv, Mtot, Ntot, part, P);
    hipLaunchKernelGGL(k_recheck_fin, dim3((B + 63) / 64), dim3(64), 0, st, ctrl, part, B, P);
    return hipGetLastError();
}

hipError_t launch_recheck_csr(const int32_t* rp, const int32_t* ci, const double* va, const int32_t* rpt,
                              const int32_t* cit, const double* vat, int m, int n, LPCtrl* ctrl, const double* b,
                              const double* y, const double* c, const double* x, const double* s, double* part,
                              int P, hipStream_t st) {
    hipLaunchKernelGGL(k_recheck_csr, dim3(P), dim3(256), 0, st, rp, ci, va, rpt, cit, vat, m, n, ctrl, b, y, c, x, s,
                       part, P);
    hipLaunchKernelGGL(k_recheck_fin, dim3(1), dim3(64), 0, st, ctrl, part, 1, P);
    return hipGetLastError();
}
