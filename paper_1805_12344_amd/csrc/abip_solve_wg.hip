// Persistent batched ABIP solver: one workgroup owns one LP for its whole
// solve (Algorithm 2 with the Section 4.2 relaxation, Section 4.1 tests and the
// Section 5 restart), LPs are taken largest-first from a device work queue.
//
// One inner iteration, with w = u + v = (y, x + s, tau + kappa, theta - (n+1)):
//   t  = y - A f                      (A f of the current state is already known)
//   a  = G^{-1} t                     (column dot products over the cached G^{-1})
//   p  = K^{-1}(w_q + H^T z)          (2x2 border; c^T d = c^T f + (A c)^T a, so the
//                                      border needs no pass over d)
//   y' = alpha (a - Z_y p) + (1-alpha) y,   theta', tau', kappa' (scalars)
//   column pass over A (one read per iteration): for every column j
//       (A^T a)_j, (A^T y')_j  -> d_j, the relaxed x-coordinate, the prox root
//       x'_j, the dual update s'_j, and the accumulation of A[:,j] (x'_j + s'_j)
//       and A[:,j] x'_j, which are the products the next iteration and the
//       next check need.
// The check of Section 4.1 and the inner test ||Qu - v||^2 <= mu of each new
// iterate is therefore exact and costs no extra pass over A.
#include <hip/hip_runtime.h>
#include "abip_internal.h"

#define UNR 4

struct WGShared {
    double* y;      // ld
    double* a;      // ld
    double* t;      // ld
    double* Af;     // ld
    double* Ax;     // ld
    double* red;    // 2 * W * ld
    double* scal;   // W * 8
    double* buf;    // W * 8
};

// One pass over the columns of A.  op: OP_REFRESH (recompute products of the
// current state), OP_PROX (the inner update), OP_RESTART (Section 5 / eq.
// update-next-iterate rescaling of x and s).  Leaves A(x+s) and A x of the new
// state in sh.Af / sh.Ax and the column-side sums in cs[7]:
//   c^T x, cbar^T x, c^T s, cbar^T s, ||A^T y + s - c tau||^2, ||A^T y + s||^2,
//   ||-A^T y + c tau - cbar theta - s||^2.
template <int NCH, typename T>
__device__ void column_pass(const T* __restrict__ A, int m, int n, int ld,
                            double* __restrict__ X, double* __restrict__ S,
                            const double* __restrict__ C, const double* __restrict__ CB,
                            const double* __restrict__ ZX0, const double* __restrict__ ZX1,
                            const WGShared& sh, int op, double p0, double p1, double tmu,
                            double alpha, double gamma, int rule, double tau, double theta,
                            double (&cs)[7]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, W = blockDim.x >> 6;
    constexpr int R = NCH * 4;
    double ra[R], ry[R], accf[R], accx[R];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = ch * 256 + lane * 4 + q;
            ra[ch * 4 + q] = (r < ld) ? sh.a[r] : 0.0;
            ry[ch * 4 + q] = (r < ld) ? sh.y[r] : 0.0;
            accf[ch * 4 + q] = 0.0;
            accx[ch * 4 + q] = 0.0;
        }
    double acc7[7] = {0, 0, 0, 0, 0, 0, 0};
    const double sg = sqrt(gamma);
    for (int cblk = wave; cblk * 64 < n; cblk += W) {
        const int j0 = cblk * 64;
        const int cnt = min(64, n - j0);
        double xj = 0, sj = 0, cj = 0, cbj = 0, z0 = 0, z1 = 0;
        if (lane < cnt) {
            xj = X[j0 + lane]; sj = S[j0 + lane];
            cj = C[j0 + lane]; cbj = CB[j0 + lane];
            if (op == OP_PROX) { z0 = ZX0[j0 + lane]; z1 = ZX1[j0 + lane]; }
        }
        double xn = xj, sn = sj;
        for (int kk = 0; kk < cnt; kk += UNR) {
            double v[UNR][R];
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                const int col = j0 + kk + u;
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) {
                    const int r0 = ch * 256 + lane * 4;
                    if (kk + u < cnt && r0 < ld) {
                        load4(A + (int64_t)col * ld + r0, &v[u][ch * 4]);
                    } else {
#pragma unroll
                        for (int q = 0; q < 4; ++q) v[u][ch * 4 + q] = 0.0;
                    }
                }
            }
            double dots[2 * UNR];
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                double da = 0.0, dy = 0.0;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    da = fma(v[u][r], ra[r], da);
                    dy = fma(v[u][r], ry[r], dy);
                }
                dots[2 * u] = da;
                dots[2 * u + 1] = dy;
            }
            wave_sum_n<2 * UNR>(dots);
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                const int l = kk + u;
                if (l < cnt) {
                    const double x0 = bcast_lane(xj, l), s0 = bcast_lane(sj, l);
                    const double c0 = bcast_lane(cj, l), cb0 = bcast_lane(cbj, l);
                    double x1, s1;
                    if (op == OP_PROX) {
                        const double zz0 = bcast_lane(z0, l), zz1 = bcast_lane(z1, l);
                        const double dj = (x0 + s0) + dots[2 * u];          // M^{-1} block, x part
                        const double ut = dj - zz0 * p0 - zz1 * p1;           // u~_x
                        const double uh = alpha * ut + (1.0 - alpha) * x0;    // relaxation
                        x1 = prox_root(uh - s0, tmu);                         // barrier prox
                        s1 = s0 - uh + x1;                                    // dual update
                    } else if (op == OP_RESTART) {
                        if (rule == 0) {
                            if (x0 >= s0) { x1 = x0; s1 = gamma * s0; }
                            else { x1 = gamma * x0; s1 = s0; }
                        } else {
                            x1 = sg * x0; s1 = sg * s0;
                        }
                    } else {
                        x1 = x0; s1 = s0;
                    }
                    if (lane == l) { xn = x1; sn = s1; }
                    const double f1 = x1 + s1;
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        accf[r] = fma(v[u][r], f1, accf[r]);
                        accx[r] = fma(v[u][r], x1, accx[r]);
                    }
                    const double aty = dots[2 * u + 1];
                    const double r1 = aty + s1 - c0 * tau;
                    const double r2 = aty + s1;
                    const double r3 = -aty + c0 * tau - cb0 * theta - s1;
                    acc7[0] = fma(c0, x1, acc7[0]);
                    acc7[1] = fma(cb0, x1, acc7[1]);
                    acc7[2] = fma(c0, s1, acc7[2]);
                    acc7[3] = fma(cb0, s1, acc7[3]);
                    acc7[4] = fma(r1, r1, acc7[4]);
                    acc7[5] = fma(r2, r2, acc7[5]);
                    acc7[6] = fma(r3, r3, acc7[6]);
                }
            }
        }
        if (lane < cnt && op != OP_REFRESH) { X[j0 + lane] = xn; S[j0 + lane] = sn; }
    }
    // cross-wave reduction (fixed order: deterministic)
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = ch * 256 + lane * 4 + q;
            if (r < ld) {
                sh.red[(2 * wave) * ld + r] = accf[ch * 4 + q];
                sh.red[(2 * wave + 1) * ld + r] = accx[ch * 4 + q];
            }
        }
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < 7; ++q) sh.scal[wave * 8 + q] = acc7[q];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < ld; i += blockDim.x) {
        double f = 0.0, x = 0.0;
        for (int w = 0; w < W; ++w) { f += sh.red[(2 * w) * ld + i]; x += sh.red[(2 * w + 1) * ld + i]; }
        sh.Af[i] = f;
        sh.Ax[i] = x;
    }
#pragma unroll
    for (int q = 0; q < 7; ++q) {
        double s = 0.0;
        for (int w = 0; w < W; ++w) s += sh.scal[w * 8 + q];
        cs[q] = s;
    }
    __syncthreads();
}

// a = G^{-1} t by column dot products over the symmetric G^{-1} (ld x m).
template <int NCH, typename T>
__device__ void ginv_pass(const T* __restrict__ G, int m, int ld, const WGShared& sh) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, W = blockDim.x >> 6;
    constexpr int R = NCH * 4;
    double rt[R];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = ch * 256 + lane * 4 + q;
            rt[ch * 4 + q] = (r < ld) ? sh.t[r] : 0.0;
        }
    for (int cblk = wave; cblk * 64 < m; cblk += W) {
        const int j0 = cblk * 64;
        const int cnt = min(64, m - j0);
        double an = 0.0;
        for (int kk = 0; kk < cnt; kk += UNR) {
            double dots[UNR];
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                const int col = j0 + kk + u;
                double v[R];
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) {
                    const int r0 = ch * 256 + lane * 4;
                    if (kk + u < cnt && r0 < ld) load4(G + (int64_t)col * ld + r0, &v[ch * 4]);
                    else {
#pragma unroll
                        for (int q = 0; q < 4; ++q) v[ch * 4 + q] = 0.0;
                    }
                }
                double s = 0.0;
#pragma unroll
                for (int r = 0; r < R; ++r) s = fma(v[r], rt[r], s);
                dots[u] = s;
            }
            wave_sum_n<UNR>(dots);
#pragma unroll
            for (int u = 0; u < UNR; ++u)
                if (lane == kk + u) an = dots[u];
        }
        if (lane < cnt) sh.a[j0 + lane] = an;
    }
    for (int i = m + threadIdx.x; i < ld; i += blockDim.x) sh.a[i] = 0.0;
    __syncthreads();
}


// Solve (or iterate) one LP with the calling workgroup.
// fixed_iters > 0: run exactly that many PROX iterations with no tests and no
// restarts (phase taken from ctrl.phase), for step-level parity checks.
template <int NCH>
__device__ void solve_one(int k, const LPDesc& d, LPCtrl* __restrict__ ctrl, const PoolPtrs& P,
                          const SolveParams& prm, int64_t fixed_iters, const WGShared& sh) {
    const int m = d.m, n = d.n, ld = d.ld;
    const int tid = threadIdx.x;
    const double* b = P.Mv + MF_B * P.Mtot + d.om;
    const double* bbar = P.Mv + MF_BBAR * P.Mtot + d.om;
    const double* Ac = P.Mv + MF_AC * P.Mtot + d.om;
    const double* Acb = P.Mv + MF_ACBAR * P.Mtot + d.om;
    const double* Zy0 = P.Mv + MF_ZY0 * P.Mtot + d.om;
    const double* Zy1 = P.Mv + MF_ZY1 * P.Mtot + d.om;
    double* Yg = P.Mv + MF_Y * P.Mtot + d.om;
    const double* C = P.Nv + NF_C * P.Ntot + d.on;
    const double* CBv = P.Nv + NF_CBAR * P.Ntot + d.on;
    const double* ZX0 = P.Nv + NF_ZX0 * P.Ntot + d.on;
    const double* ZX1 = P.Nv + NF_ZX1 * P.Ntot + d.on;
    double* X = P.Nv + NF_X * P.Ntot + d.on;
    double* S = P.Nv + NF_S * P.Ntot + d.on;
    const double* A64 = P.A64 + d.oA;
    const float* A32 = P.A32 + d.oA;
    const double* G64 = P.G64 + d.oG;
    const float* G32 = P.G32 + d.oG;

    LPCtrl cl = ctrl[k];
    double tau = cl.tau, kappa = cl.kappa, theta = cl.theta, mu = cl.mu;
    int64_t iters = cl.iters, iters64 = cl.iters64, ipm = cl.ipm;
    int phase = cl.phase;
    int op = cl.mode;          // first pass: OP_REFRESH of the loaded state
    int status = cl.status;
    const int check_final_first = cl.flags & 1;   // a loaded post-update state: test it
    double pres = cl.pres, dres = cl.dres, gap = cl.gap, pobj = cl.pobj, dobj = cl.dobj;
    double by_last = cl.by, cx_last = cl.cx;
    const double zbar = cl.zbar, nb = cl.nb, nc = cl.nc;
    const double alpha = prm.alpha, gamma = prm.gamma, beta = prm.beta, eps = prm.eps;
    const double np1 = (double)n + 1.0;

    for (int i = tid; i < ld; i += blockDim.x) sh.y[i] = (i < m) ? Yg[i] : 0.0;
    for (int i = tid; i < ld; i += blockDim.x) sh.a[i] = 0.0;
    __syncthreads();

    double p0 = 0.0, p1 = 0.0;
    int pass_kind = op;          // what the column pass does
    bool first = true;
    int64_t done_fixed = 0;
    // every pass is an update, a restart or a refresh; restarts and refreshes
    // without updates are bounded by this cap so the loop always ends
    int64_t passes = 0;
    const int64_t pass_cap = prm.max_iters + 4096;
    while (true) {
        if (++passes > pass_cap && fixed_iters == 0) { status = 4; break; }
        const double tmu = mu / beta;
        double cs[7];
        if (phase == 0)
            column_pass<NCH, float>(A32, m, n, ld, X, S, C, CBv, ZX0, ZX1, sh, pass_kind, p0, p1, tmu,
                                    alpha, gamma, prm.restart_rule, tau, theta, cs);
        else
            column_pass<NCH, double>(A64, m, n, ld, X, S, C, CBv, ZX0, ZX1, sh, pass_kind, p0, p1, tmu,
                                     alpha, gamma, prm.restart_rule, tau, theta, cs);
        const bool post_update = (pass_kind == OP_PROX) || (first && check_final_first) ||
                                 (pass_kind == OP_REFRESH && !first);
        if (pass_kind == OP_PROX) {
            ++iters;
            if (phase == 1) ++iters64;
            ++done_fixed;
        }
        first = false;
        if (fixed_iters > 0 && done_fixed >= fixed_iters) break;

        // ---- m-side sums of the check (Section 4.1) and of ||Qu - v||^2
        double ms[5] = {0, 0, 0, 0, 0};
        for (int i = tid; i < m; i += blockDim.x) {
            const double ax = sh.Ax[i], bi = b[i], bbi = bbar[i], yi = sh.y[i];
            const double r1 = ax - bi * tau;
            const double r3 = r1 + bbi * theta;
            ms[0] = fma(bi, yi, ms[0]);
            ms[1] = fma(bbi, yi, ms[1]);
            ms[2] = fma(r1, r1, ms[2]);
            ms[3] = fma(ax, ax, ms[3]);
            ms[4] = fma(r3, r3, ms[4]);
        }
        block_sum_n<5>(ms, sh.buf);
        const double by = ms[0], bby = ms[1];
        const double cx = cs[0], cbx = cs[1];

        if (fixed_iters == 0) {
            // ---- final test on a post-update iterate
            if (post_update) {
                int st = 0;
                if (tau > 0.0) {
                    pres = sqrt(ms[2]) / tau;
                    dres = sqrt(cs[4]) / tau;
                    pobj = cx / tau;
                    dobj = by / tau;
                    gap = fabs(pobj - dobj);
                    if (pres <= eps * (1.0 + nb) && dres <= eps * (1.0 + nc) &&
                        gap <= eps * (1.0 + fabs(pobj) + fabs(dobj)))
                        st = 1;
                    pres /= (1.0 + nb);
                    dres /= (1.0 + nc);
                    gap /= (1.0 + fabs(pobj) + fabs(dobj));
                }
                if (!st && nb > 0.0 && by > 0.0 && sqrt(cs[5]) <= eps * by / nb) st = 2;
                if (!st && nc > 0.0 && cx < 0.0 && sqrt(ms[3]) <= eps * (-cx) / nc) st = 3;
                by_last = by;
                cx_last = cx;
                if (st) {
                    if (phase == 0) {          // FP32 verdict: confirm with FP64 data
                        phase = 1;
                        pass_kind = OP_REFRESH;
                        continue;
                    }
                    status = st;
                    break;
                }
            }
            if (phase == 0 && iters >= prm.fp32_max_iters) {
                phase = 1;
                pass_kind = OP_REFRESH;
                continue;
            }
            // ---- inner test ||Q u - v||^2 <= mu (eq. inner-stop)
            const double rt = by - cx + zbar * theta - kappa;
            const double rth = -bby + cbx - zbar * tau + np1;
            const double inner = ms[4] + cs[6] + rt * rt + rth * rth;
            if (inner <= mu) {
                mu *= gamma;
                ++ipm;
                if (prm.restart_rule == 0) {
                    if (tau >= kappa) kappa *= gamma;
                    else tau *= gamma;
                } else {
                    const double sg = sqrt(gamma);
                    tau *= sg; kappa *= sg; theta *= sg;
                    for (int i = tid; i < m; i += blockDim.x) sh.y[i] *= sg;
                    __syncthreads();
                }
                pass_kind = OP_RESTART;
                continue;
            }
            if (iters >= prm.max_iters) { status = 4; break; }
        }

        // ---- the inner update: t = y - A f, a = G^{-1} t, border, scalars, y'
        for (int i = tid; i < ld; i += blockDim.x) sh.t[i] = (i < m) ? sh.y[i] - sh.Af[i] : 0.0;
        __syncthreads();
        if (phase == 0) ginv_pass<NCH, float>(G32, m, ld, sh);
        else ginv_pass<NCH, double>(G64, m, ld, sh);
        double bs[4] = {0, 0, 0, 0};
        for (int i = tid; i < m; i += blockDim.x) {
            const double ai = sh.a[i];
            bs[0] = fma(b[i], ai, bs[0]);
            bs[1] = fma(bbar[i], ai, bs[1]);
            bs[2] = fma(Ac[i], ai, bs[2]);
            bs[3] = fma(Acb[i], ai, bs[3]);
        }
        block_sum_n<4>(bs, sh.buf);
        const double cs_f = cx + cs[2];        // c^T (x + s)
        const double cbs_f = cbx + cs[3];      // cbar^T (x + s)
        const double h1z = -bs[0] + cs_f + bs[2];      // h1^T z, c^T d = c^T f + (A c)^T a
        const double h2z = bs[1] - cbs_f - bs[3];      // h2^T z
        const double q0 = (tau + kappa) + h1z;
        const double q1 = (theta - np1) + h2z;
        p0 = cl.K00 * q0 + cl.K01 * q1;
        p1 = cl.K10 * q0 + cl.K11 * q1;
        const double uh_tau = alpha * p0 + (1.0 - alpha) * tau;
        const double uh_theta = alpha * p1 + (1.0 - alpha) * theta;
        const double tau1 = prox_root(uh_tau - kappa, tmu);
        kappa = kappa - uh_tau + tau1;
        tau = tau1;
        theta = uh_theta;
        for (int i = tid; i < m; i += blockDim.x) {
            const double ut = sh.a[i] - Zy0[i] * p0 - Zy1[i] * p1;
            sh.y[i] = alpha * ut + (1.0 - alpha) * sh.y[i];
        }
        __syncthreads();
        pass_kind = OP_PROX;
    }

    for (int i = tid; i < m; i += blockDim.x) Yg[i] = sh.y[i];
    if (tid == 0) {
        LPCtrl& o = ctrl[k];
        o.tau = tau; o.kappa = kappa; o.theta = theta; o.mu = mu;
        o.pres = pres; o.dres = dres; o.gap = gap; o.pobj = pobj; o.dobj = dobj;
        o.by = by_last; o.cx = cx_last;
        o.iters = iters; o.iters64 = iters64; o.ipm = ipm;
        o.status = status; o.phase = phase;
        o.mode = OP_REFRESH;
        o.flags = (fixed_iters > 0) ? 1 : 0;
    }
    __syncthreads();
}

template <int NCH>
__global__ __launch_bounds__(512) void k_solve_wg(const LPDesc* __restrict__ desc, LPCtrl* __restrict__ ctrl,
                                                  PoolPtrs P, SolveParams prm, const int32_t* __restrict__ order,
                                                  int32_t B, int32_t* __restrict__ queue, int64_t fixed_iters,
                                                  int32_t ldmax) {
    extern __shared__ double smem[];
    __shared__ int s_lp;
    const int W = blockDim.x >> 6;
    WGShared sh;
    sh.y = smem;
    sh.a = sh.y + ldmax;
    sh.t = sh.a + ldmax;
    sh.Af = sh.t + ldmax;
    sh.Ax = sh.Af + ldmax;
    sh.red = sh.Ax + ldmax;
    sh.scal = sh.red + 2 * W * ldmax;
    sh.buf = sh.scal + 8 * W;
    while (true) {
        if (threadIdx.x == 0) s_lp = atomicAdd(queue, 1);
        __syncthreads();
        const int q = s_lp;
        __syncthreads();
        if (q >= B) break;
        const int k = order[q];
        const LPDesc d = desc[k];
        solve_one<NCH>(k, d, ctrl, P, prm, fixed_iters, sh);
    }
}

// LDS bytes for a launch
size_t wg_smem_bytes(int ldmax, int W) {
    return sizeof(double) * ((size_t)5 * ldmax + (size_t)2 * W * ldmax + 16 * (size_t)W);
}

hipError_t launch_solve_wg(int nch, int grid, int threads, hipStream_t st, const LPDesc* desc, LPCtrl* ctrl,
                           const PoolPtrs& P, const SolveParams& prm, const int32_t* order, int32_t B,
                           int32_t* queue, int64_t fixed_iters, int32_t ldmax) {
    const size_t smem = wg_smem_bytes(ldmax, threads / 64);
    switch (nch) {
    case 1: hipLaunchKernelGGL(k_solve_wg<1>, dim3(grid), dim3(threads), smem, st, desc, ctrl, P, prm, order, B, queue, fixed_iters, ldmax); break;
    case 2: hipLaunchKernelGGL(k_solve_wg<2>, dim3(grid), dim3(threads), smem, st, desc, ctrl, P, prm, order, B, queue, fixed_iters, ldmax); break;
    case 3: hipLaunchKernelGGL(k_solve_wg<3>, dim3(grid), dim3(threads), smem, st, desc, ctrl, P, prm, order, B, queue, fixed_iters, ldmax); break;
    case 4: hipLaunchKernelGGL(k_solve_wg<4>, dim3(grid), dim3(threads), smem, st, desc, ctrl, P, prm, order, B, queue, fixed_iters, ldmax); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t set_solve_wg_smem_limit(size_t bytes) {
    hipError_t e;
    if ((e = hipFuncSetAttribute((const void*)k_solve_wg<1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes)) != hipSuccess) return e;
    if ((e = hipFuncSetAttribute((const void*)k_solve_wg<2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes)) != hipSuccess) return e;
    if ((e = hipFuncSetAttribute((const void*)k_solve_wg<3>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes)) != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_solve_wg<4>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}
