// Grid engine: one LP spread over the whole GPU, four kernels per inner
// iteration of Algorithm 2 (Section 4.2 relaxation, Section 4.1 tests,
// Section 5 restart), replayed as hipGraphs of 16 iterations and driven from
// the host in chunks of iterations.
//
//   k_grid_col   columns split over NB workgroups.  Each workgroup first forms
//                y' = alpha (a - Z_y p) + (1-alpha) y redundantly from the
//                border p of the pending update, then streams its columns of A
//                once: (A^T a)_j, (A^T y')_j, the
//                relaxed prox / dual update of x_j, s_j, and the accumulation of
//                A[:,j](x'_j + s'_j) and A[:,j] x'_j into per-workgroup partial
//                m-vectors (waves own disjoint row ranges, so no cross-wave
//                reduction of the partials is needed).
//   k_grid_red   rows split over workgroups: sums the partials into A(x+s), A x,
//                forms t = y' - A(x+s) and the row-side sums of the check.
//   k_grid_ginv  every workgroup reduces the sums in a fixed order and takes the
//                same decision (final test, inner test, restart, phase switch);
//                for an update it computes its slice of a = G^{-1} t and the
//                partial border dots; workgroup 0 publishes the decision.
//   k_grid_border one workgroup: the 2x2 border (Section 4.4) and the relaxed
//                tau, kappa, theta of the update, published as the control
//                block of the next column pass.
// All sums are reduced in a fixed order, so runs are bitwise reproducible.
#include <hip/hip_runtime.h>
#include "abip_internal.h"
#include "abip_grid.h"

#define GRID_W 8               // waves per workgroup (512 threads)
#define GRID_UNR 8             // columns per step in the column kernels
#define GRID_RED_ROWS 32       // rows per workgroup of the partial-sum reduction

// Border, scalars and y' of a pending update, computed identically by every
// workgroup from the published partial dots.
struct Pending {
    double p0, p1, tau1, kappa1, theta1;
};

__device__ __forceinline__ Pending finish_border(const GridArgs& g, const GridCtl& c, const double* cs4,
                                                const double* ad4) {
    // cs4: c^T x, cbar^T x, c^T s, cbar^T s of the current state; ad4: b^T a,
    // bbar^T a, (A c)^T a, (A cbar)^T a
    const LPCtrl& L = *g.lc;
    const double alpha = g.prm.alpha;
    const double np1 = (double)g.n + 1.0;
    const double h1z = -ad4[0] + (cs4[0] + cs4[2]) + ad4[2];
    const double h2z = ad4[1] - (cs4[1] + cs4[3]) - ad4[3];
    const double q0 = (c.tau + c.kappa) + h1z;
    const double q1 = (c.theta - np1) + h2z;
    Pending P;
    P.p0 = L.K00 * q0 + L.K01 * q1;
    P.p1 = L.K10 * q0 + L.K11 * q1;
    const double tmu = c.mu / g.prm.beta;
    const double uh_tau = alpha * P.p0 + (1.0 - alpha) * c.tau;
    P.theta1 = alpha * P.p1 + (1.0 - alpha) * c.theta;
    P.tau1 = prox_root(uh_tau - c.kappa, tmu);
    P.kappa1 = c.kappa - uh_tau + P.tau1;
    return P;
}

// ---------------------------------------------------------------------------
// k_grid_col
// ---------------------------------------------------------------------------
template <int NCHW, typename T, int U>
__device__ void grid_col_body(const GridArgs& g, const GridCtl& c, int op, const T* __restrict__ A,
                              double p0, double p1, double tau, double theta, double* sy, double* sa,
                              double* sd, double* sx) {
    const int lane = threadIdx.x & 63, wave = wave_id();
    constexpr int R = NCHW * 4;
    const int ld = g.ld, n = g.n;
    // rows owned by this lane: wave w, chunk ch -> rows (ch*GRID_W + w)*256 + 4*lane + q
    double ra[R], ry[R], accf[R], accx[R];
#pragma unroll
    for (int ch = 0; ch < NCHW; ++ch)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = (ch * GRID_W + wave) * 256 + lane * 4 + q;
            ra[ch * 4 + q] = (r < ld) ? sa[r] : 0.0;
            ry[ch * 4 + q] = (r < ld) ? sy[r] : 0.0;
            accf[ch * 4 + q] = 0.0;
            accx[ch * 4 + q] = 0.0;
        }
    const bool prox = (op == OP_PROX);
    const double alpha = g.prm.alpha, gamma = g.prm.gamma;
    const double tmu = c.mu / g.prm.beta;
    const double sg = sqrt(gamma);
    const int rule = g.prm.restart_rule;
    const int j_begin = blockIdx.x * g.cw;
    const int j_end = min(n, j_begin + g.cw);
    double acc7[7] = {0, 0, 0, 0, 0, 0, 0};
    T va[U][R], vb[U][R];
    // per-column data of a group, loaded with it by lanes u < U (lane u: column
    // col0 + u; the other lanes load a valid neighbour and ignore it)
    struct ColData { double x, s, z0, z1, c, cb; };
    ColData da_, db_;
    // unmasked loads from clamped addresses: rows past ld have zero weights,
    // columns past j_end are skipped with a uniform test in step()
    const int rl = min(lane * 4, ld - 4);
    auto load_cols = [&](int col0, ColData& cd) {
        const int j = min(col0 + (lane < U ? lane : 0), j_end - 1);
        cd.x = g.X[j]; cd.s = g.S[j]; cd.z0 = g.Zx0[j]; cd.z1 = g.Zx1[j]; cd.c = g.C[j]; cd.cb = g.CB[j];
    };
    auto load = [&](int col0, T (&v)[U][R]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int col = min(col0 + u, j_end - 1);
#pragma unroll
            for (int ch = 0; ch < NCHW; ++ch) {
                const int r0 = (ch * GRID_W + wave) * 256 + lane * 4;
                const int rr = (r0 < ld) ? r0 : rl;
                if constexpr (sizeof(T) == 4) {
                    const float4 q4 = *reinterpret_cast<const float4*>(A + (int64_t)col * ld + rr);
                    v[u][ch * 4 + 0] = q4.x; v[u][ch * 4 + 1] = q4.y;
                    v[u][ch * 4 + 2] = q4.z; v[u][ch * 4 + 3] = q4.w;
                } else {
                    const double2 q0 = reinterpret_cast<const double2*>(A + (int64_t)col * ld + rr)[0];
                    const double2 q1 = reinterpret_cast<const double2*>(A + (int64_t)col * ld + rr)[1];
                    v[u][ch * 4 + 0] = q0.x; v[u][ch * 4 + 1] = q0.y;
                    v[u][ch * 4 + 2] = q1.x; v[u][ch * 4 + 3] = q1.y;
                }
            }
        }
    };
    auto step = [&](int col0, T (&v)[U][R], const ColData& cd) {
        // partial dots over this wave's rows, reduced over the wave, then over waves
        double dots[2 * U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            double da = 0.0, dy = 0.0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                da = fma((double)v[u][r], ra[r], da);
                dy = fma((double)v[u][r], ry[r], dy);
            }
            dots[2 * u] = da;
            dots[2 * u + 1] = dy;
        }
        // reduce-scatter: lanes u*LPC .. u*LPC+LPC-1 end with column u's (A^T a, A^T y')
        // over this wave's rows
        constexpr int LPC = 64 / U;
        wave_rs<2 * U, 2>(dots);
        if ((lane % LPC) == 0) {
            const int u = lane / LPC;
            sd[wave * 2 * U + 2 * u] = dots[0];
            sd[wave * 2 * U + 2 * u + 1] = dots[1];
        }
        __syncthreads();
        if (threadIdx.x < U) {
            const int u = threadIdx.x;
            const int j = col0 + u;
            double ata = 0.0, aty = 0.0;
            for (int w = 0; w < GRID_W; ++w) { ata += sd[w * 2 * U + 2 * u]; aty += sd[w * 2 * U + 2 * u + 1]; }
            double x1 = 0.0, s1 = 0.0;
            if (j < j_end) {
                const double x0 = cd.x, s0 = cd.s;
                x1 = x0; s1 = s0;
                if (prox) {
                    const double ut = (x0 + s0) + ata - cd.z0 * p0 - cd.z1 * p1;
                    const double uh = alpha * ut + (1.0 - alpha) * x0;
                    x1 = prox_root(uh - s0, tmu);
                    s1 = s0 - uh + x1;
                } else if (op == OP_RESTART) {
                    if (rule == 0) {
                        if (x0 >= s0) s1 = gamma * s0;
                        else x1 = gamma * x0;
                    } else {
                        x1 = sg * x0; s1 = sg * s0;
                    }
                }
                if (op != OP_REFRESH) { g.X[j] = x1; g.S[j] = s1; }
                const double c0 = cd.c, cb0 = cd.cb;
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
            sx[2 * u] = x1;
            sx[2 * u + 1] = x1 + s1;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool cv = (col0 + u) < j_end;           // uniform
            const double xu = cv ? sx[2 * u] : 0.0, fu = cv ? sx[2 * u + 1] : 0.0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                accf[r] = fma((double)v[u][r], fu, accf[r]);
                accx[r] = fma((double)v[u][r], xu, accx[r]);
            }
        }
    };
    // The next group's loads are issued without a condition (past j_end they
    // re-read the last column, which step() ignores): with a fixed number of
    // loads in flight the waits for one group leave the next group's loads
    // outstanding, so they overlap the reductions and the prox of this one.
    int c0 = j_begin;
    if (c0 < j_end) { load(c0, va); load_cols(c0, da_); }
    while (c0 < j_end) {
        const int c1 = c0 + U;
        load(c1, vb); load_cols(c1, db_);
        step(c0, va, da_);
        if (c1 >= j_end) break;
        const int c2 = c1 + U;
        load(c2, va); load_cols(c2, da_);
        step(c1, vb, db_);
        c0 = c2;
    }
    // partial m-vectors of this workgroup
    double* pf = g.Pf + (int64_t)blockIdx.x * ld;
    double* px = g.Px + (int64_t)blockIdx.x * ld;
#pragma unroll
    for (int ch = 0; ch < NCHW; ++ch)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = (ch * GRID_W + wave) * 256 + lane * 4 + q;
            if (r < ld) { pf[r] = accf[ch * 4 + q]; px[r] = accx[ch * 4 + q]; }
        }
    // column-side sums (only threads < U hold them)
    double t8[8] = {acc7[0], acc7[1], acc7[2], acc7[3], acc7[4], acc7[5], acc7[6], 0.0};
    block_sum_n<8>(t8, sd);
    if (threadIdx.x == 0)
        for (int q = 0; q < 8; ++q) g.pcol[blockIdx.x * 8 + q] = t8[q];
}

template <int NCHW>
__global__ __launch_bounds__(512) void k_grid_col(GridArgs g) {
    extern __shared__ double smem[];
    __shared__ double sd[GRID_W * 2 * GRID_UNR + 64];
    __shared__ double sx[2 * GRID_UNR];
    const GridCtl c = *g.ctl;
    if (c.status != 0) return;
    const int ld = g.ld, m = g.m;
    double* sy = smem;          // y of the state this pass produces
    double* sa = smem + ld;     // a of the pending update
    const double* ycur = g.Y2 + (int64_t)c.ybuf * ld;
    double* ynext = g.Y2 + (int64_t)(1 - c.ybuf) * ld;
    int op = c.mode;
    double p0 = 0.0, p1 = 0.0, tau = c.tau, theta = c.theta;
    if (op == OP_PROX) {
        p0 = c.p0; p1 = c.p1;
        // scalars of the new state were published by the decision kernel
        tau = c.tau_n; theta = c.theta_n;
        const double alpha = g.prm.alpha;
        for (int i = threadIdx.x; i < ld; i += blockDim.x) {
            double yv = 0.0, av = 0.0;
            if (i < m) {
                av = g.a[i];
                const double ut = av - g.Zy0[i] * p0 - g.Zy1[i] * p1;
                yv = alpha * ut + (1.0 - alpha) * ycur[i];
            }
            sy[i] = yv;
            sa[i] = av;
        }
    } else {
        const double f = (op == OP_RESTART && g.prm.restart_rule == 1) ? sqrt(g.prm.gamma) : 1.0;
        if (op == OP_RESTART) { tau = c.tau_n; theta = c.theta_n; }
        for (int i = threadIdx.x; i < ld; i += blockDim.x) {
            sy[i] = (i < m) ? f * ycur[i] : 0.0;
            sa[i] = 0.0;
        }
    }
    __syncthreads();
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < ld; i += blockDim.x) ynext[i] = sy[i];
    if (c.phase == 0) grid_col_body<NCHW, float, (NCHW == 1 ? 8 : 4)>(g, c, op, g.A32, p0, p1, tau, theta, sy, sa, sd, sx);
    else grid_col_body<NCHW, double, (NCHW == 1 ? 4 : 2)>(g, c, op, g.A64, p0, p1, tau, theta, sy, sa, sd, sx);
}

// ---------------------------------------------------------------------------
// k_grid_red: rows
// ---------------------------------------------------------------------------
// 32 rows per workgroup, 8 thread groups per row sum every 8th partial (4 per
// round so the loads overlap), then the 8 group sums are added in order.
__global__ __launch_bounds__(256) void k_grid_red(GridArgs g) {
    __shared__ double sbuf[8 * 8];
    __shared__ double sf[8][GRID_RED_ROWS], sx[8][GRID_RED_ROWS];
    const GridCtl c = *g.ctl;
    if (c.status != 0) return;
    const int r = threadIdx.x % GRID_RED_ROWS, grp = threadIdx.x / GRID_RED_ROWS;
    const int i = blockIdx.x * GRID_RED_ROWS + r;
    const int ld = g.ld, m = g.m, NB = g.NB;
    double f = 0.0, x = 0.0;
    if (i < ld) {
        int q = grp;
        for (; q + 24 < NB; q += 32) {
            const double f0 = g.Pf[(int64_t)q * ld + i], f1 = g.Pf[(int64_t)(q + 8) * ld + i];
            const double f2 = g.Pf[(int64_t)(q + 16) * ld + i], f3 = g.Pf[(int64_t)(q + 24) * ld + i];
            const double x0 = g.Px[(int64_t)q * ld + i], x1 = g.Px[(int64_t)(q + 8) * ld + i];
            const double x2 = g.Px[(int64_t)(q + 16) * ld + i], x3 = g.Px[(int64_t)(q + 24) * ld + i];
            f += f0; f += f1; f += f2; f += f3;
            x += x0; x += x1; x += x2; x += x3;
        }
        for (; q < NB; q += 8) { f += g.Pf[(int64_t)q * ld + i]; x += g.Px[(int64_t)q * ld + i]; }
    }
    sf[grp][r] = f;
    sx[grp][r] = x;
    __syncthreads();
    const double* y = g.Y2 + (int64_t)(1 - c.ybuf) * ld;    // y of the new state
    const double tau = c.tau_n, theta = c.theta_n;
    double ms[5] = {0, 0, 0, 0, 0};
    if (grp == 0 && i < ld) {
        double F = 0.0, X = 0.0;
#pragma unroll
        for (int k = 0; k < 8; ++k) { F += sf[k][r]; X += sx[k][r]; }
        g.t[i] = (i < m) ? y[i] - F : 0.0;
        if (i < m) {
            const double bi = g.b[i], bbi = g.bbar[i], yi = y[i];
            const double r1 = X - bi * tau;
            const double r3 = r1 + bbi * theta;
            ms[0] = bi * yi;
            ms[1] = bbi * yi;
            ms[2] = r1 * r1;
            ms[3] = X * X;
            ms[4] = r3 * r3;
        }
    }
    block_sum_n<5>(ms, sbuf);
    if (threadIdx.x == 0)
        for (int q = 0; q < 5; ++q) g.prow[blockIdx.x * 8 + q] = ms[q];
}

// ---------------------------------------------------------------------------
// k_grid_ginv: decision + slice of a = G^{-1} t
// ---------------------------------------------------------------------------
// One group of GRID_UNR columns of G^{-1}: this lane's four rows of every
// 256-row chunk of this wave, in the precision of the phase.
template <int NCHW, typename T>
struct GinvGroup {
    T v[GRID_UNR][NCHW * 4];
};

// Load the group starting at column col0 (columns clamped to j_end - 1, rows
// past ld to a valid row: their weights are 0).
template <int NCHW, typename T>
__device__ __forceinline__ void ginv_load(const T* __restrict__ G, int col0, int j_end, int ld,
                                          GinvGroup<NCHW, T>& P) {
    const int lane = threadIdx.x & 63, wave = wave_id();
#pragma unroll
    for (int u = 0; u < GRID_UNR; ++u) {
        const int col = min(col0 + u, j_end - 1);
#pragma unroll
        for (int ch = 0; ch < NCHW; ++ch) {
            const int r0 = (ch * GRID_W + wave) * 256 + lane * 4;
            const int rr = (r0 < ld) ? r0 : min(lane * 4, ld - 4);
            if constexpr (sizeof(T) == 4) {
                const float4 q4 = *reinterpret_cast<const float4*>(G + (int64_t)col * ld + rr);
                P.v[u][ch * 4 + 0] = q4.x; P.v[u][ch * 4 + 1] = q4.y;
                P.v[u][ch * 4 + 2] = q4.z; P.v[u][ch * 4 + 3] = q4.w;
            } else {
                const double2 q0 = reinterpret_cast<const double2*>(G + (int64_t)col * ld + rr)[0];
                const double2 q1 = reinterpret_cast<const double2*>(G + (int64_t)col * ld + rr)[1];
                P.v[u][ch * 4 + 0] = q0.x; P.v[u][ch * 4 + 1] = q0.y;
                P.v[u][ch * 4 + 2] = q1.x; P.v[u][ch * 4 + 3] = q1.y;
            }
        }
    }
}

// a = G^{-1} t on this workgroup's columns.  With PRE, `first` holds its first
// group, loaded by the caller before the decision so that its latency overlaps
// it (for NCHW <= 2: the larger groups would not stay in registers).
template <int NCHW, typename T, bool PRE>
__device__ __forceinline__ void grid_ginv_body(const GridArgs& g, const T* __restrict__ G,
                                               const GinvGroup<NCHW, T>& first, double* st, double* sd) {
    const int lane = threadIdx.x & 63, wave = wave_id();
    constexpr int R = NCHW * 4;
    constexpr int U = GRID_UNR;
    const int ld = g.ld, m = g.m;
    double rt[R];
#pragma unroll
    for (int ch = 0; ch < NCHW; ++ch)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = (ch * GRID_W + wave) * 256 + lane * 4 + q;
            rt[ch * 4 + q] = (r < ld) ? st[r] : 0.0;
        }
    const int j_begin = blockIdx.x * g.gw;
    const int j_end = min(m, j_begin + g.gw);
    double bs[4] = {0, 0, 0, 0};
    auto process = [&](const GinvGroup<NCHW, T>& P, int col0) {
        double dots[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            double s = 0.0;
#pragma unroll
            for (int r = 0; r < R; ++r) s = fma((double)P.v[u][r], rt[r], s);
            dots[u] = s;
        }
        wave_rs<U, 1>(dots);                          // lanes 8u..8u+7: column u of this wave
        if ((lane & 7) == 0) sd[wave * U + (lane >> 3)] = dots[0];
        __syncthreads();
        if (threadIdx.x < U) {
            const int j = col0 + threadIdx.x;
            if (j < j_end) {
                double a = 0.0;
                for (int w = 0; w < GRID_W; ++w) a += sd[w * U + threadIdx.x];
                g.a[j] = a;
                bs[0] = fma(g.b[j], a, bs[0]);
                bs[1] = fma(g.bbar[j], a, bs[1]);
                bs[2] = fma(g.Ac[j], a, bs[2]);
                bs[3] = fma(g.Acb[j], a, bs[3]);
            }
        }
        __syncthreads();
    };
    if constexpr (PRE) {
        if (j_begin < j_end) process(first, j_begin);
    }
    for (int col0 = PRE ? j_begin + U : j_begin; col0 < j_end; col0 += U) {
        GinvGroup<NCHW, T> P;
        ginv_load<NCHW, T>(G, col0, j_end, ld, P);
        process(P, col0);
    }
    block_sum_n<4>(bs, sd);
    if (threadIdx.x == 0)
        for (int q = 0; q < 4; ++q) g.pa[blockIdx.x * 4 + q] = bs[q];
}

template <int NCHW, typename T>
__device__ __forceinline__ void grid_ginv_step(const GridArgs& g, GridCtl c, const T* __restrict__ G, double* smem,
                                               double* sd) {
    const int ld = g.ld, n = g.n;
    // ---- sums of the state the last column pass produced, reduced in a fixed
    // order by the whole block: every workgroup gets bitwise the same totals
    double sums[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) sums[k] = 0.0;
    for (int q = threadIdx.x; q < g.NB; q += blockDim.x)
#pragma unroll
        for (int k = 0; k < 7; ++k) sums[k] += g.pcol[q * 8 + k];
    for (int q = threadIdx.x; q < g.NR; q += blockDim.x)
#pragma unroll
        for (int k = 0; k < 5; ++k) sums[7 + k] += g.prow[q * 8 + k];
    // this workgroup's first group of G^{-1} columns, issued after the partial
    // sums and without a condition (every launched workgroup has a column; a
    // pass that does not update leaves it unused): the waits for the sums
    // leave these loads in flight through the decision below
    constexpr bool PRE = NCHW <= 2;
    GinvGroup<NCHW, T> first;
    if constexpr (PRE) {
        const int j0 = blockIdx.x * g.gw;
        ginv_load<NCHW, T>(G, j0, min(g.m, j0 + g.gw), ld, first);
    }
    block_sum_n<12>(sums, sd);
    const double* cs = sums;          // c^T x, cbar^T x, c^T s, cbar^T s, D1, D2, Rx
    const double* ms = sums + 7;      // b^T y, bbar^T y, P1, P2, Ry
    const LPCtrl& L = *g.lc;
    const SolveParams& prm = g.prm;
    const double eps = prm.eps, nb = L.nb, nc = L.nc, zbar = L.zbar, gamma = prm.gamma;
    const int pass = c.mode;
    if (c.phase == 0) ++c.cp32; else ++c.cp64;
    if (pass == OP_PROX) { ++c.iters; if (c.phase == 1) ++c.iters64; }
    ++c.passes;
    c.tau = c.tau_n; c.kappa = c.kappa_n; c.theta = c.theta_n;
    c.ybuf = 1 - c.ybuf;
    const double tau = c.tau, kappa = c.kappa, theta = c.theta;
    const double by = ms[0], bby = ms[1], cx = cs[0], cbx = cs[1];
    int next = OP_PROX;
    if (c.fixed_mode) {
        if (pass == OP_PROX) --c.fixed_left;
        if (c.fixed_left <= 0) c.status = -1;
    } else {
        const bool post_update = (pass == OP_PROX) || (pass == OP_REFRESH && !c.first);
        bool decided = false;
        if (post_update) {
            int st = 0;
            if (tau > 0.0) {
                const double pres = sqrt(ms[2]) / tau, dres = sqrt(cs[4]) / tau;
                const double pobj = cx / tau, dobj = by / tau;
                const double gap = fabs(pobj - dobj);
                if (pres <= eps * (1.0 + nb) && dres <= eps * (1.0 + nc) &&
                    gap <= eps * (1.0 + fabs(pobj) + fabs(dobj)))
                    st = 1;
                c.pres = pres / (1.0 + nb);
                c.dres = dres / (1.0 + nc);
                c.gap = gap / (1.0 + fabs(pobj) + fabs(dobj));
                c.pobj = pobj;
                c.dobj = dobj;
                if (c.exit_pend && c.phase == 1) {     // the FP32 phase's last iterate, FP64 data
                    c.kfx = fmax(c.pres, fmax(c.dres, c.gap));
                    c.exit_pend = 0;
                }
            }
            if (!st && nb > 0.0 && by > 0.0 && sqrt(cs[5]) <= eps * by / nb) st = 2;
            if (!st && nc > 0.0 && cx < 0.0 && sqrt(ms[3]) <= eps * (-cx) / nc) st = 3;
            c.by = by;
            c.cx = cx;
            if (st) {
                if (c.phase == 0) { c.phase = 1; c.exit_pend = 1; next = OP_REFRESH; }   // confirm with FP64 data
                else c.status = st;
                decided = true;
            }
        }
        if (!decided && c.phase == 0 && c.iters >= prm.fp32_max_iters) {
            c.phase = 1; c.exit_pend = 1; next = OP_REFRESH; decided = true;
        }
        if (!decided) {
            const double rt = by - cx + zbar * theta - kappa;
            const double rth = -bby + cbx - zbar * tau + ((double)n + 1.0);
            const double inner = ms[4] + cs[6] + rt * rt + rth * rth;
            if (inner <= c.mu) {                                     // eq. (inner-stop)
                c.mu *= gamma;
                ++c.ipm;
                double tn = tau, kn = kappa, hn = theta;
                if (prm.restart_rule == 0) { if (tau >= kappa) kn *= gamma; else tn *= gamma; }
                else { const double sg = sqrt(gamma); tn *= sg; kn *= sg; hn *= sg; }
                c.tau_n = tn; c.kappa_n = kn; c.theta_n = hn;
                stall_reset(c.stall);
                next = OP_RESTART;
                decided = true;
            } else if (c.phase == 0 && pass == OP_PROX && stall_sample(c.stall, inner, c.mu)) {
                c.phase = 1;                   // FP32 precision floor reached
                c.exit_pend = 1;
                next = OP_REFRESH;
                decided = true;
            } else if (c.iters >= prm.max_iters || c.passes > prm.max_iters + 4096) {
                c.status = 4;
                decided = true;
            }
        }
    }
    c.first = 0;
    c.mode = next;
    if (c.status == 0 && next == OP_PROX) {    // the phase is unchanged on this path
        double* st = smem;
        for (int i = threadIdx.x; i < ld; i += blockDim.x) st[i] = g.t[i];
        __syncthreads();
        grid_ginv_body<NCHW, T, PRE>(g, G, first, st, sd);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *g.ctl_next = c;
}

template <int NCHW>
__global__ __launch_bounds__(512) void k_grid_ginv(GridArgs g) {
    extern __shared__ double smem[];
    __shared__ double sd[GRID_W * GRID_UNR + 64];
    const GridCtl c = *g.ctl;
    if (c.status != 0) return;
    if (c.phase == 0) grid_ginv_step<NCHW, float>(g, c, g.G32, smem, sd);
    else grid_ginv_step<NCHW, double>(g, c, g.G64, smem, sd);
}

// After every slice of a exists: the 2x2 border, the new scalars, and the
// control block for the next column pass.  One workgroup.
__global__ __launch_bounds__(256) void k_grid_border(GridArgs g) {
    __shared__ double sd[8 * 8];
    GridCtl c = *g.ctl_next;
    if (c.status == 0 && c.mode == OP_PROX) {
        double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int q = threadIdx.x; q < g.NG; q += blockDim.x)
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] += g.pa[q * 4 + k];
        for (int q = threadIdx.x; q < g.NB; q += blockDim.x)
#pragma unroll
            for (int k = 0; k < 4; ++k) v[4 + k] += g.pcol[q * 8 + k];
        block_sum_n<8>(v, sd);
        const Pending P = finish_border(g, c, v + 4, v);
        c.p0 = P.p0; c.p1 = P.p1;
        c.tau_n = P.tau1; c.kappa_n = P.kappa1; c.theta_n = P.theta1;
    } else if (c.mode == OP_REFRESH) {
        c.tau_n = c.tau; c.kappa_n = c.kappa; c.theta_n = c.theta;
    }
    if (threadIdx.x == 0) *g.ctl = c;
}

// Initial control block: Algorithm 2's start, first pass = refresh.
__global__ void k_grid_init(GridArgs g, double beta, int phase, int64_t fixed) {
    const int tid = threadIdx.x + blockIdx.x * blockDim.x;
    for (int i = tid; i < 2 * g.ld; i += blockDim.x * gridDim.x) g.Y2[i] = 0.0;
    for (int j = tid; j < g.n; j += blockDim.x * gridDim.x) { g.X[j] = 1.0; g.S[j] = 1.0; }
    if (tid == 0) {
        GridCtl c;
        c.tau = c.kappa = c.theta = 1.0;
        c.mu = beta;
        c.p0 = c.p1 = 0.0;
        c.mode = OP_REFRESH; c.phase = phase; c.status = 0; c.ybuf = 0; c.first = 1; c.exit_pend = 0;
        c.iters = c.iters64 = c.ipm = c.cp32 = c.cp64 = c.passes = 0;
        stall_reset(c.stall);
        c.fixed_left = fixed;
        c.fixed_mode = fixed > 0 ? 1 : 0;
        c.pad2 = 0;
        c.pres = c.dres = c.gap = c.pobj = c.dobj = NAN;
        c.by = c.cx = 0.0;
        c.kfx = NAN;
        c.tau_n = c.kappa_n = c.theta_n = 1.0;
        *g.ctl = c;
        *g.ctl_next = c;
    }
}

// Control block from an iterate loaded into the LP's pools (step-level API):
// first pass = refresh of that state, then `fixed` updates with no tests.
__global__ void k_grid_from_state(GridArgs g, const double* Yslice, const LPCtrl* lc, int phase, int64_t fixed) {
    const int tid = threadIdx.x + blockIdx.x * blockDim.x;
    for (int i = tid; i < g.ld; i += blockDim.x * gridDim.x) {
        const double v = (i < g.m) ? Yslice[i] : 0.0;
        g.Y2[i] = v;
        g.Y2[g.ld + i] = v;
    }
    if (tid == 0) {
        const LPCtrl& L = *lc;
        GridCtl c;
        c.tau = L.tau; c.kappa = L.kappa; c.theta = L.theta; c.mu = L.mu;
        c.p0 = c.p1 = 0.0;
        c.mode = OP_REFRESH; c.phase = phase; c.status = 0; c.ybuf = 0; c.first = 1; c.exit_pend = 0;
        c.iters = c.iters64 = c.ipm = c.cp32 = c.cp64 = c.passes = 0;
        stall_reset(c.stall);
        c.fixed_left = fixed;
        c.fixed_mode = fixed > 0 ? 1 : 0;
        c.pad2 = 0;
        c.pres = c.dres = c.gap = c.pobj = c.dobj = NAN;
        c.by = c.cx = 0.0;
        c.kfx = NAN;
        c.tau_n = L.tau; c.kappa_n = L.kappa; c.theta_n = L.theta;
        *g.ctl = c;
        *g.ctl_next = c;
    }
}

// Final iterate into the LP's pools and LPCtrl (so the common output and
// backward code see the same state as for the one-workgroup engine).
__global__ void k_grid_finish(GridArgs g, double* Ypool_slice, LPCtrl* lc) {
    const GridCtl c = *g.ctl;
    const double* y = g.Y2 + (int64_t)c.ybuf * g.ld;
    for (int i = threadIdx.x; i < g.m; i += blockDim.x) Ypool_slice[i] = y[i];
    if (threadIdx.x == 0) {
        LPCtrl& o = *lc;
        o.tau = c.tau; o.kappa = c.kappa; o.theta = c.theta; o.mu = c.mu;
        o.pres = c.pres; o.dres = c.dres; o.gap = c.gap; o.pobj = c.pobj; o.dobj = c.dobj;
        o.by = c.by; o.cx = c.cx;
        o.iters = c.iters; o.iters64 = c.iters64; o.ipm = c.ipm; o.cp32 = c.cp32; o.cp64 = c.cp64;
        o.cpl32 = 0; o.cpl64 = 0;
        o.gh64 = c.iters64; o.gh32 = c.iters - c.iters64;   // one pass over G^{-1} per update
        o.kfx = c.kfx;
        o.status = (c.status < 0) ? 0 : c.status;
        o.phase = c.phase;
        o.mode = OP_REFRESH;
    }
}

int grid_nchw(int ld) { return (ld + 256 * GRID_W - 1) / (256 * GRID_W); }

hipError_t grid_launch_iteration(int nchw, const GridArgs& g, hipStream_t st) {
    const size_t smem_col = sizeof(double) * 2 * g.ld;
    const size_t smem_ginv = sizeof(double) * g.ld;
    switch (nchw) {
    case 1: hipLaunchKernelGGL(k_grid_col<1>, dim3(g.NB), dim3(512), smem_col, st, g); break;
    case 2: hipLaunchKernelGGL(k_grid_col<2>, dim3(g.NB), dim3(512), smem_col, st, g); break;
    case 3: hipLaunchKernelGGL(k_grid_col<3>, dim3(g.NB), dim3(512), smem_col, st, g); break;
    case 4: hipLaunchKernelGGL(k_grid_col<4>, dim3(g.NB), dim3(512), smem_col, st, g); break;
    default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k_grid_red, dim3(g.NR), dim3(256), 0, st, g);
    switch (nchw) {
    case 1: hipLaunchKernelGGL(k_grid_ginv<1>, dim3(g.NG), dim3(512), smem_ginv, st, g); break;
    case 2: hipLaunchKernelGGL(k_grid_ginv<2>, dim3(g.NG), dim3(512), smem_ginv, st, g); break;
    case 3: hipLaunchKernelGGL(k_grid_ginv<3>, dim3(g.NG), dim3(512), smem_ginv, st, g); break;
    case 4: hipLaunchKernelGGL(k_grid_ginv<4>, dim3(g.NG), dim3(512), smem_ginv, st, g); break;
    default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k_grid_border, dim3(1), dim3(256), 0, st, g);
    return hipGetLastError();
}

hipError_t grid_set_smem(int ld) {
    const int bytes = (int)(sizeof(double) * 2 * ld);
    hipError_t e;
    if ((e = hipFuncSetAttribute((const void*)k_grid_col<1>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes)) != hipSuccess) return e;
    if ((e = hipFuncSetAttribute((const void*)k_grid_col<2>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes)) != hipSuccess) return e;
    if ((e = hipFuncSetAttribute((const void*)k_grid_col<3>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes)) != hipSuccess) return e;
    if ((e = hipFuncSetAttribute((const void*)k_grid_col<4>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes)) != hipSuccess) return e;
    if ((e = hipFuncSetAttribute((const void*)k_grid_ginv<1>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes)) != hipSuccess) return e;
    if ((e = hipFuncSetAttribute((const void*)k_grid_ginv<2>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes)) != hipSuccess) return e;
    if ((e = hipFuncSetAttribute((const void*)k_grid_ginv<3>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes)) != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_grid_ginv<4>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}
