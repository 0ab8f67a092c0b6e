// Grid engine: one LP spread over the whole GPU, three kernels per inner
// iteration of Algorithm 2 (Section 4.2 relaxation, Section 4.1 tests,
// Section 5 restart), replayed as hipGraphs of 16 iterations and driven from
// the host in chunks of iterations.  Kernel boundaries are the only
// synchronisation between workgroups.
//
//   k_grid_col   columns split over NB workgroups.  Each workgroup issues its
//                first group of columns, then reduces the partial sums of the
//                last pass (check sums, border dots of a) in a fixed order and
//                takes the decision on it (final test, inner test, restart,
//                phase switch) and, for an update, solves its 2x2 border
//                (Section 4.4) -- every workgroup the same, redundantly -- and
//                forms its lanes' rows of y' = alpha (a - Z_y p) + (1-alpha) y;
//                workgroup 0 publishes the state and y'.  Then it streams its
//                columns of A once: (A^T a)_j, (A^T y')_j, the relaxed prox /
//                dual update of x_j, s_j, and the accumulation of
//                A[:,j](x'_j + s'_j) and A[:,j] x'_j into per-workgroup partial
//                m-vectors (waves own disjoint row ranges, so no cross-wave
//                reduction of the partials is needed).
//   k_grid_red   rows split over workgroups: sums the partials into A(x+s), A x,
//                forms t = y' - A(x+s) and the row-side sums of the check.
//   k_grid_ginv  every workgroup its slice of a = G^{-1} t and the partial
//                border dots (whatever the coming decision: an unused a costs
//                less than waiting for the decision); workgroup 0 hands the
//                pass's state on to the next column pass.
// The column pass's own sums alternate between two buffers by pass parity, so
// no workgroup reads sums that its launch is writing.  For A = [A0, -A0] the
// column pass reads A0 alone and handles column j and j + n/2 together.  With
// the adaptive beta (Section 4.3) a decision that reaches a step of the beta
// choice pauses the pass; workgroup 0 of the k_grid_ginv launch that follows
// takes the step and the next column pass resumes from the paused pass's sums.
// All sums are reduced in a fixed order, so runs are bitwise reproducible.
#include <hip/hip_runtime.h>
#include "abip_internal.h"
#include "abip_grid.h"

#define GRID_W 8               // waves per workgroup (512 threads)
#define GRID_UNR 8             // columns per step in the column kernels

__device__ __forceinline__ void grid_bb_step(const GridArgs& g, const GridCtl& c, double* sbuf, bool write_ctl);

// Border, scalars and y' of a pending update, computed identically by every
// workgroup from the published partial dots.
struct Pending {
    double p0, p1, tau1, kappa1, theta1;
};

// cs0..cs3: c^T x, cbar^T x, c^T s, cbar^T s of the current state; ad0..ad3:
// b^T a, bbar^T a, (A c)^T a, (A cbar)^T a (scalars, so nothing needs an address)
__device__ __forceinline__ Pending finish_border(const GridArgs& g, const GridCtl& c, double cs0, double cs1,
                                                double cs2, double cs3, double ad0, double ad1, double ad2,
                                                double ad3) {
    const LPCtrl& L = *g.lc;
    const double alpha = g.prm.alpha;
    const double np1 = (double)g.n + 1.0;
    const double h1z = -ad0 + (cs0 + cs2) + ad2;
    const double h2z = ad1 - (cs1 + cs3) - ad3;
    const double q0 = (c.tau + c.kappa) + h1z;
    const double q1 = (c.theta - np1) + h2z;
    Pending P;
    P.p0 = L.K00 * q0 + L.K01 * q1;
    P.p1 = L.K10 * q0 + L.K11 * q1;
    const double tmu = c.mu / c.beta;
    const double uh_tau = alpha * P.p0 + (1.0 - alpha) * c.tau;
    P.theta1 = alpha * P.p1 + (1.0 - alpha) * c.theta;
    P.tau1 = prox_root(uh_tau - c.kappa, tmu);
    P.kappa1 = c.kappa - uh_tau + P.tau1;
    return P;
}

// The decision after a column pass: the Section 4.1 tests, the inner test
// (eq. inner-stop), the restart, the FP32 -> FP64 switch.  Taken at the start
// of the next column pass by every thread of every workgroup from the same
// sums (sm: c^T x, cbar^T x, c^T s, cbar^T s, D1, D2, Rx of the column side;
// b^T y, bbar^T y, P1, P2, Ry of the row side), so all reach the same c.
__device__ __forceinline__ void grid_decide(const GridArgs& g, GridCtl& c, const double (&sm)[16]) {
    const int n = g.n;
    const double* cs = sm;
    const double* ms = sm + 7;
    const LPCtrl& L = *g.lc;
    const SolveParams& prm = g.prm;
    const double eps = prm.eps, nb = L.nb, nc = L.nc, zbar = L.zbar, gamma = prm.gamma;
    const int pass = c.mode;
    const bool bb_on = (c.bbf & GBB_ON) != 0;
    const bool bb_pass = bb_on && ((c.bbf >> GBB_STAGE_SHIFT) & 3) != 0;   // a probe or the restored start: no tests
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
        bool decided = bb_pass;
        if (post_update && !bb_pass) {
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
                if (bb_on) c.bbf |= GBB_PEND;                        // the new outer iteration chooses its beta
                next = OP_RESTART;
                decided = true;
            } else if (c.phase == 0 && pass == OP_PROX && stall_sample(c.stall, inner, c.mu)) {
                c.phase = 1;                   // FP32 precision floor reached
                c.exit_pend = 1;
                next = OP_REFRESH;
                decided = true;
            } else if ((c.iters >= prm.max_iters && !(bb_on && (c.bbf & GBB_PEND))) || c.passes > prm.max_iters + 4096) {
                c.status = 4;
                decided = true;
            }
        }
        // a beta step (Section 4.3) after the tests of an outer iteration's first pass
        // or of a probe: the grid pauses (status -2) and the host runs k_grid_bb_step
        if ((!decided || bb_pass) && c.status == 0 && bb_on && ((c.bbf & GBB_PEND) || bb_pass)) {
            c.bbf = (c.bbf & ~GBB_WAS_UPDATE) | (pass == OP_PROX ? GBB_WAS_UPDATE : 0);
            c.status = -2;
        }
    }
    c.first = 0;
    c.mode = next;
}

// ---------------------------------------------------------------------------
// k_grid_col
// ---------------------------------------------------------------------------
// Takes the pending decision of the last pass first.  Returns true when that
// decision moves the LP to FP64 data: the caller then runs the FP64
// instantiation, which takes the same decision again from the same inputs.
// MIR (A = [A0, -A0], g.n2 = n / 2 column pairs): the pass reads the columns of
// A0 only; column j + n2 of A takes the negated products of column j, and the
// pair adds A0 (f_j - f_{j+n2}) to the row sums.
template <int NCHW, typename T, int U, bool MIR>
__device__ bool grid_col_body(const GridArgs& g, const T* __restrict__ A, double* sd) {
    GridCtl c = *g.ctl_next;                   // the last pass, its decision pending (c.decide)
    const bool decide = c.decide != 0;
    const bool resume = (c.bbf & GBB_RESUME) != 0;   // decided before a beta step: take its sums only
    const int lane = threadIdx.x & 63, wave = wave_id();
    constexpr int R = NCHW * 4;
    const int ld = g.ld, n = g.n, m = g.m;
    // the pass's operation and scalars, set once the border of the pending
    // update is known (below)
    int op = OP_REFRESH;
    bool prox = false;
    double p0 = 0.0, p1 = 0.0, tau = 0.0, theta = 0.0, tmu = 0.0;
    // this lane's rows (wave w, chunk ch -> rows (ch*GRID_W + w)*256 + 4*lane + q):
    // a of the pending update, the y' this pass produces, the partial sums
    double ra[R], ry[R], accf[R], accx[R];
    const double alpha = g.prm.alpha, gamma = g.prm.gamma;
    const double sg = sqrt(gamma);
    const int rule = g.prm.restart_rule;
    const int ncol = MIR ? g.n2 : n;               // columns (pairs) the pass walks
    const int j_begin = blockIdx.x * g.cw;
    const int j_end = min(ncol, j_begin + g.cw);
    constexpr int LU = MIR ? 2 * U : U;            // lanes that own a column of a group
    double acc7[7] = {0, 0, 0, 0, 0, 0, 0};
    T va[U][R], vb[U][R];
    // per-column data of a group, loaded with it by lanes u < LU (lane u: column
    // col0 + u, with MIR lane U + u: its pair col0 + u + n2; the other lanes load
    // a valid neighbour and ignore it)
    struct ColData { double x, s, z0, z1, c, cb; };
    ColData da_, db_;
    // unmasked loads from clamped addresses: rows past ld have zero weights,
    // columns past j_end are skipped with a uniform test in step()
    const int rl = min(lane * 4, ld - 4);
    auto load_cols = [&](int col0, ColData& cd) {
        int j;
        if constexpr (MIR) {
            j = min(col0 + (lane < LU ? (lane & (U - 1)) : 0), j_end - 1);
            if (lane >= U && lane < LU) j += g.n2;
        } else {
            j = min(col0 + (lane < U ? lane : 0), j_end - 1);
        }
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
    // One barrier per group: the waves' partial dots go to one of two halves of
    // sd (alternating, so a wave can start writing the next group's while a
    // slower one still reads this group's); then every wave finishes the group's
    // columns itself (lanes u < U: column u, the same values in every wave) and
    // hands x', x'+s' to its lanes by readlane.  Wave 0 alone stores x', s' and
    // accumulates the column-side sums.
    int half = 0;
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
        double* sdh = sd + half * (GRID_W * 2 * GRID_UNR);
        half ^= 1;
        if ((lane % LPC) == 0) {
            const int u = lane / LPC;
            sdh[wave * 2 * U + 2 * u] = dots[0];
            sdh[wave * 2 * U + 2 * u + 1] = dots[1];
        }
        __syncthreads();
        double x1 = 0.0, s1 = 0.0;
        if (lane < LU) {
            const int u = MIR ? (lane & (U - 1)) : lane;
            const int j = col0 + u;
            double ata = 0.0, aty = 0.0;
            for (int w = 0; w < GRID_W; ++w) { ata += sdh[w * 2 * U + 2 * u]; aty += sdh[w * 2 * U + 2 * u + 1]; }
            if (MIR && lane >= U) { ata = -ata; aty = -aty; }   // column j + n2 = -(column j)
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
                if (wave == 0) {
                    const int jj = (MIR && lane >= U) ? j + g.n2 : j;
                    if (op != OP_REFRESH) { g.X[jj] = x1; g.S[jj] = s1; }
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
            }
        }
        const double f1 = x1 + s1;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            double xu = bcast_lane(x1, u), fu = bcast_lane(f1, u);   // 0 past j_end
            if constexpr (MIR) { xu -= bcast_lane(x1, U + u); fu -= bcast_lane(f1, U + u); }
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
    // the partial sums of the last pass (check sums of the column and row
    // passes, border dots of a), issued first so that waiting for them leaves
    // the first group of columns (issued next) in flight
    // The partial sums of the last pass (check sums of the column and row
    // passes, border dots of a: at most 2 x 512 workgroups each, two per
    // thread), then with one row chunk per lane this lane's rows of a, Z_y and
    // the current y, then the first group of columns.  No loop among them, so
    // waiting for the first loads leaves the later ones in flight.
    // The column sums sit in two buffers by the parity of the pass count: this
    // pass reads the last pass's while its own workgroups, which may finish
    // before a late one starts, write the other.
    double sm[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) sm[k] = 0.0;
    if (decide) {
        const double* pc = g.pcol + ((resume ? c.passes - 1 : c.passes) & 1) * (int64_t)g.pcol_stride;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int q = threadIdx.x + h * 512;
            if (q < g.NB) {
#pragma unroll
                for (int k = 0; k < 7; ++k) sm[k] += pc[q * 8 + k];
            }
            if (q < g.NR) {
#pragma unroll
                for (int k = 0; k < 5; ++k) sm[7 + k] += g.prow[q * 8 + k];
            }
            if (q < g.NG) {
#pragma unroll
                for (int k = 0; k < 4; ++k) sm[12 + k] += g.pa[q * 4 + k];
            }
        }
    }
    constexpr bool EARLY = NCHW == 1;
    constexpr int RE = EARLY ? 4 : 1;
    double ea[RE], ez0[RE], ez1[RE], ey[RE];
    if constexpr (EARLY) {
        const double* yc0 = g.Y2 + (int64_t)(decide && !resume ? 1 - c.ybuf : c.ybuf) * ld;   // a decision flips it
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = wave * 256 + lane * 4 + q;
            const bool in = r < m;
            ea[q] = in ? g.a[r] : 0.0;
            ez0[q] = in ? g.Zy0[r] : 0.0;
            ez1[q] = in ? g.Zy1[r] : 0.0;
            ey[q] = in ? yc0[r] : 0.0;
        }
    }
    int c0 = j_begin;
    if (c0 < j_end) { load(c0, va); load_cols(c0, da_); }
    if (decide) {
        block_sum_n<16>(sm, sd);
        if (!resume) grid_decide(g, c, sm);
        c.bbf &= ~GBB_RESUME;
        if (c.status != 0) {
            if (blockIdx.x == 0 && threadIdx.x == 0) *g.ctl = c;
            return false;
        }
        if (c.phase != (sizeof(T) == 4 ? 0 : 1)) return true;
    }
    // the border (Section 4.4) of an update, from the same sums in the same
    // order in every workgroup
    op = c.mode;
    prox = (op == OP_PROX);
    if (prox) {
        const Pending P = finish_border(g, c, sm[0], sm[1], sm[2], sm[3], sm[12], sm[13], sm[14], sm[15]);
        c.p0 = P.p0; c.p1 = P.p1;
        c.tau_n = P.tau1; c.kappa_n = P.kappa1; c.theta_n = P.theta1;
    } else if (op == OP_REFRESH) {
        c.tau_n = c.tau; c.kappa_n = c.kappa; c.theta_n = c.theta;
    }
    c.decide = 1;                                  // this pass's decision comes next
    if (blockIdx.x == 0 && threadIdx.x == 0) *g.ctl = c;      // the state k_grid_red / k_grid_ginv read
    // the buffer this pass's column sums go to (pass parity after its decision)
    const int pw = __builtin_amdgcn_readfirstlane((int)(c.passes & 1));
    tau = c.tau; theta = c.theta;
    if (prox) { p0 = c.p0; p1 = c.p1; tau = c.tau_n; theta = c.theta_n; }   // scalars of the new state
    else if (op == OP_RESTART) { tau = c.tau_n; theta = c.theta_n; }
    tmu = c.mu / c.beta;
    // the same in every lane: scalar registers for the column loop
    op = __builtin_amdgcn_readfirstlane(op);
    prox = op == OP_PROX;
    p0 = bcast_first(p0); p1 = bcast_first(p1);
    tau = bcast_first(tau); theta = bcast_first(theta); tmu = bcast_first(tmu);
    // y' = alpha (a - Z_y p) + (1 - alpha) y for an update, sqrt(gamma) y or y
    // otherwise, for this lane's rows (past m: 0); workgroup 0 publishes it as
    // the next y
    {
        const double* ycur = g.Y2 + (int64_t)c.ybuf * ld;
        double* ynext = g.Y2 + (int64_t)(1 - c.ybuf) * ld;
        const double f = (op == OP_RESTART && rule == 1) ? sg : 1.0;
#pragma unroll
        for (int ch = 0; ch < NCHW; ++ch) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = ch * 4 + q;
                const int r = (ch * GRID_W + wave) * 256 + lane * 4 + q;
                double yv = 0.0, av = 0.0;
                if (r < m) {
                    double ya, yz0, yz1, yc;
                    if constexpr (EARLY) { ya = ea[q]; yz0 = ez0[q]; yz1 = ez1[q]; yc = ey[q]; }
                    else { ya = g.a[r]; yz0 = g.Zy0[r]; yz1 = g.Zy1[r]; yc = ycur[r]; }
                    if (prox) {
                        av = ya;
                        yv = alpha * (av - yz0 * p0 - yz1 * p1) + (1.0 - alpha) * yc;
                    } else {
                        yv = f * yc;
                    }
                }
                ra[k] = av;
                ry[k] = yv;
                accf[k] = 0.0;
                accx[k] = 0.0;
                if (blockIdx.x == 0 && r < ld) ynext[r] = yv;
            }
        }
    }
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
    block_sum_n<8>(t8, sd + 2 * GRID_W * 2 * GRID_UNR);      // apart from the halves the last group read
    if (threadIdx.x == 0) {
        double* pc = g.pcol + pw * (int64_t)g.pcol_stride;
        for (int q = 0; q < 8; ++q) pc[blockIdx.x * 8 + q] = t8[q];
    }
    return false;
}

template <int NCHW, bool MIR>
__global__ __launch_bounds__(512) void k_grid_col(GridArgs g) {
    __shared__ double sd[2 * GRID_W * 2 * GRID_UNR + 64];
    const GridCtl& c = *g.ctl_next;
    if (c.status != 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) *g.ctl = c;
        return;
    }
    // paired: half the columns per group (each owns two columns of the pass)
    constexpr int U32 = (NCHW == 1 && !MIR) ? 8 : 4, U64 = NCHW == 1 ? 4 : 2;
    if (c.phase == 0) {
        if (grid_col_body<NCHW, float, U32, MIR>(g, g.A32, sd))
            grid_col_body<NCHW, double, U64, MIR>(g, g.A64, sd);     // switched to FP64 data
    } else {
        grid_col_body<NCHW, double, U64, MIR>(g, g.A64, sd);
    }
}

// ---------------------------------------------------------------------------
// k_grid_red: rows
// ---------------------------------------------------------------------------
// GRID_RED_ROWS rows per workgroup; 32 thread groups per row each sum every
// 32nd partial vector (four per round so the loads overlap), then the group
// sums of a row are added in group order.
#define GRID_RED_G (256 / GRID_RED_ROWS)

__global__ __launch_bounds__(256) void k_grid_red(GridArgs g) {
    __shared__ double sbuf[5 * 4];
    __shared__ double sf[GRID_RED_G][GRID_RED_ROWS], sx[GRID_RED_G][GRID_RED_ROWS];
    const int r = threadIdx.x % GRID_RED_ROWS, grp = threadIdx.x / GRID_RED_ROWS;
    const int i = blockIdx.x * GRID_RED_ROWS + r;
    const int ld = g.ld, m = g.m, NB = g.NB;
    constexpr int GS = GRID_RED_G;
    double f = 0.0, x = 0.0;
    if (i < ld) {
        int q = grp;
        for (; q + 3 * GS < NB; q += 4 * GS) {
            const double f0 = g.Pf[(int64_t)q * ld + i], f1 = g.Pf[(int64_t)(q + GS) * ld + i];
            const double f2 = g.Pf[(int64_t)(q + 2 * GS) * ld + i], f3 = g.Pf[(int64_t)(q + 3 * GS) * ld + i];
            const double x0 = g.Px[(int64_t)q * ld + i], x1 = g.Px[(int64_t)(q + GS) * ld + i];
            const double x2 = g.Px[(int64_t)(q + 2 * GS) * ld + i], x3 = g.Px[(int64_t)(q + 3 * GS) * ld + i];
            f += f0; f += f1; f += f2; f += f3;
            x += x0; x += x1; x += x2; x += x3;
        }
        for (; q < NB; q += GS) { f += g.Pf[(int64_t)q * ld + i]; x += g.Px[(int64_t)q * ld + i]; }
    }
    // the partial sums above are read whatever the state (a finished solve
    // leaves them unused), so their loads do not wait for the control block
    const GridCtl& c = *g.ctl;
    if (c.status != 0) return;
    sf[grp][r] = f;
    sx[grp][r] = x;
    __syncthreads();
    const double* y = g.Y2 + (int64_t)(1 - c.ybuf) * ld;    // y of the new state
    const double tau = c.tau_n, theta = c.theta_n;
    double ms[5] = {0, 0, 0, 0, 0};
    if (grp == 0 && i < ld) {
        double F = 0.0, X = 0.0;
#pragma unroll
        for (int k = 0; k < GS; ++k) { F += sf[k][r]; X += sx[k][r]; }
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
// k_grid_ginv: slice of a = G^{-1} t
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

// a = G^{-1} t on this workgroup's columns, computed whatever the decision (a
// pass that is not followed by an update leaves it unused); the first group of
// columns and this lane's rows of t are loaded together at the start.
template <int NCHW, typename T>
__device__ void grid_ginv_body(const GridArgs& g, const T* __restrict__ G, double* sd) {
    const int lane = threadIdx.x & 63, wave = wave_id();
    constexpr int R = NCHW * 4;
    constexpr int U = GRID_UNR;
    const int ld = g.ld, m = g.m;
    const int j_begin = blockIdx.x * g.gw;
    const int j_end = min(m, j_begin + g.gw);
    GinvGroup<NCHW, T> first;
    ginv_load<NCHW, T>(G, j_begin, j_end, ld, first);       // every launched workgroup has a column
    double rt[R];
#pragma unroll
    for (int ch = 0; ch < NCHW; ++ch) {
        const int r0 = (ch * GRID_W + wave) * 256 + lane * 4;
        double2 t01 = make_double2(0.0, 0.0), t23 = make_double2(0.0, 0.0);
        if (r0 < ld) {                                   // ld is a multiple of 4
            t01 = reinterpret_cast<const double2*>(g.t + r0)[0];
            t23 = reinterpret_cast<const double2*>(g.t + r0)[1];
        }
        rt[ch * 4 + 0] = t01.x; rt[ch * 4 + 1] = t01.y; rt[ch * 4 + 2] = t23.x; rt[ch * 4 + 3] = t23.y;
    }
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
    process(first, j_begin);
    for (int col0 = j_begin + U; col0 < j_end; col0 += U) {
        GinvGroup<NCHW, T> P;
        ginv_load<NCHW, T>(G, col0, j_end, ld, P);
        process(P, col0);
    }
    block_sum_n<4>(bs, sd);
    if (threadIdx.x == 0)
        for (int q = 0; q < 4; ++q) g.pa[blockIdx.x * 4 + q] = bs[q];
}

template <int NCHW>
__global__ __launch_bounds__(512) void k_grid_ginv(GridArgs g) {
    __shared__ double sd[GRID_W * GRID_UNR + 64];
    const GridCtl& c = *g.ctl;
    // the pass's state, for the next column pass (which decides on it)
    if (blockIdx.x == 0 && threadIdx.x == 0) *g.ctl_next = c;
    if (c.status != 0) {
        if (c.status == -2 && blockIdx.x == 0) {   // the decision paused for a beta step: take it here
            __syncthreads();
            grid_bb_step(g, c, sd, false);
        }
        return;
    }
    if (c.phase == 0) grid_ginv_body<NCHW, float>(g, g.G32, sd);
    else grid_ginv_body<NCHW, double>(g, g.G64, sd);
}

// Initial control block: Algorithm 2's start, first pass = refresh.
// One step of the choice of an outer iteration's beta (Section 4.3), run by one
// workgroup while the grid is paused (status -2) after the tests of the pass
// that starts the outer iteration (stage 0) or of a probe pass; the same steps
// as the one-workgroup engines':
//   stage 0 -> 1: the start point (y, x, s, tau, kappa, theta) is kept, the first
//                 probe update follows;
//   stage 1, after the first probe's pass -> 2: its iterate is kept;
//   stage 2, after the second probe's pass: the five sums of the estimate, the
//                 selection rule, the start point restored; -> 1 (a redo: the
//                 probes again with the estimate) or 3 (final), the next pass a
//                 refresh of the restored point;
//   stage 3, after that refresh -> 0: the outer iteration's own updates begin.
// Then the grid resumes: the next column pass takes the paused pass's sums.
// Run by workgroup 0 of the k_grid_ginv launch that follows the pausing
// decision (the other workgroups have nothing to do then), so a step costs no
// kernel and no host round trip; k_grid_bb_step runs it for a pause that a
// solve left to the host.  sbuf: 5 doubles per wave.  Inside k_grid_ginv the
// resumed state goes to ctl_next alone: the launch's other workgroups read ctl
// and must keep seeing the pause (their slice of a would use a stale t).
__device__ __forceinline__ void grid_bb_step(const GridArgs& g, const GridCtl& c, double* sbuf, bool write_ctl) {
    // the fields the step reads, before any thread writes (thread 0 writes at the end)
    const int tid = threadIdx.x, nt = blockDim.x, m = g.m, n = g.n;
    double* y = g.Y2 + (int64_t)c.ybuf * g.ld;
    const double alpha = g.prm.alpha;
    const int bbf = c.bbf;
    const int64_t iters = c.iters;
    double tau = c.tau, kappa = c.kappa, theta = c.theta, beta = c.beta;
    double bbs[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) bbs[q] = g.bb->bbs[q];
    int64_t bbp = g.bb->bbp;
    int est = g.bb->est, bbe = g.bb->bbe;
    int stage = (bbf >> GBB_STAGE_SHIFT) & 3;
    const int prev = stage;
    const bool bb_pass = stage != 0;
    const bool was_update = (bbf & GBB_WAS_UPDATE) != 0;
    bool pend = (bbf & GBB_PEND) != 0;
    if (bb_pass && was_update) ++bbp;          // a probe update
    if (!bb_pass) pend = false;
    bool restored = false;
    if (stage == 0) {
        for (int i = tid; i < m; i += nt) g.Y0[i] = y[i];
        for (int j = tid; j < n; j += nt) { g.X0[j] = g.X[j]; g.S0[j] = g.S[j]; }
        bbs[0] = tau; bbs[1] = kappa; bbs[2] = theta;
        stage = 1;
    } else if (stage == 1 && was_update) {
        for (int i = tid; i < m; i += nt) g.Y1[i] = y[i];
        for (int j = tid; j < n; j += nt) { g.X1[j] = g.X[j]; g.S1[j] = g.S[j]; }
        bbs[3] = tau; bbs[4] = kappa; bbs[5] = theta;
        stage = 2;
    } else if (stage == 2) {
        double q[5] = {0, 0, 0, 0, 0};
        for (int i = tid; i < m; i += nt) bb_acc(y[i] - g.Y1[i], 0.0, 0.0, alpha, q);
        for (int j = tid; j < n; j += nt) bb_acc(g.X[j] - g.X1[j], g.S[j] - g.S1[j], g.S1[j] - g.S0[j], alpha, q);
        __syncthreads();
        block_sum_n<5>(q, sbuf);
        bb_acc(tau - bbs[3], kappa - bbs[4], bbs[4] - bbs[1], alpha, q);
        bb_acc(theta - bbs[5], 0.0, 0.0, alpha, q);
        bbe += 1;
        est += 1;
        const double hat = bb_hat(q, beta, g.prm.eps_cor);
        const bool fin = bb_choose(beta, hat, g.prm.eps_pen, est, g.prm.bb_max_redo);
        for (int i = tid; i < m; i += nt) y[i] = g.Y0[i];
        for (int j = tid; j < n; j += nt) { g.X[j] = g.X0[j]; g.S[j] = g.S0[j]; }
        tau = bbs[0]; kappa = bbs[1]; theta = bbs[2];
        stage = fin ? 3 : 1;
        restored = true;
    } else if (stage == 3) {
        stage = 0;
        est = 0;
    }
    int status = 0, mode = OP_PROX;
    if (restored) mode = OP_REFRESH;           // the products of the restored point
    else if (prev == 3 && iters >= g.prm.max_iters) status = 4;
    const int nbbf = GBB_ON | (pend ? GBB_PEND : 0) | (stage << GBB_STAGE_SHIFT) | GBB_RESUME;
    __syncthreads();
    if (tid == 0) {
        for (int t = 0; t < (write_ctl ? 2 : 1); ++t) {
            GridCtl* o = (t == 0) ? g.ctl_next : g.ctl;
            o->tau = tau; o->kappa = kappa; o->theta = theta; o->beta = beta;
            if (restored) { o->tau_n = tau; o->kappa_n = kappa; o->theta_n = theta; }
            o->status = status;
            o->mode = mode;
            o->bbf = nbbf;
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) g.bb->bbs[q] = bbs[q];
        g.bb->bbp = bbp; g.bb->est = est; g.bb->bbe = bbe;
    }
}

__global__ __launch_bounds__(1024) void k_grid_bb_step(GridArgs g) {
    __shared__ double sbuf[16 * 5];
    const GridCtl& c = *g.ctl_next;
    if (c.status != -2) return;                // not paused: nothing to do
    grid_bb_step(g, c, sbuf, true);
}

// Column pairing test of one large LP: sets bit 16 of *flag unless column
// j + n2 of A equals the negated column j exactly for every j < n2 (one
// workgroup per pair; A column-major with leading dimension ld).
__global__ void k_grid_pair_check(const double* __restrict__ A, int m, int ld, int n2, int* flag) {
    const int j = blockIdx.x;
    const double* a0 = A + (int64_t)j * ld;
    const double* a1 = A + (int64_t)(j + n2) * ld;
    int bad = 0;
    for (int i = threadIdx.x; i < m; i += blockDim.x)
        if (a1[i] != -a0[i]) bad = 1;
    if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(flag, 16);
}

__global__ void k_grid_init(GridArgs g, double beta, int phase, int64_t fixed, int bb) {
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
        c.decide = 0;
        c.pres = c.dres = c.gap = c.pobj = c.dobj = NAN;
        c.by = c.cx = 0.0;
        c.kfx = NAN;
        c.tau_n = c.kappa_n = c.theta_n = 1.0;
        c.beta = beta;
        c.bbf = (bb && fixed == 0) ? (GBB_ON | GBB_PEND) : 0;
        *g.ctl = c;
        *g.ctl_next = c;
        GridBB B;
        for (int q = 0; q < 6; ++q) B.bbs[q] = 0.0;
        B.bbp = 0; B.est = 0; B.bbe = 0;
        *g.bb = B;
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
        c.decide = 0;
        c.pres = c.dres = c.gap = c.pobj = c.dobj = NAN;
        c.by = c.cx = 0.0;
        c.kfx = NAN;
        c.tau_n = L.tau; c.kappa_n = L.kappa; c.theta_n = L.theta;
        c.beta = g.prm.beta;
        c.bbf = 0;
        *g.ctl = c;
        *g.ctl_next = c;
        GridBB B;
        for (int q = 0; q < 6; ++q) B.bbs[q] = 0.0;
        B.bbp = 0; B.est = 0; B.bbe = 0;
        *g.bb = B;
    }
}

// Final iterate into the LP's pools and LPCtrl (so the common output and
// backward code see the same state as for the one-workgroup engine).
__global__ void k_grid_finish(GridArgs g, double* Ypool_slice, LPCtrl* lc) {
    const GridCtl c = *g.ctl_next;
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
        o.beta = c.beta; o.bbp = g.bb->bbp; o.bbe = g.bb->bbe;
        o.status = (c.status < 0) ? 0 : c.status;
        o.phase = c.phase;
        o.mode = OP_REFRESH;
    }
}

int grid_nchw(int ld) { return (ld + 256 * GRID_W - 1) / (256 * GRID_W); }

template <int NCHW>
static void launch_col(const GridArgs& g, hipStream_t st) {
    if (g.n2 > 0) hipLaunchKernelGGL((k_grid_col<NCHW, true>), dim3(g.NB), dim3(512), 0, st, g);
    else hipLaunchKernelGGL((k_grid_col<NCHW, false>), dim3(g.NB), dim3(512), 0, st, g);
}

hipError_t grid_launch_iteration(int nchw, const GridArgs& g, hipStream_t st) {
    switch (nchw) {
    case 1: launch_col<1>(g, st); break;
    case 2: launch_col<2>(g, st); break;
    case 3: launch_col<3>(g, st); break;
    case 4: launch_col<4>(g, st); break;
    default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k_grid_red, dim3(g.NR), dim3(256), 0, st, g);
    switch (nchw) {
    case 1: hipLaunchKernelGGL(k_grid_ginv<1>, dim3(g.NG), dim3(512), 0, st, g); break;
    case 2: hipLaunchKernelGGL(k_grid_ginv<2>, dim3(g.NG), dim3(512), 0, st, g); break;
    case 3: hipLaunchKernelGGL(k_grid_ginv<3>, dim3(g.NG), dim3(512), 0, st, g); break;
    case 4: hipLaunchKernelGGL(k_grid_ginv<4>, dim3(g.NG), dim3(512), 0, st, g); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
