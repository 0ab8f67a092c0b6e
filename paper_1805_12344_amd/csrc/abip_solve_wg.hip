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
#include "abip_small.h"

struct WGShared {
    double* y;      // ld
    double* a;      // ld
    double* t;      // ld
    double* Af;     // ld
    double* Ax;     // ld
    double* red;    // 2 * W * max(ld, 32) (at least 64 W: the triangular solves' block partials)
    double* scal;   // W * 8
    double* buf;    // W * 8
};

// One pass over the columns of A.  op: OP_REFRESH (recompute products of the
// current state), OP_PROX (the inner update), OP_RESTART (Section 5 / eq.
// update-next-iterate rescaling of x and s).  Leaves A(x+s) and A x of the new
// state in sh.Af / sh.Ax and the column-side sums in cs[7]:
//   c^T x, cbar^T x, c^T s, cbar^T s, ||A^T y + s - c tau||^2, ||A^T y + s||^2,
//   ||-A^T y + c tau - cbar theta - s||^2.
// Layout: a wave owns whole columns (chunks of 64 consecutive columns, round
// robin over the waves); lane l holds rows 4l..4l+3 of every 256-row chunk.
// PROXPASS: the pass is an update (op == OP_PROX); its group body is then
// straight-line code (no branches on op, write-backs of the lanes that do not
// lead a valid column go to the spare slot X[n], S[n] past the LP's columns).
template <int NCH, int UNR, typename T, bool PROXPASS>
__device__ __forceinline__ void column_pass(const T* __restrict__ A, int m, int n, int ld,
                                         double* __restrict__ X, double* __restrict__ S,
                                         const double* __restrict__ C, const double* __restrict__ CB,
                                         const double* __restrict__ ZX0, const double* __restrict__ ZX1,
                                         const WGShared& sh, int op, double p0, double p1, double tmu,
                                         double alpha, double gamma, int rule, double tau, double theta,
                                         double* __restrict__ cs) {
    const int lane = threadIdx.x & 63, wave = wave_id(), W = num_waves();
    constexpr int R = NCH * 4;
    constexpr int K = 2 * UNR;
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
    // column-side sums, accumulated by the lane that owns the column update
    double acc7[7] = {0, 0, 0, 0, 0, 0, 0};
    const double sg = sqrt(gamma);
    const bool prox = PROXPASS || (op == OP_PROX);
    // Groups of UNR consecutive columns go round robin over the waves, so every
    // wave has work even when n is small.  Group g+1 is loaded before group g
    // is computed: one group of column loads is always in flight behind the
    // arithmetic.  After the reduce-scatter of the column dots, the LPC lanes
    // myu*LPC .. myu*LPC+LPC-1 hold column myu of the group; the first of
    // them writes it back.
    constexpr int LPC = 64 / UNR;
    const int myu = lane / LPC;
    const bool lead = (lane % LPC) == 0;
    auto group_col = [&](int g) { return (wave + g * W) * UNR; };
    struct Grp {
        T v[UNR][R];
        double x0, s0, c0, cb0, z0, z1;
    };
    // Loads are unconditional and unmasked (addresses clamped into the LP's
    // own data): with nothing consuming them at load time the compiler keeps
    // the next group's loads in flight while the current group is computed.
    // Rows past ld carry zero weights (ra, ry) and are never written back;
    // columns past n are skipped with a wave-uniform test in compute().
    const int rl = min(lane * 4, ld - 4);             // valid row start for every lane
    auto load = [&](int col0, Grp& G) {
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const int col = min(col0 + u, n - 1);
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                const int r0 = ch * 256 + lane * 4;
                const int rr = (r0 < ld) ? r0 : rl;
                if constexpr (sizeof(T) == 4) {
                    const float4 q4 = *reinterpret_cast<const float4*>(A + (int64_t)col * ld + rr);
                    G.v[u][ch * 4 + 0] = q4.x; G.v[u][ch * 4 + 1] = q4.y;
                    G.v[u][ch * 4 + 2] = q4.z; G.v[u][ch * 4 + 3] = q4.w;
                } else {
                    const double2 q0 = reinterpret_cast<const double2*>(A + (int64_t)col * ld + rr)[0];
                    const double2 q1 = reinterpret_cast<const double2*>(A + (int64_t)col * ld + rr)[1];
                    G.v[u][ch * 4 + 0] = q0.x; G.v[u][ch * 4 + 1] = q0.y;
                    G.v[u][ch * 4 + 2] = q1.x; G.v[u][ch * 4 + 3] = q1.y;
                }
            }
        }
        // the column this lane updates (clamped: lanes past n compute and drop)
        const int jl = min(col0 + myu, n - 1);
        G.x0 = X[jl]; G.s0 = S[jl]; G.c0 = C[jl]; G.cb0 = CB[jl];
        G.z0 = ZX0[jl]; G.z1 = ZX1[jl];
    };
    auto compute = [&](int col0, const Grp& G) {
        double dots[K];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            double da = 0.0, dy = 0.0;
#pragma unroll
            for (int r = 0; r < R; ++r) {        // (A^T a)_j is only used by updates
                da = fma((double)G.v[u][r], ra[r], da);
                dy = fma((double)G.v[u][r], ry[r], dy);
            }
            dots[2 * u] = da;
            dots[2 * u + 1] = dy;
        }
        wave_rs<K, 2>(dots);
        const double ata = dots[0], aty = dots[1];        // column col0 + myu
        // the column update, computed by all LPC lanes of the column
        const int jl = col0 + myu;
        const double x0 = G.x0, s0 = G.s0, c0 = G.c0, cb0 = G.cb0;
        double x1 = x0, s1 = s0;
        if (PROXPASS || prox) {
            const double dj = (x0 + s0) + ata;                     // M^{-1} block, x part
            const double ut = dj - G.z0 * p0 - G.z1 * p1;         // u~_x
            const double uh = alpha * ut + (1.0 - alpha) * x0;    // relaxation
            x1 = prox_root(uh - s0, tmu);                         // barrier prox
            s1 = s0 - uh + x1;                                    // dual update
        } else if (op == OP_RESTART) {
            if (rule == 0) {
                if (x0 >= s0) s1 = gamma * s0;
                else x1 = gamma * x0;
            } else {
                x1 = sg * x0; s1 = sg * s0;
            }
        }
        if (PROXPASS) {
            const bool mine = lead && jl < n;
            const int js = mine ? jl : n;                          // spare slot
            X[js] = x1;
            S[js] = s1;
            const double mk = mine ? 1.0 : 0.0;
            const double r1 = (aty + s1 - c0 * tau) * mk;
            const double r2 = (aty + s1) * mk;
            const double r3 = (-aty + c0 * tau - cb0 * theta - s1) * mk;
            const double c0m = c0 * mk, cb0m = cb0 * mk;
            acc7[0] = fma(c0m, x1, acc7[0]);
            acc7[1] = fma(cb0m, x1, acc7[1]);
            acc7[2] = fma(c0m, s1, acc7[2]);
            acc7[3] = fma(cb0m, s1, acc7[3]);
            acc7[4] = fma(r1, r1, acc7[4]);
            acc7[5] = fma(r2, r2, acc7[5]);
            acc7[6] = fma(r3, r3, acc7[6]);
        } else if (lead && jl < n) {
            if (op != OP_REFRESH) { X[jl] = x1; S[jl] = s1; }
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
        // A[:, col] (x'+s') and A[:, col] x' for every row this lane holds
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const bool cv = (col0 + u) < n;                   // wave-uniform
            const double xu = cv ? bcast_lane(x1, u * LPC) : 0.0;
            const double fu = cv ? xu + bcast_lane(s1, u * LPC) : 0.0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                accf[r] = fma((double)G.v[u][r], fu, accf[r]);
                accx[r] = fma((double)G.v[u][r], xu, accx[r]);
            }
        }
    };
    // the next group's loads are issued without a condition (past n they
    // re-read column n-1 and are not used), so the number of loads in flight
    // is fixed and the waits for one group leave the next group outstanding
    Grp ga, gb;
    int g = 0;
    int c0 = group_col(0);
    if (c0 < n) load(c0, ga);
    while (c0 < n) {
        const int c1 = group_col(g + 1);
        load(c1, gb);
        compute(c0, ga);
        if (c1 >= n) break;
        const int c2 = group_col(g + 2);
        load(c2, ga);
        compute(c1, gb);
        c0 = c2;
        g += 2;
    }
    // column-side sums live in the lead lanes: one reduction per pass
    {
        double t8[8] = {acc7[0], acc7[1], acc7[2], acc7[3], acc7[4], acc7[5], acc7[6], 0.0};
        wave_sum_n<8>(t8);
#pragma unroll
        for (int q = 0; q < 7; ++q) acc7[q] = t8[q];
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

// a = G^{-1} t by column dot products over the symmetric G^{-1} (ld x m): groups
// of UNR columns go round robin over the waves, lane l holds rows 4l..4l+3 of
// every 256-row chunk, and the next group is loaded before the current one is
// reduced.
template <int NCH, int UNR, typename T>
__device__ __forceinline__ void ginv_pass(const T* __restrict__ G, int m, int ld, const WGShared& sh) {
    const int lane = threadIdx.x & 63, wave = wave_id(), W = num_waves();
    constexpr int R = NCH * 4;
    constexpr int LPC = 64 / UNR;
    double rt[R];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = ch * 256 + lane * 4 + q;
            rt[ch * 4 + q] = (r < ld) ? sh.t[r] : 0.0;
        }
    auto group_col = [&](int g) { return (wave + g * W) * UNR; };
    struct Grp { T v[UNR][R]; };
    const int rl = min(lane * 4, ld - 4);
    // unmasked loads from clamped addresses (rows past ld have zero weight rt,
    // columns past m are not written)
    auto load = [&](int col0, Grp& Gr) {
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const int col = min(col0 + u, m - 1);
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                const int r0 = ch * 256 + lane * 4;
                const int rr = (r0 < ld) ? r0 : rl;
                if constexpr (sizeof(T) == 4) {
                    const float4 q4 = *reinterpret_cast<const float4*>(G + (int64_t)col * ld + rr);
                    Gr.v[u][ch * 4 + 0] = q4.x; Gr.v[u][ch * 4 + 1] = q4.y;
                    Gr.v[u][ch * 4 + 2] = q4.z; Gr.v[u][ch * 4 + 3] = q4.w;
                } else {
                    const double2 q0 = reinterpret_cast<const double2*>(G + (int64_t)col * ld + rr)[0];
                    const double2 q1 = reinterpret_cast<const double2*>(G + (int64_t)col * ld + rr)[1];
                    Gr.v[u][ch * 4 + 0] = q0.x; Gr.v[u][ch * 4 + 1] = q0.y;
                    Gr.v[u][ch * 4 + 2] = q1.x; Gr.v[u][ch * 4 + 3] = q1.y;
                }
            }
        }
    };
    auto compute = [&](int col0, const Grp& Gr) {
        double dots[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            double s = 0.0;
#pragma unroll
            for (int r = 0; r < R; ++r) s = fma((double)Gr.v[u][r], rt[r], s);
            dots[u] = s;
        }
        wave_rs<UNR, 1>(dots);               // lanes u*LPC.. hold column col0 + u
        const int j = col0 + lane / LPC;
        if ((lane % LPC) == 0 && j < m) sh.a[j] = dots[0];
    };
    // next group issued without a condition, as in the column pass
    Grp ga, gb;
    int g = 0;
    int c0 = group_col(0);
    if (c0 < m) load(c0, ga);
    while (c0 < m) {
        const int c1 = group_col(g + 1);
        load(c1, gb);
        compute(c0, ga);
        if (c1 >= m) break;
        const int c2 = group_col(g + 2);
        load(c2, ga);
        compute(c1, gb);
        c0 = c2;
        g += 2;
    }
    for (int i = m + threadIdx.x; i < ld; i += blockDim.x) sh.a[i] = 0.0;
    __syncthreads();
}

// a = G^{-1} t with one thread per row (coalesced: column j of the symmetric
// G^{-1} is contiguous); when the block has more threads than rows, P thread
// groups split the columns and their partial sums are added in a fixed order.
// Used by the adjoint, whose kernel is not specialised on the row count.
template <typename T>
__device__ __forceinline__ void ginv_rows(const T* __restrict__ G, int m, int ld, const WGShared& sh) {
    const int nthr = blockDim.x;
    int P = nthr / ld;
    if (P < 1) P = 1;
    const int Pmax = 2 * (nthr >> 6);
    if (P > Pmax) P = Pmax;
    for (int e = threadIdx.x; e < ld * P; e += nthr) {
        const int r = e % ld, g = e / ld;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int j = g;
        for (; j + 3 * P < m; j += 4 * P) {
            s0 = fma((double)G[(int64_t)j * ld + r], sh.t[j], s0);
            s1 = fma((double)G[(int64_t)(j + P) * ld + r], sh.t[j + P], s1);
            s2 = fma((double)G[(int64_t)(j + 2 * P) * ld + r], sh.t[j + 2 * P], s2);
            s3 = fma((double)G[(int64_t)(j + 3 * P) * ld + r], sh.t[j + 3 * P], s3);
        }
        for (; j < m; j += P) s0 = fma((double)G[(int64_t)j * ld + r], sh.t[j], s0);
        sh.red[g * ld + r] = (s0 + s1) + (s2 + s3);
    }
    __syncthreads();
    for (int r = threadIdx.x; r < ld; r += nthr) {
        double s = 0.0;
        for (int g = 0; g < P; ++g) s += sh.red[g * ld + r];
        sh.a[r] = (r < m) ? s : 0.0;
    }
    __syncthreads();
}

// ---- the linear step by triangular solves (ABIP_LIN_TRSV) -----------------
// a = G^{-1} t with the cached factor G = L L^T kept instead of G^{-1}:
// L z = t, then L^T a = z, by blocked substitution over 64-row blocks.  A
// block's unknowns come from the inverse of its diagonal block of L (a 64 x 64
// product, so no step is sequential within a block); the rows below it
// (forward) or above it (backward, through the column-major copy of L^T) then
// lose the block's contribution.  L, Lt: ld x m column-major at the LP's G
// offset; Li, Lit: the diagonal blocks' inverses and their transposes, 64 x 64
// column-major each.  t (sh.t) is overwritten by z; the result goes to sh.a.
// Three barriers per block and direction.
template <typename T>
__device__ void trsv_pass(const T* __restrict__ L, const T* __restrict__ Lt, const T* __restrict__ Li,
                          const T* __restrict__ Lit, int m, int ld, const WGShared& sh) {
    const int tid = threadIdx.x, NT = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6, W = NT >> 6;
    const int nb = (m + 63) >> 6;
    const int kw = 64 / W;                     // contraction share of a wave in the block product
    double* t = sh.t;
    double* a = sh.a;
    double* part = sh.red;                     // W x 64 partial sums
    for (int dir = 0; dir < 2; ++dir) {
        const T* Lm = dir == 0 ? L : Lt;
        const T* Id = dir == 0 ? Li : Lit;
        double* v = dir == 0 ? t : a;          // the block's unknowns land here
        const double* rhs = t;                 // forward: t; backward: z, kept in t
        for (int s = 0; s < nb; ++s) {
            const int p = dir == 0 ? s : nb - 1 - s;
            const int r0 = 64 * p, rb = min(64, m - r0);
            // unknowns of block p: Id(64 x 64) times the block's right-hand side
            const T* Ib = Id + (int64_t)p * 4096;
            double acc = 0.0;
            for (int k = wave * kw; k < (wave + 1) * kw; ++k)
                if (k < rb) acc = fma((double)Ib[lane + 64 * k], rhs[r0 + k], acc);
            part[wave * 64 + lane] = acc;
            __syncthreads();
            if (tid < rb) {
                double z = 0.0;
                for (int q = 0; q < W; ++q) z += part[q * 64 + tid];
                v[r0 + tid] = z;
            }
            __syncthreads();
            // the other rows lose the block's contribution: forward the rows below
            // (L's block column p), backward the rows above (L^T's block column p)
            const int i0 = dir == 0 ? r0 + rb : 0, i1 = dir == 0 ? m : r0;
            for (int i = i0 + tid; i < i1; i += NT) {
                const T* col = Lm + (int64_t)r0 * ld + i;
                double acc2 = 0.0;
                for (int k = 0; k < rb; ++k) acc2 = fma((double)col[(int64_t)k * ld], v[r0 + k], acc2);
                t[i] -= acc2;
            }
            __syncthreads();
        }
    }
}

// ---- adaptive beta (Section 4.3) -------------------------------------------
// One step of the choice of an outer iteration's beta, called after the tests
// of a pass that starts the outer iteration (stage 0) or of a probe pass:
//   stage 0 -> 1: the initial point (y, x, s, tau, kappa, theta) is kept, the
//                 first probe update follows;
//   stage 1, after the first probe's pass -> 2: its iterate is kept;
//   stage 2, after the second probe's pass: the five sums of the estimate (every
//                 thread gets the totals), the selection rule, the initial point
//                 restored; -> 1 (a redo: the probes again with the estimate) or
//                 3 (final); restored = true: the caller refreshes the products;
//   stage 3, the refresh of the initial point -> 0: the outer iteration's own
//                 updates begin.
// The copies live in the pools (MF_BBY*, NF_BB*) and the scalars in ctrl[k].bbs.
struct BBStep {
    double tau, kappa, theta, beta;
    int stage, est, bbe;
    bool restored;
};
__device__ __noinline__ BBStep bb_advance_wg(int k, const LPDesc& d, const PoolPtrs& P, LPCtrl* __restrict__ ctrl,
                                             const WGShared& sh, int stage, bool was_update, double tau,
                                             double kappa, double theta, double beta, const SolveParams& prm,
                                             int est, int bbe) {
    BBStep r{tau, kappa, theta, beta, stage, est, bbe, false};
    const int m = d.m, n = d.n, tid = threadIdx.x;
    double* X = P.Nv + NF_X * P.Ntot + d.on;
    double* S = P.Nv + NF_S * P.Ntot + d.on;
    double* Y0 = P.Mv + MF_BBY0 * P.Mtot + d.om;
    double* Y1 = P.Mv + MF_BBY1 * P.Mtot + d.om;
    double* X0 = P.Nv + NF_BBX0 * P.Ntot + d.on;
    double* S0 = P.Nv + NF_BBS0 * P.Ntot + d.on;
    double* X1 = P.Nv + NF_BBX1 * P.Ntot + d.on;
    double* S1 = P.Nv + NF_BBS1 * P.Ntot + d.on;
    double* bbs = ctrl[k].bbs;             // every thread writes the same values
    const double alpha = prm.alpha;
    if (stage == 0) {
        for (int i = tid; i < m; i += blockDim.x) Y0[i] = sh.y[i];
        for (int j = tid; j < n; j += blockDim.x) { X0[j] = X[j]; S0[j] = S[j]; }
        bbs[0] = tau; bbs[1] = kappa; bbs[2] = theta;
        r.stage = 1;
    } else if (stage == 1 && was_update) {
        for (int i = tid; i < m; i += blockDim.x) Y1[i] = sh.y[i];
        for (int j = tid; j < n; j += blockDim.x) { X1[j] = X[j]; S1[j] = S[j]; }
        bbs[3] = tau; bbs[4] = kappa; bbs[5] = theta;
        r.stage = 2;
    } else if (stage == 2) {
        double q[5] = {0, 0, 0, 0, 0};
        for (int i = tid; i < m; i += blockDim.x) bb_acc(sh.y[i] - Y1[i], 0.0, 0.0, alpha, q);
        for (int j = tid; j < n; j += blockDim.x) bb_acc(X[j] - X1[j], S[j] - S1[j], S1[j] - S0[j], alpha, q);
        __syncthreads();
        block_sum_n<5>(q, sh.buf);
        bb_acc(tau - bbs[3], kappa - bbs[4], bbs[4] - bbs[1], alpha, q);
        bb_acc(theta - bbs[5], 0.0, 0.0, alpha, q);
        r.bbe = bbe + 1;
        r.est = est + 1;
        const double hat = bb_hat(q, beta, prm.eps_cor);
        const bool fin = bb_choose(r.beta, hat, prm.eps_pen, r.est, prm.bb_max_redo);
        for (int i = tid; i < m; i += blockDim.x) sh.y[i] = Y0[i];
        for (int j = tid; j < n; j += blockDim.x) { X[j] = X0[j]; S[j] = S0[j]; }
        r.tau = bbs[0]; r.kappa = bbs[1]; r.theta = bbs[2];
        __syncthreads();
        r.stage = fin ? 3 : 1;
        r.restored = true;
    } else if (stage == 3) {
        r.stage = 0;
        r.est = 0;
    }
    return r;
}

// Solve (or iterate) one LP with the calling workgroup.
// fixed_iters > 0: run exactly that many PROX iterations with no tests and no
// restarts (phase taken from ctrl.phase), for step-level parity checks.
// NCH: 256-row chunks the LP needs; MAXT: the launch's largest block (512 leaves
// 256 registers per lane, 256 leaves room for 8-column groups).
// BB: the adaptive beta of Section 4.3 is compiled in (launches with
// settings.bb); the plain variant carries none of its code in the loop.
template <int NCH, int MAXT, bool BB, bool TRSV>
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

    const LPCtrl cl = ctrl[k];
    double tau = cl.tau, kappa = cl.kappa, theta = cl.theta, mu = cl.mu;
    int64_t iters = cl.iters, iters64 = cl.iters64, ipm = cl.ipm;
    int64_t cp32 = cl.cp32, cp64 = cl.cp64;
    int64_t gh32 = cl.gh32, gh64 = cl.gh64;
    double kfx = cl.kfx;
    bool exit_pend = (cl.flags & 8) != 0;     // the next FP64 check measures the FP32 exit
    int phase = cl.phase;
    int op = cl.mode;          // first pass: OP_REFRESH of the loaded state
    int status = cl.status;
    const int check_final_first = cl.flags & 1;   // a loaded post-update state: test it
    double pres = cl.pres, dres = cl.dres, gap = cl.gap, pobj = cl.pobj, dobj = cl.dobj;
    // raw sums of the last final test; the reported ratios are formed once at the end
    double l_ms2 = 0.0, l_cs4 = 0.0, l_tau = 0.0;
    bool l_have = false;
    double by_last = cl.by, cx_last = cl.cx;
    const double zbar = cl.zbar, nb = cl.nb, nc = cl.nc;
    const double alpha = prm.alpha, gamma = prm.gamma, eps = prm.eps;
    const double np1 = (double)n + 1.0;
    // Section 4.3: beta of the current outer iteration; bb_pend: the outer
    // iteration has not chosen it yet; bb_stage 1 / 2: the first / second probe
    // update has run (its pass computes the probe iterate's x, s), 3: the
    // initial point is restored after the final estimate
    double beta = BB ? cl.beta : prm.beta;
    bool bb_pend = BB && (cl.flags & 16) != 0;
    int bb_stage = 0, bbe = cl.bbe, bb_est_run = 0;
    int64_t bbp = cl.bbp;

    for (int i = tid; i < ld; i += blockDim.x) sh.y[i] = (i < m) ? Yg[i] : 0.0;
    for (int i = tid; i < ld; i += blockDim.x) sh.a[i] = 0.0;
    __syncthreads();

    double p0 = 0.0, p1 = 0.0;
    int pass_kind = op;          // what the column pass does
    bool first = true;
    int64_t done_fixed = 0;
    StallTrack stall;
    stall_reset(stall);
    // every pass is an update, a restart or a refresh; restarts and refreshes
    // without updates are bounded by this cap so the loop always ends
    int64_t passes = 0;
    const int64_t pass_cap = prm.max_iters + 4096;
    int64_t cyc_col = 0, cyc_ginv = 0, cyc_all = 0, cyc_chk = 0, cyc_upd = 0;
    const int64_t t_start = wall_clock64();
    while (true) {
        if (++passes > pass_cap && fixed_iters == 0) { status = 4; break; }
        const double tmu = mu / beta;      // t = mu / beta, eq. (Simple-Update:Barrier-X)
        double cs[7];
        const int64_t t0 = wall_clock64();
        if (phase == 0) {
            if (pass_kind == OP_PROX)
                column_pass<NCH, (NCH == 1 ? (MAXT <= 256 ? 8 : 4) : NCH == 2 ? 4 : 2), float, true>(
                    A32, m, n, ld, X, S, C, CBv, ZX0, ZX1, sh, pass_kind, p0, p1, tmu, alpha, gamma,
                    prm.restart_rule, tau, theta, cs);
            else
                column_pass<NCH, (NCH <= 2 ? 4 : 2), float, false>(
                    A32, m, n, ld, X, S, C, CBv, ZX0, ZX1, sh, pass_kind, p0, p1, tmu, alpha, gamma,
                    prm.restart_rule, tau, theta, cs);
        } else {
            if (pass_kind == OP_PROX)
                column_pass<NCH, (NCH == 1 ? 4 : 2), double, true>(
                    A64, m, n, ld, X, S, C, CBv, ZX0, ZX1, sh, pass_kind, p0, p1, tmu, alpha, gamma,
                    prm.restart_rule, tau, theta, cs);
            else
                column_pass<NCH, 2, double, false>(
                    A64, m, n, ld, X, S, C, CBv, ZX0, ZX1, sh, pass_kind, p0, p1, tmu, alpha, gamma,
                    prm.restart_rule, tau, theta, cs);
        }
        cyc_col += wall_clock64() - t0;
        if (phase == 0) ++cp32; else ++cp64;
        const bool post_update = (pass_kind == OP_PROX) || (first && check_final_first) ||
                                 (pass_kind == OP_REFRESH && !first);
        const bool was_update = (pass_kind == OP_PROX);
        const bool bb_pass = BB && bb_stage != 0;  // a probe iterate or the restored start: no tests
        if (pass_kind == OP_PROX) {
            ++iters;
            if (phase == 1) ++iters64;
            if (BB && bb_pass) ++bbp;
            ++done_fixed;
        }
        first = false;
        if (fixed_iters > 0 && done_fixed >= fixed_iters) break;

        // ---- m-side sums of the check (Section 4.1) and of ||Qu - v||^2
        const int64_t tc = wall_clock64();
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

        if (fixed_iters == 0 && !bb_pass) {
            // ---- final test on a post-update iterate
            if (post_update) {
                int st = 0;
                // Section 4.1's tests multiplied through by tau (> 0) and
                // squared: no square roots or divisions on the per-iteration path
                if (tau > 0.0) {
                    const double ep = eps * (1.0 + nb) * tau, ed = eps * (1.0 + nc) * tau;
                    if (ms[2] <= ep * ep && cs[4] <= ed * ed &&
                        fabs(cx - by) <= eps * (tau + fabs(cx) + fabs(by)))
                        st = 1;
                }
                if (!st && nb > 0.0 && by > 0.0 && cs[5] * (nb * nb) <= (eps * by) * (eps * by)) st = 2;
                if (!st && nc > 0.0 && cx < 0.0 && ms[3] * (nc * nc) <= (eps * cx) * (eps * cx)) st = 3;
                l_ms2 = ms[2]; l_cs4 = cs[4]; l_tau = tau; l_have = true;
                by_last = by;
                cx_last = cx;
                if (exit_pend && phase == 1) {     // the FP32 phase's last iterate, FP64 data
                    kfx = kkt_rel(ms[2], cs[4], cx, by, tau, nb, nc);
                    exit_pend = false;
                }
                if (st) {
                    if (phase == 0) {          // FP32 verdict: confirm with FP64 data
                        phase = 1;
                        exit_pend = true;
                        pass_kind = OP_REFRESH;
                        continue;
                    }
                    status = st;
                    break;
                }
            }
            if (phase == 0 && iters >= prm.fp32_max_iters) {
                phase = 1;
                exit_pend = true;
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
                stall_reset(stall);
                bb_pend = BB;
                pass_kind = OP_RESTART;
                continue;
            }
            if (phase == 0 && was_update && stall_sample(stall, inner, mu)) {
                phase = 1;                     // FP32 precision floor reached
                exit_pend = true;
                pass_kind = OP_REFRESH;
                continue;
            }
            // (an outer iteration that starts with a beta choice takes its probes first)
            if (iters >= prm.max_iters && !(BB && bb_pend)) { status = 4; break; }
        }
        if (BB && fixed_iters == 0 && (bb_pend || bb_pass)) {
            // ---- adaptive beta (Section 4.3), out of line: rare passes
            const int prev = bb_stage;
            if (!bb_pass) bb_pend = false;
            const BBStep r = bb_advance_wg(k, d, P, ctrl, sh, bb_stage, was_update, tau, kappa, theta, beta, prm,
                                           bb_est_run, bbe);
            tau = r.tau; kappa = r.kappa; theta = r.theta; beta = r.beta;
            bb_stage = r.stage; bb_est_run = r.est; bbe = r.bbe;
            if (r.restored) {
                pass_kind = OP_REFRESH;        // the passes' products of the initial point
                continue;
            }
            if (prev == 3 && iters >= prm.max_iters) { status = 4; break; }
        }
        // ---- the inner update: t = y - A f, a = G^{-1} t, border, scalars, y'
        cyc_chk += wall_clock64() - tc;
        for (int i = tid; i < ld; i += blockDim.x) sh.t[i] = (i < m) ? sh.y[i] - sh.Af[i] : 0.0;
        __syncthreads();
        const int64_t t1 = wall_clock64();
        if constexpr (TRSV) {
            if (phase == 0) {
                trsv_pass<float>(P.L32 + d.oG, P.Lt32 + d.oG, P.Li32 + d.oL, P.Lit32 + d.oL, m, ld, sh);
                ++gh32;
            } else {
                trsv_pass<double>(P.L64 + d.oG, P.Lt64 + d.oG, P.Li64 + d.oL, P.Lit64 + d.oL, m, ld, sh);
                ++gh64;
            }
        } else {
            if (phase == 0) { ginv_pass<NCH, (NCH == 1 ? 8 : NCH == 2 ? 4 : 2), float>(G32, m, ld, sh); ++gh32; }
            else { ginv_pass<NCH, (NCH == 1 ? 4 : 2), double>(G64, m, ld, sh); ++gh64; }
        }
        const int64_t t2 = wall_clock64();
        cyc_ginv += t2 - t1;
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
        cyc_upd += wall_clock64() - t2;
        pass_kind = OP_PROX;
    }

    cyc_all = wall_clock64() - t_start;
    if (l_have && l_tau > 0.0) {           // the relative residuals of the last test
        pobj = cx_last / l_tau;
        dobj = by_last / l_tau;
        pres = sqrt(l_ms2) / l_tau / (1.0 + nb);
        dres = sqrt(l_cs4) / l_tau / (1.0 + nc);
        gap = fabs(pobj - dobj) / (1.0 + fabs(pobj) + fabs(dobj));
    }
    for (int i = tid; i < m; i += blockDim.x) Yg[i] = sh.y[i];
    if (tid == 0) {
        LPCtrl& o = ctrl[k];
        o.clk[0] += cyc_col; o.clk[1] += cyc_ginv; o.clk[2] += cyc_all;
        o.clk[3] += cyc_chk; o.clk[4] += cyc_upd;
        o.tau = tau; o.kappa = kappa; o.theta = theta; o.mu = mu;
        o.pres = pres; o.dres = dres; o.gap = gap; o.pobj = pobj; o.dobj = dobj;
        o.by = by_last; o.cx = cx_last;
        o.iters = iters; o.iters64 = iters64; o.ipm = ipm;
        o.cp32 = cp32; o.cp64 = cp64;
        o.gh32 = gh32; o.gh64 = gh64; o.kfx = kfx;
        if (BB) { o.beta = beta; o.bbp = bbp; o.bbe = bbe; }
        o.status = status; o.phase = phase;
        o.mode = OP_REFRESH;
        o.flags = ((fixed_iters > 0) ? 1 : 0) | (cl.flags & 4) | (bb_pend ? 16 : 0);
    }
    __syncthreads();
}

template <int NCH, int MAXT, bool BB, bool TRSV>
__global__ __launch_bounds__(MAXT) void k_solve_wg(const LPDesc* __restrict__ desc, LPCtrl* __restrict__ ctrl,
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
    sh.scal = sh.red + 2 * W * max(ldmax, 32);
    sh.buf = sh.scal + 8 * W;
    while (true) {
        if (threadIdx.x == 0) s_lp = atomicAdd(queue, 1);
        __syncthreads();
        const int q = s_lp;
        __syncthreads();
        if (q >= B) break;
        const int k = order[q];
        const LPDesc d = desc[k];
        // an LP whose current phase fits in LDS runs LDS-resident; it comes
        // back here (state in ctrl[k] and the pools) only to hand over to FP64
        // data that does not fit
        if (!TRSV && MAXT == 256 && d.lds != 0) {
            if (solve_small_any<BB>(k, d, ctrl, P, prm, fixed_iters)) continue;
        }
        // each LP runs the variant for its own row count (the launch's NCH is
        // the batch maximum): a small LP in a mixed batch holds no idle rows
        const int nch = (d.ld + 255) >> 8;
        if (NCH == 1 || nch <= 1) solve_one<1, MAXT, BB, TRSV>(k, d, ctrl, P, prm, fixed_iters, sh);
        else if (NCH == 2 || nch == 2)
            solve_one<(NCH >= 2 ? 2 : 1), MAXT, BB, TRSV>(k, d, ctrl, P, prm, fixed_iters, sh);
        else if (NCH == 3 || nch == 3)
            solve_one<(NCH >= 3 ? 3 : 1), MAXT, BB, TRSV>(k, d, ctrl, P, prm, fixed_iters, sh);
        else solve_one<NCH, MAXT, BB, TRSV>(k, d, ctrl, P, prm, fixed_iters, sh);
    }
}

// LDS bytes for a launch
size_t wg_smem_bytes(int ldmax, int W) {
    return sizeof(double) * ((size_t)5 * ldmax + (size_t)2 * W * (ldmax > 32 ? ldmax : 32) + 16 * (size_t)W);
}

// smem: at least wg_smem_bytes(ldmax, threads / 64), and the LDS-resident
// footprint of every LP whose descriptor asks for it
hipError_t launch_solve_wg(int nch, int grid, int threads, hipStream_t st, const LPDesc* desc, LPCtrl* ctrl,
                           const PoolPtrs& P, const SolveParams& prm, const int32_t* order, int32_t B,
                           int32_t* queue, int64_t fixed_iters, int32_t ldmax, size_t smem) {
    if (threads > 256 && nch != 1) return hipErrorInvalidValue;      // only NCH = 1 has a 512-thread build
    // the adaptive beta (Section 4.3) has kernels of its own: the plain ones
    // carry none of its code
    const int key = nch * 1000 + threads;
#define ABIP_LAUNCH_WG(N, T, BBV, TRV) \
    hipLaunchKernelGGL((k_solve_wg<N, T, BBV, TRV>), dim3(grid), dim3(threads), smem, st, desc, ctrl, P, prm, order, \
                       B, queue, fixed_iters, ldmax)
    if (prm.bb) {
        switch (key) {
        case 1512: ABIP_LAUNCH_WG(1, 512, true, false); break;
        case 1256: ABIP_LAUNCH_WG(1, 256, true, false); break;
        case 2256: ABIP_LAUNCH_WG(2, 256, true, false); break;
        case 3256: ABIP_LAUNCH_WG(3, 256, true, false); break;
        case 4256: ABIP_LAUNCH_WG(4, 256, true, false); break;
        default: return hipErrorInvalidValue;
        }
    } else if (prm.trsv) {
        switch (key) {
        case 1512: ABIP_LAUNCH_WG(1, 512, false, true); break;
        case 1256: ABIP_LAUNCH_WG(1, 256, false, true); break;
        case 2256: ABIP_LAUNCH_WG(2, 256, false, true); break;
        case 3256: ABIP_LAUNCH_WG(3, 256, false, true); break;
        case 4256: ABIP_LAUNCH_WG(4, 256, false, true); break;
        default: return hipErrorInvalidValue;
        }
    } else {
        switch (key) {
        case 1512: ABIP_LAUNCH_WG(1, 512, false, false); break;
        case 1256: ABIP_LAUNCH_WG(1, 256, false, false); break;
        case 2256: ABIP_LAUNCH_WG(2, 256, false, false); break;
        case 3256: ABIP_LAUNCH_WG(3, 256, false, false); break;
        case 4256: ABIP_LAUNCH_WG(4, 256, false, false); break;
        default: return hipErrorInvalidValue;
        }
    }
#undef ABIP_LAUNCH_WG
    return hipGetLastError();
}

hipError_t set_solve_wg_smem_limit(size_t bytes) {
    const void* fns[] = {
        (const void*)k_solve_wg<1, 512, false, false>, (const void*)k_solve_wg<1, 256, false, false>,
        (const void*)k_solve_wg<2, 256, false, false>, (const void*)k_solve_wg<3, 256, false, false>,
        (const void*)k_solve_wg<4, 256, false, false>, (const void*)k_solve_wg<1, 512, true, false>,
        (const void*)k_solve_wg<1, 256, true, false>, (const void*)k_solve_wg<2, 256, true, false>,
        (const void*)k_solve_wg<3, 256, true, false>, (const void*)k_solve_wg<4, 256, true, false>,
        (const void*)k_solve_wg<1, 512, false, true>, (const void*)k_solve_wg<1, 256, false, true>,
        (const void*)k_solve_wg<2, 256, false, true>, (const void*)k_solve_wg<3, 256, false, true>,
        (const void*)k_solve_wg<4, 256, false, true>};
    for (const void* f : fns) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ===========================================================================
// Adjoint of the converged HSD fixed point (project extension).
//
// One inner iteration is a map T on z = (y, x, tau, theta, s, kappa).  At the
// final iterate L(z) = w^T x / tau, and dL/dp = lam^T dT/dp where lam solves
// lam = J_T^T lam + dL/dz (J_T = dT/dz).  One application of J_T^T, from the
// adjoint (ybar', xbar', taubar', thetabar', sbar', kappabar') of T's output:
//   rho_x = x/(x+s), rho_t = tau/(tau+kappa) (derivative of the prox root,
//   using x o s = t e and tau kappa = t, Theorem 3.1)
//   wx = rho_x xbar' + (rho_x - 1) sbar',  wt = rho_t taubar' + (rho_t - 1) kappabar'
//   wb = (I - Q)^{-1} alpha (ybar', wx, wt, thetabar')     ((I+Q)^T = I - Q)
//   J_T^T(.) = ((1-a) ybar' + wb_y, (1-a) wx + wb_x, (1-a) wt + wb_tau,
//               (1-a) thetabar' + wb_theta, -wx + wb_x, -wt + wb_tau)
// (I - Q)^{-1} reuses G^{-1} (I - Q has the same G = I + A A^T) and the border
// Z', K' of I - Q cached at setup.  The linear system (I - J_T^T) lam = dL/dz is
// solved by BiCGSTAB; then dL/dp = -zeta^T d(Q u)/dp with zeta = wb(lam).
// ===========================================================================

struct AdjArgs {
    double* ws;                       // per-LP workspace pool
    const int64_t* ows;               // offsets into ws
    const double* const* gin;         // dL/dx* per LP
    double* const* dc;                // outputs per LP (device)
    double* const* db;
    double* const* dA;                // may hold nulls
    int64_t max_iters;
    double tol;
    int64_t* iters_out;               // per LP: BiCGSTAB iterations
    double* resid_out;                // per LP: final relative residual
};

// out = in - J_T^T(in); also leaves wb = (I-Q)^{-1}(...) in WB.
__device__ void adj_op(const LPDesc& d, const LPCtrl& cl, const PoolPtrs& P, const WGShared& sh,
                       const double* __restrict__ in, double* __restrict__ out, double* __restrict__ WX,
                       double* __restrict__ Dv, double* __restrict__ WB, double alpha) {
    const int m = d.m, n = d.n, ld = d.ld, tid = threadIdx.x, lane = threadIdx.x & 63;
    const int wave = wave_id(), W = num_waves();
    const int OX = m, OT = m + n, OH = m + n + 1, OS = m + n + 2, OK = m + 2 * n + 2;
    const double* A = P.A64 + d.oA;
    const double* X = P.Nv + NF_X * P.Ntot + d.on;
    const double* S = P.Nv + NF_S * P.Ntot + d.on;
    const double* b = P.Mv + MF_B * P.Mtot + d.om;
    const double* bbar = P.Mv + MF_BBAR * P.Mtot + d.om;
    const double* C = P.Nv + NF_C * P.Ntot + d.on;
    const double* CBv = P.Nv + NF_CBAR * P.Ntot + d.on;
    const double* zy0 = P.Mv + MF_ZY0A * P.Mtot + d.om;
    const double* zy1 = P.Mv + MF_ZY1A * P.Mtot + d.om;
    const double* zx0 = P.Nv + NF_ZX0A * P.Ntot + d.on;
    const double* zx1 = P.Nv + NF_ZX1A * P.Ntot + d.on;
    const double rt = cl.tau / (cl.tau + cl.kappa);
    const double wt = rt * in[OT] + (rt - 1.0) * in[OK];
    for (int j = tid; j < n; j += blockDim.x) {
        const double rx = X[j] / (X[j] + S[j]);
        WX[j] = rx * in[OX + j] + (rx - 1.0) * in[OS + j];
    }
    __threadfence_block();
    __syncthreads();
    // t = alpha (in_y + A wx): one thread per row, columns split over P groups
    {
        int Pg = blockDim.x / ld;
        if (Pg < 1) Pg = 1;
        if (Pg > 2 * W) Pg = 2 * W;
        for (int e = tid; e < ld * Pg; e += blockDim.x) {
            const int r = e % ld, g = e / ld;
            double s0 = 0.0, s1 = 0.0;
            int j = g;
            for (; j + Pg < n; j += 2 * Pg) {
                s0 = fma(A[(int64_t)j * ld + r], WX[j], s0);
                s1 = fma(A[(int64_t)(j + Pg) * ld + r], WX[j + Pg], s1);
            }
            for (; j < n; j += Pg) s0 = fma(A[(int64_t)j * ld + r], WX[j], s0);
            sh.red[g * ld + r] = s0 + s1;
        }
        __syncthreads();
        for (int r = tid; r < ld; r += blockDim.x) {
            double s = 0.0;
            for (int g = 0; g < Pg; ++g) s += sh.red[g * ld + r];
            sh.t[r] = (r < m) ? alpha * (in[r] + s) : 0.0;
        }
        __syncthreads();
    }
    ginv_rows<double>(P.G64 + d.oG, m, ld, sh);          // sh.a = G^{-1} t
    // d_j = alpha wx_j - (A^T a)_j, four columns per wave step
    double cd = 0.0, cbd = 0.0;
    for (int j0 = wave * 4; j0 < n; j0 += 4 * W) {
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            double s = 0.0;
            if (j0 + u < n)
                for (int i = lane; i < m; i += 64) s = fma(A[(int64_t)(j0 + u) * ld + i], sh.a[i], s);
            v[u] = s;
        }
        wave_sum_n<4>(v);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double tot = v[u];
            if (lane == u && j0 + u < n) {
                const double dj = alpha * WX[j0 + u] - tot;
                Dv[j0 + u] = dj;
                cd = fma(C[j0 + u], dj, cd);
                cbd = fma(CBv[j0 + u], dj, cbd);
            }
        }
    }
    double dots[4] = {0.0, 0.0, cd, cbd};
    for (int i = tid; i < m; i += blockDim.x) {
        dots[0] = fma(b[i], sh.a[i], dots[0]);
        dots[1] = fma(bbar[i], sh.a[i], dots[1]);
    }
    block_sum_n<4>(dots, sh.buf);      // also orders the Dv writes before their reads
    // H'^T z with H' = -H:  (b^T a - c^T d, -bbar^T a + cbar^T d)
    const double q0 = alpha * wt + (dots[0] - dots[2]);
    const double q1 = alpha * in[OH] + (-dots[1] + dots[3]);
    const double p0 = cl.KA00 * q0 + cl.KA01 * q1;
    const double p1 = cl.KA10 * q0 + cl.KA11 * q1;
    for (int i = tid; i < m; i += blockDim.x) {
        const double wby = sh.a[i] - zy0[i] * p0 - zy1[i] * p1;
        WB[i] = wby;
        out[i] = in[i] - ((1.0 - alpha) * in[i] + wby);
    }
    for (int j = tid; j < n; j += blockDim.x) {
        const double wbx = Dv[j] - zx0[j] * p0 - zx1[j] * p1;
        const double wx = WX[j];
        WB[m + j] = wbx;
        out[OX + j] = in[OX + j] - ((1.0 - alpha) * wx + wbx);
        out[OS + j] = in[OS + j] - (-wx + wbx);
    }
    if (tid == 0) {
        WB[m + n] = p0;
        WB[m + n + 1] = p1;
        out[OT] = in[OT] - ((1.0 - alpha) * wt + p0);
        out[OH] = in[OH] - ((1.0 - alpha) * in[OH] + p1);
        out[OK] = in[OK] - (-wt + p0);
    }
    __threadfence_block();
    __syncthreads();
}

__device__ double adj_dot(const double* a, const double* b, int N, const WGShared& sh) {
    double v[1] = {0.0};
    for (int i = threadIdx.x; i < N; i += blockDim.x) v[0] = fma(a[i], b[i], v[0]);
    block_sum_n<1>(v, sh.buf);
    return v[0];
}

__device__ void adjoint_one(int k, const LPDesc& d, const LPCtrl* __restrict__ ctrl, const PoolPtrs& P,
                            const SolveParams& prm, const AdjArgs& aa, const WGShared& sh) {
    const int m = d.m, n = d.n, tid = threadIdx.x;
    const int Nz = m + 2 * n + 3;
    const LPCtrl cl = ctrl[k];
    double* base = aa.ws + aa.ows[k];
    double* LAM = base;
    double* Rv = LAM + Nz;
    double* R0 = Rv + Nz;
    double* Pv = R0 + Nz;
    double* V = Pv + Nz;
    double* Sv = V + Nz;
    double* Tv = Sv + Nz;
    double* WX = Tv + Nz;
    double* Dv = WX + n;
    double* WB = Dv + n;
    const double* X = P.Nv + NF_X * P.Ntot + d.on;
    const double* Y = P.Mv + MF_Y * P.Mtot + d.om;
    const double* win = aa.gin[k];
    const double alpha = prm.alpha;
    const double tau = cl.tau, theta = cl.theta;
    if ((cl.status != 1 && !(cl.flags & 4)) || !(tau > 0.0)) {   // nothing to differentiate
        double* dc = aa.dc[k];
        double* db = aa.db[k];
        double* dA = aa.dA[k];
        for (int j = tid; j < n; j += blockDim.x) dc[j] = NAN;
        for (int i = tid; i < m; i += blockDim.x) db[i] = NAN;
        if (dA)
            for (int64_t e = tid; e < (int64_t)m * n; e += blockDim.x) dA[e] = NAN;
        if (tid == 0) { aa.iters_out[k] = 0; aa.resid_out[k] = NAN; }
        __syncthreads();
        return;
    }
    // g = dL/dz = (0, w/tau, -w^T x/tau^2, 0, 0, 0)
    double wx1[1] = {0.0};
    for (int j = tid; j < n; j += blockDim.x) wx1[0] = fma(win[j], X[j], wx1[0]);
    block_sum_n<1>(wx1, sh.buf);
    for (int i = tid; i < Nz; i += blockDim.x) {
        double g = 0.0;
        if (i >= m && i < m + n) g = win[i - m] / tau;
        else if (i == m + n) g = -wx1[0] / (tau * tau);
        LAM[i] = (aa.max_iters == 0) ? g : 0.0;   // 0 iterations: contract one step of dL/dz
        Rv[i] = g; R0[i] = g; Pv[i] = 0.0; V[i] = 0.0;
    }
    __threadfence_block();
    __syncthreads();
    const double gnorm = sqrt(adj_dot(Rv, Rv, Nz, sh));
    double rho = 1.0, al = 1.0, om = 1.0, rel = 1.0;
    double rr = gnorm * gnorm;                  // ||r||^2
    int64_t it = 0;
    bool restart = false;
    if (gnorm > 0.0) {
        for (it = 1; it <= aa.max_iters; ++it) {
            double rho1 = adj_dot(R0, Rv, Nz, sh);
            // breakdown of the two-sided recurrence (r0^ orthogonal to r, or a zero /
            // non-finite step): restart with the current residual as the shadow
            if (restart || !(fabs(rho1) > 0.0) || !isfinite(rho1)) {
                restart = false;
                for (int i = tid; i < Nz; i += blockDim.x) { R0[i] = Rv[i]; Pv[i] = 0.0; V[i] = 0.0; }
                __threadfence_block();
                __syncthreads();
                rho1 = rr;
                rho = 1.0; al = 1.0; om = 1.0;
            }
            const double beta = (rho1 / rho) * (al / om);
            for (int i = tid; i < Nz; i += blockDim.x) Pv[i] = Rv[i] + beta * (Pv[i] - om * V[i]);
            __threadfence_block();
            __syncthreads();
            adj_op(d, cl, P, sh, Pv, V, WX, Dv, WB, alpha);
            const double rv = adj_dot(R0, V, Nz, sh);
            if (!(fabs(rv) > 0.0) || !isfinite(rv)) { restart = true; continue; }
            al = rho1 / rv;
            if (!isfinite(al)) { restart = true; continue; }
            for (int i = tid; i < Nz; i += blockDim.x) Sv[i] = Rv[i] - al * V[i];
            __threadfence_block();
            __syncthreads();
            const double sn = sqrt(adj_dot(Sv, Sv, Nz, sh));
            if (sn <= aa.tol * gnorm) {
                for (int i = tid; i < Nz; i += blockDim.x) LAM[i] += al * Pv[i];
                rel = sn / gnorm;
                break;
            }
            adj_op(d, cl, P, sh, Sv, Tv, WX, Dv, WB, alpha);
            const double tt = adj_dot(Tv, Tv, Nz, sh);
            const double ts = adj_dot(Tv, Sv, Nz, sh);
            om = (tt > 0.0 && isfinite(ts / tt)) ? ts / tt : 0.0;     // 0: half step, then restart
            for (int i = tid; i < Nz; i += blockDim.x) {
                LAM[i] += al * Pv[i] + om * Sv[i];
                Rv[i] = Sv[i] - om * Tv[i];
            }
            __threadfence_block();
            __syncthreads();
            rr = adj_dot(Rv, Rv, Nz, sh);
            rel = sqrt(rr) / gnorm;
            if (rel <= aa.tol) break;
            rho = rho1;
            if (om == 0.0) restart = true;         // stagnation
        }
    }
    __threadfence_block();
    __syncthreads();
    // zeta = wb(lam): one more application (its "out" is discarded into Tv)
    adj_op(d, cl, P, sh, LAM, Tv, WX, Dv, WB, alpha);
    const double zt = WB[m + n], zh = WB[m + n + 1];
    double* dc = aa.dc[k];
    double* db = aa.db[k];
    double* dA = aa.dA[k];
    for (int j = tid; j < n; j += blockDim.x) {
        const double xj = X[j];
        dc[j] = -(WB[m + j] * (tau - theta) + zt * (theta - xj) + zh * (xj - tau));
    }
    for (int i = tid; i < m; i += blockDim.x) {
        const double yi = Y[i];
        db[i] = -(WB[i] * (theta - tau) + zt * yi - zh * yi);
    }
    if (dA) {
        for (int64_t e = tid; e < (int64_t)m * n; e += blockDim.x) {
            const int i = (int)(e / n), j = (int)(e % n);
            const double yi = Y[i];
            dA[e] = -(WB[i] * (X[j] - theta) - WB[m + j] * yi + zh * yi);
        }
    }
    if (tid == 0) {
        aa.iters_out[k] = it;
        aa.resid_out[k] = rel;
    }
    __syncthreads();
}

__global__ __launch_bounds__(512) void k_adjoint(const LPDesc* __restrict__ desc, const LPCtrl* __restrict__ ctrl,
                                                 PoolPtrs P, SolveParams prm, AdjArgs aa, const int32_t* order,
                                                 int32_t B, int32_t* queue, int32_t ldmax) {
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
    sh.scal = sh.red + 2 * W * max(ldmax, 32);
    sh.buf = sh.scal + 8 * W;
    while (true) {
        if (threadIdx.x == 0) s_lp = atomicAdd(queue, 1);
        __syncthreads();
        const int q = s_lp;
        __syncthreads();
        if (q >= B) break;
        const int k = order[q];
        const LPDesc d = desc[k];
        adjoint_one(k, d, ctrl, P, prm, aa, sh);
    }
}

hipError_t launch_adjoint(int grid, int threads, hipStream_t st, const LPDesc* desc, const LPCtrl* ctrl,
                          const PoolPtrs& P, const SolveParams& prm, const AdjArgs& aa, const int32_t* order,
                          int32_t B, int32_t* queue, int32_t ldmax) {
    const size_t smem = wg_smem_bytes(ldmax, threads / 64);
    hipError_t e = hipFuncSetAttribute((const void*)k_adjoint, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_adjoint, dim3(grid), dim3(threads), smem, st, desc, ctrl, P, prm, aa, order, B, queue, ldmax);
    return hipGetLastError();
}
