// LDS-resident variant of the one-workgroup solve, for LPs whose A and G^{-1}
// fit in one workgroup's LDS in the precision of the current phase.  It runs
// the same iteration as the streamed variant (Algorithm 2 with the Section 4.2
// relaxation, the Section 4.1 tests on every update, the inner test
// ||Qu - v||^2 <= mu, the Section 5 restart, the FP32 -> FP64 handover) and
// takes the same decisions; what differs is where the data lives and how the
// products are organised:
//   * A and G^{-1} are copied into LDS once per precision phase, so an
//     iteration touches no global memory.  When A fits but A and G^{-1}
//     together do not, G^{-1} stays in the pool and the G^{-1} t sweep reads
//     its columns from global memory (L2 / MALL); the rest is unchanged.
//   * wave w owns a block of ceil(n/4) columns and a block of ceil(m/4) rows.
//     A column's owner lane keeps x_j, s_j, c_j, cbar_j, the border entries
//     and (A^T y)_j in registers: (A^T a)_j is one LDS dot product (split over
//     a lane pair when n <= 128) and the prox root and dual update need no
//     lane exchange.  A row's owner lane keeps y_i and the m-vectors of the
//     border.
//   * A f and A x: each wave sweeps its own columns with lanes over all rows
//     and leaves a partial vector; G^{-1} t: each wave sweeps the columns of
//     G^{-1} that match its own rows.  A wave only reads the f and t values
//     its own lanes wrote, so neither sweep waits for the other waves; the row
//     owners add the four partial vectors in a fixed order (deterministic).
//   * (A^T y)_j of the relaxed y update y' = alpha (a - Zy p) + (1 - alpha) y
//     (Section 4.2 applied to the y block) is carried by
//         A^T y' = alpha (A^T a - p0 A^T Zy0 - p1 A^T Zy1) + (1 - alpha) A^T y,
//     so an update needs one dot product per column instead of two.  It is
//     recomputed exactly by every refresh and restart pass, and old rounding
//     errors are multiplied by |1 - alpha| < 1 at every step, so they stay
//     bounded.
// Three workgroup barriers per update: after the A f sweep, in the check's
// sums (which also publishes the G^{-1} t partials, computed before the tests
// are taken) and in the border sums (which publishes a).
#pragma once
#include <hip/hip_runtime.h>
#include "abip_internal.h"

// four waves (256-thread launches)
#define SMALL_W 4

// For a phase that runs LDS-resident: G^{-1} is read from the pool (only A
// fits in LDS), and A is held as doubles (always in the FP64 phase; in the FP32
// phase when the FP64 layout of the same kind fits: the same values, no
// conversion per use).
__device__ __forceinline__ bool small_gs(int lds, int phase) {
    return phase == 0 ? (lds & DESC_LDS32) == 0 : (lds & DESC_LDS64) == 0;
}
__device__ __forceinline__ bool small_wide(int lds, int phase) {
    if (phase != 0) return true;
    return small_gs(lds, 0) ? (lds & DESC_LDSA64) != 0 : (lds & DESC_LDS64) != 0;
}

struct SmallCol {
    double x, s, c, cb, z0, z1;     // iterate, c, cbar, border columns of x
    double aty, atz0, atz1;         // (A^T y)_j, (A^T Zy0)_j, (A^T Zy1)_j
};

// dot of one LDS column with an LDS vector (rows past m are zero in both)
__device__ __forceinline__ double small_dot(const float* __restrict__ col, const double* __restrict__ v, int m4) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll 2
    for (int i = 0; i < m4; i += 4) {
        const float4 a = *reinterpret_cast<const float4*>(col + i);
        const double2 v0 = *reinterpret_cast<const double2*>(v + i);
        const double2 v1 = *reinterpret_cast<const double2*>(v + i + 2);
        s0 = fma((double)a.x, v0.x, s0);
        s1 = fma((double)a.y, v0.y, s1);
        s2 = fma((double)a.z, v1.x, s2);
        s3 = fma((double)a.w, v1.y, s3);
    }
    return (s0 + s1) + (s2 + s3);
}
__device__ __forceinline__ double small_dot(const double* __restrict__ col, const double* __restrict__ v, int m4) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll 2
    for (int i = 0; i < m4; i += 4) {
        const double2 a0 = *reinterpret_cast<const double2*>(col + i);
        const double2 a1 = *reinterpret_cast<const double2*>(col + i + 2);
        const double2 v0 = *reinterpret_cast<const double2*>(v + i);
        const double2 v1 = *reinterpret_cast<const double2*>(v + i + 2);
        s0 = fma(a0.x, v0.x, s0);
        s1 = fma(a0.y, v0.y, s1);
        s2 = fma(a1.x, v1.x, s2);
        s3 = fma(a1.y, v1.y, s3);
    }
    return (s0 + s1) + (s2 + s3);
}

// Wave-uniform copy of an integer (keeps sizes and loop bounds in scalar
// registers inside this out-of-line function).
__device__ __forceinline__ int small_uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Column ownership: wave w owns columns w*cb .. w*cb + cb - 1 (cb = ceil(n/4));
// lane l owns column w*cb + l + 64 q (q < CPT), or, with PAIR (cb <= 32),
// lanes 2l and 2l+1 share column w*cb + l: each takes every other group of
// four rows and the halves are added across the lane pair (both lanes then
// hold bitwise the same dot product).  Returns -1 for a lane with no column.
template <int CPT, bool PAIR>
__device__ __forceinline__ int small_col(int q, int cb, int n) {
    const int lane = threadIdx.x & 63;
    const int lo = PAIR ? (lane >> 1) : lane + 64 * q;
    const int j = wave_id() * cb + lo;
    return (lo < cb && j < n) ? j : -1;
}
template <typename T>
__device__ __forceinline__ double small_dot_half(const T* __restrict__ col, const double* __restrict__ v, int m4,
                                                 int h) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll 2
    for (int i = 4 * h; i < m4; i += 8) {
        double a[4];
        load4(col + i, a);
        const double2 v0 = *reinterpret_cast<const double2*>(v + i);
        const double2 v1 = *reinterpret_cast<const double2*>(v + i + 2);
        s0 = fma(a[0], v0.x, s0);
        s1 = fma(a[1], v0.y, s1);
        s2 = fma(a[2], v1.x, s2);
        s3 = fma(a[3], v1.y, s3);
    }
    return (s0 + s1) + (s2 + s3);
}

// Copy this phase's A and (unless gs) G^{-1} from the pools into LDS (zero
// rows m..lda-1).  FP32 data may be held as doubles (the same values, no
// conversion per use).
template <typename Td, typename Ts>
__device__ __forceinline__ void small_fill(Td* __restrict__ As, int lda, Td* __restrict__ Gs, int ldg,
                                           const Ts* __restrict__ Ag, const Ts* __restrict__ Gg, int m, int n,
                                           int ld, bool gs) {
    const int NT = blockDim.x;
    for (int e = threadIdx.x; e < lda * n; e += NT) {
        const int j = e / lda, i = e - j * lda;
        As[e] = (i < m) ? (Td)Ag[(int64_t)j * ld + i] : Td(0);
    }
    for (int e = threadIdx.x; e < (gs ? 0 : ldg * m); e += NT) {
        const int j = e / ldg, i = e - j * ldg;
        Gs[e] = (i < m) ? (Td)Gg[(int64_t)j * ld + i] : Td(0);
    }
}

// Block sum of K values (K = 4, 8, 12 or 16) over the four waves; every
// thread gets the totals, added in a fixed order.  A reduce-scatter leaves lane
// group g (16 lanes) of each wave with values K/4*g .. K/4*g + K/4 - 1; red
// holds them as [value][wave], read back with 16-byte loads.  One barrier.
// The two sums of an update use disjoint parts of red (the check's sums at 0,
// the border's at 12 * 4), so neither overwrites what a slower wave may still
// be reading.
template <int K>
__device__ __forceinline__ void small_bsum(double (&v)[K], double* __restrict__ red) {
    static_assert(K % 4 == 0 && K <= 16, "small_bsum: K = 4, 8, 12 or 16");
    constexpr int V = K / 4;
    const int lane = threadIdx.x & 63, wave = wave_id();
    wave_rs<K, V>(v);
    if ((lane & 15) == 0) {
        const int g = lane >> 4;
#pragma unroll
        for (int q = 0; q < V; ++q) red[(V * g + q) * SMALL_W + wave] = v[q];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double2 r0 = *reinterpret_cast<const double2*>(red + k * SMALL_W);
        const double2 r1 = *reinterpret_cast<const double2*>(red + k * SMALL_W + 2);
        v[k] = (r0.x + r0.y) + (r1.x + r1.y);
    }
}

// Column pass: op OP_PROX (av = a: the update of x_j, s_j), OP_REFRESH or
// OP_RESTART (av = y: exact A^T y; the restart rescales x_j, s_j).  Writes
// (x'+s', x') to fx and adds the column-side sums of the check to acc:
//   c^T x, cbar^T x, c^T s, cbar^T s, ||A^T y + s - c tau||^2, ||A^T y + s||^2,
//   ||-A^T y + c tau - cbar theta - s||^2.
template <typename T, int CPT, bool PAIR>
__device__ __forceinline__ void small_colpass(const T* __restrict__ As, int lda, int m4, int n, int cb,
                                              const double* __restrict__ av, SmallCol (&col)[CPT],
                                              double2* __restrict__ fx, int op, double p0, double p1, double tmu,
                                              double alpha, double gamma, int rule, double tau, double theta,
                                              double (&acc)[7]) {
    const double sg = sqrt(gamma);
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        const int j = small_col<CPT, PAIR>(q, cb, n);
        if (j >= 0) {
            SmallCol& C = col[q];
            double dv;
            if constexpr (PAIR) {
                const double hv = small_dot_half(As + (int64_t)j * lda, av, m4, (int)(threadIdx.x & 1));
                dv = hv + dpp_partner<0xB1>(hv);                      // lane pair 2j, 2j+1
            } else {
                dv = small_dot(As + (int64_t)j * lda, av, m4);
            }
            double x1 = C.x, s1 = C.s, aty;
            if (op == OP_PROX) {
                const double dj = (C.x + C.s) + dv;                    // M^{-1} block, x part
                const double ut = dj - C.z0 * p0 - C.z1 * p1;         // u~_x
                const double uh = alpha * ut + (1.0 - alpha) * C.x;   // relaxation
                x1 = prox_root(uh - C.s, tmu);                        // barrier prox
                s1 = C.s - uh + x1;                                   // dual update
                aty = alpha * (dv - p0 * C.atz0 - p1 * C.atz1) + (1.0 - alpha) * C.aty;
            } else {
                aty = dv;
                if (op == OP_RESTART) {
                    if (rule == 0) {
                        if (C.x >= C.s) s1 = gamma * C.s;
                        else x1 = gamma * C.x;
                    } else {
                        x1 = sg * C.x;
                        s1 = sg * C.s;
                    }
                }
            }
            C.x = x1; C.s = s1; C.aty = aty;
            const bool lead = !PAIR || (threadIdx.x & 1) == 0;        // one contribution per column
            const double mk = lead ? 1.0 : 0.0;
            const double r1 = (aty + s1 - C.c * tau) * mk;
            const double r2 = (aty + s1) * mk;
            const double r3 = (-aty + C.c * tau - C.cb * theta - s1) * mk;
            const double cm = C.c * mk, cbm = C.cb * mk;
            acc[0] = fma(cm, x1, acc[0]);
            acc[1] = fma(cbm, x1, acc[1]);
            acc[2] = fma(cm, s1, acc[2]);
            acc[3] = fma(cbm, s1, acc[3]);
            acc[4] = fma(r1, r1, acc[4]);
            acc[5] = fma(r2, r2, acc[5]);
            acc[6] = fma(r3, r3, acc[6]);
            if (lead) fx[j] = make_double2(x1 + s1, x1);
        }
    }
}

// Partial A f and A x over this wave's own column block (columns whose f the
// wave's lanes wrote, so no barrier precedes the sweep), lanes over all rows
// (RPL rows per lane, m <= 64 RPL): pf[(2w) m4 + i], pf[(2w+1) m4 + i].
// Steps of eight columns issue every LDS read before the arithmetic; the
// addresses advance by lda per column; two accumulator chains per output.
template <typename T, int RPL>
__device__ __forceinline__ void small_rowpass(const T* __restrict__ As, int lda, int m, int n, int m4, int cb,
                                              const double2* __restrict__ fx, double* __restrict__ pf) {
    constexpr int U = 8;
    const int lane = threadIdx.x & 63, wave = wave_id();
    const int j0 = small_uni(min(n, wave * cb)), j1 = small_uni(min(n, (wave + 1) * cb));
    double af0[RPL], ax0[RPL], af1[RPL], ax1[RPL];
    const T* cp = As + j0 * lda;
    int row[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        af0[r] = 0.0; ax0[r] = 0.0; af1[r] = 0.0; ax1[r] = 0.0;
        row[r] = min(lane + 64 * r, m - 1);
    }
    int j = j0;
    for (; j + U <= j1; j += U) {
        double2 f[U];
        double a[U][RPL];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            f[u] = fx[j + u];
#pragma unroll
            for (int r = 0; r < RPL; ++r) a[u][r] = (double)cp[u * lda + row[r]];
        }
#pragma unroll
        for (int u = 0; u < U; u += 2) {
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                af0[r] = fma(a[u][r], f[u].x, af0[r]);
                ax0[r] = fma(a[u][r], f[u].y, ax0[r]);
                af1[r] = fma(a[u + 1][r], f[u + 1].x, af1[r]);
                ax1[r] = fma(a[u + 1][r], f[u + 1].y, ax1[r]);
            }
        }
        cp += U * lda;
    }
    for (; j < j1; ++j) {
        const double2 f = fx[j];
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const double a = (double)cp[row[r]];
            af0[r] = fma(a, f.x, af0[r]);
            ax0[r] = fma(a, f.y, ax0[r]);
        }
        cp += lda;
    }
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int i = lane + 64 * r;
        if (i < m) {
            pf[(2 * wave) * m4 + i] = af0[r] + af1[r];
            pf[(2 * wave + 1) * m4 + i] = ax0[r] + ax1[r];
        }
    }
}

// Partial G^{-1} t over the columns of the symmetric G^{-1} that match this
// wave's own row block (t values the wave's lanes wrote), lanes over all rows
// as in the row pass: pg[w m4 + i].
template <typename T, int RPL>
__device__ __forceinline__ void small_gpass(const T* __restrict__ Gs, int ldg, int m, int m4, int rb,
                                            const double* __restrict__ tv, double* __restrict__ pg) {
    constexpr int U = 8;
    const int lane = threadIdx.x & 63, wave = wave_id();
    const int k0 = small_uni(min(m, wave * rb)), k1 = small_uni(min(m, (wave + 1) * rb));
    double ag0[RPL], ag1[RPL];
    const T* cp = Gs + k0 * ldg;
    int row[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        ag0[r] = 0.0; ag1[r] = 0.0;
        row[r] = min(lane + 64 * r, m - 1);
    }
    int k = k0;
    for (; k + U <= k1; k += U) {
        double t[U];
        double g[U][RPL];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            t[u] = tv[k + u];
#pragma unroll
            for (int r = 0; r < RPL; ++r) g[u][r] = (double)cp[u * ldg + row[r]];
        }
#pragma unroll
        for (int u = 0; u < U; u += 2) {
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                ag0[r] = fma(g[u][r], t[u], ag0[r]);
                ag1[r] = fma(g[u + 1][r], t[u + 1], ag1[r]);
            }
        }
        cp += U * ldg;
    }
    for (; k < k1; ++k) {
        const double t = tv[k];
#pragma unroll
        for (int r = 0; r < RPL; ++r) ag0[r] = fma((double)cp[row[r]], t, ag0[r]);
        cp += ldg;
    }
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int i = lane + 64 * r;
        if (i < m) pg[wave * m4 + i] = ag0[r] + ag1[r];
    }
}

// Copy this phase's A and G^{-1} into LDS (layout L is set for the phase)
// and form (A^T Zy0)_j, (A^T Zy1)_j for the owned columns.  Starts and ends
// with a barrier.
template <int CPT, bool PAIR>
__device__ __forceinline__ void small_load_phase(int phase, const LPDesc& d, int cb, const PoolPtrs& P,
                                                 const double* __restrict__ Zy0, const double* __restrict__ Zy1,
                                                 unsigned char* __restrict__ smem, SmallLayout& L,
                                                 SmallCol (&col)[CPT]) {
    const int m = d.m, n = d.n, tid = threadIdx.x;
    // LDS entries are doubles in the FP64 phase, and in the FP32 phase too when
    // the FP64 layout fits (FP32-rounded values held exactly as doubles)
    const bool wide = small_wide(d.lds, phase), gs = small_gs(d.lds, phase);
    L = small_layout(m, n, wide ? 8 : 4, SMALL_W, gs);
    double* av = reinterpret_cast<double*>(smem + L.oav);
    double* tv = reinterpret_cast<double*>(smem + L.otv);
    __syncthreads();                       // earlier readers of the LDS are done
    if (!wide)
        small_fill<float, float>(reinterpret_cast<float*>(smem + L.oA), L.lda, reinterpret_cast<float*>(smem + L.oG),
                                 L.ldg, P.A32 + d.oA, P.G32 + d.oG, m, n, d.ld, gs);
    else if (phase == 0)
        small_fill<double, float>(reinterpret_cast<double*>(smem + L.oA), L.lda,
                                  reinterpret_cast<double*>(smem + L.oG), L.ldg, P.A32 + d.oA, P.G32 + d.oG, m, n,
                                  d.ld, gs);
    else
        small_fill<double, double>(reinterpret_cast<double*>(smem + L.oA), L.lda,
                                   reinterpret_cast<double*>(smem + L.oG), L.ldg, P.A64 + d.oA, P.G64 + d.oG, m, n,
                                   d.ld, gs);
    for (int i = tid; i < L.m4; i += blockDim.x) {
        av[i] = (i < m) ? Zy0[i] : 0.0;
        tv[i] = (i < m) ? Zy1[i] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        const int j = small_col<CPT, PAIR>(q, cb, n);
        if (j >= 0) {
            if (!wide) {
                const float* cp = reinterpret_cast<const float*>(smem + L.oA) + (int64_t)j * L.lda;
                col[q].atz0 = small_dot(cp, av, L.m4);
                col[q].atz1 = small_dot(cp, tv, L.m4);
            } else {
                const double* cp = reinterpret_cast<const double*>(smem + L.oA) + (int64_t)j * L.lda;
                col[q].atz0 = small_dot(cp, av, L.m4);
                col[q].atz1 = small_dot(cp, tv, L.m4);
            }
        }
    }
    __syncthreads();                       // av / tv are rewritten next
}

// ---- adaptive beta (Section 4.3), the LDS-resident variant's step ----------
// The same stages as the streamed variant's (0 -> 1 keep the initial point,
// 1 -> 2 keep the first probe's iterate, 2: estimate, choose, restore, 3 -> 0),
// with the iterate in the owners' registers: lane values in, lane values out
// (x0/s0: the lane's first column, x1/s1: its last; equal when CPT = 1).  The
// copies go to the pools (each read back by the lane that wrote it) and the
// scalars to ctrl[k].bbs; red: the LDS of the block sums (the caller's last
// readers of it are past a barrier).
struct SmallBB {
    double y, x0, s0, x1, s1, tau, kappa, theta, beta;
    int stage, est, bbe;
    bool restored;
};
template <int CPT, bool PAIR>
__device__ __noinline__ SmallBB bb_advance_small(int k, int m, int n, int64_t om, int64_t on, const PoolPtrs& P,
                                                 LPCtrl* __restrict__ ctrl, double* __restrict__ red, int stage,
                                                 bool was_update, int cb, int ri, bool rown, double y, double x0,
                                                 double s0, double x1, double s1, double tau, double kappa,
                                                 double theta, double beta, const SolveParams& prm, int est,
                                                 int bbe) {
    SmallBB r{y, x0, s0, x1, s1, tau, kappa, theta, beta, stage, est, bbe, false};
    const int tid = threadIdx.x;
    double* Y0 = P.Mv + MF_BBY0 * P.Mtot + om;
    double* Y1 = P.Mv + MF_BBY1 * P.Mtot + om;
    double* X0 = P.Nv + NF_BBX0 * P.Ntot + on;
    double* S0 = P.Nv + NF_BBS0 * P.Ntot + on;
    double* X1 = P.Nv + NF_BBX1 * P.Ntot + on;
    double* S1 = P.Nv + NF_BBS1 * P.Ntot + on;
    double* bbs = ctrl[k].bbs;             // every thread writes the same values
    const int ja = small_col<CPT, PAIR>(0, cb, n), jb = small_col<CPT, PAIR>(CPT - 1, cb, n);
    const bool lead = !PAIR || (tid & 1) == 0;
    if (stage == 0) {
        if (rown) Y0[ri] = y;
        if (ja >= 0) { X0[ja] = x0; S0[ja] = s0; }
        if (CPT > 1 && jb >= 0) { X0[jb] = x1; S0[jb] = s1; }
        bbs[0] = tau; bbs[1] = kappa; bbs[2] = theta;
        r.stage = 1;
    } else if (stage == 1 && was_update) {
        if (rown) Y1[ri] = y;
        if (ja >= 0) { X1[ja] = x0; S1[ja] = s0; }
        if (CPT > 1 && jb >= 0) { X1[jb] = x1; S1[jb] = s1; }
        bbs[3] = tau; bbs[4] = kappa; bbs[5] = theta;
        r.stage = 2;
    } else if (stage == 2) {
        double q[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        double qq[5] = {0, 0, 0, 0, 0};
        if (rown) bb_acc(y - Y1[ri], 0.0, 0.0, prm.alpha, qq);
        if (ja >= 0 && lead) bb_acc(x0 - X1[ja], s0 - S1[ja], S1[ja] - S0[ja], prm.alpha, qq);
        if (CPT > 1 && jb >= 0 && lead) bb_acc(x1 - X1[jb], s1 - S1[jb], S1[jb] - S0[jb], prm.alpha, qq);
#pragma unroll
        for (int e = 0; e < 5; ++e) q[e] = qq[e];
        __syncthreads();
        small_bsum<8>(q, red);
#pragma unroll
        for (int e = 0; e < 5; ++e) qq[e] = q[e];
        bb_acc(tau - bbs[3], kappa - bbs[4], bbs[4] - bbs[1], prm.alpha, qq);
        bb_acc(theta - bbs[5], 0.0, 0.0, prm.alpha, qq);
        r.bbe = bbe + 1;
        r.est = est + 1;
        const double hat = bb_hat(qq, beta, prm.eps_cor);
        const bool fin = bb_choose(r.beta, hat, prm.eps_pen, r.est, prm.bb_max_redo);
        if (rown) r.y = Y0[ri];
        if (ja >= 0) { r.x0 = X0[ja]; r.s0 = S0[ja]; }
        if (CPT > 1 && jb >= 0) { r.x1 = X0[jb]; r.s1 = S0[jb]; }
        r.tau = bbs[0]; r.kappa = bbs[1]; r.theta = bbs[2];
        r.stage = fin ? 3 : 1;
        r.restored = true;
    } else if (stage == 3) {
        r.stage = 0;
        r.est = 0;
    }
    return r;
}

// Solve one LP LDS-resident from the state in ctrl[k] and the pools.  Returns
// true when the LP is finished here; false when the current phase does not fit
// (on entry, or at the handover to FP64 data): then ctrl[k] and the pools hold
// the state, with a tested FP64 refresh as the next pass, for the streamed
// variant.  Requires four waves, m <= 64 RPL (and m <= 256) and
// ceil(n/4) <= 64 CPT (<= 32 with PAIR).
// BB: the adaptive beta of Section 4.3 compiled in (launches with settings.bb).
template <int CPT, int RPL, bool PAIR, bool GS, bool BB>
__device__ __noinline__ bool solve_small(int k, const LPDesc& d_in, LPCtrl* __restrict__ ctrl, const PoolPtrs& P_in,
                                         const SolveParams& prm_in, int64_t fixed_iters) {
    static_assert(!PAIR || CPT == 1, "column pairs own one column");
    // the launch's dynamic LDS, named here so that every access is an LDS access
    extern __shared__ __align__(16) unsigned char small_lds[];
    unsigned char* const smem = small_lds;
    // private copies: the loop must not reload the caller's structs through
    // generic pointers after every LDS store
    const LPDesc d = d_in;
    const PoolPtrs P = P_in;
    const SolveParams prm = prm_in;
    const int m = small_uni(d.m), n = small_uni(d.n);
    const int tid = threadIdx.x, lane = tid & 63, wave = wave_id();
    const LPCtrl cl = ctrl[k];
    int phase = cl.phase;
    // this variant runs a phase held in LDS with (GS false) or without (GS true) G^{-1}
    auto runs_here = [&](int ph) {
        const int full = ph == 0 ? DESC_LDS32 : DESC_LDS64, aonly = ph == 0 ? DESC_LDSA32 : DESC_LDSA64;
        return GS ? ((d.lds & full) == 0 && (d.lds & aonly) != 0) : (d.lds & full) != 0;
    };
    if (num_waves() != SMALL_W || !runs_here(phase)) return false;
    const int cb = small_uni((n + SMALL_W - 1) / SMALL_W);      // columns per wave
    const int rb = small_uni((m + SMALL_W - 1) / SMALL_W);      // rows per wave

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

    double tau = cl.tau, kappa = cl.kappa, theta = cl.theta, mu = cl.mu;
    int64_t iters = cl.iters, iters64 = cl.iters64, ipm = cl.ipm;
    int64_t cp32 = cl.cp32, cp64 = cl.cp64;
    int64_t cpl32 = cl.cpl32, cpl64 = cl.cpl64, gh32 = cl.gh32, gh64 = cl.gh64;
    double kfx = cl.kfx;
    bool exit_pend = (cl.flags & 8) != 0;     // the next FP64 check measures the FP32 exit
    int status = cl.status;
    const int check_final_first = cl.flags & 1;
    double l_ms2 = 0.0, l_cs4 = 0.0, l_tau = 0.0;
    bool l_have = false;
    double by_last = cl.by, cx_last = cl.cx;
    const double zbar = cl.zbar, nb = cl.nb, nc = cl.nc;
    const double alpha = prm.alpha, gamma = prm.gamma, eps = prm.eps;
    const double np1 = (double)n + 1.0;
    // Section 4.3 (as in the streamed variant): the outer iteration's beta, a
    // pending choice, the probe stage (1 / 2: first / second probe update done,
    // 3: initial point restored after the final estimate)
    double beta = BB ? cl.beta : prm.beta;
    bool bb_pend = BB && (cl.flags & 16) != 0;
    int bb_stage = 0, bbe = cl.bbe, bb_est_run = 0;
    int64_t bbp = cl.bbp;

    // row owner registers: lane l of wave w owns row w*rb + l (lanes past the
    // block or past m hold zeros and add nothing)
    const int ri = wave * rb + lane;
    const bool rown = lane < rb && ri < m;
    const int rr = rown ? ri : 0;
    double y = rown ? Yg[rr] : 0.0;
    const double rbv = rown ? b[rr] : 0.0, rbb = rown ? bbar[rr] : 0.0;
    const double rac = rown ? Ac[rr] : 0.0, racb = rown ? Acb[rr] : 0.0;
    const double rz0 = rown ? Zy0[rr] : 0.0, rz1 = rown ? Zy1[rr] : 0.0;
    // column owner registers
    SmallCol col[CPT];
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        const int j = small_col<CPT, PAIR>(q, cb, n);
        const int jj = (j >= 0) ? j : 0;
        col[q].x = X[jj]; col[q].s = S[jj]; col[q].c = C[jj]; col[q].cb = CBv[jj];
        col[q].z0 = ZX0[jj]; col[q].z1 = ZX1[jj];
        col[q].aty = 0.0; col[q].atz0 = 0.0; col[q].atz1 = 0.0;
    }

    bool wide = small_wide(d.lds, phase);    // LDS entries are doubles
    SmallLayout L = small_layout(m, n, wide ? 8 : 4, SMALL_W, GS);
    const int m4 = L.m4;                   // the same in both precisions
    double* av = reinterpret_cast<double*>(smem + L.oav);
    double2* fx = reinterpret_cast<double2*>(smem + L.ofx);
    double* tv = reinterpret_cast<double*>(smem + L.otv);
    double* pf = reinterpret_cast<double*>(smem + L.opf);
    double* pg = reinterpret_cast<double*>(smem + L.opg);
    double* red = reinterpret_cast<double*>(smem + L.ored);

    // this phase's matrices into LDS, and A^T Zy0, A^T Zy1 for the y recurrence
    small_load_phase<CPT, PAIR>(phase, d, cb, P, Zy0, Zy1, smem, L, col);

    double p0 = 0.0, p1 = 0.0;
    int pass_kind = (cl.mode == OP_PROX) ? OP_REFRESH : cl.mode;   // a state enters with a refresh
    bool first = true;
    int64_t done_fixed = 0;
    StallTrack stall;
    stall_reset(stall);
    int64_t passes = 0;
    const int64_t pass_cap = prm.max_iters + 4096;
    int64_t cyc_col = 0, cyc_ginv = 0, cyc_chk = 0, cyc_upd = 0;
    const int64_t t_start = wall_clock64();
    bool handover = false;
    while (true) {
        if (++passes > pass_cap && fixed_iters == 0) { status = 4; break; }
        const double tmu = mu / beta;      // t = mu / beta, eq. (Simple-Update:Barrier-X)
        const int64_t t0 = wall_clock64();
        if (pass_kind != OP_PROX) {        // exact A^T y of the (rescaled) state
            if (rown) av[ri] = y;
            __syncthreads();
        }
        // ---- column pass (own columns), then A f, A x over the own columns
        double acc[7] = {0, 0, 0, 0, 0, 0, 0};
        if (!wide) {
            small_colpass<float, CPT, PAIR>(reinterpret_cast<const float*>(smem + L.oA), L.lda, m4, n, cb, av, col,
                                            fx, pass_kind, p0, p1, tmu, alpha, gamma, prm.restart_rule, tau,
                                            theta, acc);
            small_rowpass<float, RPL>(reinterpret_cast<const float*>(smem + L.oA), L.lda, m, n, m4, cb, fx, pf);
        } else {
            small_colpass<double, CPT, PAIR>(reinterpret_cast<const double*>(smem + L.oA), L.lda, m4, n, cb, av,
                                             col, fx, pass_kind, p0, p1, tmu, alpha, gamma, prm.restart_rule, tau,
                                             theta, acc);
            small_rowpass<double, RPL>(reinterpret_cast<const double*>(smem + L.oA), L.lda, m, n, m4, cb, fx, pf);
        }
        __syncthreads();
        // ---- row owner: A f, A x of the new state, t = y - A f, m-side sums
        double v12[12];
        {
            double Af = 0.0, Ax = 0.0;
            if (rown) {
#pragma unroll
                for (int w = 0; w < SMALL_W; ++w) {
                    Af += pf[(2 * w) * m4 + ri];
                    Ax += pf[(2 * w + 1) * m4 + ri];
                }
                tv[ri] = y - Af;
            }
            const double r1 = Ax - rbv * tau;
            const double r3 = r1 + rbb * theta;
#pragma unroll
            for (int q = 0; q < 7; ++q) v12[q] = acc[q];
            v12[7] = rbv * y;
            v12[8] = rbb * y;
            v12[9] = r1 * r1;
            v12[10] = Ax * Ax;
            v12[11] = r3 * r3;
        }
        cyc_col += wall_clock64() - t0;
        // ---- G^{-1} t over the own rows, before the tests (a restart or a
        // verdict leaves it unused); the sums' barrier publishes its partials
        const int64_t t1 = wall_clock64();
        if constexpr (GS) {            // G^{-1} columns from the pool (L2 / MALL)
            if (phase == 0) small_gpass<float, RPL>(P.G32 + d.oG, d.ld, m, m4, rb, tv, pg);
            else small_gpass<double, RPL>(P.G64 + d.oG, d.ld, m, m4, rb, tv, pg);
        } else {
            if (!wide) small_gpass<float, RPL>(reinterpret_cast<const float*>(smem + L.oG), L.ldg, m, m4, rb, tv, pg);
            else small_gpass<double, RPL>(reinterpret_cast<const double*>(smem + L.oG), L.ldg, m, m4, rb, tv, pg);
        }
        cyc_ginv += wall_clock64() - t1;
        const int64_t tc = wall_clock64();
        small_bsum<12>(v12, red);
        if (phase == 0) { ++cp32; ++cpl32; } else { ++cp64; ++cpl64; }
        if constexpr (GS) { if (phase == 0) ++gh32; else ++gh64; }
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

        const double cx = v12[0], cbx = v12[1];
        const double by = v12[7], bby = v12[8];
        const double ms2 = v12[9], ms3 = v12[10], ms4 = v12[11];
        const double cs4 = v12[4], cs5 = v12[5], cs6 = v12[6];
        if (fixed_iters == 0 && !bb_pass) {
            int to_phase1 = 0;
            if (post_update) {
                int st = 0;
                // Section 4.1's tests multiplied through by tau (> 0) and squared
                if (tau > 0.0) {
                    const double ep = eps * (1.0 + nb) * tau, ed = eps * (1.0 + nc) * tau;
                    if (ms2 <= ep * ep && cs4 <= ed * ed && fabs(cx - by) <= eps * (tau + fabs(cx) + fabs(by)))
                        st = 1;
                }
                if (!st && nb > 0.0 && by > 0.0 && cs5 * (nb * nb) <= (eps * by) * (eps * by)) st = 2;
                if (!st && nc > 0.0 && cx < 0.0 && ms3 * (nc * nc) <= (eps * cx) * (eps * cx)) st = 3;
                l_ms2 = ms2; l_cs4 = cs4; l_tau = tau; l_have = true;
                by_last = by;
                cx_last = cx;
                if (exit_pend && phase == 1) {     // the FP32 phase's last iterate, FP64 data
                    kfx = kkt_rel(ms2, cs4, cx, by, tau, nb, nc);
                    exit_pend = false;
                }
                if (st) {
                    if (phase == 0) to_phase1 = 1;     // FP32 verdict: confirm with FP64 data
                    else { status = st; break; }
                }
            }
            if (!to_phase1 && phase == 0 && iters >= prm.fp32_max_iters) to_phase1 = 1;
            if (!to_phase1) {
                // ---- inner test ||Q u - v||^2 <= mu (eq. inner-stop)
                const double rt = by - cx + zbar * theta - kappa;
                const double rth = -bby + cbx - zbar * tau + np1;
                const double inner = ms4 + cs6 + rt * rt + rth * rth;
                if (inner <= mu) {
                    mu *= gamma;
                    ++ipm;
                    if (prm.restart_rule == 0) {
                        if (tau >= kappa) kappa *= gamma;
                        else tau *= gamma;
                    } else {
                        const double sg = sqrt(gamma);
                        tau *= sg; kappa *= sg; theta *= sg;
                        y *= sg;
                    }
                    stall_reset(stall);
                    bb_pend = BB;
                    pass_kind = OP_RESTART;
                    cyc_chk += wall_clock64() - tc;
                    continue;
                }
                if (phase == 0 && was_update && stall_sample(stall, inner, mu)) to_phase1 = 1;
            }
            if (to_phase1) {                   // FP32 verdict or precision floor: FP64 data
                phase = 1;
                exit_pend = true;
                pass_kind = OP_REFRESH;
                cyc_chk += wall_clock64() - tc;
                // FP64 data held the other way (or not at all): hand over; the
                // caller continues with the matching variant or streams
                if (!runs_here(1)) { handover = true; break; }
                small_load_phase<CPT, PAIR>(phase, d, cb, P, Zy0, Zy1, smem, L, col);
                wide = true;
                av = reinterpret_cast<double*>(smem + L.oav);
                fx = reinterpret_cast<double2*>(smem + L.ofx);
                tv = reinterpret_cast<double*>(smem + L.otv);
                pf = reinterpret_cast<double*>(smem + L.opf);
                pg = reinterpret_cast<double*>(smem + L.opg);
                red = reinterpret_cast<double*>(smem + L.ored);
                continue;
            }
            // (an outer iteration that starts with a beta choice takes its probes first)
            if (iters >= prm.max_iters && !(BB && bb_pend)) { status = 4; break; }
        }
        if (BB && fixed_iters == 0 && (bb_pend || bb_pass)) {
            // ---- adaptive beta (Section 4.3), out of line: rare passes
            const int prev = bb_stage;
            if (!bb_pass) bb_pend = false;
            const SmallBB r = bb_advance_small<CPT, PAIR>(
                k, m, n, d.om, d.on, P_in, ctrl, red, bb_stage, was_update, cb, ri, rown, y, col[0].x, col[0].s,
                col[CPT - 1].x, col[CPT - 1].s, tau, kappa, theta, beta, prm_in, bb_est_run, bbe);
            tau = r.tau; kappa = r.kappa; theta = r.theta; beta = r.beta;
            bb_stage = r.stage; bb_est_run = r.est; bbe = r.bbe;
            if (r.restored) {
                y = r.y;
                col[0].x = r.x0; col[0].s = r.s0;
                if constexpr (CPT > 1) { col[CPT - 1].x = r.x1; col[CPT - 1].s = r.s1; }
                pass_kind = OP_REFRESH;        // exact A^T y and the products of the initial point
                cyc_chk += wall_clock64() - tc;
                continue;
            }
            if (prev == 3 && iters >= prm.max_iters) { status = 4; break; }
        }
        cyc_chk += wall_clock64() - tc;

        // ---- the inner update: a = G^{-1} t, border, scalars, y'
        const int64_t t2 = wall_clock64();
        double a = 0.0;
        if (rown) {
#pragma unroll
            for (int w = 0; w < SMALL_W; ++w) a += pg[w * m4 + ri];
            av[ri] = a;
        }
        double bs[4] = {rbv * a, rbb * a, rac * a, racb * a};
        small_bsum<4>(bs, red + 12 * SMALL_W);
        const double cs_f = cx + v12[2];        // c^T (x + s)
        const double cbs_f = cbx + v12[3];      // cbar^T (x + s)
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
        if (rown) y = alpha * (a - rz0 * p0 - rz1 * p1) + (1.0 - alpha) * y;
        cyc_upd += wall_clock64() - t2;
        pass_kind = OP_PROX;
    }

    // state back to the pools
    if (rown) Yg[ri] = y;
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        const int j = small_col<CPT, PAIR>(q, cb, n);
        if (j >= 0 && (!PAIR || (tid & 1) == 0)) { X[j] = col[q].x; S[j] = col[q].s; }
    }
    if (handover) {
        // the streamed variant continues with a tested refresh in FP64
        if (tid == 0) {
            LPCtrl& o = ctrl[k];
            o.clk[0] += cyc_col; o.clk[1] += cyc_ginv; o.clk[2] += wall_clock64() - t_start;
            o.clk[3] += cyc_chk; o.clk[4] += cyc_upd;
            o.tau = tau; o.kappa = kappa; o.theta = theta; o.mu = mu;
            o.by = by_last; o.cx = cx_last;
            o.iters = iters; o.iters64 = iters64; o.ipm = ipm;
            o.cp32 = cp32; o.cp64 = cp64;
            o.cpl32 = cpl32; o.cpl64 = cpl64; o.gh32 = gh32; o.gh64 = gh64; o.kfx = kfx;
            if (BB) { o.beta = beta; o.bbp = bbp; o.bbe = bbe; }
            o.status = 0; o.phase = 1;
            o.mode = OP_REFRESH;
            o.flags = (cl.flags & 4) | 1 | (exit_pend ? 8 : 0) | (bb_pend ? 16 : 0);
        }
        __syncthreads();
        return false;
    }
    if (tid == 0) {
        LPCtrl& o = ctrl[k];
        if (l_have && l_tau > 0.0) {       // the relative residuals of the last test
            o.pobj = cx_last / l_tau;
            o.dobj = by_last / l_tau;
            o.pres = sqrt(l_ms2) / l_tau / (1.0 + nb);
            o.dres = sqrt(l_cs4) / l_tau / (1.0 + nc);
            o.gap = fabs(o.pobj - o.dobj) / (1.0 + fabs(o.pobj) + fabs(o.dobj));
        }
        o.clk[0] += cyc_col; o.clk[1] += cyc_ginv; o.clk[2] += wall_clock64() - t_start;
        o.clk[3] += cyc_chk; o.clk[4] += cyc_upd;
        o.tau = tau; o.kappa = kappa; o.theta = theta; o.mu = mu;
        o.by = by_last; o.cx = cx_last;
        o.iters = iters; o.iters64 = iters64; o.ipm = ipm;
        o.cp32 = cp32; o.cp64 = cp64;
        o.cpl32 = cpl32; o.cpl64 = cpl64; o.gh32 = gh32; o.gh64 = gh64; o.kfx = kfx;
        if (BB) { o.beta = beta; o.bbp = bbp; o.bbe = bbe; }
        o.status = status; o.phase = phase;
        o.mode = OP_REFRESH;
        o.flags = ((fixed_iters > 0) ? 1 : 0) | (cl.flags & 4) | (bb_pend ? 16 : 0);
    }
    __syncthreads();
    return true;
}

// Pick the variant for this LP: rows per lane from m, column pairs when a
// wave owns at most 32 columns, one or two columns per lane otherwise.
template <bool GS, bool BB>
__device__ inline bool solve_small_shape(int k, const LPDesc& d, LPCtrl* __restrict__ ctrl, const PoolPtrs& P,
                                         const SolveParams& prm, int64_t fixed_iters) {
    const int rpl = (d.m + 63) >> 6;
    const int cb = (d.n + SMALL_W - 1) / SMALL_W;
    if (cb <= 32) {
        switch (rpl) {
        case 1: return solve_small<1, 1, true, GS, BB>(k, d, ctrl, P, prm, fixed_iters);
        case 2: return solve_small<1, 2, true, GS, BB>(k, d, ctrl, P, prm, fixed_iters);
        case 3: return solve_small<1, 3, true, GS, BB>(k, d, ctrl, P, prm, fixed_iters);
        default: return solve_small<1, 4, true, GS, BB>(k, d, ctrl, P, prm, fixed_iters);
        }
    }
    if (cb <= 64) {
        switch (rpl) {
        case 1: return solve_small<1, 1, false, GS, BB>(k, d, ctrl, P, prm, fixed_iters);
        case 2: return solve_small<1, 2, false, GS, BB>(k, d, ctrl, P, prm, fixed_iters);
        case 3: return solve_small<1, 3, false, GS, BB>(k, d, ctrl, P, prm, fixed_iters);
        default: return solve_small<1, 4, false, GS, BB>(k, d, ctrl, P, prm, fixed_iters);
        }
    }
    switch (rpl) {
    case 1: return solve_small<2, 1, false, GS, BB>(k, d, ctrl, P, prm, fixed_iters);
    case 2: return solve_small<2, 2, false, GS, BB>(k, d, ctrl, P, prm, fixed_iters);
    case 3: return solve_small<2, 3, false, GS, BB>(k, d, ctrl, P, prm, fixed_iters);
    default: return solve_small<2, 4, false, GS, BB>(k, d, ctrl, P, prm, fixed_iters);
    }
}

// A and G^{-1} in LDS first; then A alone (the current phase may be held that
// way from the start, or the FP32 -> FP64 handover of the first variant may
// have left a phase that is).  false: the streamed variant continues from the
// state in ctrl[k] and the pools.
template <bool BB>
__device__ inline bool solve_small_any(int k, const LPDesc& d, LPCtrl* __restrict__ ctrl, const PoolPtrs& P,
                                       const SolveParams& prm, int64_t fixed_iters) {
    if (solve_small_shape<false, BB>(k, d, ctrl, P, prm, fixed_iters)) return true;
    return solve_small_shape<true, BB>(k, d, ctrl, P, prm, fixed_iters);
}
