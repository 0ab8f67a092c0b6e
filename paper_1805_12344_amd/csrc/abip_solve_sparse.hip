// Sparse engine: Algorithm 2 on one LP whose A is given in CSR.  The linear
// step u~ = (I+Q)^{-1} w keeps the Schur reduction of Section 4.4 (with the
// theta column, so a rank-2 border), and solves G a = w_y - A w_x,
// G = I + A A^T, by Jacobi-preconditioned CG (the indirect variant of Section
// 4.4: every CG iteration is one product with A^T and one with A).  CG starts
// from the previous solution a, whose A^T a is kept from the last update.
//
// One cooperative launch runs the whole solve.  Rows of A and columns (rows of
// CSR(A^T)) are split into contiguous ranges over the workgroups; phases are
// separated by a grid barrier; every workgroup reduces the per-workgroup
// partial sums in the same fixed order and takes the same decisions, so runs
// are bitwise reproducible.  Per update: the column pass (prox, dual update,
// A^T y of the new iterate, column sums of the check), the row pass (A x, A s,
// the row sums of the check, the CG right-hand side and start), then 2
// barriers per CG iteration.  A workgroup whose rows of CSR(A) and CSR(A^T)
// fit in the launch's LDS keeps them there for the CG passes.
#include <hip/hip_runtime.h>
#include <algorithm>
#include <cmath>
#include "abip_internal.h"
#include "abip_sparse.h"

#define SP_THREADS 256

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------

// Sum over aligned groups of L consecutive lanes (L a power of two <= 64);
// every lane of a group receives the group total (same DPP / permlane steps
// as the wave sums, stopped after log2 L of them).  All 64 lanes must be active.
__device__ __forceinline__ double group_sum(double v, int L) {
    if (L >= 2) v = v + dpp_partner<0xB1>(v);
    if (L >= 4) v = v + dpp_partner<0x4E>(v);
    if (L >= 8) v = v + dpp_partner<0x141>(v);
    if (L >= 16) v = v + dpp_partner<0x140>(v);
    if (L >= 32) v = swap16_sum(v);
    if (L >= 64) v = swap32_sum(v);
    return v;
}

// Grid-wide barrier for a cooperative launch (all workgroups co-resident).
// Counter + generation; the last arrival resets the counter and bumps the
// generation.  A wait that outlasts ~2^22 polls sets *err and returns (the
// solver loop then exits), so no wave can spin forever.  Each workgroup
// releases before it counts itself in (an L2 write-back) and acquires after
// the wait (an L2 invalidate); a full fence on both sides took both each time
// (47 -> 39 us per CG iteration of the 10000 x 30000 LP with the split).
__device__ __forceinline__ void grid_sync(unsigned* bar, int* err) {
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned* cnt = bar;
        unsigned* gen = bar + 1;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");   // release this workgroup's writes
        const unsigned g0 = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned arrived = atomicAdd(cnt, 1u);
        if (arrived == gridDim.x - 1) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // the others' releases, before ours
            __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            // relaxed polls (an acquire per poll would invalidate this XCD's L2
            // under the workgroups still computing); one acquire fence after
            int polls = 0;
            while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g0) {
                __builtin_amdgcn_s_sleep(2);
                if (++polls > (1 << 22)) { atomicExch(err, 1); break; }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // acquire the other workgroups' writes
    }
    __syncthreads();
}

__device__ __forceinline__ bool grid_failed(int* err) {
    return __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// Block sum of K per-thread values written to this workgroup's partial slots.
template <int K>
__device__ __forceinline__ void put_parts(double (&v)[K], double* part, int nbp, int slot, double* sbuf) {
    block_sum_n<K>(v, sbuf);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) part[(int64_t)(slot + k) * nbp + blockIdx.x] = v[k];
    }
}

// Totals of K partial slots over all workgroups, in a fixed order (lane l
// adds workgroups l, l+64, l+128, l+192 as two pairs, then every 256th; then
// the wave sum); one value per wave at a time, every load of a value issued
// together.  Every thread gets the totals.
template <int K>
__device__ __forceinline__ void get_parts(const double* part, int nbp, int slot, double (&out)[K], double* sbuf) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, W = blockDim.x >> 6;
    const int nb = gridDim.x;
    for (int k = wave; k < K; k += W) {
        const double* pk = part + (int64_t)(slot + k) * nbp;
        double s0 = 0.0, s1 = 0.0;
        for (int b0 = lane; b0 < nb; b0 += 256) {
            const double v0 = pk[b0];
            const double v1 = (b0 + 64 < nb) ? pk[b0 + 64] : 0.0;
            const double v2 = (b0 + 128 < nb) ? pk[b0 + 128] : 0.0;
            const double v3 = (b0 + 192 < nb) ? pk[b0 + 192] : 0.0;
            s0 += v0 + v1;
            s1 += v2 + v3;
        }
        double s = wave_sum(s0 + s1);
        if (lane == 0) sbuf[k] = s;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) out[k] = sbuf[k];
    __syncthreads();
}

// Sums over one CSR row of val[e] * f(idx[e]) (NV sums, f returns NV values)
// for e = kb+sub, kb+sub+L, ... < ke, in that order, four entries per round so
// that their index / value loads and the gathers behind them are in flight
// together.  Entries past ke read index 0 with weight 0.
template <int NV, typename F>
__device__ __forceinline__ void row_sums(const int32_t* idx, const double* val, int kb, int ke, int sub, int L,
                                         F f, double (&out)[NV]) {
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v] = 0.0;
    for (int e = kb + sub; e < ke; e += 4 * L) {
        int ii[4];
        double ww[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int eu = e + u * L;
            const bool ok = eu < ke;
            ii[u] = ok ? idx[eu] : 0;
            ww[u] = ok ? val[eu] : 0.0;
        }
        double fv[4][NV];
#pragma unroll
        for (int u = 0; u < 4; ++u) f(ii[u], fv[u]);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < NV; ++v) out[v] = fma(ww[u], fv[u][v], out[v]);
    }
}

struct Range { int lo, hi; };
__device__ __forceinline__ Range my_range(int total) {
    Range r;
    sp_share(total, (int)blockIdx.x, (int)gridDim.x, &r.lo, &r.hi);
    return r;
}

// ---------------------------------------------------------------------------
// LDS-resident slices.  A workgroup owns the same columns (rows of CSR(A^T))
// and rows of CSR(A) for the whole launch, so it copies those rows of both
// matrices into LDS once; the CG passes then read no matrix entry from global
// memory (a grid barrier's acquire leaves the L2 cold for them otherwise).
// A pass forms every product val[e] * f(idx[e]) of the slice with all the
// gathers of a round in flight, stores them in LDS, and the owner of each row
// adds its products in entry order (deterministic).
// ---------------------------------------------------------------------------
struct SpSlice {
    int n, ne;                 // rows, entries
    const int32_t* ptr;        // n + 1 offsets (LDS)
    const int32_t* idx;        // ne column indices (LDS)
    const double* val;         // ne values (LDS)
};
struct SpLds {
    bool on;
    SpSlice t, a;              // CSR(A^T) rows of the workgroup's columns, CSR(A) rows of its rows
    double* prod;              // max(t.ne, a.ne) products
};

// Copy the slices when they fit in the launch's dynamic LDS (the decision is
// the workgroup's own; the others may run the global-memory passes).  Ends
// with a workgroup barrier when it copies.
__device__ SpLds sp_lds_init(const SpArgs& g, Range R, Range Cc, unsigned char* lds) {
    SpLds L;
    L.on = false;
    if (g.lds_bytes <= 0) return L;
    const int tid = threadIdx.x;
    const int tb = g.rpt[Cc.lo], te = g.rpt[Cc.hi], ab = g.rp[R.lo], ae = g.rp[R.hi];
    const int tnc = Cc.hi - Cc.lo, tne = te - tb, anr = R.hi - R.lo, ane = ae - ab;
    if (sp_slice_bytes(tnc, tne, anr, ane) > (int64_t)g.lds_bytes) return L;
    double* tval = reinterpret_cast<double*>(lds);
    double* aval = tval + tne;
    double* prod = aval + ane;
    int32_t* tidx = reinterpret_cast<int32_t*>(prod + max(tne, ane));
    int32_t* aidx = tidx + tne;
    int32_t* tptr = aidx + ane;
    int32_t* aptr = tptr + (tnc + 1);
    for (int e = tid; e < tne; e += SP_THREADS) { tidx[e] = g.cit[tb + e]; tval[e] = g.vat[tb + e]; }
    for (int e = tid; e < ane; e += SP_THREADS) { aidx[e] = g.ci[ab + e]; aval[e] = g.va[ab + e]; }
    for (int c = tid; c <= tnc; c += SP_THREADS) tptr[c] = g.rpt[Cc.lo + c] - tb;
    for (int r = tid; r <= anr; r += SP_THREADS) aptr[r] = g.rp[R.lo + r] - ab;
    __syncthreads();
    L.on = true;
    L.t = {tnc, tne, tptr, tidx, tval};
    L.a = {anr, ane, aptr, aidx, aval};
    L.prod = prod;
    return L;
}

// prod[e] = val[e] * f(idx[e]) for every entry of the slice, eight entries per
// thread and round with their gathers issued together; ends with a workgroup
// barrier.
template <typename F>
__device__ __forceinline__ void slice_products(const SpSlice& S, double* __restrict__ prod, F f) {
    constexpr int U = 8;
    const int tid = threadIdx.x;
    for (int e0 = 0; e0 < S.ne; e0 += U * SP_THREADS) {
        int ii[U];
        double vv[U], fv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * SP_THREADS + tid;
            const bool ok = e < S.ne;
            ii[u] = ok ? S.idx[e] : 0;
            vv[u] = ok ? S.val[e] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) fv[u] = f(ii[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * SP_THREADS + tid;
            if (e < S.ne) prod[e] = vv[u] * fv[u];
        }
    }
    __syncthreads();
}

// Sum of row r's products, in entry order.
__device__ __forceinline__ double slice_row_sum(const SpSlice& S, const double* __restrict__ prod, int r) {
    const int kb = S.ptr[r], ke = S.ptr[r + 1];
    double s0 = 0.0, s1 = 0.0;
    int e = kb;
    for (; e + 1 < ke; e += 2) {
        s0 += prod[e];
        s1 += prod[e + 1];
    }
    if (e < ke) s0 += prod[e];
    return s0 + s1;
}

// ---------------------------------------------------------------------------
// CG on G a = t, G = I + A A^T, Jacobi preconditioned, in the Chronopoulos-Gear
// arrangement (both inner products of an iteration come out of one
// reduction), with the vector recurrences folded into the gathers so that an
// iteration needs two grid barriers:
//   P1 (columns):  u' = (r - al (w + be s)) / diag(G) formed on the fly,
//                  q1 = A^T u'                                   -> barrier
//   P2 (rows):     p = u + be p, s = w + be s, a += al p, r -= al s,
//                  u = r / diag(G), w = u + A q1 (= G u),
//                  partial (r,u), (w,u), (r,r), border dots of a  -> barrier
//   then every workgroup forms be = g'/g, al = g' / (d - be g' / al).
// r, w, s of a row sit in one record (SpRow) with 1 / diag(G), so the gather
// of P1 is one 32-byte load; the division by diag(G) is a product with that
// reciprocal on both sides, so q1 = A^T u exactly for the stored u.
// On entry (set by the caller) r = t - G a, u = 0, w = 0, s = 0, p = 0, and
// al = be = 0, so the first P1/P2 pair computes u0 = r / diag(G), w0 = G u0.
// Returns the number of updates of a.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double sp_u_next(const SpRow& q, double al, double be) {
    return fma(-al, fma(be, q.s, q.w), q.r) * q.idg;
}

// The same iteration with G~ = A A^T given explicitly: one pass and one grid
// barrier per iteration.  Each workgroup forms d_i = sum_j G~_ij u'_j for its
// rows (u' of every row from its record, as the column pass above does) and
// updates its rows right away; so that no row's record changes while another
// workgroup still gathers it, the records alternate between two buffers
// (read one, write the other).  On return the records are back in g.rw.
__device__ int cg_loop_gram(const SpArgs& g, double rr, double tol2, double (&bd)[4], double* sbuf, int maxit,
                            int64_t (&tk)[4]) {
    const Range R = my_range(g.m);
    const int tid = threadIdx.x;
    double al = 0.0, be = 0.0, gam_old = 1.0;
    SpRow* rd = g.rw;
    SpRow* wr = g.rw2;
    int k = -1;
    while (k < maxit && (k < 0 || rr > tol2) && !grid_failed(g.err)) {
        int64_t t0 = wall_clock64();
        double v[7] = {0, 0, 0, 0, 0, 0, 0};
        const int Lg = g.LG, per = SP_THREADS / Lg;
        for (int i0 = R.lo; i0 < R.hi; i0 += per) {
            const int i = i0 + tid / Lg, sub = tid % Lg;
            double d = 0.0;
            if (i < R.hi) {
                double o[1];
                row_sums<1>(g.gci, g.gva, g.grp[i], g.grp[i + 1], sub, Lg,
                            [&](int j, double* fv) { fv[0] = sp_u_next(rd[j], al, be); }, o);
                d = o[0];
            }
            d = group_sum(d, Lg);
            if (i < R.hi && sub == 0) {
                const double pi = fma(be, g.p[i], g.z[i]);
                const SpRow o = rd[i];
                const double si = fma(be, o.s, o.w);
                const double ai = fma(al, pi, g.a[i]);
                const double ri = fma(-al, si, o.r);
                const double ui = ri * o.idg;
                const double wi = ui + d;
                g.p[i] = pi; g.a[i] = ai; g.z[i] = ui;
                wr[i] = SpRow{ri, wi, si, o.idg};
                v[0] = fma(ri, ui, v[0]);
                v[1] = fma(wi, ui, v[1]);
                v[2] = fma(ri, ri, v[2]);
                v[3] = fma(g.b[i], ai, v[3]);
                v[4] = fma(g.bbar[i], ai, v[4]);
                v[5] = fma(g.Ac[i], ai, v[5]);
                v[6] = fma(g.Acb[i], ai, v[6]);
            }
        }
        put_parts<7>(v, g.part, g.nbp, SP_CG, sbuf);
        int64_t t1 = wall_clock64();
        tk[1] += t1 - t0;
        grid_sync(g.bar, g.err);
        t0 = wall_clock64();
        tk[2] += t0 - t1;
        double t7[7];
        get_parts<7>(g.part, g.nbp, SP_CG, t7, sbuf);
        tk[3] += wall_clock64() - t0;
        bd[0] = t7[3]; bd[1] = t7[4]; bd[2] = t7[5]; bd[3] = t7[6];
        const double gam = t7[0], del = t7[1];
        rr = t7[2];
        if (k < 0) { be = 0.0; al = gam / del; }
        else { be = gam / gam_old; al = gam / (del - be * gam / al); }
        gam_old = gam;
        ++k;
        SpRow* tmp = rd; rd = wr; wr = tmp;
    }
    if (rd != g.rw) {
        for (int i = R.lo + tid; i < R.hi; i += SP_THREADS) g.rw[i] = rd[i];
        __syncthreads();
    }
    return k < 0 ? 0 : k;
}

__device__ int cg_loop(const SpArgs& g, const SpLds& L, double rr, double tol2, double (&bd)[4], double* sbuf,
                       int maxit, int64_t (&tk)[4]) {
    if (g.grp) return cg_loop_gram(g, rr, tol2, bd, sbuf, maxit, tk);
    const Range R = my_range(g.m), Cc = my_range(g.n);
    const int tid = threadIdx.x;
    double al = 0.0, be = 0.0, gam_old = 1.0;
    int k = -1;                     // -1: the start-up pair (no update of a yet)
    while (k < maxit && (k < 0 || rr > tol2) && !grid_failed(g.err)) {
        int64_t t0 = wall_clock64();
        // P1: q1_j = sum_i A_ij u'_i
        if (L.on) {
            slice_products(L.t, L.prod, [&](int i) { return sp_u_next(g.rw[i], al, be); });
            for (int c = tid; c < L.t.n; c += SP_THREADS) g.q1[Cc.lo + c] = slice_row_sum(L.t, L.prod, c);
        } else {
            const int Lt = g.LT, per = SP_THREADS / Lt;
            for (int j0 = Cc.lo; j0 < Cc.hi; j0 += per) {
                const int j = j0 + tid / Lt, sub = tid % Lt;
                double d = 0.0;
                if (j < Cc.hi) {
                    double o[1];
                    row_sums<1>(g.cit, g.vat, g.rpt[j], g.rpt[j + 1], sub, Lt,
                                [&](int i, double* fv) { fv[0] = sp_u_next(g.rw[i], al, be); }, o);
                    d = o[0];
                }
                d = group_sum(d, Lt);
                if (j < Cc.hi && sub == 0) g.q1[j] = d;
            }
        }
        int64_t t1 = wall_clock64();
        tk[0] += t1 - t0;
        grid_sync(g.bar, g.err);
        t0 = wall_clock64();
        tk[2] += t0 - t1;
        // P2: this workgroup's rows
        double v[7] = {0, 0, 0, 0, 0, 0, 0};
        auto row_update = [&](int i, double d) {
            const double pi = fma(be, g.p[i], g.z[i]);
            const SpRow o = g.rw[i];
            const double si = fma(be, o.s, o.w);
            const double ai = fma(al, pi, g.a[i]);
            const double ri = fma(-al, si, o.r);
            const double ui = ri * o.idg;
            const double wi = ui + d;
            g.p[i] = pi; g.a[i] = ai; g.z[i] = ui;
            g.rw[i] = SpRow{ri, wi, si, o.idg};
            v[0] = fma(ri, ui, v[0]);
            v[1] = fma(wi, ui, v[1]);
            v[2] = fma(ri, ri, v[2]);
            v[3] = fma(g.b[i], ai, v[3]);
            v[4] = fma(g.bbar[i], ai, v[4]);
            v[5] = fma(g.Ac[i], ai, v[5]);
            v[6] = fma(g.Acb[i], ai, v[6]);
        };
        if (L.on) {
            slice_products(L.a, L.prod, [&](int j) { return g.q1[j]; });
            for (int r = tid; r < L.a.n; r += SP_THREADS) row_update(R.lo + r, slice_row_sum(L.a, L.prod, r));
        } else {
            const int La = g.LA, per = SP_THREADS / La;
            for (int i0 = R.lo; i0 < R.hi; i0 += per) {
                const int i = i0 + tid / La, sub = tid % La;
                double d = 0.0;
                if (i < R.hi) {
                    double o[1];
                    row_sums<1>(g.ci, g.va, g.rp[i], g.rp[i + 1], sub, La,
                                [&](int jj, double* fv) { fv[0] = g.q1[jj]; }, o);
                    d = o[0];
                }
                d = group_sum(d, La);
                if (i < R.hi && sub == 0) row_update(i, d);
            }
        }
        put_parts<7>(v, g.part, g.nbp, SP_CG, sbuf);
        t1 = wall_clock64();
        tk[1] += t1 - t0;
        grid_sync(g.bar, g.err);
        t0 = wall_clock64();
        tk[2] += t0 - t1;
        double t7[7];
        get_parts<7>(g.part, g.nbp, SP_CG, t7, sbuf);
        tk[3] += wall_clock64() - t0;
        bd[0] = t7[3]; bd[1] = t7[4]; bd[2] = t7[5]; bd[3] = t7[6];
        const double gam = t7[0], del = t7[1];
        rr = t7[2];
        if (k < 0) { be = 0.0; al = gam / del; }
        else { be = gam / gam_old; al = gam / (del - be * gam / al); }
        gam_old = gam;
        ++k;
    }
    return k < 0 ? 0 : k;
}

// ---------------------------------------------------------------------------
// the solver
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(SP_THREADS) void k_sp_solve(SpArgs g) {
    __shared__ double sbuf[64];
    extern __shared__ __align__(16) unsigned char sp_lds[];
    const int tid = threadIdx.x;
    const int m = g.m, n = g.n;
    const Range R = my_range(m), Cc = my_range(n);
    const SpLds L = sp_lds_init(g, R, Cc, sp_lds);
    const LPCtrl cl = *g.lc;
    const SolveParams& prm = g.prm;
    const double alpha = prm.alpha, gamma = prm.gamma, eps = prm.eps;
    const double zbar = cl.zbar, nb = cl.nb, nc = cl.nc, np1 = (double)n + 1.0;
    const double sg = sqrt(gamma);
    double tau = cl.tau, kappa = cl.kappa, theta = cl.theta, mu = cl.mu;
    int64_t iters = cl.iters, ipm = cl.ipm, cgit = cl.cg, done = 0;
    int status = 0;
    int op = OP_REFRESH;
    const bool check_final_first = (cl.flags & 1) != 0;
    bool first = true;
    double p0 = 0.0, p1 = 0.0;
    double l_ms2 = 0.0, l_cs4 = 0.0, l_tau = 0.0, l_by = cl.by, l_cx = cl.cx;
    bool l_have = false;
    const int64_t t_start = wall_clock64();
    int64_t tk[4] = {0, 0, 0, 0};      // ticks: column passes, row passes, barriers, reductions
    // Section 4.3: the outer iteration's beta and the state of its choice (every
    // workgroup holds the same values); bb_stage 1 / 2: first / second probe,
    // 3: start point restored
    const bool bb_on = prm.bb != 0 && g.fixed_iters == 0;
    double beta = bb_on ? cl.beta : prm.beta;
    bool bb_pend = bb_on && (cl.flags & 16) != 0;
    int bb_stage = 0, bb_est = 0, bbe = cl.bbe;
    int64_t bbp = cl.bbp;
    double bbs[6] = {0, 0, 0, 0, 0, 0};

    while (true) {
        if (grid_failed(g.err)) { status = -1; break; }
        const double tmu = mu / beta;
        // ---- column pass: x, s per op; A^T y of the state; 7 column sums
        int64_t ta = wall_clock64();
        double cs[7] = {0, 0, 0, 0, 0, 0, 0};
        {
            const int L = g.LT, per = SP_THREADS / L;
            const double* V = (op == OP_PROX) ? g.a : g.Y;
            for (int j0 = Cc.lo; j0 < Cc.hi; j0 += per) {
                const int j = j0 + tid / L, sub = tid % L;
                double d = 0.0;
                if (j < Cc.hi) {
                    double o[1];
                    row_sums<1>(g.cit, g.vat, g.rpt[j], g.rpt[j + 1], sub, L,
                                [&](int i, double* fv) { fv[0] = V[i]; }, o);
                    d = o[0];
                }
                d = group_sum(d, L);
                if (j < Cc.hi && sub == 0) {
                    const double x0 = g.X[j], s0 = g.S[j];
                    double x1 = x0, s1 = s0, aty;
                    if (op == OP_PROX) {
                        // d = (A^T a)_j; u~_x = (x + s) + A^T a - Z_x p (Section 4.4)
                        const double ut = (x0 + s0) + d - g.Zx0[j] * p0 - g.Zx1[j] * p1;
                        const double uh = alpha * ut + (1.0 - alpha) * x0;          // Section 4.2
                        x1 = prox_root(uh - s0, tmu);                               // barrier prox
                        s1 = s0 - uh + x1;                                          // dual update
                        // A^T y' with y' = alpha (a - Z_y p) + (1 - alpha) y
                        aty = alpha * (d - g.ATZy0[j] * p0 - g.ATZy1[j] * p1) + (1.0 - alpha) * g.ATY[j];
                        g.ATA[j] = d;
                    } else if (op == OP_RESTART) {
                        if (prm.restart_rule == 0) {
                            if (x0 >= s0) s1 = gamma * s0;
                            else x1 = gamma * x0;
                            aty = d;
                        } else {
                            x1 = sg * x0; s1 = sg * s0;
                            aty = sg * d;            // y is scaled by sqrt(gamma) in the row pass
                        }
                    } else {
                        aty = d;
                    }
                    if (op != OP_REFRESH) { g.X[j] = x1; g.S[j] = s1; }
                    g.ATY[j] = aty;
                    const double c0 = g.C[j], cb0 = g.CB[j];
                    const double r1 = aty + s1 - c0 * tau;
                    const double r2 = aty + s1;
                    const double r3 = -aty + c0 * tau - cb0 * theta - s1;
                    cs[0] = fma(c0, x1, cs[0]);
                    cs[1] = fma(cb0, x1, cs[1]);
                    cs[2] = fma(c0, s1, cs[2]);
                    cs[3] = fma(cb0, s1, cs[3]);
                    cs[4] = fma(r1, r1, cs[4]);
                    cs[5] = fma(r2, r2, cs[5]);
                    cs[6] = fma(r3, r3, cs[6]);
                }
            }
        }
        if (op == OP_PROX) {         // y' = alpha (a - Z_y p) + (1 - alpha) y on this workgroup's rows
            for (int i = R.lo + tid; i < R.hi; i += SP_THREADS)
                g.Y[i] = alpha * (g.a[i] - g.Zy0[i] * p0 - g.Zy1[i] * p1) + (1.0 - alpha) * g.Y[i];
        }
        put_parts<7>(cs, g.part, g.nbp, SP_COL, sbuf);
        const bool was_update = (op == OP_PROX);
        const bool bb_pass = bb_on && bb_stage != 0;   // a probe or the restored start: no tests
        if (was_update) { ++iters; ++done; if (bb_pass) ++bbp; }
        int64_t tb = wall_clock64();
        tk[0] += tb - ta;
        grid_sync(g.bar, g.err);
        ta = wall_clock64();
        tk[2] += ta - tb;

        // ---- row pass: A x, A s, A (A^T a); row sums; CG right-hand side and start
        double rs[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        {
            const int L = g.LA, per = SP_THREADS / L;
            for (int i0 = R.lo; i0 < R.hi; i0 += per) {
                const int i = i0 + tid / L, sub = tid % L;
                double ax = 0.0, as = 0.0, aa = 0.0;
                if (i < R.hi) {
                    double o[3];
                    row_sums<3>(g.ci, g.va, g.rp[i], g.rp[i + 1], sub, L,
                                [&](int j, double* fv) { fv[0] = g.X[j]; fv[1] = g.S[j]; fv[2] = g.ATA[j]; }, o);
                    ax = o[0]; as = o[1]; aa = o[2];
                }
                ax = group_sum(ax, L);
                as = group_sum(as, L);
                aa = group_sum(aa, L);
                if (i < R.hi && sub == 0) {
                    double yi = g.Y[i];
                    if (op == OP_RESTART && prm.restart_rule != 0) { yi *= sg; g.Y[i] = yi; }
                    const double bi = g.b[i], bbi = g.bbar[i];
                    const double r1 = ax - bi * tau;
                    const double r3 = r1 + bbi * theta;
                    rs[0] = fma(bi, yi, rs[0]);
                    rs[1] = fma(bbi, yi, rs[1]);
                    rs[2] = fma(r1, r1, rs[2]);
                    rs[3] = fma(ax, ax, rs[3]);
                    rs[4] = fma(r3, r3, rs[4]);
                    // t = y - A (x + s);  r = t - G a = t - a - A (A^T a)
                    const double ti = yi - (ax + as);
                    const double ai = g.a[i];
                    const double ri = ti - ai - aa;
                    SpRow* o = g.rw + i;
                    o->r = ri; o->w = 0.0; o->s = 0.0;
                    g.z[i] = 0.0; g.p[i] = 0.0;
                    rs[5] = 0.0;
                    rs[6] = fma(ri, ri, rs[6]);
                    rs[7] = fma(ti, ti, rs[7]);
                    rs[8] = fma(bi, ai, rs[8]);
                    rs[9] = fma(bbi, ai, rs[9]);
                    rs[10] = fma(g.Ac[i], ai, rs[10]);
                    rs[11] = fma(g.Acb[i], ai, rs[11]);
                }
            }
        }
        put_parts<12>(rs, g.part, g.nbp, SP_ROW, sbuf);
        tb = wall_clock64();
        tk[1] += tb - ta;
        grid_sync(g.bar, g.err);
        ta = wall_clock64();
        tk[2] += ta - tb;
        double tcr[19];                 // SP_COL and SP_ROW are adjacent: one reduction
        get_parts<19>(g.part, g.nbp, SP_COL, tcr, sbuf);
        const double* tc = tcr;
        const double* tr = tcr + 7;
        tk[3] += wall_clock64() - ta;
        const double cx = tc[0], cbx = tc[1], by = tr[0], bby = tr[1];

        if (g.fixed_iters > 0) {
            if (done >= g.fixed_iters) break;
        } else {
            const bool post_update = was_update || (op == OP_REFRESH && !first) || (first && check_final_first);
            first = false;
            if (post_update && !bb_pass) {
                // Section 4.1, multiplied through by tau and squared
                int st = 0;
                if (tau > 0.0) {
                    const double ep = eps * (1.0 + nb) * tau, ed = eps * (1.0 + nc) * tau;
                    if (tr[2] <= ep * ep && tc[4] <= ed * ed && fabs(cx - by) <= eps * (tau + fabs(cx) + fabs(by)))
                        st = 1;
                }
                if (!st && nb > 0.0 && by > 0.0 && tc[5] * (nb * nb) <= (eps * by) * (eps * by)) st = 2;
                if (!st && nc > 0.0 && cx < 0.0 && tr[3] * (nc * nc) <= (eps * cx) * (eps * cx)) st = 3;
                l_ms2 = tr[2]; l_cs4 = tc[4]; l_tau = tau; l_by = by; l_cx = cx; l_have = true;
                if (st) { status = st; break; }
            }
            if (!bb_pass) {
                // inner test ||Q u - v||^2 <= mu (eq. inner-stop)
                const double rt = by - cx + zbar * theta - kappa;
                const double rth = -bby + cbx - zbar * tau + np1;
                const double inner = tr[4] + tc[6] + rt * rt + rth * rth;
                if (inner <= mu) {
                    mu *= gamma;
                    ++ipm;
                    if (prm.restart_rule == 0) {
                        if (tau >= kappa) kappa *= gamma;
                        else tau *= gamma;
                    } else {
                        tau *= sg; kappa *= sg; theta *= sg;
                    }
                    bb_pend = bb_on;             // the new outer iteration chooses its beta
                    op = OP_RESTART;
                    continue;
                }
                // (an outer iteration that starts with a beta choice takes its probes first)
                if (iters >= prm.max_iters && !(bb_on && bb_pend)) { status = 4; break; }
            }
            if (bb_on && (bb_pend || bb_pass)) {
                // ---- a step of the beta choice (Section 4.3) on this workgroup's rows
                // and columns: keep the start point, keep the first probe, or form the
                // estimate's sums over the whole LP, choose and restore the start point
                const int prev = bb_stage;
                if (!bb_pass) bb_pend = false;
                if (bb_stage == 0) {
                    for (int i = R.lo + tid; i < R.hi; i += SP_THREADS) g.Y0[i] = g.Y[i];
                    for (int j = Cc.lo + tid; j < Cc.hi; j += SP_THREADS) { g.X0[j] = g.X[j]; g.S0[j] = g.S[j]; }
                    bbs[0] = tau; bbs[1] = kappa; bbs[2] = theta;
                    bb_stage = 1;
                } else if (bb_stage == 1 && was_update) {
                    for (int i = R.lo + tid; i < R.hi; i += SP_THREADS) g.Y1[i] = g.Y[i];
                    for (int j = Cc.lo + tid; j < Cc.hi; j += SP_THREADS) { g.X1[j] = g.X[j]; g.S1[j] = g.S[j]; }
                    bbs[3] = tau; bbs[4] = kappa; bbs[5] = theta;
                    bb_stage = 2;
                } else if (bb_stage == 2) {
                    double q[5] = {0, 0, 0, 0, 0};
                    for (int i = R.lo + tid; i < R.hi; i += SP_THREADS) bb_acc(g.Y[i] - g.Y1[i], 0.0, 0.0, alpha, q);
                    for (int j = Cc.lo + tid; j < Cc.hi; j += SP_THREADS)
                        bb_acc(g.X[j] - g.X1[j], g.S[j] - g.S1[j], g.S1[j] - g.S0[j], alpha, q);
                    put_parts<5>(q, g.part, g.nbp, SP_BB, sbuf);
                    grid_sync(g.bar, g.err);
                    get_parts<5>(g.part, g.nbp, SP_BB, q, sbuf);
                    bb_acc(tau - bbs[3], kappa - bbs[4], bbs[4] - bbs[1], alpha, q);
                    bb_acc(theta - bbs[5], 0.0, 0.0, alpha, q);
                    ++bbe;
                    ++bb_est;
                    const double hat = bb_hat(q, beta, prm.eps_cor);
                    const bool fin = bb_choose(beta, hat, prm.eps_pen, bb_est, prm.bb_max_redo);
                    for (int i = R.lo + tid; i < R.hi; i += SP_THREADS) g.Y[i] = g.Y0[i];
                    for (int j = Cc.lo + tid; j < Cc.hi; j += SP_THREADS) { g.X[j] = g.X0[j]; g.S[j] = g.S0[j]; }
                    tau = bbs[0]; kappa = bbs[1]; theta = bbs[2];
                    bb_stage = fin ? 3 : 1;
                    grid_sync(g.bar, g.err);     // every row of the restored y before the next column pass
                    if (grid_failed(g.err)) { status = -1; break; }
                    op = OP_REFRESH;             // the products of the restored point
                    continue;
                } else if (bb_stage == 3) {
                    bb_stage = 0;
                    bb_est = 0;
                }
                if (prev == 3 && iters >= prm.max_iters) { status = 4; break; }
            }
        }

        // ---- the linear step: G a = t by CG from the previous a
        // stop at ||r|| <= max(cg_tol ||t||, 0.1 ||Q u - v|| / (1 + k)) (rule 0) or at the
        // relative floor alone (rule 1)
        double tol2 = g.cg_tol * g.cg_tol * tr[7];
        if (g.cg_rule == 0) {           // also in fixed-update runs, so they time a solve's CG work
            const double rt = by - cx + zbar * theta - kappa;
            const double rth = -bby + cbx - zbar * tau + np1;
            const double inner = tr[4] + tc[6] + rt * rt + rth * rth;
            const double sched = 0.01 * inner / ((1.0 + (double)iters) * (1.0 + (double)iters));
            tol2 = fmax(tol2, sched);
        }
        double bd[4] = {tr[8], tr[9], tr[10], tr[11]};
        cgit += cg_loop(g, L, tr[6], tol2, bd, sbuf, g.cg_max, tk);
        if (grid_failed(g.err)) { status = -1; break; }
        // ---- border (Section 4.4, rank 2) and the tau / kappa / theta update
        const double cs_f = cx + tc[2];
        const double cbs_f = cbx + tc[3];
        const double h1z = -bd[0] + cs_f + bd[2];      // c^T d = c^T f + (A c)^T a
        const double h2z = bd[1] - cbs_f - bd[3];
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
        op = OP_PROX;
    }

    if (blockIdx.x == 0 && tid == 0) {
        LPCtrl& o = *g.lc;
        if (l_have && l_tau > 0.0) {
            o.pobj = l_cx / l_tau;
            o.dobj = l_by / l_tau;
            o.pres = sqrt(l_ms2) / l_tau / (1.0 + nb);
            o.dres = sqrt(l_cs4) / l_tau / (1.0 + nc);
            o.gap = fabs(o.pobj - o.dobj) / (1.0 + fabs(o.pobj) + fabs(o.dobj));
        }
        o.by = l_by; o.cx = l_cx;
        o.tau = tau; o.kappa = kappa; o.theta = theta; o.mu = mu;
        o.iters = iters; o.iters64 = iters; o.ipm = ipm; o.cg = cgit;
        o.cp64 += done;
        o.status = (status < 0) ? 0 : status;
        o.phase = 1;
        o.mode = OP_REFRESH;
        o.flags = ((g.fixed_iters > 0) ? 1 : 0) | (cl.flags & 4) | (bb_pend ? 16 : 0);
        if (bb_on) { o.beta = beta; o.bbp = bbp; o.bbe = bbe; }
        o.clk[2] += wall_clock64() - t_start;
        o.clk[0] += tk[0]; o.clk[1] += tk[1]; o.clk[3] += tk[2]; o.clk[4] += tk[3];
    }
}

// CG for a right-hand side given at setup (the border columns Z).
__global__ __launch_bounds__(SP_THREADS) void k_sp_cg(SpArgs g, const double* rhs, double tol, int32_t maxit,
                                                     int64_t* iters) {
    __shared__ double sbuf[64];
    extern __shared__ __align__(16) unsigned char sp_lds[];
    const Range R = my_range(g.m), Cc = my_range(g.n);
    const SpLds L = sp_lds_init(g, R, Cc, sp_lds);
    double v[2] = {0, 0};
    for (int i = R.lo + threadIdx.x; i < R.hi; i += SP_THREADS) {
        const double ri = rhs[i];
        SpRow* o = g.rw + i;
        o->r = ri; o->w = 0.0; o->s = 0.0;
        g.a[i] = 0.0; g.z[i] = 0.0; g.p[i] = 0.0;
        v[0] = fma(ri, ri, v[0]);
    }
    v[1] = v[0];
    put_parts<2>(v, g.part, g.nbp, SP_CG, sbuf);
    grid_sync(g.bar, g.err);
    double t[2];
    get_parts<2>(g.part, g.nbp, SP_CG, t, sbuf);
    double bd[4];
    int64_t tk[4] = {0, 0, 0, 0};
    const int k = cg_loop(g, L, t[0], tol * tol * t[1], bd, sbuf, maxit, tk);
    if (blockIdx.x == 0 && threadIdx.x == 0) *iters = k;
}

// ---------------------------------------------------------------------------
// setup kernels
// ---------------------------------------------------------------------------
// flag bits: 1 row pointers, 2 column index out of range, 4 non-finite value
__global__ void k_sp_check_rows(const int32_t* rp, int32_t m, int64_t nnz, int* flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && (rp[0] != 0 || (int64_t)rp[m] != nnz)) atomicOr(flag, 1);
    if (i < m && rp[i] > rp[i + 1]) atomicOr(flag, 1);
}
__global__ void k_sp_check_entries(const int32_t* ci, const double* va, int64_t nnz, int32_t n, int* flag) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < nnz) {
        const int j = ci[e];
        if (j < 0 || j >= n) atomicOr(flag, 2);
        if (!isfinite(va[e])) atomicOr(flag, 4);
    }
}

// row pointers first (flag bit 1); the entries only once those are known good
hipError_t sp_validate_rows(const SpArgs& g, int* flag, hipStream_t st) {
    hipLaunchKernelGGL(k_sp_check_rows, dim3((g.m + 255) / 256), dim3(256), 0, st, g.rp, g.m, g.nnz, flag);
    return hipGetLastError();
}
hipError_t sp_validate_entries(const SpArgs& g, int* flag, hipStream_t st) {
    if (g.nnz > 0)
        hipLaunchKernelGGL(k_sp_check_entries, dim3((unsigned)((g.nnz + 255) / 256)), dim3(256), 0, st, g.ci, g.va,
                           g.nnz, g.n, flag);
    return hipGetLastError();
}
__global__ void k_sp_finite(const double* v, int64_t len, int* flag, int bit) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len && !isfinite(v[i])) atomicOr(flag, bit);
}
hipError_t sp_check_finite(const double* v, int64_t len, int* flag, int bit, hipStream_t st) {
    hipLaunchKernelGGL(k_sp_finite, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, st, v, len, flag, bit);
    return hipGetLastError();
}
// out[i] = a x[i] + c (elementwise)
__global__ void k_sp_affine(const double* x, double a, double c, int64_t len, double* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) out[i] = a * x[i] + c;
}
hipError_t sp_affine(const double* x, double a, double c, int64_t len, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_sp_affine, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, st, x, a, c, len, out);
    return hipGetLastError();
}

// CSR(A^T) from CSR(A): column counts, exclusive scan, scatter, then each
// column's entries sorted by row index (deterministic layout).
__global__ void k_sp_count(const int32_t* ci, int64_t nnz, int32_t* cnt) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < nnz) atomicAdd(&cnt[ci[e]], 1);
}
// exclusive scan of cnt[0..n) into rpt[0..n] by one workgroup of 1024 threads
__global__ __launch_bounds__(1024) void k_sp_scan(const int32_t* cnt, int32_t n, int32_t* rpt) {
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int per = (n + 1023) / 1024;
    const int lo = min(n, t * per), hi = min(n, lo + per);
    int64_t s = 0;
    for (int j = lo; j < hi; ++j) s += cnt[j];
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        int64_t run = 0;
        for (int k = 0; k < 1024; ++k) { const int64_t v = part[k]; part[k] = run; run += v; }
        rpt[n] = (int32_t)run;
    }
    __syncthreads();
    int64_t run = part[t];
    for (int j = lo; j < hi; ++j) { rpt[j] = (int32_t)run; run += cnt[j]; }
}
__global__ void k_sp_scatter(const int32_t* rp, const int32_t* ci, const double* va, int32_t m, int32_t* cursor,
                             int32_t* cit, double* vat) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
        const int pos = atomicAdd(&cursor[ci[e]], 1);
        cit[pos] = i;
        vat[pos] = va[e];
    }
}
__global__ void k_sp_sortseg(const int32_t* rpt, int32_t n, int32_t* cit, double* vat) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int lo = rpt[j], hi = rpt[j + 1];
    for (int e = lo + 1; e < hi; ++e) {          // insertion sort by row index
        const int key = cit[e];
        const double val = vat[e];
        int f = e - 1;
        while (f >= lo && (cit[f] > key || (cit[f] == key && vat[f] > val))) {
            cit[f + 1] = cit[f];
            vat[f + 1] = vat[f];
            --f;
        }
        cit[f + 1] = key;
        vat[f + 1] = val;
    }
}

hipError_t sp_transpose(SpArgs& g, int32_t* rpt, int32_t* cit, double* vat, int32_t* cursor, hipStream_t st) {
    hipError_t e;
    if ((e = hipMemsetAsync(cursor, 0, sizeof(int32_t) * (size_t)g.n, st)) != hipSuccess) return e;
    if (g.nnz > 0)
        hipLaunchKernelGGL(k_sp_count, dim3((unsigned)((g.nnz + 255) / 256)), dim3(256), 0, st, g.ci, g.nnz, cursor);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_sp_scan, dim3(1), dim3(1024), 0, st, cursor, g.n, rpt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(cursor, rpt, sizeof(int32_t) * (size_t)g.n, hipMemcpyDeviceToDevice, st)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_sp_scatter, dim3((g.m + 255) / 256), dim3(256), 0, st, g.rp, g.ci, g.va, g.m, cursor, cit, vat);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_sp_sortseg, dim3((g.n + 255) / 256), dim3(256), 0, st, rpt, g.n, cit, vat);
    return hipGetLastError();
}

// out = alpha * (M v) + beta * w for a CSR matrix M with `rows` rows (w may be null)
__global__ void k_sp_spmv(const int32_t* rp, const int32_t* ci, const double* va, int32_t rows, const double* v,
                          double alpha, const double* w, double beta, double* out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    double s = 0.0;
    for (int e = rp[i]; e < rp[i + 1]; ++e) s = fma(va[e], v[ci[e]], s);
    out[i] = alpha * s + (w ? beta * w[i] : 0.0);
}
hipError_t sp_spmv(const int32_t* rp, const int32_t* ci, const double* va, int32_t rows, const double* v,
                   double alpha, const double* w, double beta, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_sp_spmv, dim3((rows + 255) / 256), dim3(256), 0, st, rp, ci, va, rows, v, alpha, w, beta, out);
    return hipGetLastError();
}

// diag(G)_i = 1 + ||A_{i,:}||^2, and the CG record of row i (1 / diag(G)_i, r = w = s = 0)
__global__ void k_sp_rowsq(const int32_t* rp, const double* va, int32_t m, double* dG, SpRow* rw) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    double s = 1.0;
    for (int e = rp[i]; e < rp[i + 1]; ++e) s = fma(va[e], va[e], s);
    dG[i] = s;
    rw[i] = SpRow{0.0, 0.0, 0.0, 1.0 / s};
}
hipError_t sp_rowsq(const SpArgs& g, double* dG, hipStream_t st) {
    hipLaunchKernelGGL(k_sp_rowsq, dim3((g.m + 255) / 256), dim3(256), 0, st, g.rp, g.va, g.m, dG, g.rw);
    return hipGetLastError();
}

// partial dot products x . ys[k] per block (nblk blocks, fixed order inside);
// partial[k * nblk + blk]; the host adds the blocks in order
__global__ void k_sp_dots(const double* x, const double* const* ys, int ny, int64_t len, double* partial) {
    __shared__ double sb[8 * 4];
    for (int k = 0; k < ny; ++k) {
        double v[1] = {0.0};
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x)
            v[0] = fma(x[i], ys[k][i], v[0]);
        block_sum_n<1>(v, sb);
        if (threadIdx.x == 0) partial[(int64_t)k * gridDim.x + blockIdx.x] = v[0];
    }
}
hipError_t sp_dots(const double* x, const double* const* ys, int ny, int64_t len, double* partial, int nblk,
                   hipStream_t st) {
    hipLaunchKernelGGL(k_sp_dots, dim3(nblk), dim3(256), 0, st, x, ys, ny, len, partial);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// G~ = A A^T in CSR.  Row i: for every entry (i, k) of A and every entry (j, k)
// of row k of CSR(A^T), the product a_ik a_jk at column j.  One workgroup per
// row gathers the products with keys (j, k) into LDS in a fixed order (entries
// of row i in order, each with its column's entries in order), sorts them by
// key (bitonic), and either counts the distinct j (k_sp_gcount) or writes each
// j once with the sum of its products in k order (k_sp_gfill).  A row with
// more than SP_GCAND products reports -1 (the engine then keeps the two
// products per CG iteration).
// ---------------------------------------------------------------------------
#define SP_GCAND 2048
__device__ int sp_gram_gather(const SpArgs& g, int i, unsigned long long* key, double* val) {
    const int eb = g.rp[i], ee = g.rp[i + 1];
    int base = 0;
    for (int e = eb; e < ee; ++e) {
        const int k = g.ci[e];
        const double aik = g.va[e];
        const int fb = g.rpt[k], cnt = g.rpt[k + 1] - fb;
        if (base + cnt > SP_GCAND) return -1;
        for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
            key[base + t] = ((unsigned long long)(unsigned)g.cit[fb + t] << 32) | (unsigned)k;
            val[base + t] = aik * g.vat[fb + t];
        }
        base += cnt;
    }
    // pad to a power of two with keys past every real one, then sort
    int P = 1;
    while (P < base) P <<= 1;
    for (int t = base + threadIdx.x; t < P; t += blockDim.x) { key[t] = ~0ull; val[t] = 0.0; }
    __syncthreads();
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < P; t += blockDim.x) {
                const int u = t ^ stride;
                if (u > t) {
                    const bool up = (t & size) == 0;
                    const unsigned long long ka = key[t], kb = key[u];
                    if ((ka > kb) == up) {
                        key[t] = kb; key[u] = ka;
                        const double va = val[t];
                        val[t] = val[u]; val[u] = va;
                    }
                }
            }
            __syncthreads();
        }
    }
    return base;
}

__global__ __launch_bounds__(256) void k_sp_gcount(SpArgs g, int32_t* cnt) {
    __shared__ unsigned long long key[SP_GCAND];
    __shared__ double val[SP_GCAND];
    __shared__ int sred[4];
    const int i = blockIdx.x;
    const int nc = sp_gram_gather(g, i, key, val);
    if (nc < 0) {
        if (threadIdx.x == 0) cnt[i] = -1;
        return;
    }
    int c = 0;
    for (int t = threadIdx.x; t < nc; t += blockDim.x)
        c += (t == 0 || (key[t] >> 32) != (key[t - 1] >> 32)) ? 1 : 0;
    for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off);
    if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) cnt[i] = sred[0] + sred[1] + sred[2] + sred[3];
}

__global__ __launch_bounds__(256) void k_sp_gfill(SpArgs g, const int32_t* grp, int32_t* gci, double* gva) {
    __shared__ unsigned long long key[SP_GCAND];
    __shared__ double val[SP_GCAND];
    __shared__ int rank[SP_GCAND];
    __shared__ int scan[256];
    const int i = blockIdx.x;
    const int nc = sp_gram_gather(g, i, key, val);
    if (nc <= 0) return;
    // rank of each distinct column: exclusive scan of the segment-start flags,
    // eight consecutive positions per thread
    const int tid = threadIdx.x;
    int loc = 0;
    for (int q = 0; q < 8; ++q) {
        const int t = tid * 8 + q;
        if (t < nc && (t == 0 || (key[t] >> 32) != (key[t - 1] >> 32))) ++loc;
    }
    scan[tid] = loc;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int v = (tid >= off) ? scan[tid - off] : 0;
        __syncthreads();
        scan[tid] += v;
        __syncthreads();
    }
    int run = scan[tid] - loc;
    for (int q = 0; q < 8; ++q) {
        const int t = tid * 8 + q;
        if (t < nc && (t == 0 || (key[t] >> 32) != (key[t - 1] >> 32))) rank[t] = run++;
    }
    __syncthreads();
    const int64_t o = grp[i];
    for (int t = tid; t < nc; t += blockDim.x) {
        if (t == 0 || (key[t] >> 32) != (key[t - 1] >> 32)) {
            const unsigned j = (unsigned)(key[t] >> 32);
            double sum = 0.0;
            for (int u = t; u < nc && (unsigned)(key[u] >> 32) == j; ++u) sum += val[u];
            gci[o + rank[t]] = (int32_t)j;
            gva[o + rank[t]] = sum;
        }
    }
}

hipError_t sp_gram_count(const SpArgs& g, int32_t* cnt, hipStream_t st) {
    hipLaunchKernelGGL(k_sp_gcount, dim3(g.m), dim3(256), 0, st, g, cnt);
    return hipGetLastError();
}
hipError_t sp_gram_fill(const SpArgs& g, const int32_t* grp, int32_t* gci, double* gva, hipStream_t st) {
    hipLaunchKernelGGL(k_sp_gfill, dim3(g.m), dim3(256), 0, st, g, grp, gci, gva);
    return hipGetLastError();
}
hipError_t sp_scan(const int32_t* cnt, int32_t n, int32_t* ptr, hipStream_t st) {
    hipLaunchKernelGGL(k_sp_scan, dim3(1), dim3(1024), 0, st, cnt, n, ptr);
    return hipGetLastError();
}

// Co-resident workgroups of the cooperative kernels with `lds_bytes` of dynamic LDS.
int sp_max_blocks(int cu_count, int lds_bytes) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_sp_solve, SP_THREADS, lds_bytes) !=
            hipSuccess || per_cu < 1)
        per_cu = 1;
    int per_cu2 = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu2, (const void*)k_sp_cg, SP_THREADS, lds_bytes) ==
            hipSuccess && per_cu2 >= 1)
        per_cu = std::min(per_cu, per_cu2);
    return per_cu * cu_count;
}

hipError_t sp_set_lds_limit(int bytes) {
    hipError_t e = hipFuncSetAttribute((const void*)k_sp_solve, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_sp_cg, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

hipError_t sp_cg_solve(SpArgs g, const double* rhs, double* out, double tol, int32_t maxit, int nb,
                       int64_t* iters, hipStream_t st) {
    void* args[] = {(void*)&g, (void*)&rhs, (void*)&tol, (void*)&maxit, (void*)&iters};
    hipError_t e = hipLaunchCooperativeKernel((const void*)k_sp_cg, dim3(nb), dim3(SP_THREADS), args,
                                              (size_t)g.lds_bytes, st);
    if (e != hipSuccess) return e;
    return hipMemcpyAsync(out, g.a, sizeof(double) * (size_t)g.m, hipMemcpyDeviceToDevice, st);
}

hipError_t sp_solve(SpArgs g, int nb, hipStream_t st) {
    void* args[] = {(void*)&g};
    return hipLaunchCooperativeKernel((const void*)k_sp_solve, dim3(nb), dim3(SP_THREADS), args,
                                      (size_t)g.lds_bytes, st);
}
