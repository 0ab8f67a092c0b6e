// Setup kernels: data copies, HSD constants, the cached factorization of
// G = I + A A^T and the border of the Schur reduction of I + Q.
//
// Every kernel takes the LP index from blockIdx.y (or blockIdx.x when one
// workgroup owns one LP) and reads its layout from LPDesc, so a whole batch of
// uneven LPs is set up with one launch per step.
#include <hip/hip_runtime.h>
#include "abip_internal.h"

// ---------------------------------------------------------------------------
// A (row-major FP64, caller's buffer) -> column-major A64 / A32 with padded
// leading dimension; flags non-finite entries.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_setup_copy(const LPDesc* __restrict__ desc,
                                                    const double* const* __restrict__ Auser,
                                                    double* __restrict__ A64, float* __restrict__ A32,
                                                    int* __restrict__ errflag) {
    const int k = blockIdx.y;
    const LPDesc d = desc[k];
    const int tr = (d.m + 63) / 64, tc = (d.n + 63) / 64;
    const int tile = blockIdx.x;
    if (tile >= tr * tc) return;
    const int ti = tile / tc, tj = tile % tc;
    __shared__ double T[64][65];
    const double* A = Auser[k];
    int bad = 0;
    for (int e = threadIdx.x; e < 4096; e += blockDim.x) {
        const int r = e >> 6, c = e & 63;
        const int i = ti * 64 + r, j = tj * 64 + c;
        double v = 0.0;
        if (i < d.m && j < d.n) {
            v = A[(int64_t)i * d.n + j];
            if (!isfinite(v)) bad = 1;
        }
        T[r][c] = v;
    }
    if (bad) atomicOr(errflag, 1);
    __syncthreads();
    for (int e = threadIdx.x; e < 4096; e += blockDim.x) {
        const int c = e >> 6, r = e & 63;
        const int i = ti * 64 + r, j = tj * 64 + c;
        if (i < d.m && j < d.n) {
            const double v = T[r][c];
            A64[d.oA + (int64_t)j * d.ld + i] = v;
            A32[d.oA + (int64_t)j * d.ld + i] = (float)v;
        }
    }
}

// ---------------------------------------------------------------------------
// Ruiz equilibration (the scaling that Section 4.5's remark adds after the
// presolve): rounds of D_i *= 1/sqrt(max_j |(D_i a_ij) E_j|),
// E_j *= 1/sqrt(max_i |(D_i a_ij) E_j|), both maxima taken from the same
// matrix (a zero row or column keeps its factor); then A <- (D_i a_ij) E_j.
// A64 keeps the original entries until the last kernel.  The maxima of a round
// are kept as the bit patterns of non-negative doubles (ordered like their
// values) in the m / n scratch fields rmax / cmax, which start at 0.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_ruiz_init(const LPDesc* __restrict__ desc, double* __restrict__ Mv,
                                                   double* __restrict__ Nv, int64_t Mtot, int64_t Ntot) {
    const LPDesc d = desc[blockIdx.y];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < d.ld; i += gridDim.x * blockDim.x)
        Mv[MF_SD * Mtot + d.om + i] = 1.0;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < d.n; j += gridDim.x * blockDim.x)
        Nv[NF_SE * Ntot + d.on + j] = 1.0;
}

// Row and column maxima of one 64 x 64 tile (grid: tiles, B).
__global__ __launch_bounds__(256) void k_ruiz_max(const LPDesc* __restrict__ desc, const double* __restrict__ A64,
                                                  double* __restrict__ Mv, double* __restrict__ Nv, int64_t Mtot,
                                                  int64_t Ntot) {
    const int k = blockIdx.y;
    const LPDesc d = desc[k];
    const int tr = (d.m + 63) / 64, tc = (d.n + 63) / 64;
    const int tile = blockIdx.x;
    if (tile >= tr * tc) return;
    const int ti = tile / tc, tj = tile % tc;
    __shared__ double rm[4][64], cm[4][64];
    const double* Dv = Mv + MF_SD * Mtot + d.om;
    const double* Ev = Nv + NF_SE * Ntot + d.on;
    unsigned long long* rmax = reinterpret_cast<unsigned long long*>(Mv + MF_BBY0 * Mtot + d.om);
    unsigned long long* cmax = reinterpret_cast<unsigned long long*>(Nv + NF_BBX0 * Ntot + d.on);
    // thread (r = tid & 63, q = tid >> 6): row ti*64 + r (lanes down a column,
    // coalesced), columns q, q+4, ... of the tile
    const int r = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int i = ti * 64 + r;
    const double di = (i < d.m) ? Dv[i] : 0.0;
    double rowm = 0.0;
    for (int c = q; c < 64; c += 4) {
        const int j = tj * 64 + c;
        double v = 0.0;
        if (i < d.m && j < d.n) v = fabs((di * A64[d.oA + (int64_t)j * d.ld + i]) * Ev[j]);
        rowm = fmax(rowm, v);
        // column maxima: this wave's 64 rows of column c
        double cv = v;
        for (int off = 32; off >= 1; off >>= 1) cv = fmax(cv, __shfl_xor(cv, off));
        if (r == 0) cm[q][c >> 2] = cv;
    }
    rm[q][r] = rowm;
    __syncthreads();
    if (threadIdx.x < 64) {
        const int ii = ti * 64 + threadIdx.x;
        const double v = fmax(fmax(rm[0][threadIdx.x], rm[1][threadIdx.x]), fmax(rm[2][threadIdx.x], rm[3][threadIdx.x]));
        if (ii < d.m && v > 0.0) atomicMax(rmax + ii, (unsigned long long)__double_as_longlong(v));
    } else if (threadIdx.x < 128) {
        const int c = threadIdx.x - 64;
        const int j = tj * 64 + c;
        const double v = cm[c & 3][c >> 2];
        if (j < d.n && v > 0.0) atomicMax(cmax + j, (unsigned long long)__double_as_longlong(v));
    }
}

// Apply a round's maxima to D and E and clear them for the next round.
__global__ __launch_bounds__(256) void k_ruiz_apply(const LPDesc* __restrict__ desc, double* __restrict__ Mv,
                                                    double* __restrict__ Nv, int64_t Mtot, int64_t Ntot) {
    const LPDesc d = desc[blockIdx.y];
    double* Dv = Mv + MF_SD * Mtot + d.om;
    double* Ev = Nv + NF_SE * Ntot + d.on;
    unsigned long long* rmax = reinterpret_cast<unsigned long long*>(Mv + MF_BBY0 * Mtot + d.om);
    unsigned long long* cmax = reinterpret_cast<unsigned long long*>(Nv + NF_BBX0 * Ntot + d.on);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < d.m; i += gridDim.x * blockDim.x) {
        const double v = __longlong_as_double((long long)rmax[i]);
        if (v > 0.0) Dv[i] = Dv[i] * (1.0 / sqrt(v));
        rmax[i] = 0ull;
    }
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < d.n; j += gridDim.x * blockDim.x) {
        const double v = __longlong_as_double((long long)cmax[j]);
        if (v > 0.0) Ev[j] = Ev[j] * (1.0 / sqrt(v));
        cmax[j] = 0ull;
    }
}

// A <- (D_i a_ij) E_j in both precisions (grid: tiles, B).
__global__ __launch_bounds__(256) void k_ruiz_scale(const LPDesc* __restrict__ desc, double* __restrict__ A64,
                                                    float* __restrict__ A32, const double* __restrict__ Mv,
                                                    const double* __restrict__ Nv, int64_t Mtot, int64_t Ntot) {
    const LPDesc d = desc[blockIdx.y];
    const int tr = (d.m + 63) / 64, tc = (d.n + 63) / 64;
    const int tile = blockIdx.x;
    if (tile >= tr * tc) return;
    const int ti = tile / tc, tj = tile % tc;
    const double* Dv = Mv + MF_SD * Mtot + d.om;
    const double* Ev = Nv + NF_SE * Ntot + d.on;
    for (int e = threadIdx.x; e < 4096; e += blockDim.x) {
        const int i = ti * 64 + (e & 63), j = tj * 64 + (e >> 6);
        if (i < d.m && j < d.n) {
            const int64_t o = d.oA + (int64_t)j * d.ld + i;
            const double v = (Dv[i] * A64[o]) * Ev[j];
            A64[o] = v;
            A32[o] = (float)v;
        }
    }
}

// ---------------------------------------------------------------------------
// Per-row products with the column-major copy: bbar = b - A e, Ac = A c,
// Acbar = A cbar (eq. bar-b-c-z-re and the border dot trick); copies b, c,
// cbar into the vector pools.  Grid: (row blocks of 256, B).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_setup_rows(const LPDesc* __restrict__ desc,
                                                    const double* const* __restrict__ buser,
                                                    const double* const* __restrict__ cuser,
                                                    const double* __restrict__ A64,
                                                    double* __restrict__ Mv, double* __restrict__ Nv,
                                                    int64_t Mtot, int64_t Ntot, int* __restrict__ errflag,
                                                    int rows) {
    const int k = blockIdx.y;
    const LPDesc d = desc[k];
    const double* A = A64 + d.oA;
    const double* b = buser[k];
    const double* c = cuser[k];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    // copies of c and cbar: spread over the row blocks
    // (the LP's scaled c: E_j c_j, with E = 1 when it is not scaled)
    const double* Ev = Nv + NF_SE * Ntot + d.on;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < d.n; j += gridDim.x * blockDim.x) {
        if (!isfinite(c[j])) atomicOr(errflag, 2);
        const double cj = Ev[j] * c[j];
        Nv[NF_C * Ntot + d.on + j] = cj;
        Nv[NF_CBAR * Ntot + d.on + j] = cj - 1.0;
    }
    if (!rows || i >= d.ld) return;      // rows == 0: k_setup_rows_part / _fin form them
    if (i >= d.m) {   // zero padding rows of every m-field
        for (int f = 0; f < NMF; ++f) Mv[f * Mtot + d.om + i] = 0.0;
        return;
    }
    double se = 0.0, sc = 0.0, scb = 0.0;
    for (int j = 0; j < d.n; ++j) {
        const double a = A[(int64_t)j * d.ld + i];
        const double cj = Ev[j] * c[j];
        se += a;
        sc = fma(a, cj, sc);
        scb = fma(a, cj - 1.0, scb);
    }
    if (!isfinite(b[i])) atomicOr(errflag, 2);
    const double bi = Mv[MF_SD * Mtot + d.om + i] * b[i];
    Mv[MF_B * Mtot + d.om + i] = bi;
    Mv[MF_BBAR * Mtot + d.om + i] = bi - se;
    Mv[MF_AC * Mtot + d.om + i] = sc;
    Mv[MF_ACBAR * Mtot + d.om + i] = scb;
}

// One large LP (LP 0): the row sums of k_setup_rows (A e, A c, A cbar with the
// scaled c) over column chunks of cw columns, so that every CU takes part:
// P[(3 chunk + q) ld + i], q = 0, 1, 2 for e, c, cbar; k_setup_rows_fin adds
// the chunks of a row in chunk order.
__global__ __launch_bounds__(256) void k_setup_rows_part(const LPDesc* __restrict__ desc,
                                                         const double* const* __restrict__ cuser,
                                                         const double* __restrict__ A64,
                                                         const double* __restrict__ Nv, int64_t Ntot, int cw,
                                                         double* __restrict__ P) {
    const LPDesc d = desc[0];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.m) return;
    const double* A = A64 + d.oA;
    const double* c = cuser[0];
    const double* Ev = Nv + NF_SE * Ntot + d.on;
    const int j0 = blockIdx.y * cw, j1 = min(d.n, j0 + cw);
    double se = 0.0, sc = 0.0, scb = 0.0;
    for (int j = j0; j < j1; ++j) {
        const double a = A[(int64_t)j * d.ld + i];
        const double cj = Ev[j] * c[j];
        se += a;
        sc = fma(a, cj, sc);
        scb = fma(a, cj - 1.0, scb);
    }
    const int64_t o = (int64_t)3 * blockIdx.y * d.ld + i;
    P[o] = se;
    P[o + d.ld] = sc;
    P[o + 2 * (int64_t)d.ld] = scb;
}

__global__ __launch_bounds__(256) void k_setup_rows_fin(const LPDesc* __restrict__ desc,
                                                        const double* const* __restrict__ buser,
                                                        const double* __restrict__ P, int nch,
                                                        double* __restrict__ Mv, int64_t Mtot,
                                                        int* __restrict__ errflag) {
    const LPDesc d = desc[0];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.ld) return;
    if (i >= d.m) {   // zero padding rows of every m-field
        for (int f = 0; f < NMF; ++f) Mv[f * Mtot + d.om + i] = 0.0;
        return;
    }
    double se = 0.0, sc = 0.0, scb = 0.0;
    for (int ch = 0; ch < nch; ++ch) {
        const int64_t o = (int64_t)3 * ch * d.ld + i;
        se += P[o];
        sc += P[o + d.ld];
        scb += P[o + 2 * (int64_t)d.ld];
    }
    const double* b = buser[0];
    if (!isfinite(b[i])) atomicOr(errflag, 2);
    const double bi = Mv[MF_SD * Mtot + d.om + i] * b[i];
    Mv[MF_B * Mtot + d.om + i] = bi;
    Mv[MF_BBAR * Mtot + d.om + i] = bi - se;
    Mv[MF_AC * Mtot + d.om + i] = sc;
    Mv[MF_ACBAR * Mtot + d.om + i] = scb;
}

// ---------------------------------------------------------------------------
// Border of the Schur reduction (Section 4.4 with the theta column kept).
// sgn = +1: I + Q = [[M, H], [-H^T, I2 + S]] with M = [[I, A], [-A^T, I]],
//   H = [(-b; c), (bbar; -cbar)], S = [[0, zbar], [-zbar, 0]];
//   M^{-1}(e; f) = (a; f + A^T a), a = G^{-1}(e - A f).
// sgn = -1: the same for I - Q = (I + Q)^T, used by the adjoint: A, H, S change
//   sign, G = I + A A^T is unchanged.
// Stores Z = M^{-1} H (two M-solves) and K^{-1}, K = I2 + S + H^T Z, plus zbar,
// ||b||, ||c|| in the LP's control block.  One workgroup per LP (FP64).
// LDS: 2*ld doubles.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(512) void k_setup_border(const LPDesc* __restrict__ desc,
                                                      const double* __restrict__ A64,
                                                      const double* __restrict__ G64,
                                                      double* __restrict__ Mv, double* __restrict__ Nv,
                                                      int64_t Mtot, int64_t Ntot, LPCtrl* __restrict__ ctrl,
                                                      int sgn) {
    extern __shared__ double sm[];
    __shared__ double sbuf[8 * 8];
    const int k = blockIdx.x;
    const LPDesc d = desc[k];
    const int m = d.m, n = d.n, ld = d.ld;
    const double* A = A64 + d.oA;
    const double* G = G64 + d.oG;
    const double* b = Mv + MF_B * Mtot + d.om;
    const double* bbar = Mv + MF_BBAR * Mtot + d.om;
    const double* c = Nv + NF_C * Ntot + d.on;
    const double* cbar = Nv + NF_CBAR * Ntot + d.on;
    const int tid = threadIdx.x, lane = tid & 63, wave = wave_id(), W = num_waves();
    const int fzy = (sgn > 0) ? MF_ZY0 : MF_ZY0A;
    const int fzx = (sgn > 0) ? NF_ZX0 : NF_ZX0A;
    const double sg = (double)sgn;
    double* st = sm;          // t = e - sgn A f
    double* sa = sm + ld;     // a = G^{-1} t

    // norms and zbar
    double v3[3] = {0.0, 0.0, 0.0};
    for (int i = tid; i < m; i += blockDim.x) v3[0] = fma(b[i], b[i], v3[0]);
    for (int j = tid; j < n; j += blockDim.x) { v3[1] = fma(c[j], c[j], v3[1]); v3[2] += c[j]; }
    block_sum_n<3>(v3, sbuf);
    const double nb = sqrt(v3[0]), nc = sqrt(v3[1]), zbar = v3[2] + 1.0;

    for (int h = 0; h < 2; ++h) {
        // column h of sgn*H: h = 0: sgn*(-b; c)   h = 1: sgn*(bbar; -cbar)
        const double* ev = (h == 0) ? b : bbar;
        const double* fv = (h == 0) ? c : cbar;
        const double es = sg * ((h == 0) ? -1.0 : 1.0);
        const double fs = sg * ((h == 0) ? 1.0 : -1.0);
        for (int i = tid; i < ld; i += blockDim.x) {
            double s = 0.0;
            if (i < m) {
                for (int j = 0; j < n; ++j) s = fma(A[(int64_t)j * ld + i], fs * fv[j], s);
                s = es * ev[i] - sg * s;
            }
            st[i] = s;
        }
        __syncthreads();
        for (int i = tid; i < ld; i += blockDim.x) {
            double s = 0.0;
            if (i < m)
                for (int q = 0; q < m; ++q) s = fma(G[(int64_t)q * ld + i], st[q], s);
            sa[i] = s;
            if (i < m) Mv[(fzy + h) * Mtot + d.om + i] = s;
        }
        __syncthreads();
        for (int j = wave; j < n; j += W) {
            double s = 0.0;
            for (int i = lane; i < m; i += 64) s = fma(A[(int64_t)j * ld + i], sa[i], s);
            s = wave_sum(s);
            if (lane == 0) Nv[(fzx + h) * Ntot + d.on + j] = fs * fv[j] + sg * s;
        }
        __syncthreads();
    }
    __threadfence_block();
    __syncthreads();
    // (sgn H)^T Z: entry (r, q) = h_r^T z_q
    const double* zy0 = Mv + fzy * Mtot + d.om;
    const double* zy1 = Mv + (fzy + 1) * Mtot + d.om;
    const double* zx0 = Nv + fzx * Ntot + d.on;
    const double* zx1 = Nv + (fzx + 1) * Ntot + d.on;
    double hz[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = tid; i < m; i += blockDim.x) {
        hz[0] = fma(-b[i], zy0[i], hz[0]);
        hz[1] = fma(-b[i], zy1[i], hz[1]);
        hz[2] = fma(bbar[i], zy0[i], hz[2]);
        hz[3] = fma(bbar[i], zy1[i], hz[3]);
    }
    for (int j = tid; j < n; j += blockDim.x) {
        hz[0] = fma(c[j], zx0[j], hz[0]);
        hz[1] = fma(c[j], zx1[j], hz[1]);
        hz[2] = fma(-cbar[j], zx0[j], hz[2]);
        hz[3] = fma(-cbar[j], zx1[j], hz[3]);
    }
    block_sum_n<4>(hz, sbuf);
    if (tid == 0) {
        const double k00 = 1.0 + sg * hz[0], k01 = sg * zbar + sg * hz[1];
        const double k10 = -sg * zbar + sg * hz[2], k11 = 1.0 + sg * hz[3];
        const double det = k00 * k11 - k01 * k10;
        LPCtrl& C = ctrl[k];
        C.zbar = zbar;
        C.nb = nb;
        C.nc = nc;
        if (sgn > 0) {
            C.K00 = k11 / det; C.K01 = -k01 / det; C.K10 = -k10 / det; C.K11 = k00 / det;
        } else {
            C.KA00 = k11 / det; C.KA01 = -k01 / det; C.KA10 = -k10 / det; C.KA11 = k00 / det;
        }
    }
}
