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
// Per-row products with the column-major copy: bbar = b - A e, Ac = A c,
// Acbar = A cbar (eq. bar-b-c-z-re and the border dot trick); copies b, c,
// cbar into the vector pools.  Grid: (row blocks of 256, B).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_setup_rows(const LPDesc* __restrict__ desc,
                                                    const double* const* __restrict__ buser,
                                                    const double* const* __restrict__ cuser,
                                                    const double* __restrict__ A64,
                                                    double* __restrict__ Mv, double* __restrict__ Nv,
                                                    int64_t Mtot, int64_t Ntot, int* __restrict__ errflag) {
    const int k = blockIdx.y;
    const LPDesc d = desc[k];
    const double* A = A64 + d.oA;
    const double* b = buser[k];
    const double* c = cuser[k];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    // copies of c and cbar: spread over the row blocks
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < d.n; j += gridDim.x * blockDim.x) {
        const double cj = c[j];
        if (!isfinite(cj)) atomicOr(errflag, 2);
        Nv[NF_C * Ntot + d.on + j] = cj;
        Nv[NF_CBAR * Ntot + d.on + j] = cj - 1.0;
    }
    if (i >= d.ld) return;
    if (i >= d.m) {   // zero padding rows of every m-field
        for (int f = 0; f < NMF; ++f) Mv[f * Mtot + d.om + i] = 0.0;
        return;
    }
    double se = 0.0, sc = 0.0, scb = 0.0;
    for (int j = 0; j < d.n; ++j) {
        const double a = A[(int64_t)j * d.ld + i];
        const double cj = c[j];
        se += a;
        sc = fma(a, cj, sc);
        scb = fma(a, cj - 1.0, scb);
    }
    const double bi = b[i];
    if (!isfinite(bi)) atomicOr(errflag, 2);
    Mv[MF_B * Mtot + d.om + i] = bi;
    Mv[MF_BBAR * Mtot + d.om + i] = bi - se;
    Mv[MF_AC * Mtot + d.om + i] = sc;
    Mv[MF_ACBAR * Mtot + d.om + i] = scb;
}

// ---------------------------------------------------------------------------
// G = I + A A^T (FP64).  One 64x64 lower tile per workgroup, 4x4 outputs per
// thread, K-loop over the n columns of A staged through LDS 16 at a time.
// Writes both G[i][j] and G[j][i].
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_syrk(const LPDesc* __restrict__ desc, const double* __restrict__ A64,
                                              double* __restrict__ G64) {
    const int k = blockIdx.y;
    const LPDesc d = desc[k];
    const int nt = (d.m + 63) / 64;
    const int t = blockIdx.x;
    if (t >= nt * (nt + 1) / 2) return;
    int I = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while (I * (I + 1) / 2 > t) --I;
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    const int J = t - I * (I + 1) / 2;
    const double* A = A64 + d.oA;
    double* G = G64 + d.oG;
    __shared__ double As[16][64];
    __shared__ double Bs[16][64];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
    for (int j0 = 0; j0 < d.n; j0 += 16) {
        for (int e = threadIdx.x; e < 1024; e += 256) {
            const int jj = e >> 6, r = e & 63;
            const int j = j0 + jj;
            const int ri = I * 64 + r, rj = J * 64 + r;
            As[jj][r] = (j < d.n && ri < d.ld) ? A[(int64_t)j * d.ld + ri] : 0.0;
            Bs[jj][r] = (j < d.n && rj < d.ld) ? A[(int64_t)j * d.ld + rj] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int jj = 0; jj < 16; ++jj) {
            double a[4], b[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) { a[q] = As[jj][ty * 4 + q]; b[q] = Bs[jj][tx * 4 + q]; }
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[p][q] = fma(a[p], b[q], acc[p][q]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = I * 64 + ty * 4 + p, j = J * 64 + tx * 4 + q;
            if (i < d.m && j < d.m && j <= i) {
                const double v = acc[p][q] + (i == j ? 1.0 : 0.0);
                G[(int64_t)i * d.ld + j] = v;
                G[(int64_t)j * d.ld + i] = v;
            }
        }
}

// ---------------------------------------------------------------------------
// In-place G -> G^{-1} for one LP per workgroup (FP64):
//   blocked right-looking Cholesky G = L L^T (panel 32), W = L^{-1} by blocked
//   forward substitution (the diagonal blocks come from the panel step), and
//   G^{-1} = W^T W.  Writes G^{-1} in full into G64 and its FP32 copy into G32.
// W is an ld x ld scratch per LP (offset oW).
// ---------------------------------------------------------------------------
#define CB 32

__device__ __forceinline__ double gload(const double* M, int ld, int n, int i, int j) {
    return (i < n && j < n) ? M[(int64_t)i * ld + j] : 0.0;
}

__global__ __launch_bounds__(256) void k_chol_inv(const LPDesc* __restrict__ desc, double* __restrict__ G64,
                                                  float* __restrict__ G32, double* __restrict__ Wpool,
                                                  const int64_t* __restrict__ oW, int* __restrict__ errflag) {
    const int k = blockIdx.x;
    const LPDesc d = desc[k];
    const int m = d.m, ld = d.ld;
    double* G = G64 + d.oG;
    double* Wm = Wpool + oW[k];
    const int tid = threadIdx.x;
    __shared__ double D[CB][CB + 1];
    __shared__ double Di[CB][CB + 1];
    __shared__ double P[CB][CB + 1];
    __shared__ double Q[CB][CB + 1];
    const int nb = (m + CB - 1) / CB;
    const int r4 = tid >> 3, c4 = (tid & 7) * 4;   // 32 rows x 8 groups of 4 columns

    for (int kb = 0; kb < nb; ++kb) {
        const int k0 = kb * CB;
        const int w = min(CB, m - k0);
        // (1) diagonal block into LDS
        for (int e = tid; e < CB * CB; e += 256) {
            const int r = e / CB, c = e % CB;
            D[r][c] = (r < w && c < w) ? G[(int64_t)(k0 + r) * ld + k0 + c] : (r == c ? 1.0 : 0.0);
        }
        __syncthreads();
        // (2) unblocked Cholesky of the diagonal block
        for (int p = 0; p < CB; ++p) {
            if (tid == 0) {
                const double v = D[p][p];
                if (!(v > 0.0)) { atomicOr(errflag, 4); D[p][p] = 1.0; }
                else D[p][p] = sqrt(v);
            }
            __syncthreads();
            if (tid > p && tid < CB) D[tid][p] /= D[p][p];
            __syncthreads();
            for (int e = tid; e < CB * CB; e += 256) {
                const int i = e / CB, j = e % CB;
                if (j > p && i >= j) D[i][j] -= D[i][p] * D[j][p];
            }
            __syncthreads();
        }
        // (3) inverse of the lower-triangular diagonal block, column by column
        if (tid < CB) {
            const int j = tid;
            for (int i = 0; i < CB; ++i) Di[i][j] = 0.0;
            Di[j][j] = 1.0 / D[j][j];
            for (int i = j + 1; i < CB; ++i) {
                double s = 0.0;
                for (int p = j; p < i; ++p) s = fma(D[i][p], Di[p][j], s);
                Di[i][j] = -s / D[i][i];
            }
        }
        __syncthreads();
        for (int e = tid; e < CB * CB; e += 256) {
            const int r = e / CB, c = e % CB;
            if (r < w && c < w) {
                G[(int64_t)(k0 + r) * ld + k0 + c] = (c <= r) ? D[r][c] : 0.0;
                Wm[(int64_t)(k0 + r) * ld + k0 + c] = Di[r][c];
            }
        }
        // (4) panel below the diagonal block: L_ik = G_ik L_kk^{-T}
        for (int i = k0 + w + tid; i < m; i += 256) {
            double row[CB];
#pragma unroll
            for (int p = 0; p < CB; ++p) row[p] = (p < w) ? G[(int64_t)i * ld + k0 + p] : 0.0;
#pragma unroll 4
            for (int c = 0; c < w; ++c) {
                double s = 0.0;
                for (int p = 0; p <= c; ++p) s = fma(row[p], Di[c][p], s);
                G[(int64_t)i * ld + k0 + c] = s;
            }
        }
        __syncthreads();
        // (5) trailing update of the lower triangle: G_IJ -= L_I L_J^T
        for (int I = kb + 1; I < nb; ++I) {
            for (int J = kb + 1; J <= I; ++J) {
                for (int e = tid; e < CB * CB; e += 256) {
                    const int r = e / CB, c = e % CB;
                    P[r][c] = (c < w) ? gload(G, ld, m, I * CB + r, k0 + c) : 0.0;
                    Q[r][c] = (c < w) ? gload(G, ld, m, J * CB + r, k0 + c) : 0.0;
                }
                __syncthreads();
                double acc[4] = {0.0, 0.0, 0.0, 0.0};
                for (int p = 0; p < CB; ++p) {
                    const double a = P[r4][p];
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc[q] = fma(a, Q[c4 + q][p], acc[q]);
                }
                const int i = I * CB + r4;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int j = J * CB + c4 + q;
                    if (i < m && j < m && j <= i) G[(int64_t)i * ld + j] -= acc[q];
                }
                __syncthreads();
            }
        }
    }
    __syncthreads();
    // W = L^{-1}: W_IK = -W_II * sum_{J=K}^{I-1} L_IJ W_JK, block column by block column
    for (int K = 0; K < nb; ++K) {
        for (int I = K + 1; I < nb; ++I) {
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
            for (int J = K; J < I; ++J) {
                for (int e = tid; e < CB * CB; e += 256) {
                    const int r = e / CB, c = e % CB;
                    P[r][c] = gload(G, ld, m, I * CB + r, J * CB + c);       // L_IJ
                    Q[r][c] = gload(Wm, ld, m, J * CB + r, K * CB + c);      // W_JK
                }
                __syncthreads();
                for (int p = 0; p < CB; ++p) {
                    const double a = P[r4][p];
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc[q] = fma(a, Q[p][c4 + q], acc[q]);
                }
                __syncthreads();
            }
            for (int e = tid; e < CB * CB; e += 256) {
                const int r = e / CB, c = e % CB;
                P[r][c] = gload(Wm, ld, m, I * CB + r, I * CB + c);          // W_II
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) Q[r4][c4 + q] = acc[q];
            __syncthreads();
            double o[4] = {0.0, 0.0, 0.0, 0.0};
            for (int p = 0; p <= r4; ++p) {
                const double a = P[r4][p];
#pragma unroll
                for (int q = 0; q < 4; ++q) o[q] = fma(a, Q[p][c4 + q], o[q]);
            }
            const int i = I * CB + r4;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int j = K * CB + c4 + q;
                if (i < m && j < m) Wm[(int64_t)i * ld + j] = -o[q];
            }
            __syncthreads();
        }
    }
    // G^{-1} = W^T W: (G^{-1})_IJ = sum_{K >= I} W_KI^T W_KJ, I >= J
    for (int I = 0; I < nb; ++I) {
        for (int J = 0; J <= I; ++J) {
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
            for (int K = I; K < nb; ++K) {
                for (int e = tid; e < CB * CB; e += 256) {
                    const int r = e / CB, c = e % CB;
                    P[r][c] = gload(Wm, ld, m, K * CB + r, I * CB + c);      // W_KI
                    Q[r][c] = gload(Wm, ld, m, K * CB + r, J * CB + c);      // W_KJ
                }
                __syncthreads();
                for (int p = 0; p < CB; ++p) {
                    const double a = P[p][r4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc[q] = fma(a, Q[p][c4 + q], acc[q]);
                }
                __syncthreads();
            }
            const int i = I * CB + r4;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int j = J * CB + c4 + q;
                if (i < m && j < m) {
                    G[(int64_t)i * ld + j] = acc[q];
                    G[(int64_t)j * ld + i] = acc[q];
                    G32[d.oG + (int64_t)i * ld + j] = (float)acc[q];
                    G32[d.oG + (int64_t)j * ld + i] = (float)acc[q];
                }
            }
        }
    }
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
