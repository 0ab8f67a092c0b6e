// Border of the Schur reduction for one large dense LP (the grid engine's
// case): Z = M^{-1} H (Section 4.4, rank 2, theta column kept) and the 2 x 2
// K = I2 + S + H^T Z, for I + Q and for I - Q (the adjoint's), after the
// factorization kernels (abip_factor.hip) have left G^{-1} in G64.  The products
// with A and G^{-1} run over the whole GPU (the batched path forms the same
// border with one workgroup per LP, k_setup_border).  FP64 throughout.
#include <hip/hip_runtime.h>
#include <algorithm>
#include "abip_internal.h"

// e = es * ev, f = fs * fv
__global__ void k_lib_scale(const double* ev, double es, int m, const double* fv, double fs, int n, double* e,
                            double* f) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < m) e[t] = es * ev[t];
    if (t < n) f[t] = fs * fv[t];
}

// Partial products of a column-major M (rows < m, ld) with x over column
// chunk blockIdx.y of cw columns: P[chunk * ld + i] = sum_j M[i + j ld] x[j].
__global__ __launch_bounds__(256) void k_gemv_part(const double* __restrict__ M, int ld, int m, int n,
                                                    const double* __restrict__ x, int cw, double* __restrict__ P) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j0 = blockIdx.y * cw, j1 = min(n, j0 + cw);
    if (i >= m) return;
    double s0 = 0.0, s1 = 0.0;
    int j = j0;
    for (; j + 1 < j1; j += 2) {
        s0 = fma(M[(int64_t)j * ld + i], x[j], s0);
        s1 = fma(M[(int64_t)(j + 1) * ld + i], x[j + 1], s1);
    }
    if (j < j1) s0 = fma(M[(int64_t)j * ld + i], x[j], s0);
    P[(int64_t)blockIdx.y * ld + i] = s0 + s1;
}

// y[i] = beta yin[i] + alpha sum_chunk P[chunk * ld + i] (fixed order; yin may be null)
__global__ void k_gemv_sum(const double* __restrict__ P, int ld, int m, int nch, double alpha,
                           const double* __restrict__ yin, double beta, double* __restrict__ y) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    double s = 0.0;
    for (int c = 0; c < nch; ++c) s += P[(int64_t)c * ld + i];
    y[i] = alpha * s + (yin ? beta * yin[i] : 0.0);
}

// z[j] = beta zin[j] + alpha sum_i M[i + j ld] v[i], one wave per column
__global__ __launch_bounds__(256) void k_gemv_t(const double* __restrict__ M, int ld, int m, int n,
                                                 const double* __restrict__ v, double alpha,
                                                 const double* __restrict__ zin, double beta, double* __restrict__ z) {
    const int lane = threadIdx.x & 63;
    const int j = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (j >= n) return;
    double s = 0.0;
    for (int i = lane; i < m; i += 64) s = fma(M[(int64_t)j * ld + i], v[i], s);
    s = wave_sum(s);
    if (lane == 0) z[j] = alpha * s + (zin ? beta * zin[j] : 0.0);
}

// K = I2 + S + H^T Z for the stored border (sgn = +1: I + Q; -1: I - Q), and
// zbar, ||b||, ||c|| into the LP's control block.  One workgroup.
__global__ __launch_bounds__(512) void k_lib_border_k(const LPDesc* __restrict__ desc, const double* __restrict__ Mv,
                                                      const double* __restrict__ Nv, int64_t Mtot, int64_t Ntot,
                                                      LPCtrl* __restrict__ ctrl, int sgn) {
    __shared__ double sbuf[8 * 8];
    const LPDesc d = desc[0];
    const int m = d.m, n = d.n, tid = threadIdx.x;
    const double* b = Mv + MF_B * Mtot + d.om;
    const double* bbar = Mv + MF_BBAR * Mtot + d.om;
    const double* c = Nv + NF_C * Ntot + d.on;
    const double* cbar = Nv + NF_CBAR * Ntot + d.on;
    const int fzy = (sgn > 0) ? MF_ZY0 : MF_ZY0A, fzx = (sgn > 0) ? NF_ZX0 : NF_ZX0A;
    const double* zy0 = Mv + fzy * Mtot + d.om;
    const double* zy1 = Mv + (fzy + 1) * Mtot + d.om;
    const double* zx0 = Nv + fzx * Ntot + d.on;
    const double* zx1 = Nv + (fzx + 1) * Ntot + d.on;
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int i = tid; i < m; i += blockDim.x) {
        v[0] = fma(-b[i], zy0[i], v[0]);
        v[1] = fma(-b[i], zy1[i], v[1]);
        v[2] = fma(bbar[i], zy0[i], v[2]);
        v[3] = fma(bbar[i], zy1[i], v[3]);
        v[4] = fma(b[i], b[i], v[4]);
    }
    for (int j = tid; j < n; j += blockDim.x) {
        v[0] = fma(c[j], zx0[j], v[0]);
        v[1] = fma(c[j], zx1[j], v[1]);
        v[2] = fma(-cbar[j], zx0[j], v[2]);
        v[3] = fma(-cbar[j], zx1[j], v[3]);
        v[5] = fma(c[j], c[j], v[5]);
        v[6] += c[j];
    }
    block_sum_n<7>(v, sbuf);
    if (tid == 0) {
        const double sg = (double)sgn, zbar = v[6] + 1.0;
        const double k00 = 1.0 + sg * v[0], k01 = sg * zbar + sg * v[1];
        const double k10 = -sg * zbar + sg * v[2], k11 = 1.0 + sg * v[3];
        const double det = k00 * k11 - k01 * k10;
        LPCtrl& C = ctrl[0];
        C.zbar = zbar;
        C.nb = sqrt(v[4]);
        C.nc = sqrt(v[5]);
        if (sgn > 0) { C.K00 = k11 / det; C.K01 = -k01 / det; C.K10 = -k10 / det; C.K11 = k00 / det; }
        else { C.KA00 = k11 / det; C.KA01 = -k01 / det; C.KA10 = -k10 / det; C.KA11 = k00 / det; }
    }
}

// Scratch doubles the border of one m x n LP needs (e, f, partial products).
int64_t grid_border_scratch(int m, int n, int ld) {
    const int cw = 256;
    const int nch = std::max((n + cw - 1) / cw, (m + cw - 1) / cw);
    return (int64_t)ld + n + (int64_t)nch * ld;
}

// Z and K for I + Q and I - Q of LP desc[0]: t = e - sgn A f, a = G^{-1} t,
// z = f + sgn A^T a for the two columns of sgn H.
hipError_t grid_border(const LPDesc& d, const LPDesc* ddesc, const double* A64, const double* G64, double* Mv,
                       double* Nv, int64_t Mtot, int64_t Ntot, LPCtrl* dctrl, double* scratch, hipStream_t st) {
    const int m = d.m, n = d.n, ld = d.ld;
    const int cw = 256;
    double* e = scratch;
    double* f = e + ld;
    double* P = f + n;
    const int nchA = (n + cw - 1) / cw, nchG = (m + cw - 1) / cw;
    const dim3 rows((m + 255) / 256);
    for (int sgn = 1; sgn >= -1; sgn -= 2) {
        const double sg = (double)sgn;
        const int fzy = (sgn > 0) ? MF_ZY0 : MF_ZY0A, fzx = (sgn > 0) ? NF_ZX0 : NF_ZX0A;
        for (int hh = 0; hh < 2; ++hh) {
            const double* ev = Mv + ((hh == 0) ? MF_B : MF_BBAR) * Mtot + d.om;
            const double* fv = Nv + ((hh == 0) ? NF_C : NF_CBAR) * Ntot + d.on;
            const double es = sg * ((hh == 0) ? -1.0 : 1.0), fs = sg * ((hh == 0) ? 1.0 : -1.0);
            double* zy = Mv + (fzy + hh) * Mtot + d.om;
            double* zx = Nv + (fzx + hh) * Ntot + d.on;
            hipLaunchKernelGGL(k_lib_scale, dim3((std::max(m, n) + 255) / 256), dim3(256), 0, st, ev, es, m, fv, fs,
                               n, e, f);
            hipLaunchKernelGGL(k_gemv_part, dim3(rows.x, nchA), dim3(256), 0, st, A64, ld, m, n, f, cw, P);
            hipLaunchKernelGGL(k_gemv_sum, rows, dim3(256), 0, st, P, ld, m, nchA, -sg, e, 1.0, e);  // t = e - sg A f
            hipLaunchKernelGGL(k_gemv_part, dim3(rows.x, nchG), dim3(256), 0, st, G64, ld, m, m, e, cw, P);
            hipLaunchKernelGGL(k_gemv_sum, rows, dim3(256), 0, st, P, ld, m, nchG, 1.0, (const double*)nullptr, 0.0,
                               zy);                                                                 // a = G^{-1} t
            hipLaunchKernelGGL(k_gemv_t, dim3((n + 3) / 4), dim3(256), 0, st, A64, ld, m, n, zy, sg, f, 1.0, zx);
        }
        hipLaunchKernelGGL(k_lib_border_k, dim3(1), dim3(512), 0, st, ddesc, Mv, Nv, Mtot, Ntot, dctrl, sgn);
    }
    return hipGetLastError();
}
