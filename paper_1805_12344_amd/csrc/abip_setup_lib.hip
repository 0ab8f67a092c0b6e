// Setup of one large dense LP (the grid engine's case) with the ROCm
// libraries for the dense linear algebra that happens once per LP: G = I + A A^T
// by rocBLAS SYRK, its Cholesky factor and inverse by rocSOLVER (POTRF, POTRI),
// and the border columns Z = M^{-1} H (Section 4.4, rank 2) by GEMV products.
// FP64 throughout; the batched path keeps its own one-workgroup-per-LP kernels.
#include <hip/hip_runtime.h>
#include <algorithm>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>
#include "abip_internal.h"

__global__ void k_lib_diag(double* G, int m, int ld) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) G[(int64_t)i * ld + i] += 1.0;
}

// lower triangle -> full symmetric matrix, and its FP32 copy (rows past m stay 0)
__global__ void k_lib_symmetrize(double* G64, float* G32, int m, int ld) {
    const int j = blockIdx.y;                                     // column
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ld; i += gridDim.x * blockDim.x) {
        double v = 0.0;
        if (i < m) v = (i >= j) ? G64[(int64_t)j * ld + i] : G64[(int64_t)i * ld + j];
        G32[(int64_t)j * ld + i] = (float)v;
    }
}
__global__ void k_lib_copy_upper(double* G64, const float* G32, int m, int ld) {
    // after the FP32 copy holds the full matrix in float, restore the full FP64 one
    const int j = blockIdx.y;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x)
        if (i < j) G64[(int64_t)j * ld + i] = G64[(int64_t)i * ld + j];
}

// e = es * ev, f = fs * fv
__global__ void k_lib_scale(const double* ev, double es, int m, const double* fv, double fs, int n, double* e,
                            double* f) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < m) e[t] = es * ev[t];
    if (t < n) f[t] = fs * fv[t];
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

#define RBCHK(x) do { if ((x) != rocblas_status_success) { rc = 1; goto done; } } while (0)

// One LP (desc[0]) whose A64 (ld x n, column-major) and pools are filled and
// whose G64 / G32 are zero.  Returns 0, 1 (library error) or 2 (G not positive
// definite, which cannot happen for I + A A^T unless A is not finite).
int lib_setup_one(const LPDesc& d, const LPDesc* ddesc, const double* A64, double* G64, float* G32, double* Mv,
                  double* Nv, int64_t Mtot, int64_t Ntot, LPCtrl* dctrl, hipStream_t st) {
    rocblas_handle h = nullptr;
    int rc = 0;
    rocblas_int* dinfo = nullptr;
    double *e = nullptr, *f = nullptr;
    const int m = d.m, n = d.n, ld = d.ld;
    const double one = 1.0, zero = 0.0;
    rocblas_int hinfo = 0;
    if (rocblas_create_handle(&h) != rocblas_status_success) return 1;
    if (hipMalloc((void**)&dinfo, sizeof(rocblas_int)) != hipSuccess) { rocblas_destroy_handle(h); return 1; }
    if (hipMalloc((void**)&e, sizeof(double) * ld) != hipSuccess ||
        hipMalloc((void**)&f, sizeof(double) * n) != hipSuccess) { rc = 1; goto done; }
    RBCHK(rocblas_set_stream(h, st));
    RBCHK(rocblas_set_pointer_mode(h, rocblas_pointer_mode_host));
    // G = I + A A^T (lower triangle), factor, inverse
    hipLaunchKernelGGL(k_lib_diag, dim3((m + 255) / 256), dim3(256), 0, st, G64, m, ld);
    RBCHK(rocblas_dsyrk(h, rocblas_fill_lower, rocblas_operation_none, m, n, &one, A64, ld, &one, G64, ld));
    RBCHK(rocsolver_dpotrf(h, rocblas_fill_lower, m, G64, ld, dinfo));
    if (hipMemcpyAsync(&hinfo, dinfo, sizeof hinfo, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) { rc = 1; goto done; }
    if (hinfo != 0) { rc = 2; goto done; }
    RBCHK(rocsolver_dpotri(h, rocblas_fill_lower, m, G64, ld, dinfo));
    hipLaunchKernelGGL(k_lib_symmetrize, dim3(std::max(1, (ld + 255) / 256), m), dim3(256), 0, st, G64, G32, m, ld);
    hipLaunchKernelGGL(k_lib_copy_upper, dim3(std::max(1, (m + 255) / 256), m), dim3(256), 0, st, G64, G32, m, ld);
    // border columns for I + Q (sgn = +1) and I - Q (sgn = -1)
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
            const double msg = -sg;
            RBCHK(rocblas_dgemv(h, rocblas_operation_none, m, n, &msg, A64, ld, f, 1, &one, e, 1));   // e - sg A f
            RBCHK(rocblas_dgemv(h, rocblas_operation_none, m, m, &one, G64, ld, e, 1, &zero, zy, 1)); // a = G^-1 t
            if (hipMemcpyAsync(zx, f, sizeof(double) * n, hipMemcpyDeviceToDevice, st) != hipSuccess) { rc = 1; goto done; }
            RBCHK(rocblas_dgemv(h, rocblas_operation_transpose, m, n, &sg, A64, ld, zy, 1, &one, zx, 1)); // f + sg A^T a
        }
        hipLaunchKernelGGL(k_lib_border_k, dim3(1), dim3(512), 0, st, ddesc, Mv, Nv, Mtot, Ntot, dctrl, sgn);
    }
    if (hipStreamSynchronize(st) != hipSuccess) rc = 1;
done:
    (void)hipStreamSynchronize(st);
    (void)hipFree(dinfo);
    (void)hipFree(e);
    (void)hipFree(f);
    rocblas_destroy_handle(h);
    return rc;
}
