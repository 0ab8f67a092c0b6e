// The cached factorization of Section 4.4 on the matrix cores: G = I + A A^T,
// its Cholesky factor G = L L^T, W = L^{-1} and G^{-1} = W^T W, all FP64, for
// every LP of a work handle at once (blockIdx.y = LP; an LP with fewer tiles
// than the grid covers leaves the extra workgroups idle).
//
// Every product of 64 x 64 tiles runs on v_mfma_f64_16x16x4f64: a workgroup of
// four waves owns one 64 x 64 output tile, each wave a 32 x 32 quarter held as
// 2 x 2 accumulators of 16 x 16; the operands are staged through LDS 16 columns
// of the contraction at a time.  Layouts (all per LP, leading dimension ld):
//   A    column-major, A[i + j ld]                 (rows m..ld-1 zero)
//   G    column-major; the factorization overwrites its lower triangle with L
//        (the upper keeps G), the inverse finally overwrites all of it
//   W    row-major, W[i ld + j] (lower triangular L^{-1}), scratch
//   Lv   the inverse of each 64 x 64 diagonal block of L, column-major 64 x 64,
//        block p of the LP at oL + p * 4096, scratch
// Blocked right-looking Cholesky with 64-wide panels: for every panel p, the
// diagonal block is factored and inverted by one workgroup (VALU, in LDS), the
// blocks below become L[i,p] = G[i,p] inv(L[p,p])^T, and the trailing lower
// tiles lose L[i,p] L[j,p]^T.  Then W by block rows, W[i,p] =
// -inv(L[i,i]) sum_{k=p}^{i-1} L[i,k] W[k,p], and G^{-1}[i,j] =
// sum_{k >= i} W[k,i]^T W[k,j] on the lower tiles, mirrored.
#include <hip/hip_runtime.h>
#include "abip_internal.h"

typedef double v4d __attribute__((ext_vector_type(4)));

#define FT 64            // tile edge
#define FK 16            // contraction columns staged per step

// Lane l of a wave holds, for the 16 x 16 accumulator of a
// v_mfma_f64_16x16x4f64, element i (0..3) at row 4 i + l / 16, column l % 16
// (the A operand is (row l % 16, k l / 16), the B operand (k l / 16, column
// l % 16)).
__device__ __forceinline__ int mf_row(int lane, int i) { return 4 * i + (lane >> 4); }
__device__ __forceinline__ int mf_col(int lane) { return lane & 15; }

struct TileAcc {
    v4d c[2][2];
};

__device__ __forceinline__ void acc_zero(TileAcc& T) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) T.c[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};
}

// T += X(64 x FK) Y(FK x 64) for this wave's quarter: Xs[k][r] = X(r, k),
// Ys[k][c] = Y(k, c), both in LDS.
__device__ __forceinline__ void acc_step(TileAcc& T, const double (*Xs)[FT], const double (*Ys)[FT]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r0 = (wave >> 1) * 32, c0 = (wave & 1) * 32;
    const int kl = lane >> 4, il = lane & 15;
#pragma unroll
    for (int k4 = 0; k4 < FK; k4 += 4) {
        double xa[2], yb[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) xa[a] = Xs[k4 + kl][r0 + a * 16 + il];
#pragma unroll
        for (int b = 0; b < 2; ++b) yb[b] = Ys[k4 + kl][c0 + b * 16 + il];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) T.c[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[a], yb[b], T.c[a][b], 0, 0, 0);
    }
}

// Visit this wave's elements of the 64 x 64 tile: f(row, col, value).
template <typename F>
__device__ __forceinline__ void acc_each(const TileAcc& T, F f) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r0 = (wave >> 1) * 32, c0 = (wave & 1) * 32;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) f(r0 + a * 16 + mf_row(lane, i), c0 + b * 16 + mf_col(lane), T.c[a][b][i]);
}

// T += sum over the contraction range [k0, k1) of X(r, k) Y(k, c); the loaders
// return X(r, k) and Y(k, c) for r, c in 0..63 (0 past the data).
template <typename LX, typename LY>
__device__ __forceinline__ void tile_gemm(TileAcc& T, int k0, int k1, double (*Xs)[FT], double (*Ys)[FT], LX lx,
                                          LY ly) {
    for (int kb = k0; kb < k1; kb += FK) {
        for (int e = threadIdx.x; e < FK * FT; e += blockDim.x) {
            const int kk = e >> 6, r = e & 63;
            const int k = kb + kk;
            Xs[kk][r] = (k < k1) ? lx(r, k) : 0.0;
            Ys[kk][r] = (k < k1) ? ly(k, r) : 0.0;
        }
        __syncthreads();
        acc_step(T, Xs, Ys);
        __syncthreads();
    }
}

// lower tile t of an nt x nt tiling -> (I, J), I >= J
__device__ __forceinline__ void lower_tile(int t, int& I, int& J) {
    int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while (i * (i + 1) / 2 > t) --i;
    while ((i + 1) * (i + 2) / 2 <= t) ++i;
    I = i;
    J = t - i * (i + 1) / 2;
}

// ---------------------------------------------------------------------------
// G = I + A A^T on the lower tiles, both halves written.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fac_syrk(const LPDesc* __restrict__ desc, const double* __restrict__ A64,
                                                  double* __restrict__ G64) {
    __shared__ double Xs[FK][FT];
    __shared__ double Ys[FK][FT];
    const LPDesc d = desc[blockIdx.y];
    const int nt = (d.m + FT - 1) / FT;
    if ((int)blockIdx.x >= nt * (nt + 1) / 2) return;
    int I, J;
    lower_tile(blockIdx.x, I, J);
    const double* A = A64 + d.oA;
    double* G = G64 + d.oG;
    const int ld = d.ld, m = d.m;
    TileAcc T;
    acc_zero(T);
    tile_gemm(T, 0, d.n, Xs, Ys,
              [&](int r, int k) { const int i = I * FT + r; return i < ld ? A[(int64_t)k * ld + i] : 0.0; },
              [&](int k, int c) { const int j = J * FT + c; return j < ld ? A[(int64_t)k * ld + j] : 0.0; });
    acc_each(T, [&](int r, int c, double v) {
        const int i = I * FT + r, j = J * FT + c;
        if (i < m && j < m && j <= i) {
            v += (i == j) ? 1.0 : 0.0;
            G[(int64_t)j * ld + i] = v;
            G[(int64_t)i * ld + j] = v;
        }
    });
}

// ---------------------------------------------------------------------------
// Panel p, diagonal block: factor the 64 x 64 block of G (lower) in LDS, write
// L[p,p] into G's lower triangle, its inverse into Lv (column-major) and W
// (row-major).  One workgroup per LP; a non-positive pivot sets err bit 4.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fac_diag(const LPDesc* __restrict__ desc, double* __restrict__ G64,
                                                  double* __restrict__ Lv, const int64_t* __restrict__ oL,
                                                  double* __restrict__ Wpool, const int64_t* __restrict__ oW, int p,
                                                  int* __restrict__ err) {
    __shared__ double S[FT][FT + 1];        // S[r][c], the block (then L)
    __shared__ double V[FT][FT + 1];        // V[r][c], inv(L)
    const LPDesc d = desc[blockIdx.x];
    const int nt = (d.m + FT - 1) / FT;
    if (p >= nt) return;
    const int ld = d.ld, m = d.m, tid = threadIdx.x;
    const int b0 = p * FT, nb = min(FT, m - b0);       // rows / columns of this block that exist
    double* G = G64 + d.oG;
    for (int e = tid; e < FT * FT; e += blockDim.x) {
        const int r = e & 63, c = e >> 6;
        double v = 0.0;
        if (r < nb && c < nb) v = G[(int64_t)(b0 + c) * ld + b0 + r];
        else if (r == c) v = 1.0;                      // identity past m keeps the block regular
        S[r][c] = v;
        V[r][c] = 0.0;
    }
    __syncthreads();
    // right-looking Cholesky of S (lower)
    for (int k = 0; k < FT; ++k) {
        const double piv = S[k][k];
        __syncthreads();
        if (!(piv > 0.0)) {
            if (tid == 0) atomicOr(err, 4);
            return;
        }
        const double lk = sqrt(piv);
        if (tid == 0) S[k][k] = lk;
        for (int r = k + 1 + tid; r < FT; r += blockDim.x) S[r][k] /= lk;
        __syncthreads();
        for (int e = tid; e < (FT - k - 1) * (FT - k - 1); e += blockDim.x) {
            const int r = k + 1 + e % (FT - k - 1), c = k + 1 + e / (FT - k - 1);
            if (c <= r) S[r][c] = fma(-S[r][k], S[c][k], S[r][c]);
        }
        __syncthreads();
    }
    // inverse of the lower triangle, one column of V per thread (forward substitution)
    if (tid < FT) {
        const int c = tid;
        for (int r = c; r < FT; ++r) {
            double s = (r == c) ? 1.0 : 0.0;
            for (int q = c; q < r; ++q) s = fma(-S[r][q], V[q][c], s);
            V[r][c] = s / S[r][r];
        }
    }
    __syncthreads();
    double* L = Lv + oL[blockIdx.x] + (int64_t)p * FT * FT;
    double* W = Wpool + oW[blockIdx.x];
    for (int e = tid; e < FT * FT; e += blockDim.x) {
        const int r = e & 63, c = e >> 6;
        L[r + c * FT] = (c <= r) ? V[r][c] : 0.0;
        if (r < nb && c < nb) {
            if (c <= r) G[(int64_t)(b0 + c) * ld + b0 + r] = S[r][c];
            W[(int64_t)(b0 + r) * ld + b0 + c] = (c <= r) ? V[r][c] : 0.0;
        }
    }
}

// Panel p, blocks below the diagonal: L[i,p] = G[i,p] inv(L[p,p])^T for
// i = p+1 .. (blockIdx.x = i - p - 1).
__global__ __launch_bounds__(256) void k_fac_trsm(const LPDesc* __restrict__ desc, double* __restrict__ G64,
                                                  const double* __restrict__ Lv, const int64_t* __restrict__ oL, int p) {
    __shared__ double Xs[FK][FT];
    __shared__ double Ys[FK][FT];
    const LPDesc d = desc[blockIdx.y];
    const int nt = (d.m + FT - 1) / FT;
    const int I = p + 1 + (int)blockIdx.x;
    if (I >= nt) return;
    const int ld = d.ld, m = d.m;
    double* G = G64 + d.oG;
    const double* Li = Lv + oL[blockIdx.y] + (int64_t)p * FT * FT;
    TileAcc T;
    acc_zero(T);
    // X(r, k) = G[I*64 + r, p*64 + k], Y(k, c) = inv(L[p,p])[c][k]
    tile_gemm(T, 0, FT, Xs, Ys,
              [&](int r, int k) {
                  const int i = I * FT + r, j = p * FT + k;
                  return (i < m && j < m) ? G[(int64_t)j * ld + i] : 0.0;
              },
              [&](int k, int c) { return Li[c + k * FT]; });
    acc_each(T, [&](int r, int c, double v) {
        const int i = I * FT + r, j = p * FT + c;
        if (i < m && j < m) G[(int64_t)j * ld + i] = v;
    });
}

// Panel p, trailing lower tiles (I >= J > p): G[I,J] -= L[I,p] L[J,p]^T
// (only the lower triangle of a diagonal tile is used later).
__global__ __launch_bounds__(256) void k_fac_update(const LPDesc* __restrict__ desc, double* __restrict__ G64, int p) {
    __shared__ double Xs[FK][FT];
    __shared__ double Ys[FK][FT];
    const LPDesc d = desc[blockIdx.y];
    const int nt = (d.m + FT - 1) / FT;
    const int nr = nt - p - 1;                      // trailing tiles per side
    if (nr <= 0 || (int)blockIdx.x >= nr * (nr + 1) / 2) return;
    int I, J;
    lower_tile(blockIdx.x, I, J);
    I += p + 1;
    J += p + 1;
    const int ld = d.ld, m = d.m;
    double* G = G64 + d.oG;
    TileAcc T;
    acc_zero(T);
    tile_gemm(T, 0, FT, Xs, Ys,
              [&](int r, int k) {
                  const int i = I * FT + r, j = p * FT + k;
                  return (i < m && j < m) ? G[(int64_t)j * ld + i] : 0.0;
              },
              [&](int k, int c) {
                  const int i = J * FT + c, j = p * FT + k;
                  return (i < m && j < m) ? G[(int64_t)j * ld + i] : 0.0;
              });
    acc_each(T, [&](int r, int c, double v) {
        const int i = I * FT + r, j = J * FT + c;
        if (i < m && j < m && (I != J || c <= r)) G[(int64_t)j * ld + i] -= v;
    });
}

// Block row I of W = L^{-1}: W[I,P] = -inv(L[I,I]) sum_{k=P}^{I-1} L[I,k] W[k,P]
// for P = 0 .. I-1 (blockIdx.x = P).  W is row-major; L sits in G's lower part.
__global__ __launch_bounds__(256) void k_fac_trtri(const LPDesc* __restrict__ desc, const double* __restrict__ G64,
                                                   const double* __restrict__ Lv, const int64_t* __restrict__ oL,
                                                   double* __restrict__ Wpool, const int64_t* __restrict__ oW, int I) {
    __shared__ double Xs[FK][FT];
    __shared__ double Ys[FK][FT];
    __shared__ double Ts[FT][FT + 1];
    const LPDesc d = desc[blockIdx.y];
    const int nt = (d.m + FT - 1) / FT;
    const int P = blockIdx.x;
    if (I >= nt || P >= I) return;
    const int ld = d.ld, m = d.m;
    const double* G = G64 + d.oG;
    double* W = Wpool + oW[blockIdx.y];
    TileAcc T;
    acc_zero(T);
    // T = sum_k L[I, k] W[k, P] over rows k of blocks P .. I-1
    tile_gemm(T, P * FT, I * FT, Xs, Ys,
              [&](int r, int k) {
                  const int i = I * FT + r;
                  return (i < m && k < m) ? G[(int64_t)k * ld + i] : 0.0;
              },
              [&](int k, int c) {
                  const int j = P * FT + c;
                  return (k < m && j < m) ? W[(int64_t)k * ld + j] : 0.0;
              });
    acc_each(T, [&](int r, int c, double v) { Ts[r][c] = v; });
    __syncthreads();
    const double* Li = Lv + oL[blockIdx.y] + (int64_t)I * FT * FT;
    TileAcc U;
    acc_zero(U);
    tile_gemm(U, 0, FT, Xs, Ys, [&](int r, int k) { return Li[r + k * FT]; }, [&](int k, int c) { return Ts[k][c]; });
    acc_each(U, [&](int r, int c, double v) {
        const int i = I * FT + r, j = P * FT + c;
        if (i < m && j < m) W[(int64_t)i * ld + j] = -v;
    });
}

// G^{-1}[I,J] = sum_{k >= I} W[k,I]^T W[k,J] on the lower tiles, both halves of
// G64 written, and the FP32 copy G32 (rows m..ld-1 zero).
__global__ __launch_bounds__(256) void k_fac_lauum(const LPDesc* __restrict__ desc, const double* __restrict__ Wpool,
                                                   const int64_t* __restrict__ oW, double* __restrict__ G64,
                                                   float* __restrict__ G32) {
    __shared__ double Xs[FK][FT];
    __shared__ double Ys[FK][FT];
    const LPDesc d = desc[blockIdx.y];
    const int nt = (d.m + FT - 1) / FT;
    if ((int)blockIdx.x >= nt * (nt + 1) / 2) return;
    int I, J;
    lower_tile(blockIdx.x, I, J);
    const int ld = d.ld, m = d.m;
    const double* W = Wpool + oW[blockIdx.y];
    double* G = G64 + d.oG;
    float* G2 = G32 + d.oG;
    TileAcc T;
    acc_zero(T);
    tile_gemm(T, I * FT, m, Xs, Ys,
              [&](int r, int k) { const int i = I * FT + r; return i < m ? W[(int64_t)k * ld + i] : 0.0; },
              [&](int k, int c) { const int j = J * FT + c; return j < m ? W[(int64_t)k * ld + j] : 0.0; });
    acc_each(T, [&](int r, int c, double v) {
        const int i = I * FT + r, j = J * FT + c;
        if (i < m && j < m && j <= i) {
            G[(int64_t)j * ld + i] = v;
            G[(int64_t)i * ld + j] = v;
            G2[(int64_t)j * ld + i] = (float)v;
            G2[(int64_t)i * ld + j] = (float)v;
        }
    });
}

// ---------------------------------------------------------------------------
// Triangular-solve path: keep L (lower triangle of G after the panels, zero
// above the diagonal and in the padding rows) and L^T, both column-major ld x m
// at the LP's G offset, in FP64 and FP32; grid (tiles of an nt x nt tiling, B),
// the transpose through an LDS tile.
__global__ __launch_bounds__(256) void k_fac_keep(const LPDesc* __restrict__ desc, const double* __restrict__ G64,
                                                  double* __restrict__ L64, double* __restrict__ Lt64,
                                                  float* __restrict__ L32, float* __restrict__ Lt32) {
    const LPDesc d = desc[blockIdx.y];
    const int nt = (d.m + FT - 1) / FT;
    const int tile = blockIdx.x;
    if (tile >= nt * nt) return;
    const int ti = tile / nt, tj = tile % nt;
    __shared__ double T[FT][FT + 1];
    for (int e = threadIdx.x; e < FT * FT; e += blockDim.x) {
        const int r = e & (FT - 1), c = e / FT;
        const int i = ti * FT + r, j = tj * FT + c;
        double v = 0.0;
        if (i < d.m && j < d.m && i >= j) v = G64[d.oG + (int64_t)j * d.ld + i];
        T[r][c] = v;
        if (i < d.ld && j < d.m) {
            L64[d.oG + (int64_t)j * d.ld + i] = v;
            L32[d.oG + (int64_t)j * d.ld + i] = (float)v;
        }
    }
    __syncthreads();
    // L^T[r', c'] = L[c', r'] with r' = tj*FT + r, c' = ti*FT + c
    for (int e = threadIdx.x; e < FT * FT; e += blockDim.x) {
        const int r = e & (FT - 1), c = e / FT;
        const int i = tj * FT + r, j = ti * FT + c;
        if (i < d.ld && j < d.m) {
            const double v = (i < d.m) ? T[c][r] : 0.0;
            Lt64[d.oG + (int64_t)j * d.ld + i] = v;
            Lt32[d.oG + (int64_t)j * d.ld + i] = (float)v;
        }
    }
}

// The inverses of L's diagonal blocks and their transposes, FP64 and FP32
// (grid: blocks, B).
__global__ __launch_bounds__(256) void k_fac_keepdiag(const LPDesc* __restrict__ desc, const double* __restrict__ Lv,
                                                      const int64_t* __restrict__ oL, double* __restrict__ Li64,
                                                      double* __restrict__ Lit64, float* __restrict__ Li32,
                                                      float* __restrict__ Lit32) {
    const int k = blockIdx.y, p = blockIdx.x;
    const LPDesc d = desc[k];
    if (p >= (d.m + FT - 1) / FT) return;
    const int64_t o = oL[k] + (int64_t)p * FT * FT;
    for (int e = threadIdx.x; e < FT * FT; e += blockDim.x) {
        const int r = e & (FT - 1), c = e / FT;
        const double v = Lv[o + (int64_t)c * FT + r];
        Li64[o + (int64_t)c * FT + r] = v;
        Li32[o + (int64_t)c * FT + r] = (float)v;
        Lit64[o + (int64_t)r * FT + c] = v;
        Lit32[o + (int64_t)r * FT + c] = (float)v;
    }
}

// Host driver: the whole factorization for every LP of the handle.
// mmax: the largest m; Lv / oL, Wpool / oW: the scratch described above.
hipError_t factor_ginv(const LPDesc* ddesc, int B, int mmax, const double* A64, double* G64, float* G32, double* Lv,
                       const int64_t* oL, double* Wpool, const int64_t* oW, int* err, const FactorKeep* keep,
                       hipStream_t st) {
    const int nt = (mmax + FT - 1) / FT;
    const int tiles = nt * (nt + 1) / 2;
    hipLaunchKernelGGL(k_fac_syrk, dim3(tiles, B), dim3(256), 0, st, ddesc, A64, G64);
    for (int p = 0; p < nt; ++p) {
        hipLaunchKernelGGL(k_fac_diag, dim3(B), dim3(256), 0, st, ddesc, G64, Lv, oL, Wpool, oW, p, err);
        if (p + 1 < nt) {
            hipLaunchKernelGGL(k_fac_trsm, dim3(nt - p - 1, B), dim3(256), 0, st, ddesc, G64, Lv, oL, p);
            const int nr = nt - p - 1;
            hipLaunchKernelGGL(k_fac_update, dim3(nr * (nr + 1) / 2, B), dim3(256), 0, st, ddesc, G64, p);
        }
    }
    if (keep) {
        hipLaunchKernelGGL(k_fac_keep, dim3(nt * nt, B), dim3(256), 0, st, ddesc, G64, keep->L64, keep->Lt64,
                           keep->L32, keep->Lt32);
        hipLaunchKernelGGL(k_fac_keepdiag, dim3(nt, B), dim3(256), 0, st, ddesc, Lv, oL, keep->Li64, keep->Lit64,
                           keep->Li32, keep->Lit32);
    }
    for (int I = 1; I < nt; ++I)
        hipLaunchKernelGGL(k_fac_trtri, dim3(I, B), dim3(256), 0, st, ddesc, G64, Lv, oL, Wpool, oW, I);
    hipLaunchKernelGGL(k_fac_lauum, dim3(tiles, B), dim3(256), 0, st, ddesc, Wpool, oW, G64, G32);
    return hipGetLastError();
}
