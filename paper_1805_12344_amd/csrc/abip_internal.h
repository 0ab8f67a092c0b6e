// Internal data layout and device helpers of libabip (gfx950, wave64).
//
// Every LP of a work handle lives in shared pools:
//   * A is stored column-major with a padded leading dimension ld (a multiple
//     of 4, zero rows m..ld-1), once in FP64 (A64) and once in FP32 (A32), so a
//     wave can stream one column with 16-byte loads and one read of A feeds
//     both A^T(.) (column dot products) and A(.) (column-scaled accumulation).
//   * G^{-1} = (I + A A^T)^{-1} is stored as an ld x m symmetric array (column
//     j at offset j*ld, zero padding rows), FP64 and FP32.
//   * m-length and n-length vectors are "field-major": field f of LP k starts at
//     pool + f*Mtot + om (resp. Ntot, on).
#pragma once
#include <stdint.h>

#define ABIP_WAVE 64

// m-vector fields
enum { MF_B = 0, MF_BBAR, MF_AC, MF_ACBAR, MF_ZY0, MF_ZY1, MF_Y, MF_ZY0A, MF_ZY1A, NMF };
// n-vector fields
enum { NF_C = 0, NF_CBAR, NF_ZX0, NF_ZX1, NF_X, NF_S, NF_ZX0A, NF_ZX1A, NNF };

// column-pass operations
enum { OP_REFRESH = 0, OP_PROX = 1, OP_RESTART = 2 };

struct LPDesc {
    int32_t m, n, ld, pad;
    int64_t oA;     // element offset of column-major A (ld*n)
    int64_t oG;     // element offset of G^{-1} (ld*m)
    int64_t om;     // offset in each m-field (slice length ld)
    int64_t on;     // offset in each n-field (slice length n)
};

// Per-LP scalars kept in device memory between launches.
struct LPCtrl {
    double zbar, nb, nc;
    double K00, K01, K10, K11;        // K^{-1}, K = I2 + S + H^T Z
    double KA00, KA01, KA10, KA11;    // the same for I - Q (adjoint solves)
    double tau, kappa, theta, mu;
    double pres, dres, gap, pobj, dobj;  // last check (relative residuals)
    double by, cx;                        // b^T y, c^T x at the last check
    int64_t iters, iters64, ipm;
    int64_t cp32, cp64;                   // column passes per data precision
    int32_t status, phase, mode, flags;  // phase 0 = FP32 bulk, 1 = FP64; mode = next op
};

// Solver parameters passed by value to kernels.
struct SolveParams {
    double eps, alpha, beta, gamma;
    int64_t max_iters, fp32_max_iters;
    int32_t restart_rule, precision;
};

struct PoolPtrs {
    const double* A64; const float* A32;
    const double* G64; const float* G32;
    double* Mv; double* Nv;
    int64_t Mtot, Ntot;
};

// Positive root of z^2 - w z - t = 0, cancellation free for w < 0
// (closed form of the barrier prox, eqs. Simple-Update:Barrier-X/-tau).
__device__ __forceinline__ double prox_root(double w, double t) {
    double r = sqrt(w * w + 4.0 * t);
    return (w >= 0.0) ? 0.5 * (w + r) : (2.0 * t) / (r - w);
}

__device__ __forceinline__ double bcast_first(double v) {
    int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
    int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double bcast_lane(double v, int l) {
    int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wave; every lane receives lane 0's total, so the
// result is bitwise uniform.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return bcast_first(v);
}

template <int K>
__device__ __forceinline__ void wave_sum_n(double (&v)[K]) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] += __shfl_xor(v[k], o, 64);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = bcast_first(v[k]);
}

// Load 4 consecutive matrix entries (16-byte aligned) as doubles.
__device__ __forceinline__ void load4(const float* p, double* o) {
    float4 v = *reinterpret_cast<const float4*>(p);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
__device__ __forceinline__ void load4(const double* p, double* o) {
    double2 v0 = reinterpret_cast<const double2*>(p)[0];
    double2 v1 = reinterpret_cast<const double2*>(p)[1];
    o[0] = v0.x; o[1] = v0.y; o[2] = v1.x; o[3] = v1.y;
}

// Block-wide sum of K values; all threads receive the totals.  sbuf needs
// (blockDim/64)*K doubles of LDS.  Contains two barriers.
template <int K>
__device__ __forceinline__ void block_sum_n(double (&v)[K], double* sbuf) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, W = blockDim.x >> 6;
    wave_sum_n<K>(v);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) sbuf[wave * K + k] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (int w = 0; w < W; ++w) s += sbuf[w * K + k];
        v[k] = s;
    }
    __syncthreads();
}

__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }
__device__ __forceinline__ int num_waves() { return __builtin_amdgcn_readfirstlane(blockDim.x >> 6); }

// Reduce K values (K a power of two, 2 <= K <= 16) over the 64 lanes of a wave
// by recursive halving: at offset o the lanes with bit o set keep the upper
// half of the still-live values and the others the lower half.  Afterwards
// the total of value k sits in v[0] of lane lane_of<K>(k) (any lane of a
// 2^{6-log2 K}-lane block holds the same total); read it with bcast_lane.
template <int K>
__device__ __forceinline__ void wave_reduce_scatter(double (&v)[K]) {
    const int lane = threadIdx.x & 63;
    constexpr int L = (K >= 16) ? 4 : (K >= 8) ? 3 : (K >= 4) ? 2 : 1;
#pragma unroll
    for (int lev = 0; lev < 6; ++lev) {
        const int o = 32 >> lev;
        if (lev < L) {
            const int h = K >> (lev + 1);
            const bool up = (lane & o) != 0;
#pragma unroll
            for (int k = 0; k < h; ++k) {
                // pin both operands in registers first: otherwise the compiler turns
                // the per-lane choice into a dynamic index into v[] and lowers it as a
                // compare/select chain over the whole array
                double lo = v[k], hi = v[k + h];
                asm volatile("" : "+v"(lo), "+v"(hi));
                const double send = up ? lo : hi;
                const double keep = up ? hi : lo;
                v[k] = keep + __shfl_xor(send, o, 64);
            }
        } else {
            v[0] += __shfl_xor(v[0], o, 64);
        }
    }
}
template <int K>
__device__ __forceinline__ constexpr int lane_of(int k) {
    int lane = 0;
    for (int lev = 0; (K >> (lev + 1)) >= 1; ++lev)
        if (k & (K >> (lev + 1))) lane += 32 >> lev;
    return lane;
}
