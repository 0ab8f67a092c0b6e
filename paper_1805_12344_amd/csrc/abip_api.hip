// Host side of libabip: the C ABI declared in include/abip.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "abip.h"
#include "abip_internal.h"
#include "abip_grid.h"
#include "abip_sparse.h"
#include "abip_adjoint.h"

// defined in abip_solve_wg.hip
hipError_t launch_solve_wg(int nch, int grid, int threads, hipStream_t st, const LPDesc* desc, LPCtrl* ctrl,
                           const PoolPtrs& P, const SolveParams& prm, const int32_t* order, int32_t B,
                           int32_t* queue, int64_t fixed_iters, int32_t ldmax, size_t smem);
size_t wg_smem_bytes(int ldmax, int W);
// the cached factorization G = I + A A^T -> G^{-1} on the matrix cores (abip_factor.hip)
hipError_t factor_ginv(const LPDesc* ddesc, int B, int mmax, const double* A64, double* G64, float* G32, double* Lv,
                       const int64_t* oL, double* Wpool, const int64_t* oW, int* err, const FactorKeep* keep,
                       hipStream_t st);
// border of one large LP over the whole GPU (abip_setup_lib.hip)
int64_t grid_border_scratch(int m, int n, int ld);
hipError_t grid_border(const LPDesc& d, const LPDesc* ddesc, const double* A64, const double* G64, double* Mv,
                       double* Nv, int64_t Mtot, int64_t Ntot, LPCtrl* dctrl, double* scratch, hipStream_t st);
struct AdjArgs {
    double* ws;
    const int64_t* ows;
    const double* const* gin;
    double* const* dc;
    double* const* db;
    double* const* dA;
    int64_t max_iters;
    double tol;
    int64_t* iters_out;
    double* resid_out;
};
hipError_t launch_adjoint(int grid, int threads, hipStream_t st, const LPDesc* desc, const LPCtrl* ctrl,
                          const PoolPtrs& P, const SolveParams& prm, const AdjArgs& aa, const int32_t* order,
                          int32_t B, int32_t* queue, int32_t ldmax);
hipError_t set_solve_wg_smem_limit(size_t bytes);
// FP64 recheck of the returned point (abip_recheck.hip)
hipError_t launch_recheck_dense(const LPDesc* desc, LPCtrl* ctrl, const double* A64, const double* Mv,
                                const double* Nv, int64_t Mtot, int64_t Ntot, double* part, int B, int P,
                                hipStream_t st);
hipError_t launch_recheck_csr(const int32_t* rp, const int32_t* ci, const double* va, const int32_t* rpt,
                              const int32_t* cit, const double* vat, int m, int n, LPCtrl* ctrl, const double* b,
                              const double* y, const double* c, const double* x, const double* s, double* part,
                              int P, hipStream_t st);

// setup kernels (abip_setup.hip)
__global__ void k_setup_copy(const LPDesc*, const double* const*, double*, float*, int*);
__global__ void k_ruiz_init(const LPDesc*, double*, double*, int64_t, int64_t);
__global__ void k_ruiz_max(const LPDesc*, const double*, double*, double*, int64_t, int64_t);
__global__ void k_ruiz_apply(const LPDesc*, double*, double*, int64_t, int64_t);
__global__ void k_ruiz_scale(const LPDesc*, double*, float*, const double*, const double*, int64_t, int64_t);
__global__ void k_setup_rows(const LPDesc*, const double* const*, const double* const*, const double*,
                             double*, double*, int64_t, int64_t, int*, int);
__global__ void k_setup_rows_part(const LPDesc*, const double* const*, const double*, const double*, int64_t, int,
                                  double*);
__global__ void k_setup_rows_fin(const LPDesc*, const double* const*, const double*, int, double*, int64_t, int*);
static const int ROWS_CW = 64;     // columns per chunk of the one-large-LP row sums
static int64_t grid_rows_scratch(int n, int ld) { return (int64_t)3 * ((n + ROWS_CW - 1) / ROWS_CW) * ld; }
__global__ void k_setup_border(const LPDesc*, const double*, const double*, double*, double*, int64_t,
                               int64_t, LPCtrl*, int);

// ---------------------------------------------------------------------------
// error reporting
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

static int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    // a failed runtime call (an allocation beyond the device's memory, say) also
    // leaves HIP's last-error state set; read it here, so that the next call's
    // launch checks do not report this failure again
    (void)hipGetLastError();
    return code;
}

// the same for the library's host-only sources (presolve)
int abip_internal_fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(call)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess) {                                                                   \
            if (e_ == hipErrorOutOfMemory) return fail(ABIP_E_OOM, "%s: out of device memory", #call); \
            return fail(ABIP_E_HIP, "%s failed: %s", #call, hipGetErrorString(e_));              \
        }                                                                                         \
    } while (0)

// ---------------------------------------------------------------------------
// small device kernels
// ---------------------------------------------------------------------------
__global__ void k_reset_queue(int32_t* q) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *q = 0;
}

__global__ void k_init_state(const LPDesc* __restrict__ desc, LPCtrl* __restrict__ ctrl, double* __restrict__ Mv,
                             double* __restrict__ Nv, int64_t Mtot, int64_t Ntot, double beta, int phase,
                             int bb) {
    const int k = blockIdx.x;
    const LPDesc d = desc[k];
    for (int i = threadIdx.x; i < d.ld; i += blockDim.x) Mv[MF_Y * Mtot + d.om + i] = 0.0;
    for (int j = threadIdx.x; j < d.n; j += blockDim.x) {
        Nv[NF_X * Ntot + d.on + j] = 1.0;
        Nv[NF_S * Ntot + d.on + j] = 1.0;
    }
    if (threadIdx.x == 0) {
        LPCtrl& c = ctrl[k];
        c.tau = 1.0; c.kappa = 1.0; c.theta = 1.0; c.mu = beta;
        c.pres = c.dres = c.gap = c.pobj = c.dobj = NAN;
        c.by = c.cx = 0.0;
        c.iters = 0; c.iters64 = 0; c.ipm = 0; c.cp32 = 0; c.cp64 = 0; c.cg = 0;
        c.clk[0] = c.clk[1] = c.clk[2] = c.clk[3] = c.clk[4] = 0;
        c.cpl32 = c.cpl64 = c.gh32 = c.gh64 = 0;
        c.kfx = NAN; c.err64 = NAN;
        c.beta = beta; c.bbp = 0; c.bbe = 0;
        c.status = 0; c.phase = phase; c.mode = OP_REFRESH; c.flags = bb ? 16 : 0;
    }
}

// Scale the final iterate into the caller's buffers (Section 4.1 candidates
// and certificates).  outp: 3*B device pointers (x, y, s per LP; may be null).
__global__ void k_write_outputs(const LPDesc* __restrict__ desc, const LPCtrl* __restrict__ ctrl,
                                const double* __restrict__ Mv, const double* __restrict__ Nv, int64_t Mtot,
                                int64_t Ntot, double* const* __restrict__ outp, int32_t first) {
    const int k = blockIdx.x + first;
    const LPDesc d = desc[k];
    const LPCtrl c = ctrl[k];
    double* xo = outp[3 * blockIdx.x + 0];
    double* yo = outp[3 * blockIdx.x + 1];
    double* so = outp[3 * blockIdx.x + 2];
    const double* y = Mv + MF_Y * Mtot + d.om;
    const double* x = Nv + NF_X * Ntot + d.on;
    const double* s = Nv + NF_S * Ntot + d.on;
    double fx = 1.0 / c.tau, fy = 1.0 / c.tau, fs = 1.0 / c.tau;
    bool nx = false, ny = false, ns = false;
    if (c.status == ABIP_PRIMAL_INFEASIBLE) { fy = fs = 1.0 / c.by; nx = true; }
    else if (c.status == ABIP_DUAL_INFEASIBLE) { fx = -1.0 / c.cx; ny = ns = true; }
    // back to the LP as given: x = E x', y = D y', s = s' / E (D = E = 1 when
    // the LP was not scaled)
    const double* Dv = Mv + MF_SD * Mtot + d.om;
    const double* Ev = Nv + NF_SE * Ntot + d.on;
    for (int j = threadIdx.x; j < d.n; j += blockDim.x) {
        if (xo) xo[j] = nx ? NAN : (x[j] * fx) * Ev[j];
        if (so) so[j] = ns ? NAN : (s[j] * fs) / Ev[j];
    }
    for (int i = threadIdx.x; i < d.m; i += blockDim.x)
        if (yo) yo[i] = ny ? NAN : (y[i] * fy) * Dv[i];
}

// Copy LP k's iterate in or out (device vectors) -- step-level API.
__global__ void k_copy_state(const LPDesc* __restrict__ desc, int k, double* __restrict__ Mv,
                             double* __restrict__ Nv, int64_t Mtot, int64_t Ntot, double* y, double* x, double* s,
                             int dir) {
    const LPDesc d = desc[k];
    double* Y = Mv + MF_Y * Mtot + d.om;
    double* X = Nv + NF_X * Ntot + d.on;
    double* S = Nv + NF_S * Ntot + d.on;
    for (int i = threadIdx.x; i < d.m; i += blockDim.x) {
        if (dir == 0) Y[i] = y[i]; else if (y) y[i] = Y[i];
    }
    for (int j = threadIdx.x; j < d.n; j += blockDim.x) {
        if (dir == 0) { X[j] = x[j]; S[j] = s[j]; }
        else { if (x) x[j] = X[j]; if (s) s[j] = S[j]; }
    }
}

// (I+Q)^{-1} w for one LP with the cached data (one workgroup; FP64 or FP32
// data, FP64 arithmetic): t = w_y - A w_x, a = G^{-1} t, d = w_x + A^T a,
// border p = K^{-1}(w_q + H^T z), u~ = (z - Z p, p).
template <typename T>
__global__ __launch_bounds__(256) void k_apply_iq(const LPDesc* __restrict__ desc, const LPCtrl* __restrict__ ctrl,
                                                  int k, const T* __restrict__ Apool, const T* __restrict__ Gpool,
                                                  const double* __restrict__ Mv, const double* __restrict__ Nv,
                                                  int64_t Mtot, int64_t Ntot, const double* __restrict__ w,
                                                  double* __restrict__ out, int sgn) {
    extern __shared__ double sm[];
    __shared__ double sbuf[4 * 8];
    const LPDesc d = desc[k];
    const LPCtrl c = ctrl[k];
    const int m = d.m, n = d.n, ld = d.ld, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6,
              W = blockDim.x >> 6;
    const T* A = Apool + d.oA;
    const T* G = Gpool + d.oG;
    double* st = sm;
    double* sa = sm + ld;
    const double sg = (double)sgn;     // +1: I + Q;  -1: I - Q = (I + Q)^T
    for (int i = tid; i < ld; i += blockDim.x) {
        double s = 0.0;
        if (i < m) {
            for (int j = 0; j < n; ++j) s = fma((double)A[(int64_t)j * ld + i], w[m + j], s);
            s = w[i] - sg * s;
        }
        st[i] = s;
    }
    __syncthreads();
    for (int i = tid; i < ld; i += blockDim.x) {
        double s = 0.0;
        if (i < m)
            for (int q = 0; q < m; ++q) s = fma((double)G[(int64_t)q * ld + i], st[q], s);
        sa[i] = s;
    }
    __syncthreads();
    // d_j = w_x + (A^T a)_j into out[m + j] (temporarily)
    for (int j = wave; j < n; j += W) {
        double s = 0.0;
        for (int i = lane; i < m; i += 64) s = fma((double)A[(int64_t)j * ld + i], sa[i], s);
        s = wave_sum(s);
        if (lane == 0) out[m + j] = w[m + j] + sg * s;
    }
    __threadfence_block();
    __syncthreads();
    const double* b = Mv + MF_B * Mtot + d.om;
    const double* bbar = Mv + MF_BBAR * Mtot + d.om;
    const double* C = Nv + NF_C * Ntot + d.on;
    const double* CBv = Nv + NF_CBAR * Ntot + d.on;
    double hz[2] = {0.0, 0.0};
    for (int i = tid; i < m; i += blockDim.x) {
        hz[0] = fma(-b[i], sa[i], hz[0]);
        hz[1] = fma(bbar[i], sa[i], hz[1]);
    }
    for (int j = tid; j < n; j += blockDim.x) {
        const double dj = out[m + j];
        hz[0] = fma(C[j], dj, hz[0]);
        hz[1] = fma(-CBv[j], dj, hz[1]);
    }
    block_sum_n<2>(hz, sbuf);
    const double q0 = w[m + n] + sg * hz[0], q1 = w[m + n + 1] + sg * hz[1];
    const double k00 = sgn > 0 ? c.K00 : c.KA00, k01 = sgn > 0 ? c.K01 : c.KA01;
    const double k10 = sgn > 0 ? c.K10 : c.KA10, k11 = sgn > 0 ? c.K11 : c.KA11;
    const double p0 = k00 * q0 + k01 * q1, p1 = k10 * q0 + k11 * q1;
    const double* Zy0 = Mv + (sgn > 0 ? MF_ZY0 : MF_ZY0A) * Mtot + d.om;
    const double* Zy1 = Mv + (sgn > 0 ? MF_ZY1 : MF_ZY1A) * Mtot + d.om;
    const double* Zx0 = Nv + (sgn > 0 ? NF_ZX0 : NF_ZX0A) * Ntot + d.on;
    const double* Zx1 = Nv + (sgn > 0 ? NF_ZX1 : NF_ZX1A) * Ntot + d.on;
    for (int i = tid; i < m; i += blockDim.x) out[i] = sa[i] - Zy0[i] * p0 - Zy1[i] * p1;
    for (int j = tid; j < n; j += blockDim.x) out[m + j] = out[m + j] - Zx0[j] * p0 - Zx1[j] * p1;
    if (tid == 0) { out[m + n] = p0; out[m + n + 1] = p1; }
}

// ---------------------------------------------------------------------------
// the work handle
// ---------------------------------------------------------------------------
struct abip_work {
    int32_t B = 0;
    abip_settings set{};
    hipStream_t stream = nullptr;
    std::vector<LPDesc> hdesc;
    LPDesc* ddesc = nullptr;
    LPCtrl* dctrl = nullptr;
    double* A64 = nullptr; float* A32 = nullptr;
    double* G64 = nullptr; float* G32 = nullptr;
    double* Mv = nullptr; double* Nv = nullptr;
    int64_t Atot = 0, Gtot = 0, Mtot = 0, Ntot = 0;
    int32_t* order = nullptr;
    int32_t* queue = nullptr;
    int* errflag = nullptr;
    double** outp = nullptr;     // 3*B device pointer table
    double* rchk = nullptr;      // partial sums of the FP64 recheck (B * rchk_P * 8)
    int rchk_P = 1;              // workgroups per LP of the recheck
    // setup scratch kept with a dense handle, so abip_update_data can redo the
    // setup in place: W = L^{-1} (ld x ld per LP), the inverses of L's 64 x 64
    // diagonal blocks, the grid border's vectors, the caller's pointer tables
    double* suW = nullptr; int64_t* suoW = nullptr; double* suL = nullptr; int64_t* suoL = nullptr;
    double* suB = nullptr;
    FactorKeep keep{};               // L for the triangular-solve path (ABIP_LIN_TRSV), else null
    const double** suA = nullptr; const double** sub = nullptr; const double** suc = nullptr;
    int64_t suWtot = 0;
    int mmax = 0;
    int ldmax = 0, nch = 1, threads = 512;
    size_t wg_smem = 0;              // LDS bytes of the batched launch (streamed or LDS-resident)
    // LDS residency chosen by the autotuner: 0 = A and G^{-1}, else A alone, where
    // they fit; 1 = only A and G^{-1}; 2 = none.  lds_stream[k] != 0 streams LP k.
    int lds_policy = 0;
    std::vector<uint8_t> lds_stream;
    int lds_cap = 0;                 // the device's largest LDS allocation per workgroup
    int cu_count = 256;
    bool solved = false;
    double setup_ms = 0.0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;   // bracket the persistent solve launch
    // adjoint workspace (allocated at the first backward call)
    double* adj_ws = nullptr; int64_t* adj_ows = nullptr;
    double** adj_ptrs = nullptr;                 // 4*B device pointers: g, dc, db, dA
    int64_t* adj_iters = nullptr; double* adj_resid = nullptr;
    std::vector<int64_t> h_adj_iters; std::vector<double> h_adj_resid;
    // adjoint of a one-LP handle over the whole GPU (grid and sparse engines)
    double* big_ws = nullptr;
    double* sp_abak = nullptr;       // sparse: the solve's CG warm start, kept across a backward
    bool sp_adjb = false;            // sparse: the border of I - Q is computed
    // grid engine (one LP over the whole GPU)
    bool grid = false;
    int grid_nchw = 1;
    int grid_wgs = 0;                // workgroups per grid kernel (autotuned)
    int grid_pairs = 0;              // A = [A0, -A0] detected (settings.grid_mirror): n / 2, else 0
    GridArgs ga{};
    double* gbuf = nullptr;          // Y2, Pf, Px, pcol, prow, pa, t, a
    GridCtl* gctl = nullptr;         // 2 control blocks: the pass's state, the decision
    std::vector<LPCtrl> hctrl;
    // sparse engine (one LP, A in CSR, CG on I + A A^T)
    bool sparse = false;
    SpArgs sa{};
    int sp_nb = 1;
    int sp_nb_default = 1;          // the setup's choice (one workgroup per 256 rows or columns)
    int32_t* sp_idx = nullptr;       // rp (m+1), ci (nnz), rpt (n+1), cit (nnz), cursor (n)
    double* sp_val = nullptr;        // va (nnz), vat (nnz)
    double* sp_vec = nullptr;        // dG, a, z, p (m); CG records (2 x 4 m); ATZy0, ATZy1, ATY, ATA, q1 (n); part
    int32_t* sp_grp = nullptr;       // explicit G~ = A A^T: row pointers (m + 1), columns
    int32_t* sp_gci = nullptr;
    double* sp_gva = nullptr;        // values
    int64_t sp_gram_nnz = 0;
    std::vector<int32_t> sp_hrp, sp_hrpt;   // host copies of the row pointers of CSR(A), CSR(A^T)
    int sp_lds_cap = 0;              // dynamic LDS the cooperative kernels may use
    unsigned* sp_bar = nullptr;      // grid barrier words
    int* sp_err = nullptr;
    int64_t* sp_cgit = nullptr;
    // hipGraphs (captured on a private stream joined to the caller's by events)
    hipStream_t gstream = nullptr;
    hipEvent_t gjoin0 = nullptr, gjoin1 = nullptr;
    hipGraph_t ggraph = nullptr; hipGraphExec_t gexec = nullptr;    // grid engine: 16 iterations
    std::vector<char> gkey;
    hipGraph_t wgraph = nullptr; hipGraphExec_t wexec = nullptr;    // batched solve launch
    std::vector<char> wkey;
    // device memory taken from a caller-provided region instead of hipMalloc
    // (the allocation-free entry point): no buffer is freed, no event or graph
    // is created, launches go straight to the stream
    unsigned char* carve_base = nullptr;
    size_t carve_off = 0, carve_cap = 0;
    bool noalloc = false;
};

// Device buffer for a handle: hipMalloc, or the next 256-byte aligned slice of
// the handle's carve region.
static hipError_t dev_alloc(abip_work* w, void** p, size_t bytes) {
    if (!w->noalloc) return hipMalloc(p, bytes);
    const size_t off = (w->carve_off + 255) & ~(size_t)255;
    if (off + bytes > w->carve_cap) return hipErrorOutOfMemory;
    *p = w->carve_base + off;
    w->carve_off = off + bytes;
    return hipSuccess;
}

static void release(abip_work* w) {
    if (!w) return;
    if (w->noalloc) return;        // carved buffers belong to the region; nothing else was created
    (void)hipFree(w->ddesc); (void)hipFree(w->dctrl);
    (void)hipFree(w->A64); (void)hipFree(w->A32); (void)hipFree(w->G64); (void)hipFree(w->G32);
    (void)hipFree(w->Mv); (void)hipFree(w->Nv);
    (void)hipFree(w->order); (void)hipFree(w->queue); (void)hipFree(w->errflag); (void)hipFree(w->outp);
    (void)hipFree(w->rchk);
    (void)hipFree(w->suW); (void)hipFree(w->suoW); (void)hipFree(w->suL); (void)hipFree(w->suoL);
    (void)hipFree(w->suB); (void)hipFree((void*)w->suA); (void)hipFree((void*)w->sub); (void)hipFree((void*)w->suc);
    (void)hipFree(w->keep.L64); (void)hipFree(w->keep.Lt64); (void)hipFree(w->keep.L32); (void)hipFree(w->keep.Lt32);
    (void)hipFree(w->keep.Li64); (void)hipFree(w->keep.Lit64); (void)hipFree(w->keep.Li32); (void)hipFree(w->keep.Lit32);
    (void)hipFree(w->adj_ws); (void)hipFree(w->adj_ows); (void)hipFree(w->adj_ptrs);
    (void)hipFree(w->adj_iters); (void)hipFree(w->adj_resid);
    (void)hipFree(w->big_ws); (void)hipFree(w->sp_abak);
    (void)hipFree(w->gbuf); (void)hipFree(w->gctl);
    (void)hipFree(w->sp_idx); (void)hipFree(w->sp_val); (void)hipFree(w->sp_vec);
    (void)hipFree(w->sp_grp); (void)hipFree(w->sp_gci); (void)hipFree(w->sp_gva);
    (void)hipFree(w->sp_bar); (void)hipFree(w->sp_err); (void)hipFree(w->sp_cgit);
    if (w->gexec) (void)hipGraphExecDestroy(w->gexec);
    if (w->ggraph) (void)hipGraphDestroy(w->ggraph);
    if (w->wexec) (void)hipGraphExecDestroy(w->wexec);
    if (w->wgraph) (void)hipGraphDestroy(w->wgraph);
    if (w->gjoin0) (void)hipEventDestroy(w->gjoin0);
    if (w->gjoin1) (void)hipEventDestroy(w->gjoin1);
    if (w->gstream) (void)hipStreamDestroy(w->gstream);
    if (w->ev0) (void)hipEventDestroy(w->ev0);
    if (w->ev1) (void)hipEventDestroy(w->ev1);
}

extern "C" int abip_default_settings(abip_settings* s) {
    if (!s) return fail(ABIP_E_INVALID, "abip_default_settings: null pointer");
    memset(s, 0, sizeof *s);
    s->eps = 1e-6;
    s->alpha = 1.8;
    s->beta = 1.0;
    s->gamma = 0.5;
    s->max_admm_iters = 1000000;
    s->restart_rule = ABIP_RESTART_HEURISTIC;
    s->precision = ABIP_PREC_FP64;
    s->lin_solver = ABIP_LIN_AUTO;
    s->engine = ABIP_ENGINE_AUTO;
    s->fp32_max_iters = 1000000;
    s->cg_tol = 1e-7;
    s->cg_max_iters = 500;
    s->block_threads = 0;
    s->adjoint_tol = 1e-12;
    s->adjoint_max_iters = 200000;
    s->cg_rule = 0;
    s->use_graph = 1;
    s->lds_resident = 1;
    s->bb = 0;
    s->bb_max_redo = 10;
    s->bb_eps_cor = 0.2;
    s->bb_eps_penalty = 0.1;
    s->scale_iters = 0;
    s->sparse_gram = 0;
    s->grid_mirror = 1;
    return ABIP_OK;
}

static int check_settings(const abip_settings& s) {
    if (!(s.eps > 0.0) || !std::isfinite(s.eps)) return fail(ABIP_E_INVALID, "settings.eps must be > 0");
    if (!(s.alpha > 0.0 && s.alpha < 2.0)) return fail(ABIP_E_INVALID, "settings.alpha must lie in (0,2)");
    if (!(s.beta > 0.0) || !std::isfinite(s.beta)) return fail(ABIP_E_INVALID, "settings.beta must be > 0");
    if (!(s.gamma > 0.0 && s.gamma < 1.0)) return fail(ABIP_E_INVALID, "settings.gamma must lie in (0,1)");
    if (s.max_admm_iters < 0) return fail(ABIP_E_INVALID, "settings.max_admm_iters must be >= 0");
    if (s.restart_rule != ABIP_RESTART_HEURISTIC && s.restart_rule != ABIP_RESTART_SQRT)
        return fail(ABIP_E_INVALID, "settings.restart_rule: unknown value %d", s.restart_rule);
    if (s.precision != ABIP_PREC_FP64 && s.precision != ABIP_PREC_FP32_POLISH)
        return fail(ABIP_E_INVALID, "settings.precision: unknown value %d", s.precision);
    if (s.cg_rule != 0 && s.cg_rule != 1) return fail(ABIP_E_INVALID, "settings.cg_rule must be 0 or 1");
    if (s.use_graph != 0 && s.use_graph != 1) return fail(ABIP_E_INVALID, "settings.use_graph must be 0 or 1");
    if (s.lds_resident != 0 && s.lds_resident != 1) return fail(ABIP_E_INVALID, "settings.lds_resident must be 0 or 1");
    if (s.block_threads != 0 && s.block_threads != 256 && s.block_threads != 512)
        return fail(ABIP_E_INVALID, "settings.block_threads must be 0, 256 or 512");
    if (s.bb != 0 && s.bb != 1) return fail(ABIP_E_INVALID, "settings.bb must be 0 or 1");
    if (s.bb_max_redo < 0) return fail(ABIP_E_INVALID, "settings.bb_max_redo must be >= 0");
    if (!(s.bb_eps_cor >= 0.0 && s.bb_eps_cor < 1.0))
        return fail(ABIP_E_INVALID, "settings.bb_eps_cor must lie in [0,1)");
    if (!(s.bb_eps_penalty >= 0.0) || !std::isfinite(s.bb_eps_penalty))
        return fail(ABIP_E_INVALID, "settings.bb_eps_penalty must be >= 0");
    if (s.scale_iters < 0 || s.scale_iters > 100) return fail(ABIP_E_INVALID, "settings.scale_iters must lie in [0,100]");
    if (s.sparse_gram != 0 && s.sparse_gram != 1) return fail(ABIP_E_INVALID, "settings.sparse_gram must be 0 or 1");
    if (s.grid_mirror != 0 && s.grid_mirror != 1) return fail(ABIP_E_INVALID, "settings.grid_mirror must be 0 or 1");
    if (s.lin_solver < ABIP_LIN_AUTO || s.lin_solver > ABIP_LIN_TRSV)
        return fail(ABIP_E_INVALID, "settings.lin_solver: unknown value %d", s.lin_solver);
    if (s.lin_solver == ABIP_LIN_TRSV && s.bb)
        return fail(ABIP_E_INVALID, "settings.lin_solver = ABIP_LIN_TRSV does not combine with settings.bb");
    return ABIP_OK;
}

static SolveParams make_params(const abip_settings& s) {
    SolveParams p;
    memset(&p, 0, sizeof p);
    p.eps = s.eps; p.alpha = s.alpha; p.beta = s.beta; p.gamma = s.gamma;
    p.eps_cor = s.bb_eps_cor; p.eps_pen = s.bb_eps_penalty;
    p.bb = s.bb; p.bb_max_redo = s.bb_max_redo;
    p.trsv = (s.lin_solver == ABIP_LIN_TRSV) ? 1 : 0;
    p.max_iters = s.max_admm_iters;
    p.fp32_max_iters = (s.precision == ABIP_PREC_FP32_POLISH) ? s.fp32_max_iters : 0;
    p.restart_rule = s.restart_rule;
    p.precision = s.precision;
    return p;
}

static double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

static const int MAX_WG_M = 1024;   // largest m the one-workgroup engine holds per lane
static const int MAX_GRID_M = 8192; // 4 row chunks of 256 per wave, 8 waves
static const int64_t GRID_AUTO_MN = 4 * 1024 * 1024;   // one LP this large goes to the grid engine

// Column / row split of the grid engine for about `wgs` workgroups per kernel
// (columns per workgroup a multiple of 8); the partial buffers are sized for
// up to 4 workgroups per CU.
static void grid_config(abip_work* w, int wgs) {
    const LPDesc& d = w->hdesc[0];
    GridArgs& g = w->ga;
    const int cap = 4 * w->cu_count;
    wgs = std::max(1, std::min(wgs, cap));
    const int ncol = w->grid_pairs > 0 ? w->grid_pairs : d.n;   // the column pass walks pairs when paired
    int cw = (ncol + wgs - 1) / wgs;
    cw = ((cw + 7) / 8) * 8;
    g.cw = cw;
    g.NB = (ncol + cw - 1) / cw;
    g.n2 = w->grid_pairs;
    g.NR = (d.ld + GRID_RED_ROWS - 1) / GRID_RED_ROWS;   // workgroups of k_grid_red
    int gw = (d.m + wgs - 1) / wgs;
    gw = ((gw + 7) / 8) * 8;
    g.gw = gw;
    g.NG = (d.m + gw - 1) / gw;
    double* p = w->gbuf;
    g.Y2 = p; p += 2 * d.ld;
    g.Pf = p; p += (int64_t)cap * d.ld;
    g.Px = p; p += (int64_t)cap * d.ld;
    g.pcol = p; p += 16 * (int64_t)cap;
    g.pcol_stride = 8 * cap;
    g.prow = p; p += 8 * (int64_t)g.NR;
    g.pa = p; p += 4 * (int64_t)cap;
    g.t = p; p += d.ld;
    g.a = p; p += d.ld;
    w->grid_wgs = wgs;
}

static int grid_prepare(abip_work* w) {
    const LPDesc& d = w->hdesc[0];
    GridArgs& g = w->ga;
    g.m = d.m; g.n = d.n; g.ld = d.ld;
    w->grid_nchw = grid_nchw(d.ld);
    const int64_t cap = 4 * (int64_t)w->cu_count;
    const int64_t nbuf = 2 * (int64_t)d.ld + 2 * cap * d.ld + 16 * cap +
                         8 * (int64_t)((d.ld + GRID_RED_ROWS - 1) / GRID_RED_ROWS) + 4 * cap + 2 * (int64_t)d.ld;
    HIPCHK(hipMalloc((void**)&w->gbuf, sizeof(double) * nbuf));
    HIPCHK(hipMalloc((void**)&w->gctl, sizeof(GridCtl) * 3));   // ctl, ctl_next, then the GridBB record
    grid_config(w, w->cu_count);
    // k_grid_col reads at most two partial sums per thread of each kernel (2 x 512 workgroups)
    if (g.NR > 1024 || 4 * w->cu_count > 1024)
        return fail(ABIP_E_INVALID, "grid engine: %d rows or %d compute units exceed its partial-sum layout", d.m, w->cu_count);
    g.A64 = w->A64 + d.oA; g.A32 = w->A32 + d.oA;
    g.G64 = w->G64 + d.oG; g.G32 = w->G32 + d.oG;
    g.b = w->Mv + MF_B * w->Mtot + d.om; g.bbar = w->Mv + MF_BBAR * w->Mtot + d.om;
    g.Ac = w->Mv + MF_AC * w->Mtot + d.om; g.Acb = w->Mv + MF_ACBAR * w->Mtot + d.om;
    g.Zy0 = w->Mv + MF_ZY0 * w->Mtot + d.om; g.Zy1 = w->Mv + MF_ZY1 * w->Mtot + d.om;
    g.C = w->Nv + NF_C * w->Ntot + d.on; g.CB = w->Nv + NF_CBAR * w->Ntot + d.on;
    g.Zx0 = w->Nv + NF_ZX0 * w->Ntot + d.on; g.Zx1 = w->Nv + NF_ZX1 * w->Ntot + d.on;
    g.X = w->Nv + NF_X * w->Ntot + d.on; g.S = w->Nv + NF_S * w->Ntot + d.on;
    g.X0 = w->Nv + NF_BBX0 * w->Ntot + d.on; g.S0 = w->Nv + NF_BBS0 * w->Ntot + d.on;
    g.X1 = w->Nv + NF_BBX1 * w->Ntot + d.on; g.S1 = w->Nv + NF_BBS1 * w->Ntot + d.on;
    g.Y0 = w->Mv + MF_BBY0 * w->Mtot + d.om; g.Y1 = w->Mv + MF_BBY1 * w->Mtot + d.om;
    g.ctl = w->gctl; g.ctl_next = w->gctl + 1;
    static_assert(sizeof(GridBB) <= sizeof(GridCtl), "GridBB fits the third slot");
    g.bb = reinterpret_cast<GridBB*>(w->gctl + 2);
    g.lc = w->dctrl;
    return ABIP_OK;
}

// Private capture stream (default priority) and the events that join it to
// the caller's stream, created on first use.
static int graph_stream(abip_work* w) {
    if (!w->gstream) HIPCHK(hipStreamCreateWithFlags(&w->gstream, hipStreamNonBlocking));
    if (!w->gjoin0) HIPCHK(hipEventCreateWithFlags(&w->gjoin0, hipEventDisableTiming));
    if (!w->gjoin1) HIPCHK(hipEventCreateWithFlags(&w->gjoin1, hipEventDisableTiming));
    return ABIP_OK;
}

template <typename T>
static std::vector<char> key_bytes(const T& v, int extra) {
    std::vector<char> k(sizeof(T) + sizeof(int));
    memcpy(k.data(), &v, sizeof(T));
    memcpy(k.data() + sizeof(T), &extra, sizeof(int));
    return k;
}

// Capture `body` (stream launches only: no memsets, no host copies) into *graph /
// *exec on the private stream, unless the key matches the cached capture.
template <typename F>
static int capture_graph(abip_work* w, hipGraph_t* graph, hipGraphExec_t* exec, std::vector<char>* cached,
                         const std::vector<char>& key, F body) {
    if (*exec && *cached == key) return ABIP_OK;
    if (*exec) { (void)hipGraphExecDestroy(*exec); *exec = nullptr; }
    if (*graph) { (void)hipGraphDestroy(*graph); *graph = nullptr; }
    HIPCHK(hipStreamBeginCapture(w->gstream, hipStreamCaptureModeThreadLocal));
    const hipError_t eb = body(w->gstream);
    hipGraph_t gr = nullptr;
    const hipError_t ee = hipStreamEndCapture(w->gstream, &gr);
    if (eb != hipSuccess) { if (gr) (void)hipGraphDestroy(gr); return fail(ABIP_E_HIP, "graph capture: %s", hipGetErrorString(eb)); }
    if (ee != hipSuccess) return fail(ABIP_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(ee));
    *graph = gr;
    HIPCHK(hipGraphInstantiate(exec, gr, nullptr, nullptr, 0));
    *cached = key;
    return ABIP_OK;
}

static const int GRAPH_ITERS = 16;   // grid-engine iterations per captured graph

// Drive the grid engine: chunks of iterations, then a look at the status.
static int grid_run(abip_work* w, int64_t fixed, int phase) {
    hipStream_t st = w->stream;
    GridArgs g;
    memset(&g, 0, sizeof g);                  // padding bytes take part in the graph key
    g = w->ga;
    g.prm = make_params(w->set);
    if (fixed > 0) {
        const LPDesc& d0 = w->hdesc[0];
        hipLaunchKernelGGL(k_grid_from_state, dim3(16), dim3(256), 0, st, g, w->Mv + MF_Y * w->Mtot + d0.om,
                           w->dctrl, phase, fixed);
    } else {
        hipLaunchKernelGGL(k_grid_init, dim3(64), dim3(256), 0, st, g, w->set.beta, phase, fixed, w->set.bb);
    }
    HIPCHK(hipGetLastError());
    if (!w->ev0) HIPCHK(hipEventCreate(&w->ev0));
    if (!w->ev1) HIPCHK(hipEventCreate(&w->ev1));
    HIPCHK(hipEventRecord(w->ev0, st));
    GridCtl hc;
    if (w->set.use_graph) {
        // the iteration kernels take the same arguments every time (state lives in
        // the device control block): 16 iterations as one graph, replayed
        int rc = graph_stream(w);
        if (rc) return rc;
        const int nchw = w->grid_nchw;
        rc = capture_graph(w, &w->ggraph, &w->gexec, &w->gkey, key_bytes(g, nchw), [&](hipStream_t cs) {
            for (int i = 0; i < GRAPH_ITERS; ++i) {
                const hipError_t e = grid_launch_iteration(nchw, g, cs);
                if (e != hipSuccess) return e;
            }
            return hipSuccess;
        });
        if (rc) return rc;
        int reps = 1;
        while (true) {
            HIPCHK(hipEventRecord(w->gjoin0, st));
            HIPCHK(hipStreamWaitEvent(w->gstream, w->gjoin0, 0));
            for (int r = 0; r < reps; ++r) HIPCHK(hipGraphLaunch(w->gexec, w->gstream));
            HIPCHK(hipEventRecord(w->gjoin1, w->gstream));
            HIPCHK(hipStreamWaitEvent(st, w->gjoin1, 0));
            HIPCHK(hipMemcpyAsync(&hc, w->gctl + 1, sizeof hc, hipMemcpyDeviceToHost, st));   // the decision
            HIPCHK(hipStreamSynchronize(st));
            if (hc.status == -2) {             // paused for a beta step the iterations did not take
                hipLaunchKernelGGL(k_grid_bb_step, dim3(1), dim3(1024), 0, st, g);
                HIPCHK(hipGetLastError());
                reps = 1;
                continue;
            }
            if (hc.status != 0) break;
            if (reps < 16) reps *= 2;
        }
    } else {
        int chunk = 16;
        while (true) {
            for (int i = 0; i < chunk; ++i) HIPCHK(grid_launch_iteration(w->grid_nchw, g, st));
            HIPCHK(hipMemcpyAsync(&hc, w->gctl + 1, sizeof hc, hipMemcpyDeviceToHost, st));   // the decision
            HIPCHK(hipStreamSynchronize(st));
            if (hc.status == -2) {             // paused for a beta step the iterations did not take
                hipLaunchKernelGGL(k_grid_bb_step, dim3(1), dim3(1024), 0, st, g);
                HIPCHK(hipGetLastError());
                chunk = 16;
                continue;
            }
            if (hc.status != 0) break;
            if (chunk < 256) chunk *= 2;
        }
    }
    HIPCHK(hipEventRecord(w->ev1, st));
    const LPDesc& d = w->hdesc[0];
    hipLaunchKernelGGL(k_grid_finish, dim3(1), dim3(256), 0, st, g, w->Mv + MF_Y * w->Mtot + d.om, w->dctrl);
    HIPCHK(hipGetLastError());
    return ABIP_OK;
}

// Which phases of which LPs run LDS-resident, and the LDS bytes of the batched
// launch: with 256 threads per workgroup an LP qualifies when m <= 256,
// n <= 512 and, in that phase's precision, its A and G^{-1} fit in one
// workgroup's LDS (DESC_LDS32/64: no global memory traffic per iteration) or A
// alone fits (DESC_LDSA32/64: G^{-1} is read from the pool on every pass).
// The launch then reserves the largest such footprint.
static void assign_lds(abip_work* w) {
    const int W = w->threads / 64;
    size_t smem = wg_smem_bytes(w->ldmax, W);
    const size_t cap = (w->lds_cap > 1024) ? (size_t)w->lds_cap - 1024 : 0;   // static LDS of the kernel
    for (size_t k = 0; k < w->hdesc.size(); ++k) {
        LPDesc& d = w->hdesc[k];
        d.lds = 0;
        if (!w->set.lds_resident || w->grid || w->sparse || w->threads != 256) continue;
        if (w->set.lin_solver == ABIP_LIN_TRSV) continue;     // the LDS-resident loop multiplies by G^{-1}
        if (w->lds_policy == 2 || (k < w->lds_stream.size() && w->lds_stream[k])) continue;
        if (d.m > w->threads || d.n > 2 * w->threads) continue;
        const size_t b32 = (size_t)small_layout(d.m, d.n, 4, W).total;
        const size_t b64 = (size_t)small_layout(d.m, d.n, 8, W).total;
        const size_t a32 = (size_t)small_layout(d.m, d.n, 4, W, true).total;
        const size_t a64 = (size_t)small_layout(d.m, d.n, 8, W, true).total;
        const bool aonly = w->lds_policy == 0;
        if (b32 <= cap) { d.lds |= DESC_LDS32; smem = std::max(smem, b32); }
        else if (aonly && a32 <= cap) { d.lds |= DESC_LDSA32; smem = std::max(smem, a32); }
        if (b64 <= cap) { d.lds |= DESC_LDS64; smem = std::max(smem, b64); }
        else if (aonly && a64 <= cap) { d.lds |= DESC_LDSA64; smem = std::max(smem, a64); }
    }
    w->wg_smem = smem;
}

static int load_dense(abip_work* w, const abip_matrix* A, const double* const* b, const double* const* c);

// carve: when not null, every device buffer of the handle comes from this
// region of carve_cap bytes (no hipMalloc) and the handle creates no events or
// graphs (the allocation-free entry point).
static int setup_dense(abip_work** out, int32_t B, const abip_matrix* A, const double* const* b,
                       const double* const* c, const abip_settings* settings, void* stream,
                       unsigned char* carve = nullptr, size_t carve_cap = 0) {
    if (!out) return fail(ABIP_E_INVALID, "abip_setup: null output handle");
    *out = nullptr;
    if (B < 1) return fail(ABIP_E_DIM, "abip_setup_batch: B must be >= 1 (got %d)", B);
    if (!A || !b || !c) return fail(ABIP_E_INVALID, "abip_setup: null A, b or c");
    abip_settings s;
    if (settings) s = *settings; else abip_default_settings(&s);
    int rc = check_settings(s);
    if (rc) return rc;
    const double t0 = now_ms();
    abip_work* w = new abip_work();
    if (carve) {
        w->noalloc = true;
        w->carve_base = carve;
        w->carve_cap = carve_cap;
        s.use_graph = 0;
    }
    w->B = B;
    w->set = s;
    w->stream = (hipStream_t)stream;
    w->hdesc.resize(B);
    int64_t oA = 0, oG = 0, om = 0, on = 0;
    for (int k = 0; k < B; ++k) {
        const abip_matrix& M = A[k];
        if (M.format != ABIP_DENSE_ROWMAJOR) { delete w; return fail(ABIP_E_INVALID, "LP %d: only dense row-major A is supported by this entry point", k); }
        if (M.m < 1 || M.n < 1) { delete w; return fail(ABIP_E_DIM, "LP %d: bad dimensions m=%d n=%d", k, M.m, M.n); }
        const bool want_grid = (B == 1) && (s.engine == ABIP_ENGINE_GRID ||
                                            (s.engine == ABIP_ENGINE_AUTO &&
                                             (M.m > MAX_WG_M || (int64_t)M.m * M.n >= GRID_AUTO_MN)));
        if (want_grid) w->grid = true;
        if (want_grid && s.lin_solver == ABIP_LIN_TRSV) { delete w; return fail(ABIP_E_INVALID, "settings.lin_solver = ABIP_LIN_TRSV runs in the one-workgroup engine only (this LP takes the grid engine)"); }
        if (want_grid && M.m > MAX_GRID_M) { delete w; return fail(ABIP_E_DIM, "m=%d exceeds the grid engine limit %d", M.m, MAX_GRID_M); }
        if (!want_grid && M.m > MAX_WG_M) { delete w; return fail(ABIP_E_DIM, "LP %d: m=%d exceeds the one-workgroup engine limit %d (use abip_setup for one large LP)", k, M.m, MAX_WG_M); }
        if (!M.val || !b[k] || !c[k]) { delete w; return fail(ABIP_E_INVALID, "LP %d: null data pointer", k); }
        LPDesc& d = w->hdesc[k];
        d.m = M.m; d.n = M.n; d.ld = (M.m + 3) & ~3; d.lds = 0;
        d.oA = oA; d.oG = oG; d.om = om; d.on = on;
        oA += (int64_t)d.ld * d.n;
        oG += (int64_t)d.ld * d.m;
        om += d.ld;
        on += (d.n + 4) & ~3;          // at least one spare slot past the LP's n entries
        w->ldmax = std::max(w->ldmax, d.ld);
    }
    w->Atot = oA; w->Gtot = oG; w->Mtot = om; w->Ntot = on;
    w->nch = (w->ldmax + 255) / 256;
    // the NCH >= 2 kernels are compiled for at most 256 threads
    w->threads = (w->nch >= 2) ? 256 : (s.block_threads ? s.block_threads : 256);
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&w->cu_count, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipDeviceGetAttribute(&w->lds_cap, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    assign_lds(w);
#define ALLOC(ptr, count) do { hipError_t e_ = dev_alloc(w, (void**)&(ptr), sizeof(*(ptr)) * (size_t)(count)); \
        if (e_ != hipSuccess) { const bool nz_ = w->noalloc; release(w); delete w; return fail(e_ == hipErrorOutOfMemory ? (nz_ ? ABIP_E_DIM : ABIP_E_OOM) : ABIP_E_HIP, nz_ ? "%s (%lld elements) does not fit the scratch region" : "hipMalloc(%s, %lld elements): %s", #ptr, (long long)(count), hipGetErrorString(e_)); } } while (0)
    ALLOC(w->ddesc, B);
    ALLOC(w->dctrl, B);
    ALLOC(w->A64, oA); ALLOC(w->A32, oA);
    ALLOC(w->G64, oG); ALLOC(w->G32, oG);
    ALLOC(w->Mv, (int64_t)NMF * om); ALLOC(w->Nv, (int64_t)NNF * on);
    ALLOC(w->order, B); ALLOC(w->queue, 2); ALLOC(w->errflag, 1);     // queue[1]: abip_iterate's one-LP order
    ALLOC(w->outp, 3 * B);
    if (B == 1) {
        const int mx = std::max(w->hdesc[0].m, w->hdesc[0].n);
        w->rchk_P = std::max(1, std::min(512, (mx + 255) / 256));
    }
    ALLOC(w->rchk, (int64_t)B * w->rchk_P * 8);
    // scratch for the setup: W = L^{-1} (ld x ld per LP), the inverses of the
    // 64 x 64 diagonal blocks of L (per LP), the grid border's vectors
    std::vector<int64_t> hoW(B), hoL(B);
    int64_t wtot = 0, ltot = 0;
    int mmax = 0;
    for (int k = 0; k < B; ++k) {
        const LPDesc& d = w->hdesc[k];
        hoW[k] = wtot; wtot += (int64_t)d.ld * d.ld;
        hoL[k] = ltot; ltot += (int64_t)((d.m + 63) / 64) * 64 * 64;
        w->hdesc[k].oL = hoL[k];
        mmax = std::max(mmax, d.m);
    }
    const int64_t btot = w->grid ? std::max(grid_border_scratch(w->hdesc[0].m, w->hdesc[0].n, w->hdesc[0].ld),
                                            grid_rows_scratch(w->hdesc[0].n, w->hdesc[0].ld)) : 1;
    ALLOC(w->suW, wtot); ALLOC(w->suoW, B); ALLOC(w->suL, ltot); ALLOC(w->suoL, B); ALLOC(w->suB, btot);
    ALLOC(w->suA, B); ALLOC(w->sub, B); ALLOC(w->suc, B);
    if (s.lin_solver == ABIP_LIN_TRSV) {
        ALLOC(w->keep.L64, oG); ALLOC(w->keep.Lt64, oG); ALLOC(w->keep.L32, oG); ALLOC(w->keep.Lt32, oG);
        ALLOC(w->keep.Li64, ltot); ALLOC(w->keep.Lit64, ltot); ALLOC(w->keep.Li32, ltot); ALLOC(w->keep.Lit32, ltot);
    }
#undef ALLOC
    w->suWtot = wtot;
    w->mmax = mmax;
    hipStream_t st = w->stream;
    {
        hipError_t e1 = hipMemcpyAsync(w->suoW, hoW.data(), sizeof(int64_t) * B, hipMemcpyHostToDevice, st);
        hipError_t e2 = hipMemcpyAsync(w->suoL, hoL.data(), sizeof(int64_t) * B, hipMemcpyHostToDevice, st);
        if (e1 != hipSuccess || e2 != hipSuccess) {
            release(w); delete w;
            return fail(ABIP_E_HIP, "hipMemcpyAsync: %s", hipGetErrorString(e1 != hipSuccess ? e1 : e2));
        }
    }
    rc = load_dense(w, A, b, c);
    if (rc) { release(w); delete w; return rc; }
    hipError_t e = w->grid ? hipSuccess : set_solve_wg_smem_limit(w->wg_smem);
    if (e != hipSuccess) { release(w); delete w; return fail(ABIP_E_HIP, "hipFuncSetAttribute: %s", hipGetErrorString(e)); }
    if (w->grid) {
        int rc2 = grid_prepare(w);
        if (rc2) { release(w); delete w; return rc2; }
    }
    w->hctrl.resize(B);
    w->setup_ms = now_ms() - t0;
    *out = w;
    return ABIP_OK;
}

// Load A, b, c of every LP into a dense handle whose buffers exist and run the
// whole setup on them: copies in both precisions, HSD constants, G = I + A A^T,
// its factorization and inverse, the border.  No allocation.  Errors leave the
// handle's data undefined (the caller frees it or loads again).
static int load_dense(abip_work* w, const abip_matrix* A, const double* const* b, const double* const* c) {
    const int B = w->B;
    const int64_t oA = w->Atot, oG = w->Gtot, om = w->Mtot, on = w->Ntot;
    hipStream_t st = w->stream;
#define SCHK(call) do { hipError_t e_ = (call); if (e_ != hipSuccess) return fail(ABIP_E_HIP, "%s: %s", #call, hipGetErrorString(e_)); } while (0)
    std::vector<const double*> hA(B), hb(B), hc(B);
    for (int k = 0; k < B; ++k) { hA[k] = A[k].val; hb[k] = b[k]; hc[k] = c[k]; }
    const double** dAp = w->suA; const double** dbp = w->sub; const double** dcp = w->suc;
    SCHK(hipMemsetAsync(w->A64, 0, sizeof(double) * oA, st));
    SCHK(hipMemsetAsync(w->A32, 0, sizeof(float) * oA, st));
    SCHK(hipMemsetAsync(w->G64, 0, sizeof(double) * oG, st));
    SCHK(hipMemsetAsync(w->G32, 0, sizeof(float) * oG, st));
    SCHK(hipMemsetAsync(w->Mv, 0, sizeof(double) * NMF * om, st));
    SCHK(hipMemsetAsync(w->Nv, 0, sizeof(double) * NNF * on, st));
    SCHK(hipMemsetAsync(w->dctrl, 0, sizeof(LPCtrl) * B, st));
    SCHK(hipMemsetAsync(w->errflag, 0, sizeof(int), st));
    SCHK(hipMemcpyAsync(w->ddesc, w->hdesc.data(), sizeof(LPDesc) * B, hipMemcpyHostToDevice, st));
    SCHK(hipMemcpyAsync(dAp, hA.data(), sizeof(double*) * B, hipMemcpyHostToDevice, st));
    SCHK(hipMemcpyAsync(dbp, hb.data(), sizeof(double*) * B, hipMemcpyHostToDevice, st));
    SCHK(hipMemcpyAsync(dcp, hc.data(), sizeof(double*) * B, hipMemcpyHostToDevice, st));
    // largest first: LPT order for the persistent work queue
    std::vector<int32_t> ord(B);
    for (int k = 0; k < B; ++k) ord[k] = k;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int bb) {
        return (int64_t)w->hdesc[a].m * w->hdesc[a].n > (int64_t)w->hdesc[bb].m * w->hdesc[bb].n;
    });
    SCHK(hipMemcpyAsync(w->order, ord.data(), sizeof(int32_t) * B, hipMemcpyHostToDevice, st));
    int maxtiles = 0, maxrowblk = 0;
    for (auto& d : w->hdesc) {
        maxtiles = std::max(maxtiles, ((d.m + 63) / 64) * ((d.n + 63) / 64));
        maxrowblk = std::max(maxrowblk, (d.ld + 255) / 256);
    }
    hipLaunchKernelGGL(k_setup_copy, dim3(maxtiles, B), dim3(256), 0, st, w->ddesc, dAp, w->A64, w->A32, w->errflag);
    SCHK(hipGetLastError());
    // row / column factors of the scaled LP (all 1 unless settings.scale_iters > 0)
    hipLaunchKernelGGL(k_ruiz_init, dim3(maxrowblk + 1, B), dim3(256), 0, st, w->ddesc, w->Mv, w->Nv, w->Mtot, w->Ntot);
    SCHK(hipGetLastError());
    if (w->set.scale_iters > 0) {
        int nblk = 1;
        for (auto& d : w->hdesc) nblk = std::max(nblk, (std::max(d.m, d.n) + 255) / 256);
        for (int t = 0; t < w->set.scale_iters; ++t) {
            hipLaunchKernelGGL(k_ruiz_max, dim3(maxtiles, B), dim3(256), 0, st, w->ddesc, w->A64, w->Mv, w->Nv,
                               w->Mtot, w->Ntot);
            SCHK(hipGetLastError());
            hipLaunchKernelGGL(k_ruiz_apply, dim3(nblk, B), dim3(256), 0, st, w->ddesc, w->Mv, w->Nv, w->Mtot,
                               w->Ntot);
            SCHK(hipGetLastError());
        }
        hipLaunchKernelGGL(k_ruiz_scale, dim3(maxtiles, B), dim3(256), 0, st, w->ddesc, w->A64, w->A32, w->Mv,
                           w->Nv, w->Mtot, w->Ntot);
        SCHK(hipGetLastError());
    }
    hipLaunchKernelGGL(k_setup_rows, dim3(maxrowblk, B), dim3(256), 0, st, w->ddesc, dbp, dcp, w->A64, w->Mv, w->Nv,
                       w->Mtot, w->Ntot, w->errflag, w->grid ? 0 : 1);
    SCHK(hipGetLastError());
    if (w->grid) {     // one large LP: its row sums over column chunks, on every CU
        const LPDesc& d0 = w->hdesc[0];
        const int nch = (d0.n + ROWS_CW - 1) / ROWS_CW;
        hipLaunchKernelGGL(k_setup_rows_part, dim3((d0.m + 255) / 256, nch), dim3(256), 0, st, w->ddesc, dcp,
                           w->A64, w->Nv, w->Ntot, ROWS_CW, w->suB);
        SCHK(hipGetLastError());
        hipLaunchKernelGGL(k_setup_rows_fin, dim3((d0.ld + 255) / 256), dim3(256), 0, st, w->ddesc, dbp, w->suB, nch,
                           w->Mv, w->Mtot, w->errflag);
        SCHK(hipGetLastError());
    }
    // G = I + A A^T, its Cholesky factor and G^{-1} on the matrix cores (every LP at once)
    SCHK(factor_ginv(w->ddesc, B, w->mmax, w->A64, w->G64, w->G32, w->suL, w->suoL, w->suW, w->suoW, w->errflag,
                     w->keep.L64 ? &w->keep : nullptr, st));
    if (w->grid) {
        // one large LP: the border's products over the whole GPU
        SCHK(grid_border(w->hdesc[0], w->ddesc, w->A64, w->G64, w->Mv, w->Nv, w->Mtot, w->Ntot, w->dctrl, w->suB,
                         st));
    } else {
        for (int sgn = 1; sgn >= -1; sgn -= 2) {
            hipLaunchKernelGGL(k_setup_border, dim3(B), dim3(512), sizeof(double) * 2 * w->ldmax, st, w->ddesc,
                               w->A64, w->G64, w->Mv, w->Nv, w->Mtot, w->Ntot, w->dctrl, sgn);
            SCHK(hipGetLastError());
        }
    }
    // one large LP with an even column count: is A = [A0, -A0]? (bit 16 when not)
    const bool pair_test = w->grid && w->set.grid_mirror && w->hdesc[0].n % 2 == 0;
    if (pair_test) {
        const LPDesc& d0 = w->hdesc[0];
        hipLaunchKernelGGL(k_grid_pair_check, dim3(d0.n / 2), dim3(256), 0, st, w->A64 + d0.oA, d0.m, d0.ld,
                           d0.n / 2, w->errflag);
        SCHK(hipGetLastError());
    }
    int hflag = 0;
    SCHK(hipMemcpyAsync(&hflag, w->errflag, sizeof(int), hipMemcpyDeviceToHost, st));
    SCHK(hipStreamSynchronize(st));
#undef SCHK
    if (hflag & 3) return fail(ABIP_E_NONFINITE, "NaN or Inf in %s", (hflag & 1) ? "A" : "b or c");
    if (hflag & 4) return fail(ABIP_E_HIP, "Cholesky of I + A A^T met a non-positive pivot");
    w->grid_pairs = (pair_test && !(hflag & 16)) ? w->hdesc[0].n / 2 : 0;
    w->solved = false;
    return ABIP_OK;
}

// ---------------------------------------------------------------------------
// sparse engine: setup and run
// ---------------------------------------------------------------------------
static int lanes_for(double avg) {           // lanes per CSR row: about 4 entries per lane (one gather round)
    int L = 1;
    while (L < 64 && 4.0 * L < avg) L *= 2;
    return L;
}

// Dynamic LDS of a launch of nb workgroups: enough for the largest slices
// that fit (a workgroup whose slices do not fit runs the global-memory
// passes); 0 when none fits or the launch would not be co-resident with it.
static int sp_lds_for(const abip_work* w, int nb) {
    const SpArgs& g = w->sa;
    if (w->sp_lds_cap <= 0 || w->sp_hrp.empty() || w->sp_hrpt.empty()) return 0;
    int64_t need = 0;
    for (int b = 0; b < nb; ++b) {
        int rlo, rhi, clo, chi;
        sp_share(g.m, b, nb, &rlo, &rhi);
        sp_share(g.n, b, nb, &clo, &chi);
        const int64_t by = sp_slice_bytes(chi - clo, w->sp_hrpt[chi] - w->sp_hrpt[clo], rhi - rlo,
                                          w->sp_hrp[rhi] - w->sp_hrp[rlo]);
        if (by <= w->sp_lds_cap) need = std::max(need, by);
    }
    if (need == 0) return 0;
    const int bytes = (int)std::min<int64_t>(w->sp_lds_cap, (need + 255) & ~(int64_t)255);
    if (nb > sp_max_blocks(w->cu_count, bytes)) return 0;
    return bytes;
}

static double host_sum(const std::vector<double>& v, int k, int nblk) {
    double s = 0.0;
    for (int i = 0; i < nblk; ++i) s += v[(size_t)k * nblk + i];
    return s;
}

static int setup_sparse(abip_work** out, const abip_matrix* A, const double* b, const double* c,
                        const abip_settings* settings, void* stream) {
    *out = nullptr;
    abip_settings s;
    if (settings) s = *settings; else abip_default_settings(&s);
    int rc = check_settings(s);
    if (rc) return rc;
    const int32_t m = A->m, n = A->n;
    const int64_t nnz = A->nnz;
    if (m < 1 || n < 1) return fail(ABIP_E_DIM, "CSR: bad dimensions m=%d n=%d", m, n);
    if (nnz < 0 || nnz > (int64_t)INT32_MAX) return fail(ABIP_E_DIM, "CSR: nnz=%lld out of range", (long long)nnz);
    if (!A->rowptr || (nnz > 0 && (!A->colidx || !A->val)) || !b || !c)
        return fail(ABIP_E_INVALID, "CSR: null rowptr / colidx / val / b / c");
    if (!(s.cg_tol > 0.0) || s.cg_max_iters < 1) return fail(ABIP_E_INVALID, "settings: cg_tol > 0 and cg_max_iters >= 1 required");
    if (s.scale_iters) return fail(ABIP_E_INVALID, "settings.scale_iters: scaling is implemented for dense A only");
    if (s.lin_solver == ABIP_LIN_TRSV) return fail(ABIP_E_INVALID, "settings.lin_solver = ABIP_LIN_TRSV needs dense A");
    const double t0 = now_ms();
    abip_work* w = new abip_work();
    w->B = 1;
    w->set = s;
    w->set.precision = ABIP_PREC_FP64;        // the CG path runs in FP64
    w->stream = (hipStream_t)stream;
    w->sparse = true;
    w->hdesc.resize(1);
    LPDesc& d = w->hdesc[0];
    d.m = m; d.n = n; d.ld = (m + 3) & ~3; d.lds = 0; d.oA = 0; d.oG = 0; d.om = 0; d.on = 0; d.oL = 0;
    w->ldmax = d.ld;
    w->Mtot = d.ld;
    w->Ntot = (n + 4) & ~3;
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&w->cu_count, hipDeviceAttributeMultiprocessorCount, dev);
    hipStream_t st = w->stream;
    double* dpart = nullptr;
    const double** dptrs = nullptr;
    auto bail = [&](int code) { (void)hipFree(dpart); (void)hipFree(dptrs); dpart = nullptr; dptrs = nullptr;
                                release(w); delete w; return code; };
#define SALLOC(ptr, count) do { hipError_t e_ = hipMalloc((void**)&(ptr), sizeof(*(ptr)) * (size_t)(count)); \
        if (e_ != hipSuccess) return bail(fail(e_ == hipErrorOutOfMemory ? ABIP_E_OOM : ABIP_E_HIP, "hipMalloc(%s): %s", #ptr, hipGetErrorString(e_))); } while (0)
#define SCHK(call) do { hipError_t e_ = (call); if (e_ != hipSuccess) return bail(fail(ABIP_E_HIP, "%s: %s", #call, hipGetErrorString(e_))); } while (0)
    const int64_t nidx = (int64_t)(m + 1) + nnz + (n + 1) + nnz + n;
    const int NBLK = 64;
    const int64_t nvec = 12 * (int64_t)d.ld + 5 * (int64_t)w->Ntot + (int64_t)SP_PS * 4 * w->cu_count;
    SALLOC(w->ddesc, 1); SALLOC(w->dctrl, 1);
    SALLOC(w->Mv, (int64_t)NMF * w->Mtot); SALLOC(w->Nv, (int64_t)NNF * w->Ntot);
    SALLOC(w->errflag, 1); SALLOC(w->outp, 3);
    w->rchk_P = std::max(1, std::min(1024, (std::max(m, n) + 255) / 256));
    SALLOC(w->rchk, (int64_t)w->rchk_P * 8);
    SALLOC(w->sp_idx, nidx); SALLOC(w->sp_val, 2 * std::max<int64_t>(nnz, 1));
    SALLOC(w->sp_vec, nvec);
    SALLOC(w->sp_bar, 2); SALLOC(w->sp_err, 1); SALLOC(w->sp_cgit, 1);
    SALLOC(dpart, 8 * NBLK);
    SALLOC(dptrs, 8);
    auto freetmp = [&]() { (void)hipFree(dpart); (void)hipFree(dptrs); dpart = nullptr; dptrs = nullptr; };
    SpArgs& g = w->sa;
    g.m = m; g.n = n; g.nnz = nnz;
    int32_t* rp = w->sp_idx;
    int32_t* ci = rp + (m + 1);
    int32_t* rpt = ci + nnz;
    int32_t* cit = rpt + (n + 1);
    int32_t* cursor = cit + nnz;
    double* va = w->sp_val;
    double* vat = va + nnz;
    g.rp = rp; g.ci = ci; g.va = va; g.rpt = rpt; g.cit = cit; g.vat = vat;
    double* V = w->sp_vec;
    double* dG = V; V += d.ld;
    g.a = V; V += d.ld; g.z = V; V += d.ld; g.p = V; V += d.ld;
    g.rw = reinterpret_cast<SpRow*>(V); V += 4 * (int64_t)d.ld;     // 32-byte records (ld is a multiple of 4)
    g.rw2 = reinterpret_cast<SpRow*>(V); V += 4 * (int64_t)d.ld;
    g.grp = nullptr; g.gci = nullptr; g.gva = nullptr; g.LG = 1;
    double* ATZy0 = V; V += w->Ntot;
    double* ATZy1 = V; V += w->Ntot;
    g.ATY = V; V += w->Ntot; g.ATA = V; V += w->Ntot; g.q1 = V; V += w->Ntot;
    g.part = V; V += (int64_t)SP_PS * 4 * w->cu_count;          // partial sums of up to 4 workgroups per CU
    g.nbp = 4 * w->cu_count;
    g.lds_bytes = 0;
    g.dG = dG; g.ATZy0 = ATZy0; g.ATZy1 = ATZy1;
    double* Mv = w->Mv;
    double* Nv = w->Nv;
    double* fb = Mv + MF_B * w->Mtot;  double* fbb = Mv + MF_BBAR * w->Mtot;
    double* fAc = Mv + MF_AC * w->Mtot; double* fAcb = Mv + MF_ACBAR * w->Mtot;
    double* fZy0 = Mv + MF_ZY0 * w->Mtot; double* fZy1 = Mv + MF_ZY1 * w->Mtot;
    double* fC = Nv + NF_C * w->Ntot; double* fCB = Nv + NF_CBAR * w->Ntot;
    double* fZx0 = Nv + NF_ZX0 * w->Ntot; double* fZx1 = Nv + NF_ZX1 * w->Ntot;
    g.b = fb; g.bbar = fbb; g.Ac = fAc; g.Acb = fAcb; g.Zy0 = fZy0; g.Zy1 = fZy1;
    g.C = fC; g.CB = fCB; g.Zx0 = fZx0; g.Zx1 = fZx1;
    g.Y = Mv + MF_Y * w->Mtot; g.X = Nv + NF_X * w->Ntot; g.S = Nv + NF_S * w->Ntot;
    g.Y0 = Mv + MF_BBY0 * w->Mtot; g.X0 = Nv + NF_BBX0 * w->Ntot; g.S0 = Nv + NF_BBS0 * w->Ntot;
    g.Y1 = Mv + MF_BBY1 * w->Mtot; g.X1 = Nv + NF_BBX1 * w->Ntot; g.S1 = Nv + NF_BBS1 * w->Ntot;
    g.bar = w->sp_bar; g.err = w->sp_err; g.lc = w->dctrl;
    g.LA = lanes_for((double)nnz / m);
    g.LT = lanes_for((double)nnz / n);
    SCHK(hipMemsetAsync(w->Mv, 0, sizeof(double) * NMF * w->Mtot, st));
    SCHK(hipMemsetAsync(w->Nv, 0, sizeof(double) * NNF * w->Ntot, st));
    SCHK(hipMemsetAsync(w->sp_vec, 0, sizeof(double) * nvec, st));
    SCHK(hipMemsetAsync(w->dctrl, 0, sizeof(LPCtrl), st));
    SCHK(hipMemsetAsync(w->errflag, 0, sizeof(int), st));
    SCHK(hipMemsetAsync(w->sp_bar, 0, 2 * sizeof(unsigned), st));
    SCHK(hipMemsetAsync(w->sp_err, 0, sizeof(int), st));
    SCHK(hipMemcpyAsync(w->ddesc, &d, sizeof d, hipMemcpyHostToDevice, st));
    // scaling factors D = E = 1 (a CSR LP is not scaled): the output and recheck
    // kernels apply them
    hipLaunchKernelGGL(k_ruiz_init, dim3((std::max(d.ld, n) + 255) / 256, 1), dim3(256), 0, st, w->ddesc, w->Mv, w->Nv,
                       w->Mtot, w->Ntot);
    SCHK(hipGetLastError());
    SCHK(hipMemcpyAsync(rp, A->rowptr, sizeof(int32_t) * (size_t)(m + 1), hipMemcpyDeviceToDevice, st));
    if (nnz > 0) {
        SCHK(hipMemcpyAsync(ci, A->colidx, sizeof(int32_t) * (size_t)nnz, hipMemcpyDeviceToDevice, st));
        SCHK(hipMemcpyAsync(va, A->val, sizeof(double) * (size_t)nnz, hipMemcpyDeviceToDevice, st));
    }
    SCHK(hipMemcpyAsync(fb, b, sizeof(double) * m, hipMemcpyDeviceToDevice, st));
    SCHK(hipMemcpyAsync(fC, c, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    // validation: row pointers, then entries, then b and c
    int hflag = 0;
    SCHK(sp_validate_rows(g, w->errflag, st));
    SCHK(hipMemcpyAsync(&hflag, w->errflag, sizeof(int), hipMemcpyDeviceToHost, st));
    SCHK(hipStreamSynchronize(st));
    if (hflag) { freetmp(); return bail(fail(ABIP_E_INVALID, "CSR: row pointers are not a nondecreasing 0..nnz sequence")); }
    SCHK(sp_validate_entries(g, w->errflag, st));
    SCHK(sp_check_finite(fb, m, w->errflag, 8, st));
    SCHK(sp_check_finite(fC, n, w->errflag, 8, st));
    SCHK(hipMemcpyAsync(&hflag, w->errflag, sizeof(int), hipMemcpyDeviceToHost, st));
    SCHK(hipStreamSynchronize(st));
    if (hflag & 2) { freetmp(); return bail(fail(ABIP_E_INVALID, "CSR: column index out of range [0, %d)", n)); }
    if (hflag & 4) { freetmp(); return bail(fail(ABIP_E_NONFINITE, "NaN or Inf in A")); }
    if (hflag & 8) { freetmp(); return bail(fail(ABIP_E_NONFINITE, "NaN or Inf in b or c")); }
    // CSR(A^T), Jacobi diagonal, HSD constants (eq. bar-b-c-z-re)
    SCHK(sp_transpose(g, rpt, cit, vat, cursor, st));
    SCHK(sp_rowsq(g, dG, st));
    // G~ = A A^T explicitly (one product and one grid barrier per CG iteration)
    // when asked for (settings.sparse_gram = 1) and every row's products fit the gather
    if (s.sparse_gram == 1 && nnz > 0) {
        int32_t* gcnt = nullptr;
        SALLOC(gcnt, m);
        std::vector<int32_t> hc(m);
        hipError_t e1 = sp_gram_count(g, gcnt, st);
        if (e1 == hipSuccess) e1 = hipMemcpyAsync(hc.data(), gcnt, sizeof(int32_t) * (size_t)m, hipMemcpyDeviceToHost, st);
        if (e1 == hipSuccess) e1 = hipStreamSynchronize(st);
        (void)hipFree(gcnt);
        if (e1 != hipSuccess) return bail(fail(ABIP_E_HIP, "G = A A^T count: %s", hipGetErrorString(e1)));
        bool fits = true;
        int64_t tot = 0;
        std::vector<int32_t> hp_(m + 1);
        for (int i = 0; i < m; ++i) {
            if (hc[i] < 0) { fits = false; break; }
            hp_[i] = (int32_t)tot;
            tot += hc[i];
        }
        hp_[m] = (int32_t)tot;
        const bool want = fits && tot > 0 && tot < INT32_MAX;
        if (want) {
            SALLOC(w->sp_grp, (int64_t)m + 1);
            SALLOC(w->sp_gci, tot);
            SALLOC(w->sp_gva, tot);
            SCHK(hipMemcpyAsync(w->sp_grp, hp_.data(), sizeof(int32_t) * ((size_t)m + 1), hipMemcpyHostToDevice, st));
            SCHK(sp_gram_fill(g, w->sp_grp, w->sp_gci, w->sp_gva, st));
            g.grp = w->sp_grp; g.gci = w->sp_gci; g.gva = w->sp_gva;
            g.LG = lanes_for((double)tot / m);
            w->sp_gram_nnz = tot;
        }
    }
    // row pointers on the host, to size each launch's LDS-resident slices
    w->sp_hrp.resize((size_t)m + 1);
    w->sp_hrpt.resize((size_t)n + 1);
    SCHK(hipMemcpyAsync(w->sp_hrp.data(), rp, sizeof(int32_t) * ((size_t)m + 1), hipMemcpyDeviceToHost, st));
    SCHK(hipMemcpyAsync(w->sp_hrpt.data(), rpt, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyDeviceToHost, st));
    SCHK(hipStreamSynchronize(st));
    (void)hipDeviceGetAttribute(&w->lds_cap, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    w->sp_lds_cap = (w->lds_cap > 1024) ? w->lds_cap - 1024 : 0;      // the kernels' static LDS stays free
    if (w->sp_lds_cap > 0) SCHK(sp_set_lds_limit(w->sp_lds_cap));
    SCHK(sp_affine(fC, 0.0, 1.0, n, g.q1, st));                               // e (scratch)
    SCHK(sp_spmv(rp, ci, va, m, g.q1, -1.0, fb, 1.0, fbb, st));              // bbar = b - A e
    SCHK(sp_affine(fC, 1.0, -1.0, n, fCB, st));                               // cbar = c - e
    SCHK(sp_spmv(rp, ci, va, m, fC, 1.0, nullptr, 0.0, fAc, st));            // A c
    SCHK(sp_spmv(rp, ci, va, m, fCB, 1.0, nullptr, 0.0, fAcb, st));          // A cbar
    std::vector<double> hp(8 * NBLK);
    {
        const double* ys[2] = {g.q1, fC};
        SCHK(hipMemcpyAsync(dptrs, ys, sizeof ys, hipMemcpyHostToDevice, st));
        SCHK(sp_dots(fC, dptrs, 2, n, dpart, NBLK, st));                      // c^T e, c^T c
        SCHK(hipMemcpyAsync(hp.data(), dpart, sizeof(double) * 2 * NBLK, hipMemcpyDeviceToHost, st));
        SCHK(hipStreamSynchronize(st));
    }
    const double zbar = host_sum(hp, 0, NBLK) + 1.0, nc = std::sqrt(host_sum(hp, 1, NBLK));
    {
        const double* ys[1] = {fb};
        SCHK(hipMemcpyAsync(dptrs, ys, sizeof ys, hipMemcpyHostToDevice, st));
        SCHK(sp_dots(fb, dptrs, 1, m, dpart, NBLK, st));
        SCHK(hipMemcpyAsync(hp.data(), dpart, sizeof(double) * NBLK, hipMemcpyDeviceToHost, st));
        SCHK(hipStreamSynchronize(st));
    }
    const double nb = std::sqrt(host_sum(hp, 0, NBLK));
    // the border Z = M^{-1} H (Section 4.4, rank 2): Z_y = G^{-1}(e - A f), Z_x = f + A^T Z_y
    // for H1 = (-b; c) and H2 = (bbar; -cbar), by CG to near machine precision
    const int maxb = std::min(sp_max_blocks(w->cu_count, 0), 4 * w->cu_count);
    w->sp_nb = std::max(1, std::min<int>(maxb, (int)std::min<int64_t>(w->cu_count, (std::max<int64_t>(m, n) + 255) / 256)));
    w->sp_nb_default = w->sp_nb;
    g.lds_bytes = s.lds_resident ? sp_lds_for(w, w->sp_nb) : 0;
    double* rhs = g.Y;                                                         // scratch until the solve
    const int32_t bmax = std::max<int32_t>(5000, 20 * s.cg_max_iters);
    SCHK(sp_spmv(rp, ci, va, m, fC, -1.0, fb, -1.0, rhs, st));               // -b - A c
    SCHK(sp_cg_solve(g, rhs, fZy0, 1e-14, bmax, w->sp_nb, w->sp_cgit, st));
    SCHK(sp_spmv(rp, ci, va, m, fCB, 1.0, fbb, 1.0, rhs, st));               // bbar + A cbar
    SCHK(sp_cg_solve(g, rhs, fZy1, 1e-14, bmax, w->sp_nb, w->sp_cgit, st));
    SCHK(sp_spmv(rpt, cit, vat, n, fZy0, 1.0, nullptr, 0.0, ATZy0, st));     // A^T Z_y0
    SCHK(sp_spmv(rpt, cit, vat, n, fZy1, 1.0, nullptr, 0.0, ATZy1, st));     // A^T Z_y1
    SCHK(sp_spmv(rpt, cit, vat, n, fZy0, 1.0, fC, 1.0, fZx0, st));           // Z_x0 = c + A^T Z_y0
    SCHK(sp_spmv(rpt, cit, vat, n, fZy1, 1.0, fCB, -1.0, fZx1, st));         // Z_x1 = -cbar + A^T Z_y1
    SCHK(hipMemsetAsync(g.a, 0, sizeof(double) * d.ld, st));                  // CG warm start of the solve: 0
    int herr = 0;
    SCHK(hipMemcpyAsync(&herr, w->sp_err, sizeof(int), hipMemcpyDeviceToHost, st));
    // K = I2 + S + H^T Z
    {
        const double* ys[4] = {fZy0, fZy1, nullptr, nullptr};
        SCHK(hipMemcpyAsync(dptrs, ys, 2 * sizeof(double*), hipMemcpyHostToDevice, st));
        SCHK(sp_dots(fb, dptrs, 2, m, dpart, NBLK, st));                       // b^T Z_y0, b^T Z_y1
        SCHK(sp_dots(fbb, dptrs, 2, m, dpart + 2 * NBLK, NBLK, st));           // bbar^T Z_y0, bbar^T Z_y1
        const double* xs[2] = {fZx0, fZx1};
        SCHK(hipMemcpyAsync(dptrs + 2, xs, 2 * sizeof(double*), hipMemcpyHostToDevice, st));
        SCHK(sp_dots(fC, dptrs + 2, 2, n, dpart + 4 * NBLK, NBLK, st));        // c^T Z_x0, c^T Z_x1
        SCHK(sp_dots(fCB, dptrs + 2, 2, n, dpart + 6 * NBLK, NBLK, st));       // cbar^T Z_x0, cbar^T Z_x1
        SCHK(hipMemcpyAsync(hp.data(), dpart, sizeof(double) * 8 * NBLK, hipMemcpyDeviceToHost, st));
        SCHK(hipStreamSynchronize(st));
    }
    freetmp();
    if (herr) return bail(fail(ABIP_E_HIP, "sparse setup: a grid barrier timed out"));
    const double bZ0 = host_sum(hp, 0, NBLK), bZ1 = host_sum(hp, 1, NBLK);
    const double bbZ0 = host_sum(hp, 2, NBLK), bbZ1 = host_sum(hp, 3, NBLK);
    const double cZ0 = host_sum(hp, 4, NBLK), cZ1 = host_sum(hp, 5, NBLK);
    const double cbZ0 = host_sum(hp, 6, NBLK), cbZ1 = host_sum(hp, 7, NBLK);
    const double k00 = 1.0 + (-bZ0 + cZ0), k01 = zbar + (-bZ1 + cZ1);
    const double k10 = -zbar + (bbZ0 - cbZ0), k11 = 1.0 + (bbZ1 - cbZ1);
    const double det = k00 * k11 - k01 * k10;
    LPCtrl C{};
    C.zbar = zbar; C.nb = nb; C.nc = nc;
    C.K00 = k11 / det; C.K01 = -k01 / det; C.K10 = -k10 / det; C.K11 = k00 / det;
    C.KA00 = C.KA01 = C.KA10 = C.KA11 = NAN;
    C.phase = 1;
    SCHK(hipMemcpyAsync(w->dctrl, &C, sizeof C, hipMemcpyHostToDevice, st));
    SCHK(hipStreamSynchronize(st));
#undef SALLOC
#undef SCHK
    w->hctrl.resize(1);
    w->setup_ms = now_ms() - t0;
    *out = w;
    return ABIP_OK;
}

// one cooperative launch for the whole solve (or `fixed` updates)
static int sparse_run(abip_work* w, int64_t fixed) {
    hipStream_t st = w->stream;
    SpArgs g = w->sa;
    g.lds_bytes = w->set.lds_resident ? sp_lds_for(w, w->sp_nb) : 0;
    g.prm = make_params(w->set);
    g.cg_tol = w->set.cg_tol;
    g.cg_max = w->set.cg_max_iters;
    g.cg_rule = w->set.cg_rule;
    g.fixed_iters = fixed;
    if (fixed == 0) {          // a fresh solve starts CG from a = 0 (reproducible runs)
        HIPCHK(hipMemsetAsync(g.a, 0, sizeof(double) * (size_t)g.m, st));
        HIPCHK(hipMemsetAsync(g.ATA, 0, sizeof(double) * (size_t)g.n, st));
    }
    HIPCHK(hipMemsetAsync(w->sp_bar, 0, 2 * sizeof(unsigned), st));
    HIPCHK(hipMemsetAsync(w->sp_err, 0, sizeof(int), st));
    if (!w->ev0) HIPCHK(hipEventCreate(&w->ev0));
    if (!w->ev1) HIPCHK(hipEventCreate(&w->ev1));
    HIPCHK(hipEventRecord(w->ev0, st));
    HIPCHK(sp_solve(g, w->sp_nb, st));
    HIPCHK(hipEventRecord(w->ev1, st));
    int herr = 0;
    HIPCHK(hipMemcpyAsync(&herr, w->sp_err, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (herr) return fail(ABIP_E_HIP, "sparse solve: a grid barrier timed out");
    return ABIP_OK;
}

extern "C" int abip_setup(abip_work** out, const abip_matrix* A, const double* b, const double* c,
                          const abip_settings* settings, void* stream) {
    if (!out) return fail(ABIP_E_INVALID, "abip_setup: null output handle");
    if (!A) return fail(ABIP_E_INVALID, "abip_setup: null A");
    if (A->format == ABIP_CSR) return setup_sparse(out, A, b, c, settings, stream);
    const double* bb[1] = {b};
    const double* cc[1] = {c};
    return setup_dense(out, 1, A, bb, cc, settings, stream);
}

extern "C" int abip_setup_batch(abip_work** out, int32_t B, const abip_matrix* A, const double* const* b,
                                const double* const* c, const abip_settings* settings, void* stream) {
    return setup_dense(out, B, A, b, c, settings, stream);
}

extern "C" int abip_update_data(abip_work* w, const abip_matrix* A, const double* const* b,
                                const double* const* c) {
    if (!w) return fail(ABIP_E_INVALID, "abip_update_data: null handle");
    if (w->sparse) return fail(ABIP_E_STATE, "abip_update_data: dense handles only");
    if (!A || !b || !c) return fail(ABIP_E_INVALID, "abip_update_data: null A, b or c");
    for (int k = 0; k < w->B; ++k) {
        const abip_matrix& M = A[k];
        if (M.format != ABIP_DENSE_ROWMAJOR) return fail(ABIP_E_INVALID, "LP %d: dense row-major A only", k);
        if (M.m != w->hdesc[k].m || M.n != w->hdesc[k].n)
            return fail(ABIP_E_DIM, "LP %d: %d x %d does not match the handle's %d x %d", k, M.m, M.n,
                        w->hdesc[k].m, w->hdesc[k].n);
        if (!M.val || !b[k] || !c[k]) return fail(ABIP_E_INVALID, "LP %d: null data pointer", k);
    }
    const double t0 = now_ms();
    const int rc = load_dense(w, A, b, c);
    if (rc) return rc;
    if (w->grid) grid_config(w, w->grid_wgs);     // the column split follows the new data's pairing
    w->setup_ms = now_ms() - t0;
    return ABIP_OK;
}

static PoolPtrs pools(abip_work* w) {
    PoolPtrs P;
    P.A64 = w->A64; P.A32 = w->A32; P.G64 = w->G64; P.G32 = w->G32;
    P.Mv = w->Mv; P.Nv = w->Nv; P.Mtot = w->Mtot; P.Ntot = w->Ntot;
    P.L64 = w->keep.L64; P.Lt64 = w->keep.Lt64; P.L32 = w->keep.L32; P.Lt32 = w->keep.Lt32;
    P.Li64 = w->keep.Li64; P.Lit64 = w->keep.Lit64; P.Li32 = w->keep.Li32; P.Lit32 = w->keep.Lit32;
    return P;
}

static int run_wg(abip_work* w, int32_t B, int64_t fixed_iters, const SolveParams& prm) {
    hipStream_t st = w->stream;
    const int per_cu = (w->wg_smem <= 76 * 1024 && w->threads <= 512) ? 2 : 1;
    const int grid = std::max(1, std::min<int>(B, w->cu_count * per_cu));
    if (w->noalloc) {                     // plain launches, no events
        hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(64), 0, st, w->queue);
        HIPCHK(hipGetLastError());
        HIPCHK(launch_solve_wg(w->nch, grid, w->threads, st, w->ddesc, w->dctrl, pools(w), prm, w->order, B,
                               w->queue, fixed_iters, w->ldmax, w->wg_smem));
        return ABIP_OK;
    }
    if (!w->ev0) HIPCHK(hipEventCreate(&w->ev0));
    if (!w->ev1) HIPCHK(hipEventCreate(&w->ev1));
    if (w->set.use_graph && fixed_iters == 0 && B == w->B) {
        // queue reset + the persistent launch as one graph, kept with the handle
        int rc = graph_stream(w);
        if (rc) return rc;
        struct Key { SolveParams p; int threads, grid; size_t smem; } key;
        memset(&key, 0, sizeof key);          // padding bytes take part in the comparison
        key.p = prm; key.threads = w->threads; key.grid = grid; key.smem = w->wg_smem;
        const PoolPtrs P = pools(w);
        rc = capture_graph(w, &w->wgraph, &w->wexec, &w->wkey, key_bytes(key, B), [&](hipStream_t cs) {
            hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(64), 0, cs, w->queue);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            return launch_solve_wg(w->nch, grid, w->threads, cs, w->ddesc, w->dctrl, P, prm, w->order, B, w->queue,
                                   0, w->ldmax, w->wg_smem);
        });
        if (rc) return rc;
        HIPCHK(hipEventRecord(w->gjoin0, st));
        HIPCHK(hipStreamWaitEvent(w->gstream, w->gjoin0, 0));
        HIPCHK(hipEventRecord(w->ev0, w->gstream));
        HIPCHK(hipGraphLaunch(w->wexec, w->gstream));
        HIPCHK(hipEventRecord(w->ev1, w->gstream));
        HIPCHK(hipEventRecord(w->gjoin1, w->gstream));
        HIPCHK(hipStreamWaitEvent(st, w->gjoin1, 0));
        return ABIP_OK;
    }
    hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(64), 0, st, w->queue);
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(w->ev0, st));
    HIPCHK(launch_solve_wg(w->nch, grid, w->threads, st, w->ddesc, w->dctrl, pools(w), prm, w->order, B, w->queue,
                           fixed_iters, w->ldmax, w->wg_smem));
    HIPCHK(hipEventRecord(w->ev1, st));
    return ABIP_OK;
}

static void fill_info(abip_info* info, const LPCtrl& c, const LPDesc& d, double setup_ms, double solve_ms,
                      double kernel_ms) {
    info->colpass_lds_fp32 = c.cpl32;
    info->colpass_lds_fp64 = c.cpl64;
    info->ginv_hbm_fp32 = c.gh32;
    info->ginv_hbm_fp64 = c.gh64;
    info->lds_mode = d.lds;
    info->fp32_exit_kkt = c.kfx;
    info->err_vs_fp64 = c.err64;
    info->beta = c.beta;
    info->bb_probe_iters = c.bbp;
    info->bb_estimates = c.bbe;
    info->ticks_colpass = c.clk[0];
    info->ticks_ginv = c.clk[1];
    info->ticks_total = c.clk[2];
    info->ticks_check = c.clk[3];
    info->ticks_update = c.clk[4];
    info->colpass_fp32 = c.cp32;
    info->colpass_fp64 = c.cp64;
    info->kernel_ms = kernel_ms;
    info->status = c.status;
    info->admm_iters = c.iters;
    info->admm_iters_fp64 = c.iters64;
    info->ipm_iters = c.ipm;
    info->cg_iters = c.cg;
    info->pres = c.pres; info->dres = c.dres; info->gap = c.gap;
    info->pobj = c.pobj; info->dobj = c.dobj;
    info->tau = c.tau; info->kappa = c.kappa; info->theta = c.theta; info->mu = c.mu;
    info->setup_ms = setup_ms;
    info->solve_ms = solve_ms;
}

static int solve_all(abip_work* w, double* const* x, double* const* y, double* const* s, abip_info* info) {
    hipStream_t st = w->stream;
    const double t0 = now_ms();
    const SolveParams prm = make_params(w->set);
    const int phase = (w->set.precision == ABIP_PREC_FP32_POLISH) ? 0 : 1;
    hipLaunchKernelGGL(k_init_state, dim3(w->B), dim3(256), 0, st, w->ddesc, w->dctrl, w->Mv, w->Nv, w->Mtot, w->Ntot,
                       w->set.beta, phase, w->set.bb);
    HIPCHK(hipGetLastError());
    int rc = w->sparse ? sparse_run(w, 0) : w->grid ? grid_run(w, 0, phase) : run_wg(w, w->B, 0, prm);
    if (rc) return rc;
    std::vector<double*> tab(3 * w->B);
    for (int k = 0; k < w->B; ++k) {
        tab[3 * k] = x ? x[k] : nullptr;
        tab[3 * k + 1] = y ? y[k] : nullptr;
        tab[3 * k + 2] = s ? s[k] : nullptr;
    }
    // FP64 recheck of the point handed back (independent of the loop's own sums)
    if (w->sparse) {
        const SpArgs& g = w->sa;
        HIPCHK(launch_recheck_csr(g.rp, g.ci, g.va, g.rpt, g.cit, g.vat, g.m, g.n, w->dctrl, g.b, g.Y, g.C, g.X, g.S,
                                  w->rchk, w->rchk_P, st));
    } else {
        HIPCHK(launch_recheck_dense(w->ddesc, w->dctrl, w->A64, w->Mv, w->Nv, w->Mtot, w->Ntot, w->rchk, w->B,
                                    w->rchk_P, st));
    }
    HIPCHK(hipMemcpyAsync(w->outp, tab.data(), sizeof(double*) * 3 * w->B, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_write_outputs, dim3(w->B), dim3(256), 0, st, w->ddesc, w->dctrl, w->Mv, w->Nv, w->Mtot,
                       w->Ntot, w->outp, 0);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(w->hctrl.data(), w->dctrl, sizeof(LPCtrl) * w->B, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const double ms = now_ms() - t0;
    float kms = NAN;
    if (!w->noalloc) HIPCHK(hipEventElapsedTime(&kms, w->ev0, w->ev1));
    if (info)
        for (int k = 0; k < w->B; ++k) {
            fill_info(&info[k], w->hctrl[k], w->hdesc[k], w->setup_ms, ms, (double)kms);
            info[k].gram_nnz = w->sp_gram_nnz;
            info[k].grid_mirror = w->grid && w->grid_pairs > 0 ? 1 : 0;
        }
    w->solved = true;
    return ABIP_OK;
}

extern "C" int abip_solve(abip_work* w, double* x, double* y, double* s, abip_info* info) {
    if (!w) return fail(ABIP_E_INVALID, "abip_solve: null handle");
    if (w->B != 1) return fail(ABIP_E_STATE, "abip_solve: handle holds %d LPs; use abip_solve_batch", w->B);
    double* xs[1] = {x};
    double* ys[1] = {y};
    double* ss[1] = {s};
    return solve_all(w, xs, ys, ss, info);
}

extern "C" int abip_solve_batch(abip_work* w, double* const* x, double* const* y, double* const* s, abip_info* info) {
    if (!w) return fail(ABIP_E_INVALID, "abip_solve_batch: null handle");
    return solve_all(w, x, y, s, info);
}

// Sparse engine: the border of I - Q = (I + Q)^T for the adjoint (Section 4.4's
// Schur reduction with A, H and S changing sign; G = I + A A^T unchanged), by
// CG to near machine precision, as the setup does for I + Q:
//   Z_y0 = G^{-1}(b - A c),        Z_x0 = -c - A^T Z_y0,
//   Z_y1 = G^{-1}(A cbar - bbar),  Z_x1 = cbar - A^T Z_y1,
//   K_A = I2 - S - H^T Z,  stored inverted in the control block.
static int sparse_adjoint_border(abip_work* w, double* part) {
    hipStream_t st = w->stream;
    const SpArgs& g0 = w->sa;
    SpArgs g = g0;
    g.lds_bytes = w->set.lds_resident ? sp_lds_for(w, w->sp_nb) : 0;
    const int m = g.m, n = g.n;
    double* Mv = w->Mv;
    double* Nv = w->Nv;
    double* zy0 = Mv + MF_ZY0A * w->Mtot; double* zy1 = Mv + MF_ZY1A * w->Mtot;
    double* zx0 = Nv + NF_ZX0A * w->Ntot; double* zx1 = Nv + NF_ZX1A * w->Ntot;
    const int32_t bmax = std::max<int32_t>(5000, 20 * w->set.cg_max_iters);
    HIPCHK(sp_spmv(g.rp, g.ci, g.va, m, g.C, -1.0, g.b, 1.0, zy0, st));        // b - A c (right-hand side in place)
    HIPCHK(sp_cg_solve(g, zy0, zy0, 1e-14, bmax, w->sp_nb, w->sp_cgit, st));
    HIPCHK(sp_spmv(g.rp, g.ci, g.va, m, g.CB, 1.0, g.bbar, -1.0, zy1, st));    // A cbar - bbar
    HIPCHK(sp_cg_solve(g, zy1, zy1, 1e-14, bmax, w->sp_nb, w->sp_cgit, st));
    HIPCHK(sp_spmv(g.rpt, g.cit, g.vat, n, zy0, -1.0, g.C, -1.0, zx0, st));    // -c - A^T Z_y0
    HIPCHK(sp_spmv(g.rpt, g.cit, g.vat, n, zy1, -1.0, g.CB, 1.0, zx1, st));    // cbar - A^T Z_y1
    double bz0, bz1, bbz0, bbz1, cz0, cz1, cbz0, cbz1;
    HIPCHK(big_dot2(g.b, zy0, g.b, zy1, m, part, &bz0, &bz1, st));
    HIPCHK(big_dot2(g.bbar, zy0, g.bbar, zy1, m, part, &bbz0, &bbz1, st));
    HIPCHK(big_dot2(g.C, zx0, g.C, zx1, n, part, &cz0, &cz1, st));
    HIPCHK(big_dot2(g.CB, zx0, g.CB, zx1, n, part, &cbz0, &cbz1, st));
    int herr = 0;
    HIPCHK(hipMemcpyAsync(&herr, w->sp_err, sizeof(int), hipMemcpyDeviceToHost, st));
    LPCtrl c;
    HIPCHK(hipMemcpyAsync(&c, w->dctrl, sizeof c, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (herr) return fail(ABIP_E_HIP, "abip_backward: a grid barrier of the sparse CG timed out");
    // (H^T Z)_{rq} = h_r^T z_q with h_0 = (-b; c), h_1 = (bbar; -cbar)
    const double hz0 = -bz0 + cz0, hz1 = -bz1 + cz1, hz2 = bbz0 - cbz0, hz3 = bbz1 - cbz1;
    const double k00 = 1.0 - hz0, k01 = -c.zbar - hz1, k10 = c.zbar - hz2, k11 = 1.0 - hz3;
    const double det = k00 * k11 - k01 * k10;
    c.KA00 = k11 / det; c.KA01 = -k01 / det; c.KA10 = -k10 / det; c.KA11 = k00 / det;
    HIPCHK(hipMemcpyAsync(w->dctrl, &c, sizeof c, hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    if (!w->hctrl.empty()) {
        w->hctrl[0].KA00 = c.KA00; w->hctrl[0].KA01 = c.KA01; w->hctrl[0].KA10 = c.KA10; w->hctrl[0].KA11 = c.KA11;
    }
    w->sp_adjb = true;
    return ABIP_OK;
}

// abip_backward on a handle holding one LP for the whole GPU (grid or sparse engine)
static int backward_big(abip_work* w, const double* gin, double* dc, double* db, double* dA) {
    hipStream_t st = w->stream;
    const LPDesc& d = w->hdesc[0];
    const int m = d.m, n = d.n;
    const int ldw = w->sparse ? 0 : d.ld;
    if (!w->big_ws) HIPCHK(hipMalloc((void**)&w->big_ws, sizeof(double) * big_adj_ws_doubles(m, n, ldw)));
    if (w->h_adj_iters.size() != 1) { w->h_adj_iters.assign(1, 0); w->h_adj_resid.assign(1, 0.0); }
    BigAdj B{};
    B.m = m; B.n = n; B.ld = ldw;
    B.sparse = w->sparse;
    B.alpha = w->set.alpha;
    B.ws = w->big_ws;
    if (w->sparse) {
        if (!w->sp_abak) HIPCHK(hipMalloc((void**)&w->sp_abak, sizeof(double) * (size_t)m));
        HIPCHK(hipMemsetAsync(w->sp_bar, 0, 2 * sizeof(unsigned), st));
        HIPCHK(hipMemsetAsync(w->sp_err, 0, sizeof(int), st));
        // the last 2 x 512 doubles of the workspace serve the border's dot products
        double* part = w->big_ws + big_adj_ws_doubles(m, n, ldw) - 1024;
        HIPCHK(hipMemcpyAsync(w->sp_abak, w->sa.a, sizeof(double) * (size_t)m, hipMemcpyDeviceToDevice, st));
        if (!w->sp_adjb) {
            const int rc = sparse_adjoint_border(w, part);
            if (rc) return rc;
        }
        B.sp = w->sa;
        B.sp.lds_bytes = w->set.lds_resident ? sp_lds_for(w, w->sp_nb) : 0;
        B.sp_nb = w->sp_nb;
        B.cg_tol = std::max(1e-13, 0.1 * w->set.adjoint_tol);
        B.cg_max = std::max<int32_t>(5000, 20 * w->set.cg_max_iters);
        B.cg_iters = w->sp_cgit;
        B.A = nullptr; B.G = nullptr;
    } else {
        B.A = w->A64 + d.oA;
        B.G = w->G64 + d.oG;
    }
    double* Mv = w->Mv;
    double* Nv = w->Nv;
    B.X = Nv + NF_X * w->Ntot + d.on; B.S = Nv + NF_S * w->Ntot + d.on; B.Y = Mv + MF_Y * w->Mtot + d.om;
    B.b = Mv + MF_B * w->Mtot + d.om; B.bbar = Mv + MF_BBAR * w->Mtot + d.om;
    B.C = Nv + NF_C * w->Ntot + d.on; B.CB = Nv + NF_CBAR * w->Ntot + d.on;
    B.zy0 = Mv + MF_ZY0A * w->Mtot + d.om; B.zy1 = Mv + MF_ZY1A * w->Mtot + d.om;
    B.zx0 = Nv + NF_ZX0A * w->Ntot + d.on; B.zx1 = Nv + NF_ZX1A * w->Ntot + d.on;
    HIPCHK(hipMemcpyAsync(&B.cl, w->dctrl, sizeof(LPCtrl), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    int herr = 0;
    int64_t it = 0;
    double rel = 0.0;
    const hipError_t e = big_adjoint(B, gin, dc, db, dA, w->sparse ? w->sa.rp : nullptr,
                                     w->sparse ? w->sa.ci : nullptr, w->set.adjoint_max_iters, w->set.adjoint_tol,
                                     &it, &rel, &herr, st);
    if (w->sparse)        // the solve's CG warm start, as it was
        HIPCHK(hipMemcpyAsync(w->sa.a, w->sp_abak, sizeof(double) * (size_t)m, hipMemcpyDeviceToDevice, st));
    HIPCHK(e);
    HIPCHK(hipStreamSynchronize(st));
    if (herr) return fail(ABIP_E_HIP, "abip_backward: a grid barrier of the sparse CG timed out");
    w->h_adj_iters[0] = it;
    w->h_adj_resid[0] = rel;
    return ABIP_OK;
}

static int backward_all(abip_work* w, const double* const* g, double* const* dc, double* const* db,
                        double* const* dA) {
    if (w->set.scale_iters) return fail(ABIP_E_STATE, "abip_backward: not available for a scaled LP (settings.scale_iters)");
    if (!w->solved) return fail(ABIP_E_STATE, "abip_backward: call abip_solve first");
    for (int k = 0; k < w->B; ++k) {
        if (!g || !g[k] || !dc || !dc[k] || !db || !db[k])
            return fail(ABIP_E_INVALID, "abip_backward: null gradient or output pointer (LP %d)", k);
        if (w->hctrl[k].status != ABIP_SOLVED && !(w->hctrl[k].flags & 4) && w->B == 1)
            return fail(ABIP_E_STATE, "abip_backward: the solve ended with status %d, not SOLVED", w->hctrl[k].status);
    }
    if (w->grid || w->sparse) return backward_big(w, g[0], dc[0], db[0], dA ? dA[0] : nullptr);
    hipStream_t st = w->stream;
    if (!w->adj_ws) {
        std::vector<int64_t> ows(w->B);
        int64_t tot = 0;
        for (int k = 0; k < w->B; ++k) {
            const LPDesc& d = w->hdesc[k];
            ows[k] = tot;
            tot += 7 * (int64_t)(d.m + 2 * d.n + 3) + 2 * (int64_t)d.n + (d.m + d.n + 2);
            tot = (tot + 3) & ~(int64_t)3;
        }
        HIPCHK(hipMalloc((void**)&w->adj_ws, sizeof(double) * tot));
        HIPCHK(hipMalloc((void**)&w->adj_ows, sizeof(int64_t) * w->B));
        HIPCHK(hipMalloc((void**)&w->adj_ptrs, sizeof(double*) * 4 * w->B));
        HIPCHK(hipMalloc((void**)&w->adj_iters, sizeof(int64_t) * w->B));
        HIPCHK(hipMalloc((void**)&w->adj_resid, sizeof(double) * w->B));
        HIPCHK(hipMemcpyAsync(w->adj_ows, ows.data(), sizeof(int64_t) * w->B, hipMemcpyHostToDevice, st));
        w->h_adj_iters.resize(w->B);
        w->h_adj_resid.resize(w->B);
    }
    std::vector<double*> tab(4 * w->B);
    for (int k = 0; k < w->B; ++k) {
        tab[k] = (double*)g[k];
        tab[w->B + k] = dc[k];
        tab[2 * w->B + k] = db[k];
        tab[3 * w->B + k] = dA ? dA[k] : nullptr;
    }
    HIPCHK(hipMemcpyAsync(w->adj_ptrs, tab.data(), sizeof(double*) * 4 * w->B, hipMemcpyHostToDevice, st));
    AdjArgs aa;
    aa.ws = w->adj_ws; aa.ows = w->adj_ows;
    aa.gin = w->adj_ptrs; aa.dc = w->adj_ptrs + w->B; aa.db = w->adj_ptrs + 2 * w->B; aa.dA = w->adj_ptrs + 3 * w->B;
    aa.max_iters = w->set.adjoint_max_iters;
    aa.tol = w->set.adjoint_tol;
    aa.iters_out = w->adj_iters; aa.resid_out = w->adj_resid;
    const SolveParams prm = make_params(w->set);
    const int threads = 512;
    const int grid = std::max(1, std::min<int>(w->B, w->cu_count));
    hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(64), 0, st, w->queue);
    HIPCHK(hipGetLastError());
    HIPCHK(launch_adjoint(grid, threads, st, w->ddesc, w->dctrl, pools(w), prm, aa, w->order, w->B, w->queue,
                          w->ldmax));
    HIPCHK(hipMemcpyAsync(w->h_adj_iters.data(), w->adj_iters, sizeof(int64_t) * w->B, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(w->h_adj_resid.data(), w->adj_resid, sizeof(double) * w->B, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return ABIP_OK;
}

extern "C" int abip_backward(abip_work* w, const double* dL_dx, double* dL_dc, double* dL_db, double* dL_dA) {
    if (!w) return fail(ABIP_E_INVALID, "abip_backward: null handle");
    if (w->B != 1) return fail(ABIP_E_STATE, "abip_backward: handle holds %d LPs; use abip_backward_batch", w->B);
    const double* g[1] = {dL_dx};
    double* c[1] = {dL_dc};
    double* b[1] = {dL_db};
    double* a[1] = {dL_dA};
    return backward_all(w, g, c, b, a);
}

extern "C" int abip_backward_batch(abip_work* w, const double* const* dL_dx, double* const* dL_dc,
                                   double* const* dL_db, double* const* dL_dA) {
    if (!w) return fail(ABIP_E_INVALID, "abip_backward_batch: null handle");
    return backward_all(w, dL_dx, dL_dc, dL_db, dL_dA);
}

extern "C" int abip_backward_stats(abip_work* w, int32_t k, int64_t* iters, double* rel_resid) {
    if (!w) return fail(ABIP_E_INVALID, "abip_backward_stats: null handle");
    if (k < 0 || k >= w->B) return fail(ABIP_E_INVALID, "abip_backward_stats: LP index %d out of range", k);
    if (w->h_adj_iters.empty()) return fail(ABIP_E_STATE, "abip_backward_stats: no backward call yet");
    if (iters) *iters = w->h_adj_iters[k];
    if (rel_resid) *rel_resid = w->h_adj_resid[k];
    return ABIP_OK;
}

extern "C" int abip_apply_iq(abip_work* w, int32_t k, const double* win, double* out, int32_t use_fp32) {
    if (!w) return fail(ABIP_E_INVALID, "abip_apply_iq: null handle");
    if (k < 0 || k >= w->B) return fail(ABIP_E_INVALID, "abip_apply_iq: LP index %d out of range", k);
    if (!win || !out) return fail(ABIP_E_INVALID, "abip_apply_iq: null vector");
    if (w->sparse) return fail(ABIP_E_STATE, "abip_apply_iq: dense handles only");
    const size_t smem = sizeof(double) * 2 * w->hdesc[k].ld;
    const int sgn = (use_fp32 & 2) ? -1 : 1;
    if (use_fp32 & 1)
        hipLaunchKernelGGL(k_apply_iq<float>, dim3(1), dim3(256), smem, w->stream, w->ddesc, w->dctrl, k, w->A32,
                           w->G32, w->Mv, w->Nv, w->Mtot, w->Ntot, win, out, sgn);
    else
        hipLaunchKernelGGL(k_apply_iq<double>, dim3(1), dim3(256), smem, w->stream, w->ddesc, w->dctrl, k, w->A64,
                           w->G64, w->Mv, w->Nv, w->Mtot, w->Ntot, win, out, sgn);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(w->stream));
    return ABIP_OK;
}

extern "C" int abip_set_state(abip_work* w, int32_t k, const double* y, const double* x, const double* s,
                              double tau, double kappa, double theta, double mu) {
    if (!w) return fail(ABIP_E_INVALID, "abip_set_state: null handle");
    if (k < 0 || k >= w->B) return fail(ABIP_E_INVALID, "abip_set_state: LP index %d out of range", k);
    if (!y || !x || !s) return fail(ABIP_E_INVALID, "abip_set_state: null vector");
    if (!(tau > 0 && kappa > 0 && mu > 0)) return fail(ABIP_E_INVALID, "abip_set_state: tau, kappa, mu must be > 0");
    hipLaunchKernelGGL(k_copy_state, dim3(1), dim3(256), 0, w->stream, w->ddesc, k, w->Mv, w->Nv, w->Mtot, w->Ntot,
                       (double*)y, (double*)x, (double*)s, 0);
    HIPCHK(hipGetLastError());
    LPCtrl c;
    HIPCHK(hipMemcpyAsync(&c, w->dctrl + k, sizeof c, hipMemcpyDeviceToHost, w->stream));
    HIPCHK(hipStreamSynchronize(w->stream));
    c.tau = tau; c.kappa = kappa; c.theta = theta; c.mu = mu;
    c.status = 0; c.mode = OP_REFRESH; c.flags = 4;     // 4: loaded iterate, may be differentiated
    c.beta = w->set.beta; c.bbp = 0; c.bbe = 0;        // abip_iterate runs at the settings' beta
    if (w->sparse) {
        HIPCHK(hipMemsetAsync(w->sa.a, 0, sizeof(double) * (size_t)w->sa.m, w->stream));
        HIPCHK(hipMemsetAsync(w->sa.ATA, 0, sizeof(double) * (size_t)w->sa.n, w->stream));
    }
    c.iters = 0; c.iters64 = 0; c.ipm = 0;
    HIPCHK(hipMemcpyAsync(w->dctrl + k, &c, sizeof c, hipMemcpyHostToDevice, w->stream));
    HIPCHK(hipStreamSynchronize(w->stream));
    if (w->hctrl.size() == (size_t)w->B) w->hctrl[k] = c;
    w->solved = true;        // the loaded iterate is what abip_backward differentiates
    return ABIP_OK;
}

extern "C" int abip_get_state(abip_work* w, int32_t k, double* y, double* x, double* s, double* scalars) {
    if (!w) return fail(ABIP_E_INVALID, "abip_get_state: null handle");
    if (k < 0 || k >= w->B) return fail(ABIP_E_INVALID, "abip_get_state: LP index %d out of range", k);
    hipLaunchKernelGGL(k_copy_state, dim3(1), dim3(256), 0, w->stream, w->ddesc, k, w->Mv, w->Nv, w->Mtot, w->Ntot,
                       y, x, s, 1);
    HIPCHK(hipGetLastError());
    LPCtrl c;
    HIPCHK(hipMemcpyAsync(&c, w->dctrl + k, sizeof c, hipMemcpyDeviceToHost, w->stream));
    HIPCHK(hipStreamSynchronize(w->stream));
    if (scalars) { scalars[0] = c.tau; scalars[1] = c.kappa; scalars[2] = c.theta; scalars[3] = c.mu; }
    return ABIP_OK;
}

// iterate LP k alone: a one-LP work queue that points at k
__global__ void k_single_order(int32_t* order, int32_t k) {
    if (threadIdx.x == 0) order[0] = k;
}

extern "C" int abip_iterate(abip_work* w, int32_t k, int64_t iters, int32_t use_fp32) {
    if (!w) return fail(ABIP_E_INVALID, "abip_iterate: null handle");
    if (k < 0 || k >= w->B) return fail(ABIP_E_INVALID, "abip_iterate: LP index %d out of range", k);
    if (iters < 1) return fail(ABIP_E_INVALID, "abip_iterate: iters must be >= 1");
    LPCtrl c;
    HIPCHK(hipMemcpyAsync(&c, w->dctrl + k, sizeof c, hipMemcpyDeviceToHost, w->stream));
    HIPCHK(hipStreamSynchronize(w->stream));
    c.phase = (use_fp32 && !w->sparse) ? 0 : 1;
    c.mode = OP_REFRESH;
    c.flags &= 4;
    HIPCHK(hipMemcpyAsync(w->dctrl + k, &c, sizeof c, hipMemcpyHostToDevice, w->stream));
    if (w->sparse) return sparse_run(w, iters);
    if (w->grid) {
        int rc = grid_run(w, iters, use_fp32 ? 0 : 1);
        if (rc) return rc;
        HIPCHK(hipStreamSynchronize(w->stream));
        LPCtrl c2;
        HIPCHK(hipMemcpy(&c2, w->dctrl, sizeof c2, hipMemcpyDeviceToHost));
        c2.flags = c.flags;
        HIPCHK(hipMemcpy(w->dctrl, &c2, sizeof c2, hipMemcpyHostToDevice));
        return ABIP_OK;
    }
    int32_t* ord1 = w->queue + 1;         // the handle's one-entry order slot (no allocation per call)
    hipLaunchKernelGGL(k_single_order, dim3(1), dim3(64), 0, w->stream, ord1, k);
    SolveParams prm = make_params(w->set);
    hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(64), 0, w->stream, w->queue);
    hipError_t e = launch_solve_wg(w->nch, 1, w->threads, w->stream, w->ddesc, w->dctrl, pools(w), prm, ord1, 1,
                                   w->queue, iters, w->ldmax, w->wg_smem);
    hipError_t e2 = hipStreamSynchronize(w->stream);
    if (e != hipSuccess) return fail(ABIP_E_HIP, "abip_iterate launch: %s", hipGetErrorString(e));
    if (e2 != hipSuccess) return fail(ABIP_E_HIP, "abip_iterate: %s", hipGetErrorString(e2));
    return ABIP_OK;
}

// Launch-configuration autotuner: every candidate runs `iters` updates from
// Algorithm 2's start point (fixed-iteration mode, no tests); the best is kept
// and the iterate is reset.  Grid and sparse engines (one LP): the launch time
// (HIP events on the work stream).  One-workgroup engine: the LDS policies (A
// and G^{-1} or A alone resident, only A and G^{-1}, everything streamed) at
// 256 threads, 512 streamed threads when every LP fits the 512-thread build,
// then a per-LP mix that streams the LPs whose own clock ran faster streamed
// than resident; scored by the sum of the LPs' own clocks, since a batch's
// throughput depends on every LP's time per update while a fixed-iteration
// launch lasts as long as its largest LP alone.
extern "C" int abip_autotune(abip_work* w, int64_t iters, double* ms, int32_t max_cand, int32_t* ncand,
                             int32_t* chosen) {
    if (!w) return fail(ABIP_E_INVALID, "abip_autotune: null handle");
    if (iters < 1) return fail(ABIP_E_INVALID, "abip_autotune: iters must be >= 1");
    if (w->noalloc) return fail(ABIP_E_STATE, "abip_autotune: not available on an allocation-free handle");
    struct WgCand { int threads, policy; bool mix; };
    std::vector<int> cand;
    std::vector<WgCand> wc;
    const bool wgeng = !w->sparse && !w->grid;
    if (w->sparse) {
        const int maxb = std::min(sp_max_blocks(w->cu_count, 0), 4 * w->cu_count);
        cand.push_back(std::min(w->sp_nb_default, maxb));
        for (int nb : {32, 64, 128, 256})
            if (nb <= maxb && nb != cand[0]) cand.push_back(nb);
    } else if (w->grid) {
        for (int f : {1, 2, 4, 8}) cand.push_back(w->cu_count * f / 2);
    } else {
        wc.push_back({256, 0, false});
        if (w->set.lds_resident) {
            wc.push_back({256, 1, false});
            wc.push_back({256, 2, false});
        }
        if (w->nch == 1) wc.push_back({512, 2, false});
        if (w->set.lds_resident) wc.push_back({256, 0, true});
        for (size_t i = 0; i < wc.size(); ++i) cand.push_back((int)i);
    }
    const int phase = (w->set.precision == ABIP_PREC_FP32_POLISH && !w->sparse) ? 0 : 1;
    const SolveParams prm = make_params(w->set);
    hipStream_t st = w->stream;
    const int B = w->B;
    // per-LP clocks of the all-resident (candidate 0) and all-streamed (candidate 2) runs
    std::vector<int64_t> tk_res(B, 0), tk_str(B, 0);
    auto configure = [&](int c) -> int {
        if (w->sparse) { w->sp_nb = c; return ABIP_OK; }
        if (w->grid) { grid_config(w, c); return ABIP_OK; }
        const WgCand& C = wc[c];
        w->threads = C.threads;
        w->lds_policy = C.policy;
        w->lds_stream.assign(B, 0);
        if (C.mix)
            for (int k = 0; k < B; ++k) w->lds_stream[k] = (tk_str[k] > 0 && tk_str[k] < tk_res[k]) ? 1 : 0;
        assign_lds(w);
        HIPCHK(hipMemcpyAsync(w->ddesc, w->hdesc.data(), sizeof(LPDesc) * w->B, hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        const hipError_t e = set_solve_wg_smem_limit(w->wg_smem);
        if (e != hipSuccess) return fail(ABIP_E_HIP, "hipFuncSetAttribute: %s", hipGetErrorString(e));
        return ABIP_OK;
    };
    auto reset = [&]() -> int {
        hipLaunchKernelGGL(k_init_state, dim3(w->B), dim3(256), 0, st, w->ddesc, w->dctrl, w->Mv, w->Nv, w->Mtot,
                           w->Ntot, w->set.beta, phase, 0);
        HIPCHK(hipGetLastError());
        return ABIP_OK;
    };
    double best = 1e300;
    int bi = 0;
    for (size_t i = 0; i < cand.size(); ++i) {
        int rc = configure(cand[i]);
        if (rc) return rc;
        rc = reset();
        if (rc) return rc;
        rc = w->sparse ? sparse_run(w, iters) : w->grid ? grid_run(w, iters, phase) : run_wg(w, w->B, iters, prm);
        if (rc) return rc;
        HIPCHK(hipStreamSynchronize(st));
        float t = 0.0f;
        HIPCHK(hipEventElapsedTime(&t, w->ev0, w->ev1));
        double score = t;
        if (wgeng) {
            w->hctrl.resize(B);
            HIPCHK(hipMemcpy(w->hctrl.data(), w->dctrl, sizeof(LPCtrl) * B, hipMemcpyDeviceToHost));
            int64_t sum = 0;
            for (int k = 0; k < B; ++k) sum += w->hctrl[k].clk[2];
            score = (double)sum / 1e5;           // 100 MHz ticks -> ms
            if (i == 0 || (wc[i].policy == 2 && wc[i].threads == 256 && !wc[i].mix))
                for (int k = 0; k < B; ++k) (i == 0 ? tk_res : tk_str)[k] = w->hctrl[k].clk[2];
        }
        if (ms && (int32_t)i < max_cand) ms[i] = score;
        if (score < best) { best = score; bi = (int)i; }
    }
    int rc = configure(cand[bi]);
    if (rc) return rc;
    rc = reset();
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(st));
    w->solved = false;
    if (ncand) *ncand = (int32_t)cand.size();
    if (chosen) *chosen = cand[bi];
    return ABIP_OK;
}

// The row / column factors of LP k's scaling (device outputs D[m], E[n]; all 1
// when the LP is not scaled).
extern "C" int abip_get_scaling(abip_work* w, int32_t k, double* D, double* E) {
    if (!w) return fail(ABIP_E_INVALID, "abip_get_scaling: null handle");
    if (k < 0 || k >= w->B) return fail(ABIP_E_INVALID, "abip_get_scaling: LP index %d out of range", k);
    if (w->sparse) return fail(ABIP_E_STATE, "abip_get_scaling: dense handles only");
    const LPDesc& d = w->hdesc[k];
    if (D) HIPCHK(hipMemcpyAsync(D, w->Mv + MF_SD * w->Mtot + d.om, sizeof(double) * d.m, hipMemcpyDeviceToDevice,
                                 w->stream));
    if (E) HIPCHK(hipMemcpyAsync(E, w->Nv + NF_SE * w->Ntot + d.on, sizeof(double) * d.n, hipMemcpyDeviceToDevice,
                                 w->stream));
    HIPCHK(hipStreamSynchronize(w->stream));
    return ABIP_OK;
}

extern "C" int abip_free(abip_work* w) {
    if (!w) return ABIP_OK;
    (void)hipStreamSynchronize(w->stream);
    release(w);
    delete w;
    return ABIP_OK;
}

// ---------------------------------------------------------------------------
// allocation-free solve of one small dense LP
// ---------------------------------------------------------------------------
// Every device buffer of the solve (the library's copies of A, b, c in both
// precisions, G^{-1}, the border, the iterate, the control block, the setup's
// Cholesky workspace, the recheck's partial sums) is carved out of this
// file-scope array; each GPU the library runs on holds its own copy until the
// process ends.  The largest LP (m = 256, n = 1024) takes about 4.5 MiB.
static const size_t NOALLOC_BYTES = (size_t)5 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];
static const int NOALLOC_MAX_DEV = 64;
static unsigned char* g_scratch_ptr[NOALLOC_MAX_DEV];
static std::mutex g_scratch_mu;

// The device address of `scratch` on the current device (looked up once per
// device; host code never uses the symbol's own name as a device address).
static int scratch_address(int dev, unsigned char** out) {
    if (dev < 0 || dev >= NOALLOC_MAX_DEV) return fail(ABIP_E_INVALID, "abip_solve_noalloc: device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(ABIP_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = (unsigned char*)p;
    }
    *out = g_scratch_ptr[dev];
    return ABIP_OK;
}

extern "C" int abip_solve_noalloc(const abip_matrix* A, const double* b, const double* c, double* x, double* y,
                                  double* s, abip_info* info, const abip_settings* settings, void* stream) {
    if (!A || !b || !c) return fail(ABIP_E_INVALID, "abip_solve_noalloc: null A, b or c");
    if (A->format != ABIP_DENSE_ROWMAJOR) return fail(ABIP_E_INVALID, "abip_solve_noalloc: dense row-major A only");
    if (A->m < 1 || A->n < 1 || A->m > ABIP_NOALLOC_MAX_M || A->n > ABIP_NOALLOC_MAX_N)
        return fail(ABIP_E_DIM, "abip_solve_noalloc: m=%d n=%d outside 1..%d x 1..%d", A->m, A->n,
                    ABIP_NOALLOC_MAX_M, ABIP_NOALLOC_MAX_N);
    abip_settings st;
    if (settings) st = *settings; else abip_default_settings(&st);
    if (st.engine == ABIP_ENGINE_GRID) return fail(ABIP_E_INVALID, "abip_solve_noalloc: one-workgroup engine only");
    st.engine = ABIP_ENGINE_WG;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    unsigned char* base = nullptr;
    int rc = scratch_address(dev, &base);
    if (rc) return rc;
    const double* bb[1] = {b};
    const double* cc[1] = {c};
    abip_work* w = nullptr;
    rc = setup_dense(&w, 1, A, bb, cc, &st, stream, base, NOALLOC_BYTES);
    if (rc) return rc;
    double* xs[1] = {x};
    double* ys[1] = {y};
    double* ss[1] = {s};
    rc = solve_all(w, xs, ys, ss, info);
    release(w);                 // nothing to free: the buffers are the scratch region's
    delete w;
    return rc;
}

extern "C" const char* abip_last_error(void) { return g_err.c_str(); }

extern "C" const char* abip_version(void) { return "abip-mi355x 0.1 gfx950"; }
