// Single-GPU restarted reflected-Halpern PDHG (the D-PDLP paper's method at
// one device: Algorithm 1 with |R| = |C| = 1) behind the C ABI of dpdlp.h.
//
// Per iteration two fused kernels run on the caller's stream, each streaming
// one copy of A exactly once:
//   primal  CSC tiles: A^T y, projection, reflection, Halpern  (x, xbar)
//   dual    CSR tiles: A xbar, proj_{-S}, Halpern                (y)
// Every K-th iteration (and at the first iteration of each restart epoch)
// the two kernels also write T(z) = (xh, yh) and z - T(z); one CSR and one
// CSC check pass then produce per-tile partial sums, and a single-workgroup
// control kernel adds them in a fixed order and takes, in FP64 on the
// device, the KKT (App. B.4), restart (App. B.2) and PID primal-weight
// (App. B.3) decisions.  The host reads back a ~200-byte control block per
// check to schedule the next launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "dpdlp_internal.h"
#include "dpdlp_kernels.h"

namespace dpdlp {

// ---------------------------------------------------------------------------
// small device kernels

constexpr int kNQ = 5;              // partial quantities per check pass

template <typename T>
__global__ void k_fill(T *p, T v, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

template <typename Ti, typename To>
__global__ void k_convert(const Ti *__restrict__ in, To *__restrict__ out, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (To)in[i];
}

// d[i] *= f[i]
__global__ void k_mul(double *__restrict__ d, const double *__restrict__ f, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] *= f[i];
}

// Scale the stored values of A by (a * f_row[i]) * f_col[j] over one format's
// tiles.  csr = 1: segments are rows (fseg = f_row, fidx = f_col); csr = 0:
// segments are columns (fseg = f_col, fidx = f_row).  Both formats use the
// same multiplication order, so the two copies stay bitwise equal.
__global__ __launch_bounds__(kBlock) void k_scale_vals(const Tile *__restrict__ tiles, int ntiles,
                                                       const int *__restrict__ seg_ptr,
                                                       const int *__restrict__ idx,
                                                       double *__restrict__ val,
                                                       const double *__restrict__ fseg,
                                                       const double *__restrict__ fidx, int csr)
{
    const int t = blockIdx.x;
    if (t >= ntiles) return;
    const Tile d = tiles[t];
    const int nseg = d.seg_end - d.seg_begin;
    const int G = 1 << d.width_log2;
    const int lane = threadIdx.x & (G - 1);
    for (int s = threadIdx.x >> d.width_log2; s < nseg; s += kBlock >> d.width_log2) {
        const int seg = d.seg_begin + s;
        const int b = max(seg_ptr[seg], d.nnz_begin), e = min(seg_ptr[seg + 1], d.nnz_end);
        const double fs = fseg[seg];
        for (int p = b + lane; p < e; p += G) {
            const double fi = fidx[idx[p]];
            val[p] = csr ? val[p] * fs * fi : val[p] * fi * fs;
        }
    }
}

// Scaled problem data: c~ = D_c c, var bounds / D_c, con bounds * D_r.
__global__ void k_scale_vectors(int m, int n, const double *__restrict__ dr,
                                const double *__restrict__ dc, const double *__restrict__ c0,
                                const double *__restrict__ vlo0, const double *__restrict__ vhi0,
                                const double *__restrict__ clo0, const double *__restrict__ chi0,
                                double *c, double *vlo, double *vhi, double *clo, double *chi)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        c[i] = dc[i] * c0[i];
        vlo[i] = vlo0[i] / dc[i];
        vhi[i] = vhi0[i] / dc[i];
    }
    if (i < m) {
        clo[i] = dr[i] * clo0[i];
        chi[i] = dr[i] * chi0[i];
    }
}

// Per-block partial sums for the norms used by the KKT denominators and
// omega0: ||c||^2, ||finite [l_c,u_c]||^2 (original), the same scaled.
__global__ __launch_bounds__(kBlock) void k_norm_partials(int m, int n, const double *c0,
                                                          const double *clo0,
                                                          const double *chi0, const double *c,
                                                          const double *clo, const double *chi,
                                                          double *partials)
{
    __shared__ double s_red[4][kBlock / 64];
    double acc[4] = {0, 0, 0, 0};
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        acc[0] = c0[i] * c0[i];
        acc[2] = c[i] * c[i];
    }
    if (i < m) {
        if (isfinite(clo0[i])) acc[1] += clo0[i] * clo0[i];
        if (isfinite(chi0[i])) acc[1] += chi0[i] * chi0[i];
        if (isfinite(clo[i])) acc[3] += clo[i] * clo[i];
        if (isfinite(chi[i])) acc[3] += chi[i] * chi[i];
    }
    block_reduce<SumOp, 4>(acc, s_red);
    if (threadIdx.x == 0)
        for (int q = 0; q < 4; ++q) partials[(size_t)q * gridDim.x + blockIdx.x] = acc[q];
}

// Single-workgroup fixed-order sum of nq rows of partials[q * np + i]:
// thread t adds i = t, t + kBlock, ... in that order, then a tree over the
// threads.  The loads of U strided steps of every row are issued before
// their adds (same order, more loads in flight).
template <int NQMAX>
__device__ void sum_partials(const double *partials, int np, int nq, double *out)
{
    __shared__ double s[NQMAX][kBlock];
    constexpr int U = 8;
    double a[NQMAX];
#pragma unroll
    for (int q = 0; q < NQMAX; ++q) a[q] = 0.0;
    int i = threadIdx.x;
    for (; i + (U - 1) * kBlock < np; i += U * kBlock) {
        double v[NQMAX][U];
#pragma unroll
        for (int q = 0; q < NQMAX; ++q)
            if (q < nq) {
#pragma unroll
                for (int u = 0; u < U; ++u) v[q][u] = partials[(size_t)q * np + i + u * kBlock];
            }
#pragma unroll
        for (int q = 0; q < NQMAX; ++q)
            if (q < nq) {
#pragma unroll
                for (int u = 0; u < U; ++u) a[q] += v[q][u];
            }
    }
    for (; i < np; i += kBlock) {
#pragma unroll
        for (int q = 0; q < NQMAX; ++q)
            if (q < nq) a[q] += partials[(size_t)q * np + i];
    }
#pragma unroll
    for (int q = 0; q < NQMAX; ++q)
        if (q < nq) s[q][threadIdx.x] = a[q];
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int q = 0; q < nq; ++q) s[q][threadIdx.x] += s[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < nq; ++q) out[q] = s[q][0];
    __syncthreads();
}

__global__ __launch_bounds__(kBlock) void k_sum_rows(const double *partials, int np, int nq,
                                                     double *out)
{
    sum_partials<8>(partials, np, nq, out);
}

// Lanczos: *norm = sqrt(sum of the partials), also kept in hist[idx].
__global__ __launch_bounds__(kBlock) void k_lanczos_norm(const double *partials, int np,
                                                         double *norm, double *hist, int idx)
{
    __shared__ double tot;
    sum_partials<1>(partials, np, 1, &tot);
    if (threadIdx.x == 0) {
        const double l = sqrt(tot);
        *norm = l;
        hist[idx] = l;
    }
}

// Start point (original space -> scaled, permuted): x = clamp(x0/D_c, X),
// y = proj_Y(y0/D_r); the anchor is the same point.
template <typename T>
__global__ void k_init_x(int n, const double *x0, const int *perm, const double *dc,
                         const double *vlo, const double *vhi, T *x, T *xa)
{
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double v = x0 ? x0[perm[j]] / dc[j] : 0.0;
    v = clampv(v, vlo[j], vhi[j]);
    x[j] = (T)v;
    xa[j] = (T)v;
}
template <typename T>
__global__ void k_init_y(int m, const double *y0, const int *perm, const double *dr,
                         const double *clo, const double *chi, T *y, T *ya)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    double v = y0 ? y0[perm[i]] / dr[i] : 0.0;
    const bool lf = isfinite(clo[i]), hf = isfinite(chi[i]);
    if (!lf && !hf) v = 0.0;
    else if (!lf) v = fmin(v, 0.0);
    else if (!hf) v = fmax(v, 0.0);
    y[i] = (T)v;
    ya[i] = (T)v;
}

// out[perm[i]] = scale[i] * in[i]   (scale may be null)
template <typename T>
__global__ void k_unpermute(int n, const T *in, const int *perm, const double *scale, double *out)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double v = (double)in[i];
    out[perm[i]] = scale ? scale[i] * v : v;
}
// out[i] = in[perm[i]] / div[i]   (div may be null)
template <typename T>
__global__ void k_permute(int n, const double *in, const int *perm, const double *div, T *out)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double v = in[perm[i]];
    out[i] = (T)(div ? v / div[i] : v);
}

// Restart (App. B.2): the new anchor and iterate are T(z) = (xh, yh).
template <typename T>
__global__ void k_restart(int m, int n, const double *xh, const double *yh, T *x, T *xa, T *y,
                          T *ya)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) { x[i] = (T)xh[i]; xa[i] = (T)xh[i]; }
    if (i < m) { y[i] = (T)yh[i]; ya[i] = (T)yh[i]; }
}

// Control block: FP64 scalars kept on the device.
struct Control {
    double omega, r0, r_prev, pid_int, pid_prev;
    double r_primal, r_dual, r_gap, obj_p, obj_d, r;
    double sums[2 * kNQ];
    int32_t pid_started, restarts, restart, converged, numerical, n_checks;
};

struct CtlArgs {
    int64_t k, t;
    double eta, eps, beta_suf, beta_nec, beta_art, kp, ki, kd, c_norm, b_norm;
    int32_t mode;     // 0: decide (solver check), 1: evaluate only
    int32_t pad;
};

// KKT (App. B.4), fixed-point residual (App. B.2, D.2.1), restart decision
// and PID primal-weight update (App. B.3).  One workgroup.
__global__ __launch_bounds__(kBlock) void k_control(const double *pr, int ntr, const double *pc,
                                                    int ntc, Control *ctl, CtlArgs a)
{
    __shared__ double srow[kNQ], scol[kNQ];
    sum_partials<kNQ>(pr, ntr, kNQ, srow);
    sum_partials<kNQ>(pc, ntc, kNQ, scol);
    if (threadIdx.x != 0) return;
    Control C = *ctl;
    for (int q = 0; q < kNQ; ++q) { C.sums[q] = srow[q]; C.sums[kNQ + q] = scol[q]; }
    const double pres = srow[0], py = srow[1], dyy = srow[2], dya = srow[3], yanc = srow[4];
    const double dres = scol[0], cx = scol[1], sx = scol[2], dxx = scol[3], xanc = scol[4];
    const double rp = sqrt(pres) / (1.0 + a.b_norm);
    const double rd = sqrt(dres) / (1.0 + a.c_norm);
    const double dobj = py + sx;
    const double rg = fabs(cx - dobj) / (1.0 + fmax(fabs(cx), fabs(dobj)));
    C.r_primal = rp; C.r_dual = rd; C.r_gap = rg; C.obj_p = cx; C.obj_d = dobj;
    if (a.mode == 1) { *ctl = C; return; }
    const double w = C.omega;
    const double r2 = (w / a.eta) * dxx + dyy / (a.eta * w) + 2.0 * dya;
    const double r = sqrt(fmax(r2, 0.0));
    C.r = r;
    const double kkt = fmax(rp, fmax(rd, rg));
    C.numerical = !(isfinite(kkt) && isfinite(r));
    C.converged = (!C.numerical) && kkt <= a.eps;
    C.restart = 0;
    if (!C.converged && !C.numerical) {
        if (a.k == 0) C.r0 = r;
        else if (r <= a.beta_suf * C.r0) C.restart = 1;
        else if (r <= a.beta_nec * C.r0 && r > C.r_prev) C.restart = 2;
        else if ((double)a.k >= a.beta_art * (double)a.t) C.restart = 3;
    }
    if (C.restart) {
        const double ddx = sqrt(xanc), ddy = sqrt(yanc);
        if (!(ddx < 1e-10 || ddy < 1e-10)) {
            const double e = log(C.omega * ddx / ddy);
            if (!C.pid_started) { C.pid_prev = e; C.pid_started = 1; }
            C.pid_int += e;
            const double lw = log(C.omega) - (a.kp * e + a.ki * C.pid_int + a.kd * (e - C.pid_prev));
            C.pid_prev = e;
            C.omega = exp(lw);
        }
        C.restarts += 1;
    } else if (!C.converged) {
        C.r_prev = r;
    }
    C.n_checks += 1;
    *ctl = C;
}

// ---------------------------------------------------------------------------
// the problem handle

struct TileSet {
    Tile *d = nullptr;
    int n = 0;
    SplitSeg *splits = nullptr;     // segments split over several tiles
    int nsplit = 0;
    int *blk2tile = nullptr;        // sliced sets: workgroup -> tile (-1: idle)
    int grid = 0;                   // sliced sets: launch size
    int seg_stride = 0;             // per-slice pointer stride (0 for the compact sliced form)
    uint16_t *pos = nullptr;        // gather-sorted tiles: product position in the tile
};

// One format cut into gather slices (the XCD-sliced form of a fused step).
struct SlicedSet {
    TileSet ts;
    int S = 0;
    int *ptr = nullptr, *idx = nullptr, *src = nullptr;
    double *val = nullptr;
    float *val32 = nullptr;
    uint8_t *mask = nullptr;        // per segment: slices with nonzeros (S/8 byte planes)
    int *cbase = nullptr;           // per combine block and slice: first compact segment
    int64_t G = 0;                  // compact segments (partial sums per pass)
};

// Gathers the (scaled) values of the unsliced format into the sliced order.
template <typename T>
__global__ void k_gather_vals(const int *__restrict__ src, const double *__restrict__ val,
                              T *__restrict__ out, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (T)val[src[i]];
}

struct DevMem {
    std::vector<void *> ptrs;
    ~DevMem() { for (void *p : ptrs) (void)hipFree(p); }
};

}  // namespace dpdlp

using namespace dpdlp;

struct dpdlp_problem {
    dpdlp_params prm{};
    int32_t m = 0, n = 0;
    int64_t nnz = 0;
    DevMem mem;
    hipStream_t s = nullptr;
    // matrix (permuted, scaled)
    int *rp = nullptr, *ci = nullptr, *cp = nullptr, *ri = nullptr;
    double *v = nullptr, *vt = nullptr;
    float *v32 = nullptr, *vt32 = nullptr;
    TileSet tr, tc;
    SlicedSet sr, sc;               // XCD-sliced CSR (dual) and CSC (primal)
    void *part_slices = nullptr;    // compact per-slice segment sums
    int chk_nr = 0, chk_nc = 0;     // partial-sum entries of the last check passes
    void *carries = nullptr;
    double *part_r = nullptr, *part_c = nullptr;
    int *perm_row = nullptr, *perm_col = nullptr;
    std::vector<int32_t> h_perm_row, h_perm_col;
    // problem vectors (permuted)
    double *c0 = nullptr, *clo0 = nullptr, *chi0 = nullptr, *vlo0 = nullptr, *vhi0 = nullptr;
    double *c = nullptr, *clo = nullptr, *chi = nullptr, *vlo = nullptr, *vhi = nullptr;
    double *dr = nullptr, *dc = nullptr, *fr = nullptr, *fc = nullptr;
    // iterate, FP64
    double *x = nullptr, *y = nullptr, *xbar = nullptr, *xa = nullptr, *ya = nullptr;
    double *xh = nullptr, *yh = nullptr, *dx = nullptr, *dy = nullptr;
    // iterate and data, FP32 (mixed precision)
    float *x32 = nullptr, *y32 = nullptr, *xbar32 = nullptr, *xa32 = nullptr, *ya32 = nullptr;
    float *c32 = nullptr, *clo32 = nullptr, *chi32 = nullptr, *vlo32 = nullptr, *vhi32 = nullptr;
    double *xbest = nullptr, *ybest = nullptr;  // T(z) of the FP32 phase's best check
    // diagonal QP (Sec. 6): scaled, permuted diag(Q) (and its FP32 copy in
    // FP32-mixed mode); used when has_q
    double *qd = nullptr;
    float *q32 = nullptr;
    bool has_q = false;
    // scratch
    double *tmp_m = nullptr, *tmp_n = nullptr, *tmp_m2 = nullptr, *tmp_n2 = nullptr;
    double *scal = nullptr;         // device scalars: [4..7] norms, [8] beta, [9] alpha (Lanczos)
    double *norm_part = nullptr;
    double *sig_hist = nullptr;
    Control *ctl = nullptr;
    Control *ctl_eval = nullptr;    // scratch block for dpdlp_kkt
    Control *h_ctl = nullptr;       // pinned
    // host-side scalars
    double eta = 0, sigma_max = 0, omega0 = 0, c_norm = 0, b_norm = 0;
    int power_iters = 0;
    double omega = 1.0;
    int64_t k = 0, t = 0, fp32_iters = 0;
    int32_t status = DPDLP_RUNNING;
    bool in_fp32 = false;
    double fp32_ref_kkt = INFINITY;
    double fp32_best_kkt = INFINITY, fp32_best_omega = 1.0;
    int fp32_stall = 0;
    bool initialized = false;
    double setup_seconds = 0, solve_seconds = 0;
    std::vector<dpdlp_log_rec> log;
    // graph replay of the runs between checks
    IterDev *iterdev = nullptr;
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    hipStream_t gstream = nullptr;
    // profiling
    bool prof = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[8];
    std::vector<hipEvent_t> ev_pool;
    double prof_ms[8] = {0};
    int64_t prof_n[8] = {0};
};

namespace dpdlp {

static int hip_fail(hipError_t e, const char *what)
{
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? DPDLP_E_OOM : DPDLP_E_HIP;
}

#define HIPCHK(expr)                                              \
    do {                                                          \
        hipError_t _e = (expr);                                   \
        if (_e != hipSuccess) return hip_fail(_e, #expr);         \
    } while (0)

template <typename T>
static int dalloc(dpdlp_problem *P, T **p, size_t count)
{
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc");
    P->mem.ptrs.push_back(q);
    *p = (T *)q;
    return DPDLP_OK;
}

#define CHK(expr)                         \
    do {                                  \
        int _r = (expr);                  \
        if (_r != DPDLP_OK) return _r;    \
    } while (0)

static inline unsigned nblk(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

template <class Op>
static void launch_tiles(dpdlp_problem *P, const Op &op, const TileSet &ts, const int *seg_ptr,
                         const int *idx, const typename Op::MT *val)
{
    if (ts.n == 0) return;
    const int remap = P->prm.xcd_remap ? 1 : 0;
    const int grid = ts.blk2tile ? ts.grid : (remap ? ((ts.n + 7) / 8) * 8 : ts.n);
    hipLaunchKernelGGL(k_tile<Op>, dim3(grid), dim3(kBlock), 0, P->s, op, ts.d, ts.n, ts.blk2tile,
                       ts.seg_stride, seg_ptr, idx, val, (const uint16_t *)ts.pos,
                       (typename Op::AT *)P->carries, remap);
    if (ts.nsplit)
        hipLaunchKernelGGL(k_split_fix<Op>, dim3((ts.nsplit + 63) / 64), dim3(64), 0, P->s, op,
                           ts.splits, ts.nsplit, ts.n, (const typename Op::AT *)P->carries);
}

// ---- profiling helpers -----------------------------------------------------
static hipEvent_t prof_event(dpdlp_problem *P)
{
    if (!P->ev_pool.empty()) {
        hipEvent_t e = P->ev_pool.back();
        P->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}
struct ProfScope {
    dpdlp_problem *P;
    int cls;
    hipEvent_t b = nullptr;
    ProfScope(dpdlp_problem *P_, int c) : P(P_), cls(c)
    {
        if (P->prof) { b = prof_event(P); (void)hipEventRecord(b, P->s); }
    }
    ~ProfScope()
    {
        if (P->prof) {
            hipEvent_t e = prof_event(P);
            (void)hipEventRecord(e, P->s);
            P->ev[cls].push_back({b, e});
        }
    }
};
static void prof_collect(dpdlp_problem *P)
{
    for (int c = 0; c < 8; ++c) {
        for (auto &pr : P->ev[c]) {
            float ms = 0.f;
            if (hipEventSynchronize(pr.second) == hipSuccess &&
                hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) {
                P->prof_ms[c] += ms;
                P->prof_n[c] += 1;
            }
            P->ev_pool.push_back(pr.first);
            P->ev_pool.push_back(pr.second);
        }
        P->ev[c].clear();
    }
}

// ---- the fused steps -------------------------------------------------------
// The primal step with its epilogue Op (PrimalOp, or PrimalQPOp for a QP):
// sliced (per-slice partial sums, then the combine runs the epilogue) or on
// the CSC tiles.
template <typename T, class Op>
static void run_primal(dpdlp_problem *P, const Op &op, const T *y, const T *vt)
{
    if (P->sc.S > 0) {
        PartialOp<T> po;
        po.v = y; po.partial = (T *)P->part_slices; po.partials = nullptr;
        launch_tiles(P, po, P->sc.ts, P->sc.ptr, P->sc.idx,
                     (const T *)(sizeof(T) == 8 ? (const void *)P->sc.val : (const void *)P->sc.val32));
        hipLaunchKernelGGL(k_combine<Op>, dim3(nblk(P->n)), dim3(kBlock), 0, P->s, op, P->n,
                           P->sc.S, (const T *)P->part_slices, P->sc.mask, P->sc.cbase, P->sc.G);
        return;
    }
    launch_tiles(P, op, P->tc, P->cp, P->ri, vt);
}

template <typename T>
static void launch_primal(dpdlp_problem *P, const T *y, const T *c, const T *lo, const T *hi,
                          const T *xa, T *x, T *xbar, const T *vt, double tau, int64_t k,
                          int write_hat, const IterDev *dev = nullptr, int j = 0)
{
    PrimalOp<T> op;
    op.dev = dev;
    op.j = j;
    op.y = y; op.c = c; op.lo = lo; op.hi = hi; op.xa = xa; op.x = x; op.xbar = xbar;
    op.xh = P->xh; op.dx = P->dx; op.partials = nullptr;
    op.tau = (T)tau;
    op.a = (T)((double)(k + 1) / (double)(k + 2));
    op.b = (T)(1.0 / (double)(k + 2));
    op.gamma = (T)P->prm.gamma;
    op.write_hat = write_hat;
    if (P->has_q) {
        PrimalQPOp<T> qop;
        static_cast<PrimalOp<T> &>(qop) = op;
        if constexpr (sizeof(T) == 8) qop.q = P->qd;
        else qop.q = P->q32;
        run_primal<T>(P, qop, y, vt);
        return;
    }
    run_primal<T>(P, op, y, vt);
}

template <typename T>
static void launch_dual(dpdlp_problem *P, const T *xbar, const T *lo, const T *hi, const T *ya,
                        T *y, const T *v, double sigma, int64_t k, int write_hat,
                        const IterDev *dev = nullptr, int j = 0)
{
    DualOp<T> op;
    op.dev = dev;
    op.j = j;
    op.xbar = xbar; op.lo = lo; op.hi = hi; op.ya = ya; op.y = y;
    op.yh = P->yh; op.dy = P->dy; op.partials = nullptr;
    op.sigma = (T)sigma;
    op.a = (T)((double)(k + 1) / (double)(k + 2));
    op.b = (T)(1.0 / (double)(k + 2));
    op.gamma = (T)P->prm.gamma;
    op.write_hat = write_hat;
    if (P->sr.S > 0) {
        PartialOp<T> po;
        po.v = xbar; po.partial = (T *)P->part_slices; po.partials = nullptr;
        launch_tiles(P, po, P->sr.ts, P->sr.ptr, P->sr.idx,
                     (const T *)(sizeof(T) == 8 ? (const void *)P->sr.val : (const void *)P->sr.val32));
        hipLaunchKernelGGL(k_combine<DualOp<T>>, dim3(nblk(P->m)), dim3(kBlock), 0, P->s, op, P->m,
                           P->sr.S, (const T *)P->part_slices, P->sr.mask, P->sr.cbase, P->sr.G);
        return;
    }
    launch_tiles(P, op, P->tr, P->rp, P->ci, v);
}

// One PDHG + Halpern iteration in the current precision.  With dev set, the
// step sizes and the Halpern index (k0 + j) are read from device memory (graph
// replays); the arguments tau, sigma, k are then unused.
static void pdhg_iteration(dpdlp_problem *P, double tau, double sigma, int64_t k, int write_hat,
                           const IterDev *dev = nullptr, int j = 0)
{
    if (P->in_fp32) {
        { ProfScope ps(P, 0);
          launch_primal<float>(P, P->y32, P->c32, P->vlo32, P->vhi32, P->xa32, P->x32, P->xbar32,
                               P->vt32, tau, k, write_hat, dev, j); }
        { ProfScope ps(P, 1);
          launch_dual<float>(P, P->xbar32, P->clo32, P->chi32, P->ya32, P->y32, P->v32, sigma, k,
                             write_hat, dev, j); }
    } else {
        { ProfScope ps(P, 0);
          launch_primal<double>(P, P->y, P->c, P->vlo, P->vhi, P->xa, P->x, P->xbar, P->vt, tau,
                                k, write_hat, dev, j); }
        { ProfScope ps(P, 1);
          launch_dual<double>(P, P->xbar, P->clo, P->chi, P->ya, P->y, P->v, sigma, k,
                              write_hat, dev, j); }
    }
}

__global__ void k_set_iter(IterDev *d, double tau, double sigma, long long k0)
{
    d->tau = tau;
    d->sigma = sigma;
    d->k0 = k0;
}

// The check_period - 1 iterations between two checks as one HIP graph (one
// per precision), captured on a private stream on first use and replayed on
// the solver's stream after k_set_iter has written the run's scalars.
static int run_graph(dpdlp_problem *P, double tau, double sigma, int64_t k0, int L)
{
    hipGraphExec_t &ge = P->graph[P->in_fp32 ? 1 : 0];
    if (!ge) {
        if (!P->gstream) HIPCHK(hipStreamCreateWithFlags(&P->gstream, hipStreamNonBlocking));
        hipStream_t saved = P->s;
        P->s = P->gstream;
        HIPCHK(hipStreamBeginCapture(P->gstream, hipStreamCaptureModeThreadLocal));
        for (int j = 0; j < L; ++j) pdhg_iteration(P, 0.0, 0.0, 0, 0, P->iterdev, j);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(P->gstream, &g);
        P->s = saved;
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) { ge = nullptr; return hip_fail(e, "hipGraphInstantiate"); }
    }
    hipLaunchKernelGGL(k_set_iter, dim3(1), dim3(1), 0, P->s, P->iterdev, tau, sigma, (long long)k0);
    HIPCHK(hipGraphLaunch(ge, P->s));
    return DPDLP_OK;
}

static void drop_graphs(dpdlp_problem *P)
{
    for (auto &g : P->graph)
        if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
}

// A single-right-hand-side product pass with a per-segment epilogue (SpmvOp,
// LanczosOp: out = f(A~ in) and per-block sums of out^2), on the XCD-sliced
// format when that product has one.  transpose: A~^T (CSC, segments are
// columns).  Returns the number of partial-sum entries left in op.partials.
template <class Op>
static int launch_product(dpdlp_problem *P, bool transpose, const Op &op, const double *in)
{
    const SlicedSet &ss = transpose ? P->sc : P->sr;
    const int nseg = transpose ? P->n : P->m;
    if (ss.S > 0) {
        PartialOp<double> po;
        po.v = in; po.partial = (double *)P->part_slices; po.partials = nullptr;
        launch_tiles(P, po, ss.ts, ss.ptr, ss.idx, ss.val);
        hipLaunchKernelGGL(k_combine<Op>, dim3(nblk(nseg)), dim3(kBlock), 0, P->s, op, nseg, ss.S,
                           (const double *)P->part_slices, ss.mask, ss.cbase, ss.G);
        return (int)nblk(nseg);
    }
    if (transpose) launch_tiles(P, op, P->tc, P->cp, P->ri, P->vt);
    else launch_tiles(P, op, P->tr, P->rp, P->ci, P->v);
    return transpose ? P->tc.n : P->tr.n;
}

// Check passes at (xh, yh, dx, dy) against the anchor (xa_any, ya_any),
// on the XCD-sliced formats where the fused steps use
// them (partial sums per slice, then a combine that runs the check's
// epilogue).  Sets chk_nr / chk_nc, the number of partial-sum entries per
// quantity that k_control adds.
template <typename TA>
static void launch_checks(dpdlp_problem *P, const double *xh, const double *dx, const double *yh,
                          const double *dy, const TA *xa, const TA *ya, double tau)
{
    {
        ProfScope ps(P, 2);
        CheckRowOp<TA> op;
        op.xh = xh; op.dx = dx; op.yh = yh; op.dy = dy; op.ya = ya;
        op.dr = P->dr; op.lo0 = P->clo0; op.hi0 = P->chi0; op.partials = P->part_r;
        if (P->sr.S > 0) {
            PartialOp2 po;
            po.v = xh; po.v2 = dx; po.partial = (double *)P->part_slices; po.G = P->sr.G;
            po.partials = nullptr;
            launch_tiles(P, po, P->sr.ts, P->sr.ptr, P->sr.idx, P->sr.val);
            hipLaunchKernelGGL(k_combine<CheckRowOp<TA>>, dim3(nblk(P->m)), dim3(kBlock), 0, P->s, op,
                               P->m, P->sr.S, (const double *)P->part_slices, P->sr.mask,
                               P->sr.cbase, P->sr.G);
            P->chk_nr = nblk(P->m);
        } else {
            launch_tiles(P, op, P->tr, P->rp, P->ci, P->v);
            P->chk_nr = P->tr.n;
        }
    }
    {
        ProfScope ps(P, 3);
        CheckColOp<TA> op;
        op.yh = yh; op.xh = xh; op.dx = dx; op.xa = xa; op.c = P->c; op.c0 = P->c0;
        op.lo = P->vlo; op.hi = P->vhi; op.dc = P->dc; op.partials = P->part_c; op.tau = tau;
        op.q = P->has_q ? P->qd : nullptr;
        if (P->sc.S > 0) {
            PartialOp<double> po;
            po.v = yh; po.partial = (double *)P->part_slices; po.partials = nullptr;
            launch_tiles(P, po, P->sc.ts, P->sc.ptr, P->sc.idx, P->sc.val);
            hipLaunchKernelGGL(k_combine<CheckColOp<TA>>, dim3(nblk(P->n)), dim3(kBlock), 0, P->s, op,
                               P->n, P->sc.S, (const double *)P->part_slices, P->sc.mask,
                               P->sc.cbase, P->sc.G);
            P->chk_nc = nblk(P->n);
        } else {
            launch_tiles(P, op, P->tc, P->cp, P->ri, P->vt);
            P->chk_nc = P->tc.n;
        }
    }
}

static CtlArgs ctl_args(dpdlp_problem *P, int mode)
{
    CtlArgs a{};
    a.k = P->k; a.t = P->t; a.eta = P->eta; a.eps = P->prm.eps;
    a.beta_suf = P->prm.beta_suf; a.beta_nec = P->prm.beta_nec; a.beta_art = P->prm.beta_art;
    a.kp = P->prm.kp; a.ki = P->prm.ki; a.kd = P->prm.kd;
    a.c_norm = P->c_norm; a.b_norm = P->b_norm; a.mode = mode;
    return a;
}

static int read_ctl(dpdlp_problem *P)
{
    HIPCHK(hipMemcpyAsync(P->h_ctl, P->ctl, sizeof(Control), hipMemcpyDeviceToHost, P->s));
    HIPCHK(hipStreamSynchronize(P->s));
    return DPDLP_OK;
}

// ---- setup -----------------------------------------------------------------
static int upload(dpdlp_problem *P, void *dst, const void *src, size_t bytes)
{
    HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, P->s));
    return DPDLP_OK;
}

static int build_tileset(dpdlp_problem *P, const hvec<int32_t> &ptr, int32_t nseg,
                         TileSet &ts, std::vector<Tile> &host_tiles)
{
    build_tiles(ptr.data(), nseg, P->prm.tile_nnz, host_tiles);
    ts.n = (int)host_tiles.size();
    std::vector<SplitSeg> sp;
    for (int i = 0; i < ts.n; ++i) {
        const Tile &t = host_tiles[(size_t)i];
        if (t.npieces > 0 && t.piece == 0) sp.push_back(SplitSeg{t.seg_begin, i, t.npieces, t.slice});
    }
    ts.nsplit = (int)sp.size();
    CHK(dalloc(P, &ts.d, host_tiles.size()));
    CHK(upload(P, ts.d, host_tiles.data(), host_tiles.size() * sizeof(Tile)));
    if (ts.nsplit) {
        CHK(dalloc(P, &ts.splits, sp.size()));
        CHK(upload(P, ts.splits, sp.data(), sp.size() * sizeof(SplitSeg)));
    }
    HIPCHK(hipStreamSynchronize(P->s));     // host vectors are reused by the caller
    return DPDLP_OK;
}

// Sliced copy of one format: tiles of slice s run on XCD s % 8 (workgroup b
// runs on XCD b % 8), the slices of one XCD one after another.  gptr is the
// gathered dimension's pointer array (slices hold equal nonzero counts).
static int build_sliced(dpdlp_problem *P, const hvec<int32_t> &ptr,
                        const hvec<int32_t> &idx, const hvec<int32_t> &gptr, int32_t nseg,
                        int32_t nidx, int S, SlicedSet &ss)
{
    SlicedHost sh;
    slice_format(ptr, idx, gptr, nseg, nidx, S, P->prm.tile_nnz, sh);
    ss.S = S;
    const size_t nnz = sh.idx.size();
    // gather-sorted tiles where that cuts the cache lines one wave's gathers
    // touch by at least a quarter (16 FP64 entries per 128-byte line)
    hvec<uint16_t> pos;
    if (nnz && P->prm.gather_sort != 0) {
        const int64_t l0 = tile_gather_lines(sh.tiles, sh.idx, 16, false);
        const int64_t l1 = tile_gather_lines(sh.tiles, sh.idx, 16, true);
        if (P->prm.gather_sort > 0 || (double)l1 <= 0.75 * (double)l0) {
            sort_tiles_by_gather(sh.tiles, sh.idx, sh.src, pos);
            CHK(dalloc(P, &ss.ts.pos, nnz));
            CHK(upload(P, ss.ts.pos, pos.data(), nnz * sizeof(uint16_t)));
        }
    }
    CHK(dalloc(P, &ss.ptr, sh.ptr.size()));
    CHK(dalloc(P, &ss.idx, nnz));
    CHK(dalloc(P, &ss.src, nnz));
    CHK(dalloc(P, &ss.val, nnz));
    CHK(upload(P, ss.ptr, sh.ptr.data(), sh.ptr.size() * sizeof(int32_t)));
    ss.G = sh.G;
    CHK(dalloc(P, &ss.mask, std::max<size_t>(sh.mask.size(), 1)));
    CHK(dalloc(P, &ss.cbase, std::max<size_t>(sh.cbase.size(), 1)));
    if (!sh.mask.empty()) CHK(upload(P, ss.mask, sh.mask.data(), sh.mask.size()));
    if (!sh.cbase.empty()) CHK(upload(P, ss.cbase, sh.cbase.data(), sh.cbase.size() * sizeof(int32_t)));
    if (nnz) {
        CHK(upload(P, ss.idx, sh.idx.data(), nnz * sizeof(int32_t)));
        CHK(upload(P, ss.src, sh.src.data(), nnz * sizeof(int32_t)));
    }
    TileSet &ts = ss.ts;
    ts.n = (int)sh.tiles.size();
    ts.seg_stride = 0;              // compact segments are numbered globally
    std::vector<SplitSeg> sp;
    std::vector<std::vector<int>> per(8);
    for (int i = 0; i < ts.n; ++i) {
        const Tile &tl = sh.tiles[(size_t)i];
        if (tl.npieces > 0 && tl.piece == 0) sp.push_back(SplitSeg{tl.seg_begin, i, tl.npieces, tl.slice});
        per[(size_t)(tl.slice % 8)].push_back(i);
    }
    size_t mx = 0;
    for (auto &v : per) mx = std::max(mx, v.size());
    std::vector<int> b2t(8 * mx, -1);
    for (size_t x = 0; x < 8; ++x)
        for (size_t q = 0; q < per[x].size(); ++q) b2t[8 * q + x] = per[x][q];
    ts.grid = (int)b2t.size();
    ts.nsplit = (int)sp.size();
    CHK(dalloc(P, &ts.d, sh.tiles.size()));
    CHK(upload(P, ts.d, sh.tiles.data(), sh.tiles.size() * sizeof(Tile)));
    CHK(dalloc(P, &ts.blk2tile, b2t.size()));
    CHK(upload(P, ts.blk2tile, b2t.data(), b2t.size() * sizeof(int)));
    if (ts.nsplit) {
        CHK(dalloc(P, &ts.splits, sp.size()));
        CHK(upload(P, ts.splits, sp.data(), sp.size() * sizeof(SplitSeg)));
    }
    HIPCHK(hipStreamSynchronize(P->s));
    return DPDLP_OK;
}

// sigma_max(A~) by Golub-Kahan-Lanczos bidiagonalization from one seeded
// start (no reorthogonalisation; the largest Ritz value converges from
// below):
//   z_k = A~ v_k - beta_k u_(k-1),     alpha_k = ||z_k||,   u_k = z_k / alpha_k
//   w_k+1 = A~^T u_k - alpha_k v_k,    beta_k+1 = ||w_k+1||, v_k+1 = w_k+1 / beta_k+1
// The estimate after k steps is sigma_max of the k x k upper bidiagonal
// (alpha, beta).  It stops when the estimate grew by at most power_tol
// (relative) over the last 8 steps (k >= 16), at a breakdown (exact), or
// after max_steps steps.
static int lanczos_sigma(dpdlp_problem *P, uint64_t seed, int max_steps, double *sigma, int *steps)
{
    const int maxit = std::max(1, max_steps);
    const int32_t n = P->n;
    double *w = P->tmp_n2, *z = P->tmp_m;
    double *beta = P->scal + 8, *alpha = P->scal + 9;
    double *ha = P->sig_hist, *hb = P->sig_hist + (maxit + 2);
    {
        std::vector<double> w0((size_t)n);
        const double b1 = lanczos_start(n, seed, w0.data());
        CHK(upload(P, w, w0.data(), sizeof(double) * (size_t)n));
        CHK(upload(P, beta, &b1, sizeof(double)));
    }
    std::vector<double> al((size_t)maxit + 2, 0.0), be((size_t)maxit + 2, 0.0);
    std::vector<double> est((size_t)maxit + 2, 0.0);
    int stop = -1, k_done = 0;
    const int chunk = 16, window = 8;
    for (int k0 = 1; k0 <= maxit && stop < 0; k0 += chunk) {
        const int k1 = std::min(maxit, k0 + chunk - 1);
        for (int k = k0; k <= k1; ++k) {
            LanczosOp a;
            a.in = w; a.out = z; a.nin = beta; a.nprev = alpha; a.first = k == 1;
            a.partials = P->part_r;
            const int na = launch_product(P, false, a, w);
            hipLaunchKernelGGL(k_lanczos_norm, dim3(1), dim3(kBlock), 0, P->s, P->part_r, na,
                               alpha, ha, k);
            LanczosOp b;
            b.in = z; b.out = w; b.nin = alpha; b.nprev = beta; b.first = 0;
            b.partials = P->part_c;
            const int nb = launch_product(P, true, b, z);
            hipLaunchKernelGGL(k_lanczos_norm, dim3(1), dim3(kBlock), 0, P->s, P->part_c, nb,
                               beta, hb, k + 1);
        }
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(al.data() + k0, ha + k0, sizeof(double) * (size_t)(k1 - k0 + 1),
                              hipMemcpyDeviceToHost, P->s));
        HIPCHK(hipMemcpyAsync(be.data() + k0 + 1, hb + k0 + 1, sizeof(double) * (size_t)(k1 - k0 + 1),
                              hipMemcpyDeviceToHost, P->s));
        HIPCHK(hipStreamSynchronize(P->s));
        for (int k = k0; k <= k1; ++k) {
            if (!(al[(size_t)k] > 0.0) || !std::isfinite(al[(size_t)k])) { stop = k - 1; break; }
            est[(size_t)k] = bidiag_sigma_max(al.data() + 1, be.data() + 1, k);
            k_done = k;
            if (!(be[(size_t)k + 1] > 0.0)) { stop = k; break; }      // invariant subspace: exact
            if (k >= 2 * window &&
                est[(size_t)k] - est[(size_t)(k - window)] <= P->prm.power_tol * est[(size_t)k]) {
                stop = k;
                break;
            }
        }
    }
    if (stop < 0) stop = k_done;
    *sigma = stop >= 1 ? est[(size_t)stop] : 0.0;
    *steps = stop;
    return DPDLP_OK;
}

// sigma_max(A~): the larger of two Lanczos estimates from independent
// starts (a start nearly orthogonal to the top singular vector can settle
// on the second singular value).
static int estimate_sigma_max(dpdlp_problem *P)
{
    double s1 = 0, s2 = 0;
    int k1 = 0, k2 = 0;
    CHK(lanczos_sigma(P, P->prm.perm_seed ^ 0x5EED1A2Cull, P->prm.power_max_iters, &s1, &k1));
    CHK(lanczos_sigma(P, P->prm.perm_seed ^ 0x7A11C0DEull, P->prm.power_max_iters, &s2, &k2));
    P->sigma_max = std::max(s1, s2);
    P->power_iters = k1 + k2;
    return DPDLP_OK;
}

// Every device buffer a kernel of the solve path writes or reads must be
// allocated; a missing one is reported here instead of reaching a kernel.
static int check_buffers(dpdlp_problem *P)
{
    const void *req[] = {P->rp, P->ci, P->v, P->cp, P->ri, P->vt, P->tr.d, P->tc.d, P->carries,
                         P->part_r, P->part_c, P->perm_row, P->perm_col, P->c0, P->clo0,
                         P->chi0, P->vlo0, P->vhi0, P->c, P->clo, P->chi, P->vlo, P->vhi, P->dr,
                         P->dc, P->fr, P->fc, P->x, P->y, P->xbar, P->xa, P->ya, P->xh, P->yh,
                         P->dx, P->dy, P->tmp_m, P->tmp_n, P->tmp_m2, P->tmp_n2, P->scal,
                         P->sig_hist, P->ctl, P->ctl_eval, P->iterdev, P->h_ctl};
    for (const void *p : req)
        if (!p) { set_error("internal: a device buffer is not allocated"); return DPDLP_E_HIP; }
    if ((P->tr.nsplit && !P->tr.splits) || (P->tc.nsplit && !P->tc.splits)) {
        set_error("internal: split list not allocated");
        return DPDLP_E_HIP;
    }
    for (const SlicedSet *ss : {&P->sr, &P->sc})
        if (ss->S > 0 && (!ss->ptr || !ss->idx || !ss->val || !ss->ts.d || !ss->ts.blk2tile ||
                          !ss->mask || !ss->cbase ||
                          !P->part_slices || (ss->ts.nsplit && !ss->ts.splits))) {
            set_error("internal: sliced buffers not allocated");
            return DPDLP_E_HIP;
        }
    if (P->prm.precision == DPDLP_FP32_MIXED) {
        const void *r32[] = {P->v32, P->vt32, P->x32, P->y32, P->xbar32, P->xa32, P->ya32,
                             P->c32, P->clo32, P->chi32, P->vlo32, P->vhi32, P->xbest, P->ybest};
        for (const void *p : r32)
            if (!p) { set_error("internal: FP32 buffer not allocated"); return DPDLP_E_HIP; }
        for (const SlicedSet *ss : {&P->sr, &P->sc})
            if (ss->S > 0 && !ss->val32) { set_error("internal: FP32 sliced values"); return DPDLP_E_HIP; }
    }
    return DPDLP_OK;
}

// Scaled problem vectors (c~, bounds) and the norms used by the KKT
// denominators and omega0, from the permuted original vectors and D_r, D_c.
static int scale_data(dpdlp_problem *P)
{
    const int32_t m = P->m, n = P->n;
    hipLaunchKernelGGL(k_scale_vectors, dim3(nblk(std::max(m, n))), dim3(kBlock), 0, P->s, m, n,
                       P->dr, P->dc, P->c0, P->vlo0, P->vhi0, P->clo0, P->chi0, P->c, P->vlo,
                       P->vhi, P->clo, P->chi);
    const unsigned nb = nblk(std::max(m, n));
    if (!P->norm_part) CHK(dalloc(P, &P->norm_part, (size_t)4 * nb));
    hipLaunchKernelGGL(k_norm_partials, dim3(nb), dim3(kBlock), 0, P->s, m, n, P->c0, P->clo0,
                       P->chi0, P->c, P->clo, P->chi, P->norm_part);
    hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(kBlock), 0, P->s, P->norm_part, (int)nb, 4,
                       P->scal + 4);
    double h[4];
    HIPCHK(hipMemcpyAsync(h, P->scal + 4, sizeof(h), hipMemcpyDeviceToHost, P->s));
    HIPCHK(hipStreamSynchronize(P->s));
    P->c_norm = std::sqrt(h[0]);
    P->b_norm = std::sqrt(h[1]);
    const double cns = std::sqrt(h[2]), bns = std::sqrt(h[3]);
    if (P->prm.omega0 > 0) P->omega0 = P->prm.omega0;
    else if (cns > 1e-10 && bns > 1e-10) P->omega0 = cns / bns;
    else P->omega0 = 1.0;
    if (P->prm.precision == DPDLP_FP32_MIXED && P->c32) {
        auto cv = [&](const double *a, float *b, int64_t k) {
            hipLaunchKernelGGL((k_convert<double, float>), dim3(nblk(k)), dim3(kBlock), 0, P->s, a, b, k);
        };
        cv(P->c, P->c32, n); cv(P->vlo, P->vlo32, n); cv(P->vhi, P->vhi32, n);
        cv(P->clo, P->clo32, m); cv(P->chi, P->chi32, m);
    }
    HIPCHK(hipGetLastError());
    return DPDLP_OK;
}

static int create_impl(const dpdlp_csr_lp *lp_in, const dpdlp_params *params, void *stream,
                       dpdlp_problem **out)
{
    auto t_start = std::chrono::steady_clock::now();
    if (!lp_in || !out) { set_error("NULL argument"); return DPDLP_E_INVALID_ARG; }
    *out = nullptr;
    if (!mem_kind_ok(lp_in->mem_kind)) return bad_mem_kind();
    // Host copy of the input (device inputs are brought over for the integer
    // preprocessing).
    dpdlp_csr_lp lp = *lp_in;
    std::vector<int32_t> h_rp, h_ci;
    std::vector<double> h_v, h_c, h_clo, h_chi, h_vlo, h_vhi;
    if (lp.mem_kind == DPDLP_MEM_DEVICE) {
        if (lp.m < 1 || lp.n < 1 || !lp.row_ptr) { set_error("bad sizes"); return DPDLP_E_INVALID_ARG; }
        h_rp.resize((size_t)lp.m + 1);
        HIPCHK(hipMemcpy(h_rp.data(), lp.row_ptr, sizeof(int32_t) * h_rp.size(), hipMemcpyDeviceToHost));
        const int64_t nz = h_rp[(size_t)lp.m];
        if (nz < 0) { set_error("row_ptr[m] < 0"); return DPDLP_E_BAD_CSR; }
        h_ci.resize((size_t)nz); h_v.resize((size_t)nz);
        if (nz) {
            HIPCHK(hipMemcpy(h_ci.data(), lp.col_idx, sizeof(int32_t) * (size_t)nz, hipMemcpyDeviceToHost));
            HIPCHK(hipMemcpy(h_v.data(), lp.val, sizeof(double) * (size_t)nz, hipMemcpyDeviceToHost));
        }
        auto cpv = [&](std::vector<double> &h, const double *d, int32_t k) -> int {
            h.resize((size_t)k);
            if (!d) { set_error("NULL vector"); return DPDLP_E_INVALID_ARG; }
            HIPCHK(hipMemcpy(h.data(), d, sizeof(double) * (size_t)k, hipMemcpyDeviceToHost));
            return DPDLP_OK;
        };
        CHK(cpv(h_c, lp.c, lp.n)); CHK(cpv(h_vlo, lp.var_lo, lp.n)); CHK(cpv(h_vhi, lp.var_hi, lp.n));
        CHK(cpv(h_clo, lp.con_lo, lp.m)); CHK(cpv(h_chi, lp.con_hi, lp.m));
        lp.row_ptr = h_rp.data(); lp.col_idx = h_ci.data(); lp.val = h_v.data();
        lp.c = h_c.data(); lp.var_lo = h_vlo.data(); lp.var_hi = h_vhi.data();
        lp.con_lo = h_clo.data(); lp.con_hi = h_chi.data();
        lp.mem_kind = DPDLP_MEM_HOST;
    }
    CHK(validate_host(&lp));

    dpdlp_problem *P = new dpdlp_problem();
    std::unique_ptr<dpdlp_problem> guard(P);
    if (params) P->prm = *params; else dpdlp_params_default(&P->prm);
    if (P->prm.tile_nnz <= 0) {
        // automatic: the power of two (256..2048) nearest, on a log scale,
        // to nnz / 800, i.e. about 800 tiles per step where the problem is
        // small enough: fewer tiles than one round of resident workgroups
        // (256 CUs x 5), each long enough to hide its memory round trips
        const double tn = (double)lp.row_ptr[lp.m] / 800.0;
        int32_t p2 = 256;
        while (p2 < kTileNnzMax && tn > (double)p2 * 1.4142135623730951) p2 <<= 1;
        P->prm.tile_nnz = p2;
    }
    if (P->prm.tile_nnz > kTileNnzMax) P->prm.tile_nnz = kTileNnzMax;
    if (P->prm.check_period < 1) P->prm.check_period = 1;
    if (P->prm.perm_order < 0 || P->prm.perm_order > 3) {
        set_error("perm_order must be 0..3 (bit 0: rows hot-first, bit 1: columns hot-first)");
        return DPDLP_E_INVALID_ARG;
    }
    P->s = (hipStream_t)stream;
    P->m = lp.m; P->n = lp.n; P->nnz = lp.row_ptr[lp.m];
    const int32_t m = P->m, n = P->n;
    const size_t nnz = (size_t)P->nnz;

    // A1 + A0: block-wise random permutation, then the CSC copy (host).
    HostMatrix H;
    permute_and_transpose(&lp, P->prm.perm_block, P->prm.perm_seed, P->prm.perm_order, H);
    P->h_perm_row = H.perm_row;
    P->h_perm_col = H.perm_col;

    CHK(dalloc(P, &P->rp, (size_t)m + 1)); CHK(dalloc(P, &P->ci, nnz)); CHK(dalloc(P, &P->v, nnz));
    CHK(dalloc(P, &P->cp, (size_t)n + 1)); CHK(dalloc(P, &P->ri, nnz)); CHK(dalloc(P, &P->vt, nnz));
    CHK(upload(P, P->rp, H.rp.data(), sizeof(int32_t) * ((size_t)m + 1)));
    CHK(upload(P, P->cp, H.cp.data(), sizeof(int32_t) * ((size_t)n + 1)));
    if (nnz) {
        CHK(upload(P, P->ci, H.ci.data(), sizeof(int32_t) * nnz));
        CHK(upload(P, P->v, H.v.data(), sizeof(double) * nnz));
        CHK(upload(P, P->ri, H.ri.data(), sizeof(int32_t) * nnz));
        CHK(upload(P, P->vt, H.vt.data(), sizeof(double) * nnz));
    }
    // A2: nonzero-aware workgroup tiles for both formats
    std::vector<Tile> ht;
    CHK(build_tileset(P, H.rp, m, P->tr, ht));
    CHK(build_tileset(P, H.cp, n, P->tc, ht));
    int ntmax = std::max(P->tr.n, P->tc.n);
    // XCD-sliced fused steps: S > 0 slices both steps; S < 0 (automatic)
    // slices a step when its gathered vector exceeds one XCD's L2 (4 MB),
    // when the gathers of one XCD's resident tiles (5 workgroups on each of
    // its 32 CUs, a contiguous run of tiles) touch more than half an L2 of
    // it (so the order gives them no locality of their own), and when its
    // compact partial sums (written and read, 8 + 8 bytes, plus a 4-byte
    // pointer per compact segment) cost less than its matrix stream (12
    // bytes per nonzero); with S = 16 where 8 slices would still leave more
    // than 2 MB per slice (in the iterate's precision) of a vector that is
    // gathered at least 4 times per pass, else S = 8; never when the
    // gathered dimension is in hot-first order (the order itself gives the
    // cache locality).
    int Sd = 0, Sp = 0;                 // dual (CSR, gathers x), primal (CSC, gathers y)
    if (P->prm.gather_slices > 0) {
        if (P->prm.gather_slices % 8 != 0 || P->prm.gather_slices > 64) {
            set_error("gather_slices must be -1, 0 or a multiple of 8 up to 64");
            return DPDLP_E_INVALID_ARG;
        }
        Sd = Sp = P->prm.gather_slices;
    } else if (P->prm.gather_slices < 0) {
        const double mat = 12.0 * (double)nnz, l2 = 4.0 * (1 << 20);
        const double eb = P->prm.precision == DPDLP_FP32_MIXED ? 4.0 : 8.0;   // gathered element
        const bool hot_rows = P->prm.perm_order & 1, hot_cols = P->prm.perm_order & 2;
        auto pick = [&](const hvec<int32_t> &ptr, const hvec<int32_t> &idx,
                        const hvec<int32_t> &gptr, int32_t nseg, int32_t nidx) -> int {
            if (8.0 * nidx <= l2) return 0;
            // (the footprint is measured with FP64 entries, 16 per line, in
            // both precisions: an FP32 footprint is smaller only where
            // consecutive entries are gathered, and slicing such a step
            // still pays in FP32 - on c2's dual step 0.109 ms unsliced)
            const int64_t window = (int64_t)32 * 5 * P->prm.tile_nnz;
            if (gather_window_bytes(idx, nnz, nidx, window, 16, 16) <= l2 / 2) return 0;
            // 16 slices when 8 would leave more than half an L2 per slice and
            // each gathered element is read at least 4 times per pass
            int S = (eb * nidx / 8.0 > l2 / 2 && (double)nnz >= 4.0 * nidx) ? 16 : 8;
            for (; S >= 8; S /= 2)
                if (20.0 * (double)count_compact(ptr, idx, gptr, nseg, nidx, S) < mat) return S;
            return 0;
        };
        if (!hot_cols) Sd = pick(H.rp, H.ci, H.cp, m, n);
        if (!hot_rows) Sp = pick(H.cp, H.ri, H.rp, n, m);
    }
    if (Sd) CHK(build_sliced(P, H.rp, H.ci, H.cp, m, n, Sd, P->sr));   // dual: gathers xbar
    if (Sp) CHK(build_sliced(P, H.cp, H.ri, H.rp, n, m, Sp, P->sc));   // primal: gathers y

    if (Sd || Sp) {
        ntmax = std::max(ntmax, std::max(P->sr.ts.n, P->sc.ts.n));
        // the sliced CSR check pass keeps two right-hand sides (2 G doubles)
        const size_t ps = (size_t)std::max<int64_t>(1, std::max(2 * P->sr.G, P->sc.G));
        CHK(dalloc(P, (double **)&P->part_slices, ps));
    }
    // split-piece carries (2 right-hand sides) and per-tile partial sums
    CHK(dalloc(P, (double **)&P->carries, (size_t)2 * std::max(ntmax, 1)));
    // per-tile (or, sliced, per-combine-block) partial sums of the checks
    CHK(dalloc(P, &P->part_r, (size_t)kNQ * std::max(std::max(P->tr.n, (int)nblk(m)), 1)));
    CHK(dalloc(P, &P->part_c, (size_t)kNQ * std::max(std::max(P->tc.n, (int)nblk(n)), 1)));
    CHK(dalloc(P, &P->perm_row, (size_t)m)); CHK(dalloc(P, &P->perm_col, (size_t)n));
    CHK(upload(P, P->perm_row, H.perm_row.data(), sizeof(int32_t) * (size_t)m));
    CHK(upload(P, P->perm_col, H.perm_col.data(), sizeof(int32_t) * (size_t)n));

    // problem vectors, permuted on the host
    {
        std::vector<double> tmp((size_t)std::max(m, n));
        auto put = [&](double **d, const double *src, const std::vector<int32_t> &perm, int32_t k) -> int {
            CHK(dalloc(P, d, (size_t)k));
            for (int32_t i = 0; i < k; ++i) tmp[(size_t)i] = src[perm[(size_t)i]];
            HIPCHK(hipMemcpy(*d, tmp.data(), sizeof(double) * (size_t)k, hipMemcpyHostToDevice));
            return DPDLP_OK;
        };
        HIPCHK(hipStreamSynchronize(P->s));
        CHK(put(&P->c0, lp.c, H.perm_col, n));
        CHK(put(&P->vlo0, lp.var_lo, H.perm_col, n));
        CHK(put(&P->vhi0, lp.var_hi, H.perm_col, n));
        CHK(put(&P->clo0, lp.con_lo, H.perm_row, m));
        CHK(put(&P->chi0, lp.con_hi, H.perm_row, m));
    }
    H = HostMatrix();
    double **nvec[] = {&P->c, &P->vlo, &P->vhi, &P->dc, &P->fc, &P->x, &P->xbar, &P->xa, &P->xh,
                       &P->dx, &P->tmp_n, &P->tmp_n2};
    for (auto pp : nvec) CHK(dalloc(P, pp, (size_t)n));
    double **mvec[] = {&P->clo, &P->chi, &P->dr, &P->fr, &P->y, &P->ya, &P->yh, &P->dy,
                       &P->tmp_m, &P->tmp_m2};
    for (auto pp : mvec) CHK(dalloc(P, pp, (size_t)m));
    CHK(dalloc(P, &P->scal, 16));
    CHK(dalloc(P, &P->sig_hist, 2 * ((size_t)std::max(1, P->prm.power_max_iters) + 2)));
    CHK(dalloc(P, &P->ctl, 1));
    CHK(dalloc(P, &P->ctl_eval, 1));
    CHK(dalloc(P, &P->iterdev, 1));
    HIPCHK(hipHostMalloc((void **)&P->h_ctl, sizeof(Control), hipHostMallocDefault));

    // A3: rescaling (Ruiz passes, then one Pock-Chambolle pass)
    hipLaunchKernelGGL(k_fill<double>, dim3(nblk(m)), dim3(kBlock), 0, P->s, P->dr, 1.0, (int64_t)m);
    hipLaunchKernelGGL(k_fill<double>, dim3(nblk(n)), dim3(kBlock), 0, P->s, P->dc, 1.0, (int64_t)n);
    auto apply_scale = [&]() {
        if (P->tr.n)
            hipLaunchKernelGGL(k_scale_vals, dim3(P->tr.n), dim3(kBlock), 0, P->s, P->tr.d, P->tr.n,
                               P->rp, P->ci, P->v, P->fr, P->fc, 1);
        if (P->tc.n)
            hipLaunchKernelGGL(k_scale_vals, dim3(P->tc.n), dim3(kBlock), 0, P->s, P->tc.d, P->tc.n,
                               P->cp, P->ri, P->vt, P->fc, P->fr, 0);
        hipLaunchKernelGGL(k_mul, dim3(nblk(m)), dim3(kBlock), 0, P->s, P->dr, P->fr, m);
        hipLaunchKernelGGL(k_mul, dim3(nblk(n)), dim3(kBlock), 0, P->s, P->dc, P->fc, n);
    };
    for (int it = 0; it < P->prm.ruiz_iters; ++it) {
        hipLaunchKernelGGL(k_fill<double>, dim3(nblk(m)), dim3(kBlock), 0, P->s, P->fr, 1.0, (int64_t)m);
        hipLaunchKernelGGL(k_fill<double>, dim3(nblk(n)), dim3(kBlock), 0, P->s, P->fc, 1.0, (int64_t)n);
        AbsMaxOp a; a.f = P->fr; a.partials = nullptr;
        launch_tiles(P, a, P->tr, P->rp, P->ci, P->v);
        AbsMaxOp b; b.f = P->fc; b.partials = nullptr;
        launch_tiles(P, b, P->tc, P->cp, P->ri, P->vt);
        apply_scale();
    }
    if (P->prm.use_pc) {
        AbsPowSumOp a; a.f = P->fr; a.partials = nullptr; a.p = 2.0 - P->prm.pc_alpha;
        launch_tiles(P, a, P->tr, P->rp, P->ci, P->v);
        AbsPowSumOp b; b.f = P->fc; b.partials = nullptr; b.p = P->prm.pc_alpha;
        launch_tiles(P, b, P->tc, P->cp, P->ri, P->vt);
        apply_scale();
    }
    CHK(scale_data(P));
    if (P->sr.S > 0)
        hipLaunchKernelGGL(k_gather_vals<double>, dim3(nblk((int64_t)nnz)), dim3(kBlock), 0, P->s,
                           P->sr.src, P->v, P->sr.val, (int64_t)nnz);
    if (P->sc.S > 0)
        hipLaunchKernelGGL(k_gather_vals<double>, dim3(nblk((int64_t)nnz)), dim3(kBlock), 0, P->s,
                           P->sc.src, P->vt, P->sc.val, (int64_t)nnz);

    // A4: step size
    if (P->prm.eta > 0) {
        P->eta = P->prm.eta;
        P->sigma_max = 0;
        P->power_iters = 0;
    } else {
        CHK(estimate_sigma_max(P));
        P->eta = P->sigma_max > 0 ? P->prm.eta_safety / P->sigma_max : 1.0;
    }
    // FP32 copies for the mixed-precision form
    if (P->prm.precision == DPDLP_FP32_MIXED) {
        CHK(dalloc(P, &P->v32, nnz)); CHK(dalloc(P, &P->vt32, nnz));
        float **nf[] = {&P->x32, &P->xbar32, &P->xa32, &P->c32, &P->vlo32, &P->vhi32};
        for (auto pp : nf) CHK(dalloc(P, pp, (size_t)n));
        float **mf[] = {&P->y32, &P->ya32, &P->clo32, &P->chi32};
        for (auto pp : mf) CHK(dalloc(P, pp, (size_t)m));
        CHK(dalloc(P, &P->xbest, (size_t)n)); CHK(dalloc(P, &P->ybest, (size_t)m));
        auto cv = [&](const double *a, float *b, int64_t k) {
            if (k) hipLaunchKernelGGL((k_convert<double, float>), dim3(nblk(k)), dim3(kBlock), 0, P->s, a, b, k);
        };
        cv(P->v, P->v32, (int64_t)nnz); cv(P->vt, P->vt32, (int64_t)nnz);
        if (P->sr.S > 0) { CHK(dalloc(P, &P->sr.val32, nnz)); cv(P->sr.val, P->sr.val32, (int64_t)nnz); }
        if (P->sc.S > 0) { CHK(dalloc(P, &P->sc.val32, nnz)); cv(P->sc.val, P->sc.val32, (int64_t)nnz); }

        CHK(scale_data(P));
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(P->s));
    CHK(check_buffers(P));
    P->setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    *out = guard.release();
    return DPDLP_OK;
}

// ---- state -------------------------------------------------------------------
static void reset_ctl_host(dpdlp_problem *P)
{
    std::memset(P->h_ctl, 0, sizeof(Control));
    P->h_ctl->omega = P->omega;
}

static int init_impl(dpdlp_problem *P, const double *x0, const double *y0, int mem_kind)
{
    const int32_t m = P->m, n = P->n;
    const double *dx0 = nullptr, *dy0 = nullptr;
    if (x0) {
        if (mem_kind == DPDLP_MEM_HOST) {
            HIPCHK(hipMemcpyAsync(P->tmp_n2, x0, sizeof(double) * n, hipMemcpyHostToDevice, P->s));
            dx0 = P->tmp_n2;
        } else dx0 = x0;
    }
    if (y0) {
        if (mem_kind == DPDLP_MEM_HOST) {
            HIPCHK(hipMemcpyAsync(P->tmp_m2, y0, sizeof(double) * m, hipMemcpyHostToDevice, P->s));
            dy0 = P->tmp_m2;
        } else dy0 = y0;
    }
    hipLaunchKernelGGL(k_init_x<double>, dim3(nblk(n)), dim3(kBlock), 0, P->s, n, dx0, P->perm_col,
                       P->dc, P->vlo, P->vhi, P->x, P->xa);
    hipLaunchKernelGGL(k_init_y<double>, dim3(nblk(m)), dim3(kBlock), 0, P->s, m, dy0, P->perm_row,
                       P->dr, P->clo, P->chi, P->y, P->ya);
    HIPCHK(hipMemcpyAsync(P->xh, P->x, sizeof(double) * n, hipMemcpyDeviceToDevice, P->s));
    HIPCHK(hipMemcpyAsync(P->yh, P->y, sizeof(double) * m, hipMemcpyDeviceToDevice, P->s));
    P->in_fp32 = P->prm.precision == DPDLP_FP32_MIXED;
    if (P->in_fp32) {
        hipLaunchKernelGGL((k_convert<double, float>), dim3(nblk(n)), dim3(kBlock), 0, P->s, P->x, P->x32, (int64_t)n);
        hipLaunchKernelGGL((k_convert<double, float>), dim3(nblk(n)), dim3(kBlock), 0, P->s, P->xa, P->xa32, (int64_t)n);
        hipLaunchKernelGGL((k_convert<double, float>), dim3(nblk(m)), dim3(kBlock), 0, P->s, P->y, P->y32, (int64_t)m);
        hipLaunchKernelGGL((k_convert<double, float>), dim3(nblk(m)), dim3(kBlock), 0, P->s, P->ya, P->ya32, (int64_t)m);
    }
    P->omega = P->omega0;
    P->k = 0; P->t = 0; P->fp32_iters = 0;
    P->status = DPDLP_RUNNING;
    P->fp32_ref_kkt = INFINITY;
    P->fp32_best_kkt = INFINITY;
    P->fp32_stall = 0;
    P->solve_seconds = 0;
    P->log.clear();
    reset_ctl_host(P);
    HIPCHK(hipMemcpyAsync(P->ctl, P->h_ctl, sizeof(Control), hipMemcpyHostToDevice, P->s));
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(P->s));
    P->initialized = true;
    return DPDLP_OK;
}

// FP32 -> FP64 switch: continue in FP64 as a fresh epoch anchored at T(z)
// of the last check, or, after a divergence, at the FP32 phase's best check
// point (lowest KKT error) with the primal weight that produced it.
static int switch_to_fp64(dpdlp_problem *P, bool from_best)
{
    if (from_best) {
        HIPCHK(hipMemcpyAsync(P->xh, P->xbest, sizeof(double) * P->n, hipMemcpyDeviceToDevice, P->s));
        HIPCHK(hipMemcpyAsync(P->yh, P->ybest, sizeof(double) * P->m, hipMemcpyDeviceToDevice, P->s));
        P->omega = P->fp32_best_omega;
        // the control kernel measures r in the P-norm of this weight and
        // starts the next PID step from it, so the device copy follows
        P->h_ctl->omega = P->omega;
        HIPCHK(hipMemcpyAsync(&P->ctl->omega, &P->h_ctl->omega, sizeof(double),
                              hipMemcpyHostToDevice, P->s));
    }
    hipLaunchKernelGGL(k_restart<double>, dim3(nblk(std::max(P->m, P->n))), dim3(kBlock), 0, P->s,
                       P->m, P->n, P->xh, P->yh, P->x, P->xa, P->y, P->ya);
    P->in_fp32 = false;
    P->k = 0;
    HIPCHK(hipGetLastError());
    return DPDLP_OK;
}

static int iterate_impl(dpdlp_problem *P, int64_t n_iters)
{
    if (!P->initialized) CHK(init_impl(P, nullptr, nullptr, DPDLP_MEM_HOST));
    auto t0 = std::chrono::steady_clock::now();
    const int K = P->prm.check_period;
    int64_t done = 0;
    int rc = DPDLP_OK;
    if (P->status == DPDLP_ITER_LIMIT || P->status == DPDLP_TIME_LIMIT) P->status = DPDLP_RUNNING;
    while (done < n_iters && P->status == DPDLP_RUNNING) {
        if (P->t >= P->prm.max_iters) { P->status = DPDLP_ITER_LIMIT; break; }
        const double tau = P->eta / P->omega, sigma = P->eta * P->omega;
        const bool is_check = (P->k == 0) || ((P->t + 1) % K == 0);
        if (!is_check && P->prm.use_graphs && !P->prof && K > 1 && P->t % K == 0) {
            // a whole run t .. t+K-2 of non-check iterations, none the last of the call
            const int L = K - 1;
            if (done + L < n_iters && P->t + L < P->prm.max_iters) {
                CHK(run_graph(P, tau, sigma, P->k, L));
                if (P->in_fp32) P->fp32_iters += L;
                done += L;
                P->k += L;
                P->t += L;
                continue;
            }
        }
        const bool last = (done + 1 == n_iters) || (P->t + 1 >= P->prm.max_iters);
        pdhg_iteration(P, tau, sigma, P->k, (is_check || last) ? 1 : 0);
        if (P->in_fp32) P->fp32_iters++;
        done++;
        if (!is_check) { P->k++; P->t++; continue; }
        if (P->in_fp32) launch_checks<float>(P, P->xh, P->dx, P->yh, P->dy, P->xa32, P->ya32, tau);
        else launch_checks<double>(P, P->xh, P->dx, P->yh, P->dy, P->xa, P->ya, tau);
        {
            ProfScope ps(P, 4);
            hipLaunchKernelGGL(k_control, dim3(1), dim3(kBlock), 0, P->s, P->part_r, P->chk_nr,
                               P->part_c, P->chk_nc, P->ctl, ctl_args(P, 0));
        }
        hipError_t le = hipGetLastError();
        if (le != hipSuccess) return hip_fail(le, "kernel launch");
        CHK(read_ctl(P));
        const Control &C = *P->h_ctl;
        dpdlp_log_rec rec{};
        rec.t = P->t; rec.k = P->k; rec.r = C.r; rec.r0 = C.r0;
        rec.r_primal = C.r_primal; rec.r_dual = C.r_dual; rec.r_gap = C.r_gap;
        rec.omega = P->omega; rec.restart = C.restart;
        P->log.push_back(rec);
        if (C.numerical) { P->status = DPDLP_NUMERICAL; P->t++; break; }
        const double kkt = std::max(C.r_primal, std::max(C.r_dual, C.r_gap));
        if (P->in_fp32 && kkt < P->fp32_best_kkt) {    // keep the FP32 phase's best point
            P->fp32_best_kkt = kkt;
            P->fp32_best_omega = P->omega;
            HIPCHK(hipMemcpyAsync(P->xbest, P->xh, sizeof(double) * P->n, hipMemcpyDeviceToDevice, P->s));
            HIPCHK(hipMemcpyAsync(P->ybest, P->yh, sizeof(double) * P->m, hipMemcpyDeviceToDevice, P->s));
        }
        if (C.converged) {           // the KKT is evaluated in FP64 in both precisions
            P->status = DPDLP_CONVERGED;
            P->t++;
            break;
        }
        if (C.restart) {
            if (P->in_fp32)
                hipLaunchKernelGGL(k_restart<float>, dim3(nblk(std::max(P->m, P->n))), dim3(kBlock), 0,
                                   P->s, P->m, P->n, P->xh, P->yh, P->x32, P->xa32, P->y32, P->ya32);
            else
                hipLaunchKernelGGL(k_restart<double>, dim3(nblk(std::max(P->m, P->n))), dim3(kBlock), 0,
                                   P->s, P->m, P->n, P->xh, P->yh, P->x, P->xa, P->y, P->ya);
            P->k = 0;
            P->omega = C.omega;
        } else {
            P->k++;
        }
        P->t++;
        if (P->in_fp32) {            // FP32 -> FP64 switch rule
            // tolerance reached, divergence (KKT far above the phase's best:
            // FP32 rounding amplified by a small primal weight), or stall
            const bool diverged = P->prm.fp32_diverge > 0 && kkt > P->prm.fp32_diverge * P->fp32_best_kkt;
            bool sw = kkt <= P->prm.fp32_switch_tol || diverged;
            if (kkt <= 0.5 * P->fp32_ref_kkt || P->fp32_ref_kkt == INFINITY) {
                P->fp32_ref_kkt = kkt;
                P->fp32_stall = 0;
            } else if (++P->fp32_stall >= P->prm.fp32_stall_checks) {
                sw = true;
            }
            if (sw) CHK(switch_to_fp64(P, diverged));
        }
        if (P->prm.time_limit > 0) {
            double el = P->solve_seconds +
                        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            if (el >= P->prm.time_limit) { P->status = DPDLP_TIME_LIMIT; break; }
        }
    }
    if (P->status == DPDLP_RUNNING && P->t >= P->prm.max_iters) P->status = DPDLP_ITER_LIMIT;
    hipError_t le = hipGetLastError();
    if (le != hipSuccess) rc = hip_fail(le, "kernel launch");
    hipError_t se = hipStreamSynchronize(P->s);
    if (se != hipSuccess && rc == DPDLP_OK) rc = hip_fail(se, "hipStreamSynchronize");
    P->solve_seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (P->prof) prof_collect(P);
    return rc;
}

static int output_impl(dpdlp_problem *P, double *x_out, double *y_out, int mem_kind)
{
    const int32_t m = P->m, n = P->n;
    if (x_out) {
        double *dst = mem_kind == DPDLP_MEM_DEVICE ? x_out : P->tmp_n;
        hipLaunchKernelGGL(k_unpermute<double>, dim3(nblk(n)), dim3(kBlock), 0, P->s, n, P->xh,
                           P->perm_col, P->dc, dst);
        if (mem_kind == DPDLP_MEM_HOST)
            HIPCHK(hipMemcpyAsync(x_out, dst, sizeof(double) * n, hipMemcpyDeviceToHost, P->s));
    }
    if (y_out) {
        double *dst = mem_kind == DPDLP_MEM_DEVICE ? y_out : P->tmp_m;
        hipLaunchKernelGGL(k_unpermute<double>, dim3(nblk(m)), dim3(kBlock), 0, P->s, m, P->yh,
                           P->perm_row, P->dr, dst);
        if (mem_kind == DPDLP_MEM_HOST)
            HIPCHK(hipMemcpyAsync(y_out, dst, sizeof(double) * m, hipMemcpyDeviceToHost, P->s));
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(P->s));
    return DPDLP_OK;
}

static void fill_result(dpdlp_problem *P, dpdlp_result *r)
{
    if (!r) return;
    std::memset(r, 0, sizeof(*r));
    const Control &C = *P->h_ctl;
    r->status = P->status; r->restarts = C.restarts; r->iters = P->t;
    r->fp32_iters = P->fp32_iters;
    r->r_primal = C.r_primal; r->r_dual = C.r_dual; r->r_gap = C.r_gap;
    r->obj_primal = C.obj_p; r->obj_dual = C.obj_d;
    r->omega = P->omega; r->eta = P->eta; r->sigma_max = P->sigma_max;
    r->setup_seconds = P->setup_seconds; r->solve_seconds = P->solve_seconds;
    r->power_iters = P->power_iters; r->n_checks = C.n_checks;
    r->slices_primal = P->sc.S; r->slices_dual = P->sr.S;
}

int problem_view(dpdlp_problem *P, ProblemView *o)
{
    if (!P || !o) return DPDLP_E_INVALID_ARG;
    o->m = P->m; o->n = P->n; o->nnz = P->nnz;
    o->rp = P->rp; o->ci = P->ci; o->cp = P->cp; o->ri = P->ri; o->v = P->v; o->vt = P->vt;
    o->perm_row = P->perm_row; o->perm_col = P->perm_col; o->dr = P->dr; o->dc = P->dc;
    o->vlo0 = P->vlo0; o->vhi0 = P->vhi0;
    return DPDLP_OK;
}

}  // namespace dpdlp

// ---------------------------------------------------------------------------
// C ABI

#define ENTER(P)                                                  \
    if (!(P)) { set_error("NULL problem"); return DPDLP_E_INVALID_ARG; } \
    (P)->s = (hipStream_t)stream

extern "C" {

int dpdlp_problem_create(const dpdlp_csr_lp *lp, const dpdlp_params *params, void *stream,
                         dpdlp_problem **out)
{
    return create_impl(lp, params, stream, out);
}

int dpdlp_problem_update_data(dpdlp_problem *P, const double *c, const double *con_lo,
                              const double *con_hi, const double *var_lo, const double *var_hi,
                              int32_t mem_kind, void *stream)
{
    ENTER(P);
    if (!mem_kind_ok(mem_kind)) return bad_mem_kind();
    const int32_t m = P->m, n = P->n;
    struct Item { const double *src; int k; const std::vector<int32_t> *perm; double *dst; } items[] = {
        {c, n, &P->h_perm_col, P->c0}, {var_lo, n, &P->h_perm_col, P->vlo0},
        {var_hi, n, &P->h_perm_col, P->vhi0}, {con_lo, m, &P->h_perm_row, P->clo0},
        {con_hi, m, &P->h_perm_row, P->chi0}};
    std::vector<double> a((size_t)std::max(m, n)), b((size_t)std::max(m, n));
    // host copies for validation (device inputs are brought over)
    std::vector<std::vector<double>> host(5);
    for (int q = 0; q < 5; ++q) {
        if (!items[q].src) continue;
        host[(size_t)q].resize((size_t)items[q].k);
        if (mem_kind == DPDLP_MEM_DEVICE)
            HIPCHK(hipMemcpy(host[(size_t)q].data(), items[q].src, sizeof(double) * items[q].k,
                             hipMemcpyDeviceToHost));
        else
            std::memcpy(host[(size_t)q].data(), items[q].src, sizeof(double) * items[q].k);
    }
    if (c)
        for (int32_t j = 0; j < n; ++j)
            if (!std::isfinite(host[0][(size_t)j])) { set_error("non-finite c"); return DPDLP_E_BAD_BOUNDS; }
    for (int pair = 0; pair < 2; ++pair) {
        const int ql = pair == 0 ? 1 : 3, qh = ql + 1;
        if (!items[ql].src && !items[qh].src) continue;
        const int k = items[ql].k;
        // current values for the side not given
        std::vector<double> lo((size_t)k), hi((size_t)k);
        for (int side = 0; side < 2; ++side) {
            const int q = side == 0 ? ql : qh;
            std::vector<double> &dst = side == 0 ? lo : hi;
            if (items[q].src) { dst = host[(size_t)q]; continue; }
            std::vector<double> tmp((size_t)k);
            HIPCHK(hipMemcpy(tmp.data(), items[q].dst, sizeof(double) * k, hipMemcpyDeviceToHost));
            for (int i = 0; i < k; ++i) dst[(size_t)(*items[q].perm)[(size_t)i]] = tmp[(size_t)i];
        }
        for (int i = 0; i < k; ++i) {
            const double l = lo[(size_t)i], h = hi[(size_t)i];
            if (std::isnan(l) || std::isnan(h) || l > h || l == INFINITY || h == -INFINITY) {
                set_error("bad bounds at index " + std::to_string(i));
                return DPDLP_E_BAD_BOUNDS;
            }
        }
    }
    for (int q = 0; q < 5; ++q) {
        if (!items[q].src) continue;
        const int k = items[q].k;
        for (int i = 0; i < k; ++i) a[(size_t)i] = host[(size_t)q][(size_t)(*items[q].perm)[(size_t)i]];
        HIPCHK(hipMemcpy(items[q].dst, a.data(), sizeof(double) * k, hipMemcpyHostToDevice));
    }
    CHK(scale_data(P));
    HIPCHK(hipStreamSynchronize(P->s));
    P->initialized = false;
    return DPDLP_OK;
}

int dpdlp_problem_destroy(dpdlp_problem *P)
{
    if (!P) return DPDLP_OK;
    (void)hipDeviceSynchronize();
    if (P->h_ctl) (void)hipHostFree(P->h_ctl);
    for (int c = 0; c < 8; ++c)
        for (auto &pr : P->ev[c]) { (void)hipEventDestroy(pr.first); (void)hipEventDestroy(pr.second); }
    for (auto e : P->ev_pool) (void)hipEventDestroy(e);
    drop_graphs(P);
    if (P->gstream) (void)hipStreamDestroy(P->gstream);
    delete P;
    return DPDLP_OK;
}

int dpdlp_set_params(dpdlp_problem *P, const dpdlp_params *q)
{
    if (!P || !q) { set_error("NULL argument"); return DPDLP_E_INVALID_ARG; }
    if (q->check_period < 1 || q->max_iters < 0) { set_error("bad check_period / max_iters"); return DPDLP_E_INVALID_ARG; }
    dpdlp_params &p = P->prm;
    p.eps = q->eps; p.max_iters = q->max_iters; p.time_limit = q->time_limit;
    p.check_period = q->check_period; p.gamma = q->gamma;
    p.beta_suf = q->beta_suf; p.beta_nec = q->beta_nec; p.beta_art = q->beta_art;
    p.kp = q->kp; p.ki = q->ki; p.kd = q->kd; p.xcd_remap = q->xcd_remap;
    p.fp32_switch_tol = q->fp32_switch_tol; p.fp32_stall_checks = q->fp32_stall_checks;
    p.fp32_diverge = q->fp32_diverge;
    p.use_graphs = q->use_graphs;
    drop_graphs(P);                 // gamma is a captured kernel argument
    return DPDLP_OK;
}

int dpdlp_set_objective_diag(dpdlp_problem *P, const double *q, int32_t mem_kind, void *stream)
{
    ENTER(P);
    const int32_t n = P->n;
    if (!q) {
        P->has_q = false;
        drop_graphs(P);             // the primal step's kernel is a captured node
        return DPDLP_OK;
    }
    if (mem_kind != DPDLP_MEM_HOST && mem_kind != DPDLP_MEM_DEVICE) {
        set_error("bad mem_kind");
        return DPDLP_E_INVALID_ARG;
    }
    std::vector<double> h((size_t)n), dc((size_t)n), out((size_t)n);
    if (mem_kind == DPDLP_MEM_DEVICE)
        HIPCHK(hipMemcpy(h.data(), q, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost));
    else
        std::memcpy(h.data(), q, sizeof(double) * (size_t)n);
    for (int32_t j = 0; j < n; ++j)
        if (!std::isfinite(h[(size_t)j]) || h[(size_t)j] < 0.0) {
            set_error("diag(Q) must be finite and >= 0 (index " + std::to_string(j) + ")");
            return DPDLP_E_INVALID_ARG;
        }
    HIPCHK(hipStreamSynchronize(P->s));
    HIPCHK(hipMemcpy(dc.data(), P->dc, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost));
    // permuted column j holds original column h_perm_col[j]; the scaled
    // problem's Q is D_c Q D_c
    for (int32_t j = 0; j < n; ++j)
        out[(size_t)j] = dc[(size_t)j] * dc[(size_t)j] * h[(size_t)P->h_perm_col[(size_t)j]];
    if (!P->qd) CHK(dalloc(P, &P->qd, (size_t)n));
    HIPCHK(hipMemcpy(P->qd, out.data(), sizeof(double) * (size_t)n, hipMemcpyHostToDevice));
    if (P->prm.precision == DPDLP_FP32_MIXED) {
        // the FP32 phase's copy (its checks use the FP64 one)
        if (!P->q32) CHK(dalloc(P, &P->q32, (size_t)n));
        hipLaunchKernelGGL((k_convert<double, float>), dim3(nblk(n)), dim3(kBlock), 0, P->s, P->qd,
                           P->q32, (int64_t)n);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(P->s));
    }
    P->has_q = true;
    drop_graphs(P);
    return DPDLP_OK;
}

int dpdlp_init(dpdlp_problem *P, const double *x0, const double *y0, int32_t mem_kind, void *stream)
{
    ENTER(P);
    if (!mem_kind_ok(mem_kind)) return bad_mem_kind();
    return init_impl(P, x0, y0, mem_kind);
}

int dpdlp_iterate(dpdlp_problem *P, int64_t n_iters, void *stream)
{
    ENTER(P);
    if (n_iters < 0) { set_error("n_iters < 0"); return DPDLP_E_INVALID_ARG; }
    return iterate_impl(P, n_iters);
}

int dpdlp_solve(dpdlp_problem *P, const double *x0, const double *y0, double *x_out,
                double *y_out, int32_t mem_kind, dpdlp_result *info, void *stream)
{
    ENTER(P);
    if (!mem_kind_ok(mem_kind)) return bad_mem_kind();
    CHK(init_impl(P, x0, y0, mem_kind));
    CHK(iterate_impl(P, P->prm.max_iters));
    CHK(output_impl(P, x_out, y_out, mem_kind));
    fill_result(P, info);
    return DPDLP_OK;
}

int dpdlp_get_result(dpdlp_problem *P, double *x_out, double *y_out, int32_t mem_kind,
                     dpdlp_result *info, void *stream)
{
    ENTER(P);
    if (!mem_kind_ok(mem_kind)) return bad_mem_kind();
    CHK(output_impl(P, x_out, y_out, mem_kind));
    fill_result(P, info);
    return DPDLP_OK;
}

int dpdlp_state_export(dpdlp_problem *P, dpdlp_state *st, double *x, double *y, double *xa,
                       double *ya, double *xh, double *yh, int32_t mem_kind, void *stream)
{
    ENTER(P);
    if (!mem_kind_ok(mem_kind)) return bad_mem_kind();
    const int32_t m = P->m, n = P->n;
    struct Item { double *dst; int isx; const double *src64; const float *src32; } items[] = {
        {x, 1, P->x, P->x32}, {y, 0, P->y, P->y32}, {xa, 1, P->xa, P->xa32},
        {ya, 0, P->ya, P->ya32}, {xh, 1, P->xh, nullptr}, {yh, 0, P->yh, nullptr}};
    for (auto &it : items) {
        if (!it.dst) continue;
        const int k = it.isx ? n : m;
        const int *perm = it.isx ? P->perm_col : P->perm_row;
        double *dst = mem_kind == DPDLP_MEM_DEVICE ? it.dst : (it.isx ? P->tmp_n : P->tmp_m);
        if (P->in_fp32 && it.src32)
            hipLaunchKernelGGL(k_unpermute<float>, dim3(nblk(k)), dim3(kBlock), 0, P->s, k, it.src32,
                               perm, (const double *)nullptr, dst);
        else
            hipLaunchKernelGGL(k_unpermute<double>, dim3(nblk(k)), dim3(kBlock), 0, P->s, k, it.src64,
                               perm, (const double *)nullptr, dst);
        if (mem_kind == DPDLP_MEM_HOST)
            HIPCHK(hipMemcpyAsync(it.dst, dst, sizeof(double) * k, hipMemcpyDeviceToHost, P->s));
        HIPCHK(hipStreamSynchronize(P->s));
    }
    if (st) {
        const Control &C = *P->h_ctl;
        std::memset(st, 0, sizeof(*st));
        st->omega = P->omega; st->r0 = C.r0; st->r_prev = C.r_prev; st->pid_int = C.pid_int;
        st->pid_prev = C.pid_prev; st->k = P->k; st->t = P->t; st->pid_started = C.pid_started;
        st->restarts = C.restarts; st->status = P->status; st->n_checks = C.n_checks;
        st->r_primal = C.r_primal; st->r_dual = C.r_dual; st->r_gap = C.r_gap;
        st->obj_primal = C.obj_p; st->obj_dual = C.obj_d; st->r_fixed_point = C.r;
    }
    return DPDLP_OK;
}

int dpdlp_state_import(dpdlp_problem *P, const dpdlp_state *st, const double *x, const double *y,
                       const double *xa, const double *ya, const double *xh, const double *yh,
                       int32_t mem_kind, void *stream)
{
    ENTER(P);
    if (!st || !x || !y || !xa || !ya) { set_error("state import needs st, x, y, xa, ya"); return DPDLP_E_INVALID_ARG; }
    if (!mem_kind_ok(mem_kind)) return bad_mem_kind();
    if (P->prm.precision == DPDLP_FP32_MIXED) { set_error("state import is FP64 only"); return DPDLP_E_NOT_SUPPORTED; }
    const int32_t m = P->m, n = P->n;
    struct Item { const double *src; int isx; double *dst; } items[] = {
        {x, 1, P->x}, {y, 0, P->y}, {xa, 1, P->xa}, {ya, 0, P->ya}, {xh, 1, P->xh}, {yh, 0, P->yh}};
    for (auto &it : items) {
        if (!it.src) continue;
        const int k = it.isx ? n : m;
        const double *src = it.src;
        if (mem_kind == DPDLP_MEM_HOST) {
            double *stage = it.isx ? P->tmp_n : P->tmp_m;
            HIPCHK(hipMemcpyAsync(stage, it.src, sizeof(double) * k, hipMemcpyHostToDevice, P->s));
            src = stage;
        }
        hipLaunchKernelGGL(k_permute<double>, dim3(nblk(k)), dim3(kBlock), 0, P->s, k, src,
                           it.isx ? P->perm_col : P->perm_row, (const double *)nullptr, it.dst);
        HIPCHK(hipStreamSynchronize(P->s));
    }
    P->omega = st->omega; P->k = st->k; P->t = st->t; P->status = DPDLP_RUNNING;
    P->in_fp32 = false;
    std::memset(P->h_ctl, 0, sizeof(Control));
    Control &C = *P->h_ctl;
    C.omega = st->omega; C.r0 = st->r0; C.r_prev = st->r_prev; C.pid_int = st->pid_int;
    C.pid_prev = st->pid_prev; C.pid_started = st->pid_started; C.restarts = st->restarts;
    C.n_checks = st->n_checks; C.r_primal = st->r_primal; C.r_dual = st->r_dual;
    C.r_gap = st->r_gap; C.obj_p = st->obj_primal; C.obj_d = st->obj_dual; C.r = st->r_fixed_point;
    HIPCHK(hipMemcpyAsync(P->ctl, P->h_ctl, sizeof(Control), hipMemcpyHostToDevice, P->s));
    HIPCHK(hipStreamSynchronize(P->s));
    P->log.clear();
    P->initialized = true;
    return DPDLP_OK;
}

int dpdlp_get_log(dpdlp_problem *P, dpdlp_log_rec *recs, int32_t cap, int32_t *count)
{
    if (!P || !count) { set_error("NULL argument"); return DPDLP_E_INVALID_ARG; }
    *count = (int32_t)P->log.size();
    if (recs)
        for (int32_t i = 0; i < cap && i < (int32_t)P->log.size(); ++i) recs[i] = P->log[(size_t)i];
    return DPDLP_OK;
}

int dpdlp_spmv(dpdlp_problem *P, int32_t transpose, const double *in, double *out, void *stream)
{
    ENTER(P);
    if (!in || !out) { set_error("NULL vector"); return DPDLP_E_INVALID_ARG; }
    const int32_t m = P->m, n = P->n;
    const int kin = transpose ? m : n, kout = transpose ? n : m;
    double *pin = transpose ? P->tmp_m2 : P->tmp_n2;
    double *pout = transpose ? P->tmp_n : P->tmp_m;
    hipLaunchKernelGGL(k_permute<double>, dim3(nblk(kin)), dim3(kBlock), 0, P->s, kin, in,
                       transpose ? P->perm_row : P->perm_col, (const double *)nullptr, pin);
    SpmvOp op; op.in = pin; op.div = nullptr; op.out = pout;
    op.partials = transpose ? P->part_c : P->part_r;
    launch_product(P, transpose != 0, op, pin);
    hipLaunchKernelGGL(k_unpermute<double>, dim3(nblk(kout)), dim3(kBlock), 0, P->s, kout, pout,
                       transpose ? P->perm_col : P->perm_row, (const double *)nullptr, out);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(P->s));
    (void)kout;
    return DPDLP_OK;
}

int dpdlp_kkt(dpdlp_problem *P, const double *x, const double *y, double tau, int32_t mem_kind,
              double *out5, void *stream)
{
    ENTER(P);
    if (!out5 || (!x) != (!y)) { set_error("bad arguments"); return DPDLP_E_INVALID_ARG; }
    if (x && !mem_kind_ok(mem_kind)) return bad_mem_kind();
    const int32_t m = P->m, n = P->n;
    if (tau <= 0) tau = P->eta / P->omega;
    if (!x) {
        // the current start point (set by dpdlp_init: clamped into X, projected onto Y)
        if (!P->initialized) CHK(init_impl(P, nullptr, nullptr, DPDLP_MEM_HOST));
        if (P->in_fp32) {
            hipLaunchKernelGGL((k_convert<float, double>), dim3(nblk(n)), dim3(kBlock), 0, P->s, P->xa32, P->tmp_n, (int64_t)n);
            hipLaunchKernelGGL((k_convert<float, double>), dim3(nblk(m)), dim3(kBlock), 0, P->s, P->ya32, P->tmp_m, (int64_t)m);
        } else {
            HIPCHK(hipMemcpyAsync(P->tmp_n, P->xa, sizeof(double) * n, hipMemcpyDeviceToDevice, P->s));
            HIPCHK(hipMemcpyAsync(P->tmp_m, P->ya, sizeof(double) * m, hipMemcpyDeviceToDevice, P->s));
        }
    } else {
        const double *dxp = x, *dyp = y;
        if (mem_kind == DPDLP_MEM_HOST) {
            HIPCHK(hipMemcpyAsync(P->tmp_n2, x, sizeof(double) * n, hipMemcpyHostToDevice, P->s));
            HIPCHK(hipMemcpyAsync(P->tmp_m2, y, sizeof(double) * m, hipMemcpyHostToDevice, P->s));
            dxp = P->tmp_n2; dyp = P->tmp_m2;
        }
        // scaled, permuted copies in tmp_n / tmp_m
        hipLaunchKernelGGL(k_permute<double>, dim3(nblk(n)), dim3(kBlock), 0, P->s, n, dxp, P->perm_col,
                           P->dc, P->tmp_n);
        hipLaunchKernelGGL(k_permute<double>, dim3(nblk(m)), dim3(kBlock), 0, P->s, m, dyp, P->perm_row,
                           P->dr, P->tmp_m);
    }
    launch_checks<double>(P, P->tmp_n, P->tmp_n, P->tmp_m, P->tmp_m, P->tmp_n, P->tmp_m, tau);
    // evaluate into a scratch control block so the solver state is untouched
    HIPCHK(hipMemsetAsync(P->ctl_eval, 0, sizeof(Control), P->s));
    CtlArgs a = ctl_args(P, 1);
    hipLaunchKernelGGL(k_control, dim3(1), dim3(kBlock), 0, P->s, P->part_r, P->chk_nr, P->part_c,
                       P->chk_nc, P->ctl_eval, a);
    Control h;
    HIPCHK(hipMemcpyAsync(&h, P->ctl_eval, sizeof(Control), hipMemcpyDeviceToHost, P->s));
    HIPCHK(hipStreamSynchronize(P->s));
    out5[0] = h.r_primal; out5[1] = h.r_dual; out5[2] = h.r_gap; out5[3] = h.obj_p; out5[4] = h.obj_d;
    return DPDLP_OK;
}

int dpdlp_get_scaling(dpdlp_problem *P, double *dr, double *dc, double *eta, double *sigma_max,
                      double *omega0, void *stream)
{
    ENTER(P);
    if (dr) {
        hipLaunchKernelGGL(k_unpermute<double>, dim3(nblk(P->m)), dim3(kBlock), 0, P->s, P->m, P->dr,
                           P->perm_row, (const double *)nullptr, P->tmp_m);
        HIPCHK(hipMemcpyAsync(dr, P->tmp_m, sizeof(double) * P->m, hipMemcpyDeviceToHost, P->s));
    }
    if (dc) {
        hipLaunchKernelGGL(k_unpermute<double>, dim3(nblk(P->n)), dim3(kBlock), 0, P->s, P->n, P->dc,
                           P->perm_col, (const double *)nullptr, P->tmp_n);
        HIPCHK(hipMemcpyAsync(dc, P->tmp_n, sizeof(double) * P->n, hipMemcpyDeviceToHost, P->s));
    }
    HIPCHK(hipStreamSynchronize(P->s));
    if (eta) *eta = P->eta;
    if (sigma_max) *sigma_max = P->sigma_max;
    if (omega0) *omega0 = P->omega0;
    return DPDLP_OK;
}

int dpdlp_time_kernel(dpdlp_problem *P, int32_t which, int32_t reps, void *stream, double *avg_ms,
                      double *bytes)
{
    ENTER(P);
    if (reps < 1 || which < 0 || which > 3 || !avg_ms) { set_error("bad arguments"); return DPDLP_E_INVALID_ARG; }
    const double m = P->m, n = P->n, z = (double)P->nnz;
    const bool f32 = P->prm.precision == DPDLP_FP32_MIXED && P->in_fp32;
    const double vb = f32 ? 4.0 : 8.0;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    // scratch iterate copies so the solver state does not move
    const double tau = P->eta / P->omega, sigma = P->eta * P->omega;
    auto body = [&]() {
        if (which == 0) {
            if (f32) launch_primal<float>(P, P->y32, P->c32, P->vlo32, P->vhi32, P->xa32,
                                          (float *)P->tmp_n, (float *)P->tmp_n2, P->vt32, tau, 5, 0);
            else launch_primal<double>(P, P->y, P->c, P->vlo, P->vhi, P->xa, P->tmp_n, P->tmp_n2,
                                       P->vt, tau, 5, 0);
        } else if (which == 1) {
            if (f32) launch_dual<float>(P, P->xbar32, P->clo32, P->chi32, P->ya32, (float *)P->tmp_m,
                                        P->v32, sigma, 5, 0);
            else launch_dual<double>(P, P->xbar, P->clo, P->chi, P->ya, P->tmp_m, P->v, sigma, 5, 0);
        } else if (which == 2) {
            SpmvOp op; op.in = P->x; op.div = nullptr; op.out = P->tmp_m; op.partials = P->part_r;
            launch_product(P, false, op, P->x);
        } else {
            SpmvOp op; op.in = P->y; op.div = nullptr; op.out = P->tmp_n; op.partials = P->part_c;
            launch_product(P, true, op, P->y);
        }
    };
    // the in-place update on scratch copies needs valid data in them
    if (which == 0)
        HIPCHK(hipMemcpyAsync(P->tmp_n, f32 ? (const void *)P->x32 : (const void *)P->x,
                              (f32 ? 4 : 8) * (size_t)P->n, hipMemcpyDeviceToDevice, P->s));
    if (which == 1)
        HIPCHK(hipMemcpyAsync(P->tmp_m, f32 ? (const void *)P->y32 : (const void *)P->y,
                              (f32 ? 4 : 8) * (size_t)P->m, hipMemcpyDeviceToDevice, P->s));
    body();
    HIPCHK(hipEventRecord(e0, P->s));
    for (int r = 0; r < reps; ++r) body();
    HIPCHK(hipEventRecord(e1, P->s));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIPCHK(hipGetLastError());
    *avg_ms = ms / reps;
    if (bytes) {
        const double ib = 4.0;   // int32 index / pointer
        const double mb = f32 ? 4.0 : 8.0;
        if (which == 0) *bytes = z * (ib + mb) + ib * (n + 1) + 5 * vb * n + 2 * vb * n + vb * m;
        else if (which == 1) *bytes = z * (ib + mb) + ib * (m + 1) + 4 * vb * m + vb * m + vb * n;
        else if (which == 2) *bytes = z * 12.0 + 4.0 * (m + 1) + 8.0 * n + 8.0 * m;
        else *bytes = z * 12.0 + 4.0 * (n + 1) + 8.0 * m + 8.0 * n;
    }
    return DPDLP_OK;
}

int dpdlp_profile_enable(dpdlp_problem *P, int32_t enable)
{
    if (!P) { set_error("NULL problem"); return DPDLP_E_INVALID_ARG; }
    if (enable) {
        for (int c = 0; c < 8; ++c) { P->prof_ms[c] = 0; P->prof_n[c] = 0; }
    }
    P->prof = enable != 0;
    return DPDLP_OK;
}

int dpdlp_get_profile(dpdlp_problem *P, double *total_ms, int64_t *launches, double *bytes_per_launch)
{
    if (!P) { set_error("NULL problem"); return DPDLP_E_INVALID_ARG; }
    prof_collect(P);
    const double m = P->m, n = P->n, z = (double)P->nnz;
    const bool f32 = P->in_fp32;
    const double vb = f32 ? 4.0 : 8.0, mb = f32 ? 4.0 : 8.0;
    const double bpl[8] = {
        z * (4.0 + mb) + 4.0 * (n + 1) + (P->has_q ? 8 : 7) * vb * n + vb * m,  // primal: CSC,
                                                                  // x c l u xa (q), xbar x, y
        z * (4.0 + mb) + 4.0 * (m + 1) + 5 * vb * m + vb * n,     // dual: CSR, y l u ya, y, xbar
        z * 24.0 / 2 + 4.0 * (m + 1) + 16.0 * n + 8.0 * 7 * m,    // check CSR
        z * 24.0 / 2 + 4.0 * (n + 1) + 8.0 * m + 8.0 * 7 * n,     // check CSC
        0, 0, 0, 0};
    for (int c = 0; c < 8; ++c) {
        if (total_ms) total_ms[c] = P->prof_ms[c];
        if (launches) launches[c] = P->prof_n[c];
        if (bytes_per_launch) bytes_per_launch[c] = bpl[c];
    }
    return DPDLP_OK;
}

}  // extern "C"
