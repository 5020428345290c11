// KKT evaluation that allocates nothing (dpdlp_kkt_noalloc in dpdlp.h), for
// callers that cannot call hipMalloc: code under HIP graph capture, tight
// serving loops.  It evaluates the relative KKT error of App. B.4 of an LP
// (or a diagonal QP, Sec. 6) given in CSR and CSC directly from the caller's
// device arrays, with per-column primal steps tau * col_scale_j^2 (the
// solver's scaled-space step mapped to the original space, so the result is
// the solver's own termination measure, the one dpdlp_kkt reports).
//
// Its only device memory beyond the inputs and outputs is the per-workgroup
// partial sums, kept in the file-scope array `scratch` below.  Every
// workgroup writes all of its slots on every call before the final kernel
// reads them, so nothing needs clearing; calls that overlap on one GPU share
// the array and race.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

#include "dpdlp_internal.h"

namespace {

constexpr int kNaThreads = 256;                 // threads per workgroup
constexpr int kNaLanes = 8;                     // lanes per row / column
constexpr int kNaSegs = 256;                    // rows or columns per workgroup
constexpr int kNaMaxBlocks = 65536;             // workgroups per pass
constexpr int kNaRowQ = 3;                      // row-pass partial quantities
constexpr int kNaColQ = 4;                      // column-pass partial quantities
constexpr int kNaMaxDevices = 64;

}  // namespace

// Partial sums of both passes: [kNaRowQ][kNaMaxBlocks] then [kNaColQ][kNaMaxBlocks]
// (3.7 MB per GPU, held until the process ends).
static __device__ __align__(256) double scratch[(kNaRowQ + kNaColQ) * kNaMaxBlocks];

namespace {

std::mutex g_na_mu;
double *g_na_ptr[kNaMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (each GPU holds its own copy of the array at its own address).
int scratch_address(double **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        dpdlp::set_error(std::string("hipGetDevice: ") + hipGetErrorString(e));
        return DPDLP_E_HIP;
    }
    if (dev < 0 || dev >= kNaMaxDevices) {
        dpdlp::set_error("dpdlp_kkt_noalloc: device ordinal beyond 63");
        return DPDLP_E_NOT_SUPPORTED;
    }
    std::lock_guard<std::mutex> lk(g_na_mu);
    if (!g_na_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            dpdlp::set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            return DPDLP_E_HIP;
        }
        g_na_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_na_ptr[dev];
    return DPDLP_OK;
}

__device__ __forceinline__ double clampd(double v, double lo, double hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

__device__ __forceinline__ double sum8(double v)
{
    v += __shfl_xor(v, 4, 64);
    v += __shfl_xor(v, 2, 64);
    v += __shfl_xor(v, 1, 64);
    return v;
}

// Fixed-order workgroup sum of NQ values; thread 0 writes part[q * nb + block].
template <int NQ>
__device__ void block_partials(double (&acc)[NQ], double *part, int nb)
{
    __shared__ double s[NQ][kNaThreads / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double v = acc[q];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) s[q][wave] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            double v = s[q][0];
            for (int w = 1; w < kNaThreads / 64; ++w) v += s[q][w];
            part[(size_t)q * nb + blockIdx.x] = v;
        }
    }
}

// Row pass: per row i, (A x)_i by 8 lanes in fixed strided order, then
//   0 sum ((A x)_i - proj_[lo_i, hi_i]((A x)_i))^2
//   1 sum (lo_i y_i^+ - hi_i y_i^-)          (= -p(-y; lo, hi))
//   2 sum of the squared finite bounds        (||[lo, hi]||^2)
__global__ __launch_bounds__(kNaThreads) void k_na_rows(
    int m, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
    const double *__restrict__ val, const double *__restrict__ x, const double *__restrict__ y,
    const double *__restrict__ lo, const double *__restrict__ hi, double *part, int nb)
{
    double acc[kNaRowQ] = {0.0, 0.0, 0.0};
    const int lane = threadIdx.x & (kNaLanes - 1);
    for (int r = 0; r < kNaSegs * kNaLanes / kNaThreads; ++r) {
        const int i = blockIdx.x * kNaSegs + r * (kNaThreads / kNaLanes) + threadIdx.x / kNaLanes;
        double s = 0.0;
        if (i < m)
            for (int p = rp[i] + lane; p < rp[i + 1]; p += kNaLanes) s += val[p] * x[ci[p]];
        s = sum8(s);
        if (i < m && lane == 0) {
            const double l = lo[i], h = hi[i];
            const double res = s - clampd(s, l, h);
            acc[0] += res * res;
            const double yi = y[i];
            if (yi > 0.0) acc[1] += l * yi;
            else if (yi < 0.0) acc[1] += h * yi;
            if (std::isfinite(l)) acc[2] += l * l;
            if (std::isfinite(h)) acc[2] += h * h;
        }
    }
    block_partials<kNaRowQ>(acc, part, nb);
}

// Column pass: per column j, g = c_j + q_j x_j - (A^T y)_j, the projected
// step u = x_j - tau_j g with tau_j = tau * dc_j^2 and s = (clamp(u) - u) / tau_j:
//   0 sum (g - s)^2   1 sum c_j x_j + q_j x_j^2 / 2   2 sum s_j x_j - q_j x_j^2 / 2
//   3 sum c_j^2
__global__ __launch_bounds__(kNaThreads) void k_na_cols(
    int n, const int32_t *__restrict__ cp, const int32_t *__restrict__ ri,
    const double *__restrict__ vt, const double *__restrict__ y, const double *__restrict__ x,
    const double *__restrict__ c, const double *__restrict__ vlo, const double *__restrict__ vhi,
    const double *__restrict__ dc, const double *__restrict__ q, double tau, double *part, int nb)
{
    double acc[kNaColQ] = {0.0, 0.0, 0.0, 0.0};
    const int lane = threadIdx.x & (kNaLanes - 1);
    for (int r = 0; r < kNaSegs * kNaLanes / kNaThreads; ++r) {
        const int j = blockIdx.x * kNaSegs + r * (kNaThreads / kNaLanes) + threadIdx.x / kNaLanes;
        double s = 0.0;
        if (j < n)
            for (int p = cp[j] + lane; p < cp[j + 1]; p += kNaLanes) s += vt[p] * y[ri[p]];
        s = sum8(s);
        if (j < n && lane == 0) {
            const double xj = x[j], cj = c[j];
            const double qx = q ? q[j] * xj : 0.0;
            const double g = cj + qx - s;
            const double tj = dc ? tau * dc[j] * dc[j] : tau;
            const double u = xj - tj * g;
            const double sj = (clampd(u, vlo[j], vhi[j]) - u) / tj;
            const double d = g - sj;
            acc[0] += d * d;
            const double half_xqx = 0.5 * qx * xj;
            acc[1] += cj * xj + half_xqx;
            acc[2] += sj * xj - half_xqx;
            acc[3] += cj * cj;
        }
    }
    block_partials<kNaColQ>(acc, part, nb);
}

// One workgroup: the partials of each quantity summed in block order, then
// r_primal, r_dual, r_gap, primal and dual objective into out5 (App. B.4).
__global__ __launch_bounds__(kNaThreads) void k_na_finish(const double *rpart, int nbr,
                                                         const double *cpart, int nbc,
                                                         double *out5)
{
    __shared__ double s[kNaRowQ + kNaColQ][kNaThreads];
    double a[kNaRowQ + kNaColQ];
    for (int q = 0; q < kNaRowQ + kNaColQ; ++q) a[q] = 0.0;
    for (int i = threadIdx.x; i < nbr; i += kNaThreads)
        for (int q = 0; q < kNaRowQ; ++q) a[q] += rpart[(size_t)q * nbr + i];
    for (int i = threadIdx.x; i < nbc; i += kNaThreads)
        for (int q = 0; q < kNaColQ; ++q) a[kNaRowQ + q] += cpart[(size_t)q * nbc + i];
    for (int q = 0; q < kNaRowQ + kNaColQ; ++q) s[q][threadIdx.x] = a[q];
    __syncthreads();
    for (int w = kNaThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int q = 0; q < kNaRowQ + kNaColQ; ++q) s[q][threadIdx.x] += s[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double pres = s[0][0], py = s[1][0], bn2 = s[2][0];
    const double dres = s[3][0], cx = s[4][0], sx = s[5][0], cn2 = s[6][0];
    const double dobj = py + sx;
    out5[0] = sqrt(pres) / (1.0 + sqrt(bn2));
    out5[1] = sqrt(dres) / (1.0 + sqrt(cn2));
    out5[2] = fabs(cx - dobj) / (1.0 + fmax(fabs(cx), fabs(dobj)));
    out5[3] = cx;
    out5[4] = dobj;
}

}  // namespace

extern "C" int dpdlp_kkt_noalloc(const dpdlp_csr_lp *lp, const int32_t *col_ptr,
                                 const int32_t *row_idx, const double *val_csc,
                                 const double *col_scale, const double *q, const double *x,
                                 const double *y, double tau, double *out5, void *stream)
{
    if (!lp || !col_ptr || !row_idx || !val_csc || !x || !y || !out5 || !lp->row_ptr ||
        !lp->col_idx || !lp->val || !lp->c || !lp->con_lo || !lp->con_hi || !lp->var_lo ||
        !lp->var_hi) {
        dpdlp::set_error("dpdlp_kkt_noalloc: NULL argument");
        return DPDLP_E_INVALID_ARG;
    }
    if (lp->mem_kind != DPDLP_MEM_DEVICE) {
        dpdlp::set_error("dpdlp_kkt_noalloc: every array must be device memory (mem_kind = DPDLP_MEM_DEVICE)");
        return DPDLP_E_INVALID_ARG;
    }
    const int64_t cap = (int64_t)kNaMaxBlocks * kNaSegs;
    if (lp->m < 1 || lp->n < 1 || lp->m > cap || lp->n > cap) {
        dpdlp::set_error("dpdlp_kkt_noalloc: m and n must lie in [1, 16777216] (the partial sums "
                         "of 65536 workgroups of 256 rows or columns fill its fixed scratch)");
        return DPDLP_E_INVALID_ARG;
    }
    if (!(tau > 0.0) || !std::isfinite(tau)) {
        dpdlp::set_error("dpdlp_kkt_noalloc: tau must be positive and finite");
        return DPDLP_E_INVALID_ARG;
    }
    double *sc = nullptr;
    const int rc = scratch_address(&sc);
    if (rc != DPDLP_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int nbr = (int)((lp->m + kNaSegs - 1) / kNaSegs);
    const int nbc = (int)((lp->n + kNaSegs - 1) / kNaSegs);
    double *rpart = sc, *cpart = sc + (size_t)kNaRowQ * kNaMaxBlocks;
    hipLaunchKernelGGL(k_na_rows, dim3(nbr), dim3(kNaThreads), 0, s, lp->m, lp->row_ptr,
                       lp->col_idx, lp->val, x, y, lp->con_lo, lp->con_hi, rpart, nbr);
    hipLaunchKernelGGL(k_na_cols, dim3(nbc), dim3(kNaThreads), 0, s, lp->n, col_ptr, row_idx,
                       val_csc, y, x, lp->c, lp->var_lo, lp->var_hi, col_scale, q, tau, cpart,
                       nbc);
    hipLaunchKernelGGL(k_na_finish, dim3(1), dim3(kNaThreads), 0, s, rpart, nbr, cpart, nbc, out5);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        dpdlp::set_error(std::string("dpdlp_kkt_noalloc launch: ") + hipGetErrorString(e));
        return DPDLP_E_HIP;
    }
    return DPDLP_OK;
}
