// Learned warm start: a bipartite message-passing network on the row/column
// graph of the scaled constraint matrix A~, trained on the GPU by the kernels
// in this file, predicting a start point (x0, y0) for the PDHG solver.
//
// Network (hidden width H = 128, L layers, BF16 activations and weights,
// FP32 accumulation; FP32 master weights, gradients and Adam moments):
//   H_c^0 = relu(X_c W_cin)                 X_c: n x 16 column features
//   H_r^0 = relu(X_r W_rin)                 X_r: m x 16 row features
//   layer l = 1..L:
//     S_r = A~ H_c^{l-1}                    (CSR SpMM)
//     H_r^l = relu([H_r^{l-1}, S_r] W_r^l)  (256 x 128 weights, MFMA GEMM)
//     S_c = A~^T H_r^l                      (CSC SpMM)
//     H_c^l = relu([H_c^{l-1}, S_c] W_c^l)
//   x~0 = x~ref + H_c^L w_x,  y~0 = y~ref + H_r^L w_y   (scaled space)
// (x~ref, y~ref) is a reference point supplied by the caller (the family's
// mean solution); with w_x = w_y = 0 the network returns it exactly.
// Loss: mean((x~0 - x~*)^2) + mean((y~0 - y~*)^2).
//
// Activations are stored so that each layer's GEMM input [H^{l-1}, S] is one
// contiguous m x 256 (n x 256) BF16 array: a layer writes its output straight
// into the left half of the next layer's input.  Every reduction runs in a
// fixed order (no atomics), so training is bitwise reproducible.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "dpdlp_internal.h"

namespace dpdlp {
namespace gnn {

constexpr int kH = 128;
constexpr int kF = 16;
constexpr int kKC = 2048;             // split-K chunk of the weight-gradient GEMMs
typedef uint16_t bf16;
typedef short short4v __attribute__((ext_vector_type(4)));
typedef float float4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf16 f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u)                  // inf / nan
        return (bf16)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);                       // round to nearest even
    return (bf16)(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16 h) { return __uint_as_float(((uint32_t)h) << 16); }

enum { G_RELU = 1, G_OUT_BF16 = 2, G_ACCUM = 4 };

// C[M x Nc] = A[M x K] B[K x Nc] on the matrix cores (v_mfma_f32_16x16x16_bf16).
// A(i,k) = A[i*a_rs + k*a_cs], B(k,j) = B[k*b_rs + j*b_cs]: the strides cover
// X W, dZ W^T and X^T dZ without transposed copies.  A workgroup (4 wave64)
// owns a 64 x 64 output tile, each wave a 32 x 32 sub-tile (2 x 2 MFMA
// tiles); 64 x 32 slices of A and B are staged in LDS per K step.  blockIdx.z
// selects a K chunk [z*kc, (z+1)*kc) whose result goes to C + z*c_zs (split K;
// the chunks are added afterwards in chunk order).
__global__ __launch_bounds__(256) void k_gemm(const bf16 *__restrict__ A, long a_rs, long a_cs,
                                              const bf16 *__restrict__ B, long b_rs, long b_cs,
                                              void *__restrict__ C, long ldc, long c_zs, int M,
                                              int Nc, int K, int kc, int flags)
{
    __shared__ bf16 As[64][40];
    __shared__ bf16 Bs[64][40];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int bm = blockIdx.x * 64, bn = blockIdx.y * 64;
    const int k0 = blockIdx.z * kc, k1 = min(K, k0 + kc);
    const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
    float4v acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = float4v{0.f, 0.f, 0.f, 0.f};
    for (int kk = k0; kk < k1; kk += 32) {
        for (int e = tid; e < 64 * 32; e += 256) {
            int i, k;
            if (a_cs == 1) { i = e >> 5; k = e & 31; } else { i = e & 63; k = e >> 6; }
            const int gi = bm + i, gk = kk + k;
            As[i][k] = (gi < M && gk < k1) ? A[(long)gi * a_rs + (long)gk * a_cs] : (bf16)0;
        }
        for (int e = tid; e < 64 * 32; e += 256) {
            int j, k;
            if (b_cs == 1) { j = e & 63; k = e >> 6; } else { j = e >> 5; k = e & 31; }
            const int gj = bn + j, gk = kk + k;
            Bs[j][k] = (gj < Nc && gk < k1) ? B[(long)gk * b_rs + (long)gj * b_cs] : (bf16)0;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < 32; ks += 16) {
            short4v fa[2], fb[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const bf16 *pa = &As[wm + t * 16 + (lane & 15)][ks + 4 * (lane >> 4)];
                fa[t] = short4v{(short)pa[0], (short)pa[1], (short)pa[2], (short)pa[3]};
                const bf16 *pb = &Bs[wn + t * 16 + (lane & 15)][ks + 4 * (lane >> 4)];
                fb[t] = short4v{(short)pb[0], (short)pb[1], (short)pb[2], (short)pb[3]};
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(fa[a], fb[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }
    float *C32 = (float *)C;
    bf16 *C16 = (bf16 *)C;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = bm + wm + a * 16 + 4 * (lane >> 4) + v;
                const int j = bn + wn + b * 16 + (lane & 15);
                if (i >= M || j >= Nc) continue;
                const long off = (long)blockIdx.z * c_zs + (long)i * ldc + j;
                float r = acc[a][b][v];
                if (flags & G_ACCUM) r += (flags & G_OUT_BF16) ? bf2f(C16[off]) : C32[off];
                if (flags & G_RELU) r = fmaxf(r, 0.f);
                if (flags & G_OUT_BF16) C16[off] = f2bf(r);
                else C32[off] = r;
            }
}

// out[e] (+)= sum_z part[z * stride + e], z in chunk order.
__global__ void k_sum_chunks(const float *__restrict__ part, long stride, int nz, float *out, long n,
                             int accum)
{
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    float s = 0.f;
    for (int z = 0; z < nz; ++z) s += part[(long)z * stride + e];
    out[e] = accum ? out[e] + s : s;
}

// out[s, :] (+)= sum_{p in segment s} a_p in[idx_p, :]; one wave per segment,
// each lane two of the 128 features; FP32 accumulation in stored order.
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_spmm(const int *__restrict__ ptr, const int *__restrict__ idx,
                                              const float *__restrict__ val, int nseg,
                                              const TI *__restrict__ in, long in_ld,
                                              TO *__restrict__ out, long out_ld, int accum)
{
    const int seg = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (seg >= nseg) return;
    float a0 = 0.f, a1 = 0.f;
    const int pe = ptr[seg + 1];
    for (int p = ptr[seg]; p < pe; ++p) {
        const int j = idx[p];
        const float a = val[p];
        float h0, h1;
        if constexpr (sizeof(TI) == 2) {
            const uint32_t u = *(const uint32_t *)((const bf16 *)in + (long)j * in_ld + 2 * lane);
            h0 = bf2f((bf16)(u & 0xffffu));
            h1 = bf2f((bf16)(u >> 16));
        } else {
            const float2 f = *(const float2 *)((const float *)in + (long)j * in_ld + 2 * lane);
            h0 = f.x; h1 = f.y;
        }
        a0 += a * h0;
        a1 += a * h1;
    }
    const long o = (long)seg * out_ld + 2 * lane;
    if constexpr (sizeof(TO) == 2) {
        bf16 *po = (bf16 *)out + o;
        if (accum) { a0 += bf2f(po[0]); a1 += bf2f(po[1]); }
        po[0] = f2bf(a0); po[1] = f2bf(a1);
    } else {
        float *po = (float *)out + o;
        if (accum) { a0 += po[0]; a1 += po[1]; }
        po[0] = a0; po[1] = a1;
    }
}

__global__ void k_d2f(const double *__restrict__ a, float *__restrict__ b, long n)
{
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}
__global__ void k_f2bf(const float *__restrict__ a, bf16 *__restrict__ b, long n)
{
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = f2bf(a[i]);
}

// Column features (permuted order, scaled space; see dpdlp.h):
//   [c~, c~ - c~ref, x~ref, has_lo, has_hi, lo~ or 0, hi~ or 0, 1, 0 ...]
__global__ void k_feat_col(int n, const int *perm, const double *dc, const double *c,
                           const double *cref, const double *xref, const double *vlo0,
                           const double *vhi0, bf16 *X, float *xref_s)
{
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int o = perm[j];
    const double d = dc[j];
    const double lo = vlo0[j], hi = vhi0[j];
    float f[kF] = {0};
    f[0] = (float)(d * c[o]);
    f[1] = (float)(d * (c[o] - cref[o]));
    const double xr = xref[o] / d;
    f[2] = (float)xr;
    f[3] = isfinite(lo) ? 1.f : 0.f;
    f[4] = isfinite(hi) ? 1.f : 0.f;
    f[5] = isfinite(lo) ? (float)fmin(fmax(lo / d, -1e4), 1e4) : 0.f;
    f[6] = isfinite(hi) ? (float)fmin(fmax(hi / d, -1e4), 1e4) : 0.f;
    f[7] = 1.f;
    for (int q = 0; q < kF; ++q) X[(long)j * kF + q] = f2bf(f[q]);
    xref_s[j] = (float)xr;
}
// Row features: b = finite lo, else finite hi, else 0;
//   [b~, b~ - b~ref, y~ref, is_eq, has_lo, has_hi, 0, 1, 0 ...]
__global__ void k_feat_row(int m, const int *perm, const double *dr, const double *lo,
                           const double *hi, const double *bref, const double *yref, bf16 *X,
                           float *yref_s)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const int o = perm[i];
    const double d = dr[i];
    const double l = lo[o], h = hi[o];
    const double b = isfinite(l) ? l : (isfinite(h) ? h : 0.0);
    float f[kF] = {0};
    f[0] = (float)(d * b);
    f[1] = (float)(d * (b - bref[o]));
    const double yr = yref[o] / d;
    f[2] = (float)yr;
    f[3] = (isfinite(l) && isfinite(h) && l == h) ? 1.f : 0.f;
    f[4] = isfinite(l) ? 1.f : 0.f;
    f[5] = isfinite(h) ? 1.f : 0.f;
    f[7] = 1.f;
    for (int q = 0; q < kF; ++q) X[(long)i * kF + q] = f2bf(f[q]);
    yref_s[i] = (float)yr;
}

// pred_j = ref_j + sum_f H[j, f] w[f]   (sequential over f)
__global__ void k_head(int n, const bf16 *__restrict__ Hl, long ld, const float *__restrict__ w,
                       const float *__restrict__ ref, float *__restrict__ pred)
{
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    float s = 0.f;
    for (int f = 0; f < kH; ++f) s += bf2f(Hl[(long)j * ld + f]) * w[f];
    pred[j] = ref[j] + s;
}

// Loss gradient of the head: d_j = 2 (pred_j - target_j) / n, dH[j, f] = d_j w[f];
// per-block partial sums of the squared error (for the loss) go to part[block].
__global__ __launch_bounds__(256) void k_head_bwd(int n, const float *__restrict__ pred,
                                                  const float *__restrict__ tgt,
                                                  const float *__restrict__ w,
                                                  float *__restrict__ dpred,
                                                  float *__restrict__ dH, double *part)
{
    __shared__ double s[256];
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    double e2 = 0.0;
    if (j < n) {
        const float r = pred[j] - tgt[j];
        e2 = (double)r * (double)r;
        const float d = 2.f * r / (float)n;
        dpred[j] = d;
        for (int f = 0; f < kH; ++f) dH[(long)j * kH + f] = d * w[f];
    }
    s[threadIdx.x] = e2;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// dw[f] partials over node chunks: part[c * kH + f] = sum_{j in chunk c} d_j H[j, f]
__global__ __launch_bounds__(kH) void k_head_wgrad(int n, int chunk, const bf16 *__restrict__ Hl,
                                                   long ld, const float *__restrict__ d,
                                                   float *__restrict__ part)
{
    const int f = threadIdx.x, c = blockIdx.x;
    const int j0 = c * chunk, j1 = min(n, j0 + chunk);
    float s = 0.f;
    for (int j = j0; j < j1; ++j) s += d[j] * bf2f(Hl[(long)j * ld + f]);
    part[(long)c * kH + f] = s;
}

// dZ = dH * [H > 0] (the ReLU derivative on the stored output), as a BF16
// pair hi + lo with hi = bf16(dZ), lo = bf16(dZ - hi): the gradient GEMMs run
// both on the matrix cores and add them in FP32 (about 16 mantissa bits).
__global__ void k_relu_bwd(long rows, const float *__restrict__ dH, long dld,
                           const bf16 *__restrict__ Hout, long hld, bf16 *__restrict__ dZ,
                           bf16 *__restrict__ dZlo)
{
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * kH) return;
    const long r = e / kH, f = e % kH;
    const float g = bf2f(Hout[r * hld + f]) > 0.f ? dH[r * dld + f] : 0.f;
    const bf16 hi = f2bf(g);
    dZ[r * kH + f] = hi;
    dZlo[r * kH + f] = f2bf(g - bf2f(hi));
}

// dst[r, 0:128] = src[r, 0:128] (strided f32 copy)
__global__ void k_copy_rows(long rows, const float *__restrict__ src, long sld, float *__restrict__ dst,
                            long dld)
{
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * kH) return;
    const long r = e / kH, f = e % kH;
    dst[r * dld + f] = src[r * sld + f];
}

__global__ void k_adam(long n, float *__restrict__ w, const float *__restrict__ g,
                       float *__restrict__ m1, float *__restrict__ m2, bf16 *__restrict__ wb,
                       float lr, float b1, float b2, float eps, float c1, float c2)
{
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.f - b1) * gi;
    const float b = b2 * m2[i] + (1.f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = b;
    const float wi = w[i] - lr * (a / c1) / (sqrtf(b / c2) + eps);
    w[i] = wi;
    wb[i] = f2bf(wi);
}

// out[perm[j]] = scale[j] * pred[j]  (scaled, permuted -> original; x = D_c x~,
// y = D_r y~)
__global__ void k_unperm_scale(int n, const float *pred, const int *perm, const double *scale,
                               int mul, double *out)
{
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    out[perm[j]] = mul ? scale[j] * (double)pred[j] : (double)pred[j] / scale[j];
}
// out[j] = x[perm[j]] / scale[j]  (original -> scaled, permuted)
__global__ void k_perm_scale(int n, const double *x, const int *perm, const double *scale, int mul,
                             float *out)
{
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    out[j] = (float)(mul ? x[perm[j]] * scale[j] : x[perm[j]] / scale[j]);
}
__global__ __launch_bounds__(256) void k_sum_double(const double *part, int np, double *out)
{
    __shared__ double s[256];
    double a = 0.0;
    for (int i = threadIdx.x; i < np; i += 256) a += part[i];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = s[0];
}

}  // namespace gnn
}  // namespace dpdlp

using namespace dpdlp;
using namespace dpdlp::gnn;

struct dpdlp_gnn {
    ProblemView pv;
    hipStream_t s = nullptr;
    int L = 3;
    long n_params = 0;
    std::vector<void *> mem;
    // parameters
    float *w = nullptr, *g = nullptr, *m1 = nullptr, *m2 = nullptr;
    bf16 *wb = nullptr;
    long off_cin = 0, off_rin = 0, off_wx = 0, off_wy = 0;
    std::vector<long> off_c, off_r;
    int adam_t = 0;
    // graph values in FP32
    float *vf = nullptr, *vtf = nullptr;
    // features, references, activations
    bf16 *Xc = nullptr, *Xr = nullptr;
    float *xref = nullptr, *yref = nullptr, *px = nullptr, *py = nullptr;
    float *tx = nullptr, *ty = nullptr, *dpx = nullptr, *dpy = nullptr;
    std::vector<bf16 *> INc, INr;          // index 1..L
    bf16 *Hc_last = nullptr, *Hr_last = nullptr;
    float *dHc = nullptr, *dHr = nullptr, *dINc = nullptr, *dINr = nullptr;
    bf16 *dZc = nullptr, *dZr = nullptr, *dZc_lo = nullptr, *dZr_lo = nullptr;
    float *wpart = nullptr;
    double *lpart = nullptr, *lsum = nullptr;
    double *ref_c = nullptr, *ref_b = nullptr, *ref_x = nullptr, *ref_y = nullptr;
    double *tmp_n = nullptr, *tmp_m = nullptr, *tmp_n2 = nullptr, *tmp_m2 = nullptr, *tmp_m3 = nullptr;
    bool have_ref = false, have_inst = false;
    ~dpdlp_gnn() { for (void *p : mem) (void)hipFree(p); }
};

namespace {

int gfail(hipError_t e, const char *what)
{
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? DPDLP_E_OOM : DPDLP_E_HIP;
}
#define GCHK(expr)                                           \
    do {                                                     \
        hipError_t _e = (expr);                              \
        if (_e != hipSuccess) return gfail(_e, #expr);       \
    } while (0)
#define RCHK(expr)                      \
    do {                                \
        int _r = (expr);                \
        if (_r != DPDLP_OK) return _r;  \
    } while (0)

template <typename T>
int galloc(dpdlp_gnn *G, T **p, size_t count)
{
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
    if (e != hipSuccess) return gfail(e, "hipMalloc");
    G->mem.push_back(q);
    *p = (T *)q;
    return DPDLP_OK;
}

inline unsigned nb(long n, int b = 256) { return (unsigned)((n + b - 1) / b); }

void gemm(dpdlp_gnn *G, const bf16 *A, long a_rs, long a_cs, const bf16 *B, long b_rs, long b_cs,
          void *C, long ldc, int M, int Nc, int K, int flags)
{
    hipLaunchKernelGGL(k_gemm, dim3(nb(M, 64), nb(Nc, 64), 1), dim3(256), 0, G->s, A, a_rs, a_cs, B,
                       b_rs, b_cs, C, ldc, 0L, M, Nc, K, K, flags);
}

// weight gradient  out[M x Nc] (+)= A^T[M x K] dZ[K x Nc]  (split K, chunk order)
void wgrad1(dpdlp_gnn *G, const bf16 *A, long a_ld, int M, const bf16 *dZ, int K, float *out,
            int accum)
{
    const int nz = (K + kKC - 1) / kKC;
    const long zs = (long)M * kH;
    hipLaunchKernelGGL(k_gemm, dim3(nb(M, 64), nb(kH, 64), nz), dim3(256), 0, G->s, A, 1L, a_ld, dZ,
                       (long)kH, 1L, (void *)G->wpart, (long)kH, zs, M, kH, K, kKC, 0);
    hipLaunchKernelGGL(k_sum_chunks, dim3(nb(zs)), dim3(256), 0, G->s, G->wpart, zs, nz, out, zs,
                       accum);
}
// with dZ given as the BF16 pair (hi, lo)
void wgrad(dpdlp_gnn *G, const bf16 *A, long a_ld, int M, const bf16 *dZ, const bf16 *dZlo, int K,
           float *out)
{
    wgrad1(G, A, a_ld, M, dZ, K, out, 0);
    wgrad1(G, A, a_ld, M, dZlo, K, out, 1);
}
// data gradient  out[N x 256] = dZ W^T with dZ = hi + lo (FP32 output)
void dgrad(dpdlp_gnn *G, const bf16 *dZ, const bf16 *dZlo, const bf16 *W, float *out, int N)
{
    gemm(G, dZ, kH, 1, W, 1, kH, out, 2 * kH, N, 2 * kH, kH, 0);
    gemm(G, dZlo, kH, 1, W, 1, kH, out, 2 * kH, N, 2 * kH, kH, G_ACCUM);
}

template <typename TI, typename TO>
void spmm(dpdlp_gnn *G, bool csr, const TI *in, long in_ld, TO *out, long out_ld, int accum)
{
    const ProblemView &P = G->pv;
    const int nseg = csr ? P.m : P.n;
    hipLaunchKernelGGL((k_spmm<TI, TO>), dim3(nb(nseg, 4)), dim3(256), 0, G->s, csr ? P.rp : P.cp,
                       csr ? P.ci : P.ri, csr ? G->vf : G->vtf, nseg, in, in_ld, out, out_ld, accum);
}

const bf16 *Hc_of(dpdlp_gnn *G, int l, long *ld)
{
    if (l < G->L) { *ld = 2 * kH; return G->INc[(size_t)l + 1]; }
    *ld = kH;
    return G->Hc_last;
}
const bf16 *Hr_of(dpdlp_gnn *G, int l, long *ld)
{
    if (l < G->L) { *ld = 2 * kH; return G->INr[(size_t)l + 1]; }
    *ld = kH;
    return G->Hr_last;
}

void forward(dpdlp_gnn *G)
{
    const int m = G->pv.m, n = G->pv.n, L = G->L;
    const int RB = G_RELU | G_OUT_BF16;
    gemm(G, G->Xc, kF, 1, G->wb + G->off_cin, kH, 1, G->INc[1], 2 * kH, n, kH, kF, RB);
    gemm(G, G->Xr, kF, 1, G->wb + G->off_rin, kH, 1, G->INr[1], 2 * kH, m, kH, kF, RB);
    for (int l = 1; l <= L; ++l) {
        spmm<bf16, bf16>(G, true, G->INc[l], 2 * kH, G->INr[l] + kH, 2 * kH, 0);
        long ldr;
        bf16 *Hr = (bf16 *)Hr_of(G, l, &ldr);
        gemm(G, G->INr[l], 2 * kH, 1, G->wb + G->off_r[(size_t)l - 1], kH, 1, Hr, ldr, m, kH, 2 * kH, RB);
        spmm<bf16, bf16>(G, false, Hr, ldr, G->INc[l] + kH, 2 * kH, 0);
        long ldc;
        bf16 *Hc = (bf16 *)Hc_of(G, l, &ldc);
        gemm(G, G->INc[l], 2 * kH, 1, G->wb + G->off_c[(size_t)l - 1], kH, 1, Hc, ldc, n, kH, 2 * kH, RB);
    }
    hipLaunchKernelGGL(k_head, dim3(nb(n)), dim3(256), 0, G->s, n, G->Hc_last, (long)kH,
                       G->w + G->off_wx, G->xref, G->px);
    hipLaunchKernelGGL(k_head, dim3(nb(m)), dim3(256), 0, G->s, m, G->Hr_last, (long)kH,
                       G->w + G->off_wy, G->yref, G->py);
}

void backward(dpdlp_gnn *G)
{
    const int m = G->pv.m, n = G->pv.n, L = G->L;
    const unsigned bn_ = nb(n), bm_ = nb(m);
    hipLaunchKernelGGL(k_head_bwd, dim3(bn_), dim3(256), 0, G->s, n, G->px, G->tx, G->w + G->off_wx,
                       G->dpx, G->dHc, G->lpart);
    hipLaunchKernelGGL(k_head_bwd, dim3(bm_), dim3(256), 0, G->s, m, G->py, G->ty, G->w + G->off_wy,
                       G->dpy, G->dHr, G->lpart + bn_);
    hipLaunchKernelGGL(k_sum_double, dim3(1), dim3(256), 0, G->s, G->lpart, (int)bn_, G->lsum);
    hipLaunchKernelGGL(k_sum_double, dim3(1), dim3(256), 0, G->s, G->lpart + bn_, (int)bm_, G->lsum + 1);
    const int ch = 1024;
    const int ncx = (n + ch - 1) / ch, ncy = (m + ch - 1) / ch;
    hipLaunchKernelGGL(k_head_wgrad, dim3(ncx), dim3(kH), 0, G->s, n, ch, G->Hc_last, (long)kH, G->dpx, G->wpart);
    hipLaunchKernelGGL(k_sum_chunks, dim3(1), dim3(kH), 0, G->s, G->wpart, (long)kH, ncx, G->g + G->off_wx, (long)kH, 0);
    hipLaunchKernelGGL(k_head_wgrad, dim3(ncy), dim3(kH), 0, G->s, m, ch, G->Hr_last, (long)kH, G->dpy, G->wpart);
    hipLaunchKernelGGL(k_sum_chunks, dim3(1), dim3(kH), 0, G->s, G->wpart, (long)kH, ncy, G->g + G->off_wy, (long)kH, 0);

    for (int l = L; l >= 1; --l) {
        long ldc, ldr;
        const bf16 *Hc = Hc_of(G, l, &ldc);
        const bf16 *Hr = Hr_of(G, l, &ldr);
        // column update of layer l
        hipLaunchKernelGGL(k_relu_bwd, dim3(nb((long)n * kH)), dim3(256), 0, G->s, (long)n, G->dHc,
                           (long)kH, Hc, ldc, G->dZc, G->dZc_lo);
        wgrad(G, G->INc[l], 2 * kH, 2 * kH, G->dZc, G->dZc_lo, n, G->g + G->off_c[(size_t)l - 1]);
        dgrad(G, G->dZc, G->dZc_lo, G->wb + G->off_c[(size_t)l - 1], G->dINc, n);
        spmm<float, float>(G, true, G->dINc + kH, 2 * kH, G->dHr, kH, 1);   // dH_r^l += A~ dS_c
        // row update of layer l
        hipLaunchKernelGGL(k_relu_bwd, dim3(nb((long)m * kH)), dim3(256), 0, G->s, (long)m, G->dHr,
                           (long)kH, Hr, ldr, G->dZr, G->dZr_lo);
        wgrad(G, G->INr[l], 2 * kH, 2 * kH, G->dZr, G->dZr_lo, m, G->g + G->off_r[(size_t)l - 1]);
        dgrad(G, G->dZr, G->dZr_lo, G->wb + G->off_r[(size_t)l - 1], G->dINr, m);
        // gradients of the previous layer's outputs
        hipLaunchKernelGGL(k_copy_rows, dim3(nb((long)n * kH)), dim3(256), 0, G->s, (long)n, G->dINc,
                           2L * kH, G->dHc, (long)kH);
        spmm<float, float>(G, false, G->dINr + kH, 2 * kH, G->dHc, kH, 1);  // dH_c^{l-1} += A~^T dS_r
        hipLaunchKernelGGL(k_copy_rows, dim3(nb((long)m * kH)), dim3(256), 0, G->s, (long)m, G->dINr,
                           2L * kH, G->dHr, (long)kH);
    }
    // embeddings
    hipLaunchKernelGGL(k_relu_bwd, dim3(nb((long)n * kH)), dim3(256), 0, G->s, (long)n, G->dHc,
                       (long)kH, G->INc[1], 2L * kH, G->dZc, G->dZc_lo);
    wgrad(G, G->Xc, kF, kF, G->dZc, G->dZc_lo, n, G->g + G->off_cin);
    hipLaunchKernelGGL(k_relu_bwd, dim3(nb((long)m * kH)), dim3(256), 0, G->s, (long)m, G->dHr,
                       (long)kH, G->INr[1], 2L * kH, G->dZr, G->dZr_lo);
    wgrad(G, G->Xr, kF, kF, G->dZr, G->dZr_lo, m, G->g + G->off_rin);
}

// host or device double vector -> device (staging through tmp when host)
int to_dev(dpdlp_gnn *G, const double *src, int mem_kind, double *stage, long k, const double **out)
{
    if (!src) { *out = nullptr; return DPDLP_OK; }
    if (mem_kind == DPDLP_MEM_HOST) {
        GCHK(hipMemcpyAsync(stage, src, sizeof(double) * (size_t)k, hipMemcpyHostToDevice, G->s));
        *out = stage;
    } else {
        *out = src;
    }
    return DPDLP_OK;
}

}  // namespace

extern "C" {

int dpdlp_gnn_create(dpdlp_problem *prob, int32_t layers, void *stream, dpdlp_gnn **out)
{
    if (!prob || !out || layers < 1 || layers > 8) {
        set_error("bad arguments");
        return DPDLP_E_INVALID_ARG;
    }
    *out = nullptr;
    auto G = std::make_unique<dpdlp_gnn>();
    RCHK(problem_view(prob, &G->pv));
    G->s = (hipStream_t)stream;
    G->L = layers;
    const long m = G->pv.m, n = G->pv.n, nnz = G->pv.nnz;
    // parameter layout
    long off = 0;
    G->off_cin = off; off += (long)kF * kH;
    G->off_rin = off; off += (long)kF * kH;
    for (int l = 0; l < layers; ++l) {
        G->off_c.push_back(off); off += 2L * kH * kH;
        G->off_r.push_back(off); off += 2L * kH * kH;
    }
    G->off_wx = off; off += kH;
    G->off_wy = off; off += kH;
    G->n_params = off;
    RCHK(galloc(G.get(), &G->w, (size_t)off));
    RCHK(galloc(G.get(), &G->g, (size_t)off));
    RCHK(galloc(G.get(), &G->m1, (size_t)off));
    RCHK(galloc(G.get(), &G->m2, (size_t)off));
    RCHK(galloc(G.get(), &G->wb, (size_t)off));
    GCHK(hipMemsetAsync(G->w, 0, sizeof(float) * off, G->s));
    GCHK(hipMemsetAsync(G->g, 0, sizeof(float) * off, G->s));
    GCHK(hipMemsetAsync(G->m1, 0, sizeof(float) * off, G->s));
    GCHK(hipMemsetAsync(G->m2, 0, sizeof(float) * off, G->s));
    GCHK(hipMemsetAsync(G->wb, 0, sizeof(bf16) * off, G->s));
    RCHK(galloc(G.get(), &G->vf, (size_t)nnz));
    RCHK(galloc(G.get(), &G->vtf, (size_t)nnz));
    if (nnz) {
        hipLaunchKernelGGL(k_d2f, dim3(nb(nnz)), dim3(256), 0, G->s, G->pv.v, G->vf, nnz);
        hipLaunchKernelGGL(k_d2f, dim3(nb(nnz)), dim3(256), 0, G->s, G->pv.vt, G->vtf, nnz);
    }
    RCHK(galloc(G.get(), &G->Xc, (size_t)n * kF));
    RCHK(galloc(G.get(), &G->Xr, (size_t)m * kF));
    float **fv[] = {&G->xref, &G->px, &G->tx, &G->dpx};
    for (auto p : fv) RCHK(galloc(G.get(), p, (size_t)n));
    float **fm[] = {&G->yref, &G->py, &G->ty, &G->dpy};
    for (auto p : fm) RCHK(galloc(G.get(), p, (size_t)m));
    G->INc.assign((size_t)layers + 1, nullptr);
    G->INr.assign((size_t)layers + 1, nullptr);
    for (int l = 1; l <= layers; ++l) {
        RCHK(galloc(G.get(), &G->INc[(size_t)l], (size_t)n * 2 * kH));
        RCHK(galloc(G.get(), &G->INr[(size_t)l], (size_t)m * 2 * kH));
    }
    RCHK(galloc(G.get(), &G->Hc_last, (size_t)n * kH));
    RCHK(galloc(G.get(), &G->Hr_last, (size_t)m * kH));
    RCHK(galloc(G.get(), &G->dHc, (size_t)n * kH));
    RCHK(galloc(G.get(), &G->dHr, (size_t)m * kH));
    RCHK(galloc(G.get(), &G->dINc, (size_t)n * 2 * kH));
    RCHK(galloc(G.get(), &G->dINr, (size_t)m * 2 * kH));
    RCHK(galloc(G.get(), &G->dZc, (size_t)n * kH));
    RCHK(galloc(G.get(), &G->dZr, (size_t)m * kH));
    RCHK(galloc(G.get(), &G->dZc_lo, (size_t)n * kH));
    RCHK(galloc(G.get(), &G->dZr_lo, (size_t)m * kH));
    const long nzmax = (std::max(n, m) + kKC - 1) / kKC;
    RCHK(galloc(G.get(), &G->wpart, (size_t)std::max<long>(nzmax * 2 * kH * kH, (n / 1024 + 2) * kH)));
    RCHK(galloc(G.get(), &G->lpart, (size_t)(nb(n) + nb(m))));
    RCHK(galloc(G.get(), &G->lsum, 2));
    double **dn[] = {&G->ref_c, &G->ref_x, &G->tmp_n, &G->tmp_n2};
    for (auto p : dn) RCHK(galloc(G.get(), p, (size_t)n));
    double **dm[] = {&G->ref_b, &G->ref_y, &G->tmp_m, &G->tmp_m2, &G->tmp_m3};
    for (auto p : dm) RCHK(galloc(G.get(), p, (size_t)m));
    GCHK(hipGetLastError());
    GCHK(hipStreamSynchronize(G->s));
    *out = G.release();
    return DPDLP_OK;
}

int dpdlp_gnn_destroy(dpdlp_gnn *G)
{
    if (!G) return DPDLP_OK;
    (void)hipStreamSynchronize(G->s);
    delete G;
    return DPDLP_OK;
}

int64_t dpdlp_gnn_num_params(dpdlp_gnn *G) { return G ? G->n_params : -1; }

int dpdlp_gnn_set_params(dpdlp_gnn *G, const float *params, int64_t count, void *stream)
{
    if (!G || !params || count != G->n_params) { set_error("bad arguments"); return DPDLP_E_INVALID_ARG; }
    G->s = (hipStream_t)stream;
    GCHK(hipMemcpyAsync(G->w, params, sizeof(float) * count, hipMemcpyHostToDevice, G->s));
    hipLaunchKernelGGL(k_f2bf, dim3(nb(count)), dim3(256), 0, G->s, G->w, G->wb, (long)count);
    GCHK(hipMemsetAsync(G->m1, 0, sizeof(float) * count, G->s));
    GCHK(hipMemsetAsync(G->m2, 0, sizeof(float) * count, G->s));
    G->adam_t = 0;
    GCHK(hipStreamSynchronize(G->s));
    return DPDLP_OK;
}

int dpdlp_gnn_get_params(dpdlp_gnn *G, float *params, float *grads, int64_t count, void *stream)
{
    if (!G || count != G->n_params) { set_error("bad arguments"); return DPDLP_E_INVALID_ARG; }
    G->s = (hipStream_t)stream;
    if (params) GCHK(hipMemcpyAsync(params, G->w, sizeof(float) * count, hipMemcpyDeviceToHost, G->s));
    if (grads) GCHK(hipMemcpyAsync(grads, G->g, sizeof(float) * count, hipMemcpyDeviceToHost, G->s));
    GCHK(hipStreamSynchronize(G->s));
    return DPDLP_OK;
}

int dpdlp_gnn_set_reference(dpdlp_gnn *G, const double *c_ref, const double *b_ref,
                            const double *x_ref, const double *y_ref, int32_t mem_kind, void *stream)
{
    if (!G || !c_ref || !b_ref || !x_ref || !y_ref) { set_error("NULL argument"); return DPDLP_E_INVALID_ARG; }
    if (!mem_kind_ok(mem_kind)) return bad_mem_kind();
    G->s = (hipStream_t)stream;
    const long m = G->pv.m, n = G->pv.n;
    const int k = mem_kind == DPDLP_MEM_HOST ? (int)hipMemcpyHostToDevice : (int)hipMemcpyDeviceToDevice;
    GCHK(hipMemcpyAsync(G->ref_c, c_ref, sizeof(double) * n, (hipMemcpyKind)k, G->s));
    GCHK(hipMemcpyAsync(G->ref_x, x_ref, sizeof(double) * n, (hipMemcpyKind)k, G->s));
    GCHK(hipMemcpyAsync(G->ref_b, b_ref, sizeof(double) * m, (hipMemcpyKind)k, G->s));
    GCHK(hipMemcpyAsync(G->ref_y, y_ref, sizeof(double) * m, (hipMemcpyKind)k, G->s));
    GCHK(hipStreamSynchronize(G->s));
    G->have_ref = true;
    return DPDLP_OK;
}

int dpdlp_gnn_set_instance(dpdlp_gnn *G, const double *c, const double *con_lo, const double *con_hi,
                           int32_t mem_kind, void *stream)
{
    if (!G || !c || !con_lo || !con_hi) { set_error("NULL argument"); return DPDLP_E_INVALID_ARG; }
    if (!mem_kind_ok(mem_kind)) return bad_mem_kind();
    if (!G->have_ref) { set_error("dpdlp_gnn_set_reference first"); return DPDLP_E_INVALID_ARG; }
    G->s = (hipStream_t)stream;
    const int m = G->pv.m, n = G->pv.n;
    const double *dc_, *dlo, *dhi;
    RCHK(to_dev(G, c, mem_kind, G->tmp_n, n, &dc_));
    RCHK(to_dev(G, con_lo, mem_kind, G->tmp_m, m, &dlo));
    RCHK(to_dev(G, con_hi, mem_kind, G->tmp_m2, m, &dhi));
    hipLaunchKernelGGL(k_feat_col, dim3(nb(n)), dim3(256), 0, G->s, n, G->pv.perm_col, G->pv.dc, dc_,
                       G->ref_c, G->ref_x, G->pv.vlo0, G->pv.vhi0, G->Xc, G->xref);
    hipLaunchKernelGGL(k_feat_row, dim3(nb(m)), dim3(256), 0, G->s, m, G->pv.perm_row, G->pv.dr, dlo,
                       dhi, G->ref_b, G->ref_y, G->Xr, G->yref);
    GCHK(hipGetLastError());
    GCHK(hipStreamSynchronize(G->s));
    G->have_inst = true;
    return DPDLP_OK;
}

int dpdlp_gnn_forward(dpdlp_gnn *G, double *x0, double *y0, int32_t mem_kind, void *stream)
{
    if (!G) { set_error("NULL argument"); return DPDLP_E_INVALID_ARG; }
    if (!mem_kind_ok(mem_kind)) return bad_mem_kind();
    if (!G->have_inst) { set_error("dpdlp_gnn_set_instance first"); return DPDLP_E_INVALID_ARG; }
    G->s = (hipStream_t)stream;
    const int m = G->pv.m, n = G->pv.n;
    forward(G);
    if (x0) {
        double *d = mem_kind == DPDLP_MEM_DEVICE ? x0 : G->tmp_n2;
        hipLaunchKernelGGL(k_unperm_scale, dim3(nb(n)), dim3(256), 0, G->s, n, G->px, G->pv.perm_col,
                           G->pv.dc, 1, d);
        if (mem_kind == DPDLP_MEM_HOST)
            GCHK(hipMemcpyAsync(x0, d, sizeof(double) * n, hipMemcpyDeviceToHost, G->s));
    }
    if (y0) {
        double *d = mem_kind == DPDLP_MEM_DEVICE ? y0 : G->tmp_m3;
        hipLaunchKernelGGL(k_unperm_scale, dim3(nb(m)), dim3(256), 0, G->s, m, G->py, G->pv.perm_row,
                           G->pv.dr, 1, d);
        if (mem_kind == DPDLP_MEM_HOST)
            GCHK(hipMemcpyAsync(y0, d, sizeof(double) * m, hipMemcpyDeviceToHost, G->s));
    }
    GCHK(hipGetLastError());
    GCHK(hipStreamSynchronize(G->s));
    return DPDLP_OK;
}

int dpdlp_gnn_backward(dpdlp_gnn *G, const double *x_target, const double *y_target, int32_t mem_kind,
                       double *loss2, void *stream)
{
    if (!G || !x_target || !y_target) { set_error("NULL argument"); return DPDLP_E_INVALID_ARG; }
    if (!mem_kind_ok(mem_kind)) return bad_mem_kind();
    if (!G->have_inst) { set_error("dpdlp_gnn_set_instance first"); return DPDLP_E_INVALID_ARG; }
    G->s = (hipStream_t)stream;
    const int m = G->pv.m, n = G->pv.n;
    const double *dx, *dy;
    RCHK(to_dev(G, x_target, mem_kind, G->tmp_n, n, &dx));
    RCHK(to_dev(G, y_target, mem_kind, G->tmp_m, m, &dy));
    hipLaunchKernelGGL(k_perm_scale, dim3(nb(n)), dim3(256), 0, G->s, n, dx, G->pv.perm_col, G->pv.dc, 0, G->tx);
    hipLaunchKernelGGL(k_perm_scale, dim3(nb(m)), dim3(256), 0, G->s, m, dy, G->pv.perm_row, G->pv.dr, 0, G->ty);
    forward(G);
    backward(G);
    double h[2];
    GCHK(hipMemcpyAsync(h, G->lsum, sizeof(h), hipMemcpyDeviceToHost, G->s));
    GCHK(hipGetLastError());
    GCHK(hipStreamSynchronize(G->s));
    if (loss2) { loss2[0] = h[0] / n; loss2[1] = h[1] / m; }
    return DPDLP_OK;
}

int dpdlp_gnn_adam_step(dpdlp_gnn *G, double lr, double beta1, double beta2, double eps, void *stream)
{
    if (!G) { set_error("NULL argument"); return DPDLP_E_INVALID_ARG; }
    G->s = (hipStream_t)stream;
    G->adam_t += 1;
    const float c1 = (float)(1.0 - std::pow(beta1, G->adam_t));
    const float c2 = (float)(1.0 - std::pow(beta2, G->adam_t));
    hipLaunchKernelGGL(k_adam, dim3(nb(G->n_params)), dim3(256), 0, G->s, G->n_params, G->w, G->g,
                       G->m1, G->m2, G->wb, (float)lr, (float)beta1, (float)beta2, (float)eps, c1, c2);
    GCHK(hipGetLastError());
    return DPDLP_OK;
}

int dpdlp_gnn_gemm_test(const uint16_t *A, long a_rs, long a_cs, const uint16_t *B, long b_rs,
                        long b_cs, float *C, long ldc, int32_t M, int32_t Nc, int32_t K, void *stream)
{
    if (!A || !B || !C || M < 1 || Nc < 1 || K < 1) { set_error("bad arguments"); return DPDLP_E_INVALID_ARG; }
    hipLaunchKernelGGL(k_gemm, dim3(nb(M, 64), nb(Nc, 64), 1), dim3(256), 0, (hipStream_t)stream, A, a_rs,
                       a_cs, B, b_rs, b_cs, (void *)C, ldc, 0L, M, Nc, K, K, 0);
    GCHK(hipGetLastError());
    GCHK(hipStreamSynchronize((hipStream_t)stream));
    return DPDLP_OK;
}

}  // extern "C"
