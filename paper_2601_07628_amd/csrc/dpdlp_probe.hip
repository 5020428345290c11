// Random-gather rate probe (dpdlp_time_gather in dpdlp.h): the ceiling
// against which the gathers of the XCD-sliced fused steps are measured.
//
// Each workgroup gathers kProbeTile entries of v, as one tile of the sliced
// steps does: kProbeBlock threads, kProbePer indices each, loaded
// non-temporally and coalesced, then the kProbePer gathers, summed and
// written once per thread (so the stores are negligible).  The indices are
// uniform random inside one slice of v: v is cut into S equal slices, slice
// s is gathered by workgroups on XCD s % 8 (workgroup b runs on XCD b % 8),
// and the slices of one XCD come one after another, the placement of the
// sliced steps.  What is left is the cost of the gathers themselves: one
// L2 request per lane unless lanes share a line, hits in the XCD's L2 when
// its slice fits there.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <string>

#include "dpdlp_internal.h"

namespace {

constexpr int kProbeBlock = 256;
constexpr int kProbePer = 8;
constexpr int kProbeTile = kProbeBlock * kProbePer;

// splitmix64 output function (Steele, Lea and Flood, 2014)
__device__ __forceinline__ uint64_t probe_mix(uint64_t z)
{
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Index e belongs to workgroup b = e / kProbeTile; its slice is that
// workgroup's XCD plus 8 times its position among the XCD's workgroups.
__global__ void k_probe_indices(int *__restrict__ idx, int64_t n_g, int64_t n_vec, int S,
                                int64_t nb, uint64_t seed)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_g) return;
    const int64_t b = e / kProbeTile;
    const int64_t per_xcd = (nb + 7) / 8;
    const int64_t round = (b / 8) * (S / 8) / per_xcd;
    const int s = (int)(b % 8) + 8 * (int)round;
    const int64_t lo = n_vec * s / S, hi = n_vec * (s + 1) / S;
    const uint64_t r = probe_mix(seed + (uint64_t)e);
    idx[e] = (int)(lo + (int64_t)(r % (uint64_t)(hi - lo)));
}

template <typename T>
__global__ void k_probe_fill(T *__restrict__ v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = T(1) + T(0.125) * T(i & 7);
}

template <typename T>
__global__ __launch_bounds__(kProbeBlock) void k_probe_gather(const int *__restrict__ idx,
                                                              const T *__restrict__ v, int64_t n_g,
                                                              T *__restrict__ out)
{
    const int64_t base = (int64_t)blockIdx.x * kProbeTile;
    int jj[kProbePer];
#pragma unroll
    for (int q = 0; q < kProbePer; ++q) {
        const int64_t e = base + threadIdx.x + (int64_t)q * kProbeBlock;
        jj[q] = __builtin_nontemporal_load(idx + (e < n_g ? e : n_g - 1));
    }
    T acc = T(0);
#pragma unroll
    for (int q = 0; q < kProbePer; ++q) acc += v[jj[q]];
    out[(int64_t)blockIdx.x * kProbeBlock + threadIdx.x] = acc;
}

struct ProbeBuffers {
    void *v = nullptr, *out = nullptr;
    int *idx = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~ProbeBuffers()
    {
        if (v) (void)hipFree(v);
        if (out) (void)hipFree(out);
        if (idx) (void)hipFree(idx);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

int probe_hip(hipError_t e, const char *what)
{
    dpdlp::set_error(std::string(what) + ": " + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? DPDLP_E_OOM : DPDLP_E_HIP;
}

#define PROBE_HIP(call, what)                               \
    do {                                                    \
        hipError_t pe_ = (call);                            \
        if (pe_ != hipSuccess) return probe_hip(pe_, what); \
    } while (0)

template <typename T>
int time_gather(int64_t n_vec, int S, int64_t n_gathers, int reps, uint64_t seed, hipStream_t s,
                double *avg_ms, double *gathers_per_s)
{
    const int64_t nb = (n_gathers + kProbeTile - 1) / kProbeTile;
    ProbeBuffers B;
    PROBE_HIP(hipMalloc(&B.v, sizeof(T) * (size_t)n_vec), "hipMalloc");
    PROBE_HIP(hipMalloc(&B.out, sizeof(T) * (size_t)nb * kProbeBlock), "hipMalloc");
    PROBE_HIP(hipMalloc(&B.idx, sizeof(int) * (size_t)n_gathers), "hipMalloc");
    PROBE_HIP(hipEventCreate(&B.e0), "hipEventCreate");
    PROBE_HIP(hipEventCreate(&B.e1), "hipEventCreate");
    hipLaunchKernelGGL(k_probe_fill<T>, dim3((unsigned)((n_vec + 255) / 256)), dim3(256), 0, s,
                       (T *)B.v, n_vec);
    hipLaunchKernelGGL(k_probe_indices, dim3((unsigned)((n_gathers + 255) / 256)), dim3(256), 0, s,
                       B.idx, n_gathers, n_vec, S, nb, seed);
    // one launch to warm the caches and the code object, then the timed ones
    hipLaunchKernelGGL(k_probe_gather<T>, dim3((unsigned)nb), dim3(kProbeBlock), 0, s,
                       (const int *)B.idx, (const T *)B.v, n_gathers, (T *)B.out);
    PROBE_HIP(hipEventRecord(B.e0, s), "hipEventRecord");
    for (int r = 0; r < reps; ++r)
        hipLaunchKernelGGL(k_probe_gather<T>, dim3((unsigned)nb), dim3(kProbeBlock), 0, s,
                           (const int *)B.idx, (const T *)B.v, n_gathers, (T *)B.out);
    PROBE_HIP(hipEventRecord(B.e1, s), "hipEventRecord");
    PROBE_HIP(hipGetLastError(), "kernel launch");
    PROBE_HIP(hipEventSynchronize(B.e1), "hipEventSynchronize");
    float ms = 0.0f;
    PROBE_HIP(hipEventElapsedTime(&ms, B.e0, B.e1), "hipEventElapsedTime");
    *avg_ms = (double)ms / reps;
    if (gathers_per_s) *gathers_per_s = (double)n_gathers / (*avg_ms * 1e-3);
    return DPDLP_OK;
}

}  // namespace

extern "C" int dpdlp_time_gather(int64_t n_vec, int32_t slices, int64_t n_gathers,
                                 int32_t precision, int32_t reps, uint64_t seed, void *stream,
                                 double *avg_ms, double *gathers_per_s)
{
    if (!avg_ms || reps < 1 || slices < 8 || slices > 64 || slices % 8 != 0 ||
        n_vec < slices || n_vec > INT32_MAX || n_gathers < 1 || n_gathers > INT32_MAX ||
        (precision != DPDLP_FP64 && precision != DPDLP_FP32_MIXED)) {
        dpdlp::set_error("dpdlp_time_gather: bad arguments (n_vec in [slices, 2^31 - 1], slices a "
                         "multiple of 8 up to 64, n_gathers in [1, 2^31 - 1], reps >= 1, "
                         "precision FP64 or FP32_MIXED, avg_ms not NULL)");
        return DPDLP_E_INVALID_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    if (precision == DPDLP_FP64)
        return time_gather<double>(n_vec, slices, n_gathers, reps, seed, s, avg_ms, gathers_per_s);
    return time_gather<float>(n_vec, slices, n_gathers, reps, seed, s, avg_ms, gathers_per_s);
}
