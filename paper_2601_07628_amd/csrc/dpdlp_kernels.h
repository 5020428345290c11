// Device kernels of the single-GPU restarted reflected-Halpern PDHG solver,
// written for gfx950 (MI355X): wave64, 256-thread workgroups, LDS-staged
// nonzero tiles, deterministic reductions (no floating-point atomics).
//
// The tile framework: a matrix in CSR (segments = rows) or CSC (segments =
// columns) is cut on the host into tiles of at most kTileNnzMax nonzeros
// (nonzero-aware partitioning, Sec. 4.3 of the D-PDLP paper, applied to
// workgroups).  One workgroup owns one tile:
//   1. it streams the tile's (index, value) pairs once with coalesced
//      non-temporal loads, gathers the vector entry, and stages the products
//      in LDS;
//   2. groups of G = 2^width_log2 lanes (G chosen per tile from the mean
//      segment length) reduce one segment each from LDS with a fixed-order
//      strided sum and an xor-shuffle butterfly;
//   3. one thread per segment applies the fused epilogue (projection,
//      reflection, Halpern, or a residual contribution) with coalesced
//      vector loads and stores.
// Where the gathers of a tile hit the same cache lines out of order (rows of
// a transportation LP, whose columns are strided), the host may store each
// tile's nonzeros sorted by gathered index, so that one wave's lanes load
// neighbouring entries together; pos then gives every nonzero's position in
// the tile's segment order, where its product is stored in LDS, so the
// segment sums are unchanged.
// A segment longer than a tile is split into pieces; each piece's workgroup
// reduces its part and publishes it, and a small follow-up kernel adds the
// pieces in piece order and runs the epilogue.  The summation order is fixed
// by the tiling alone, so results are bitwise reproducible run to run.
//
// The XCD-sliced form (the paper's 2-D partition, Sec. 3.1 / App. D, across
// the 8 XCDs): the gathered dimension is cut into S slices, slice s runs on
// XCD s % 8 so its share of the gathered vector stays in that XCD's L2;
// PartialOp writes one sum per (segment, slice) pair that has nonzeros, and
// k_combine adds a segment's slice sums in slice order before the epilogue.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "dpdlp_internal.h"

namespace dpdlp {

template <typename T>
__device__ __forceinline__ T clampv(T v, T lo, T hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

template <typename T>
__device__ __forceinline__ T nt_load(const T *p)
{
    return __builtin_nontemporal_load(p);
}

struct SumOp {
    template <typename T> __device__ static T id() { return T(0); }
    template <typename T> __device__ static T comb(T a, T b) { return a + b; }
};
struct MaxOp {
    template <typename T> __device__ static T id() { return T(0); }
    template <typename T> __device__ static T comb(T a, T b) { return a > b ? a : b; }
};

// Tile index of this workgroup.  Workgroups are dispatched round-robin over
// the 8 XCDs (workgroup b runs on XCD b % 8); with remap on, XCD x processes a
// contiguous run of tiles so neighbouring segments share that XCD's L2.
__device__ __forceinline__ int tile_of_block(int remap)
{
    const int b = blockIdx.x;
    if (!remap) return b;
    const int per = gridDim.x >> 3;     // grid is a multiple of 8 when remapped
    return (b & 7) * per + (b >> 3);
}

// Butterfly over groups of G lanes (G a power of two <= 64).
template <class R, typename T>
__device__ __forceinline__ T group_reduce(T v, int G)
{
    for (int off = G >> 1; off > 0; off >>= 1) v = R::comb(v, __shfl_xor(v, off, 64));
    return v;
}

// Fixed-order workgroup reduction of NQ values; result valid in thread 0.
template <class R, int NQ, typename T>
__device__ __forceinline__ void block_reduce(T (&v)[NQ], T (*s_red)[kBlock / 64])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        T x = group_reduce<R>(v[q], 64);
        if (lane == 0) s_red[q][wave] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            T x = s_red[q][0];
            for (int w = 1; w < kBlock / 64; ++w) x = R::comb(x, s_red[q][w]);
            v[q] = x;
        }
    }
}

template <typename T>
__device__ __forceinline__ void nt_store(T *p, T v)
{
    __builtin_nontemporal_store(v, p);
}

// Generic tile kernel.  Op supplies:
//   MT  matrix value type, AT accumulation type, NR right-hand sides,
//   NQ  per-tile partial quantities (0 = none), R the reduction (Sum/Max),
//   Pre per-segment values loaded before the reduction (prefetch)
//   value(a, j, out[NR])          product for a nonzero a with index j
//   prefetch(seg, pre)            issue the epilogue's vector loads early
//   epilogue(seg, r[NR], pre, acc) per-segment update, adds to acc[NQ]
//   partials                      double* [NQ * ntiles] or null
// Memory-level parallelism: every thread first issues all of its index /
// value loads (kPer per thread), the segment-pointer loads and the epilogue
// prefetches, then all of its gathers, so one tile costs about two memory
// round trips before the LDS phases.
constexpr int kPer = kTileNnzMax / kBlock;     // nonzeros per thread per tile
constexpr int kPre = 2;                         // prefetched segments per thread

template <class Op>
__global__ __launch_bounds__(kBlock) void k_tile(Op op0, const Tile *__restrict__ tiles,
                                                 int ntiles, const int *__restrict__ blk2tile,
                                                 int seg_stride,
                                                 const int *__restrict__ seg_ptr,
                                                 const int *__restrict__ idx,
                                                 const typename Op::MT *__restrict__ val,
                                                 const uint16_t *__restrict__ pos,
                                                 typename Op::AT *__restrict__ carries,
                                                 int remap)
{
    using AT = typename Op::AT;
    using MT = typename Op::MT;
    using R = typename Op::R;
    constexpr int NR = Op::NR;
    constexpr int NQ = Op::NQ > 0 ? Op::NQ : 1;
    __shared__ AT s_prod[NR][kTileNnzMax];
    __shared__ AT s_seg[NR][kMaxSegs];
    __shared__ int s_ptr[kMaxSegs + 1];
    __shared__ double s_red[NQ][kBlock / 64];
    __shared__ AT s_redp[NR][kBlock / 64];

    Op op = op0;
    op.resolve();             // graph replays: its scalar loads go out with the tile's
    const int t = blk2tile ? blk2tile[blockIdx.x] : tile_of_block(remap);
    if (t < 0 || t >= ntiles) return;
    const Tile d = tiles[t];
    op.slice = d.slice;
    seg_ptr += (size_t)d.slice * seg_stride;
    const int nnz0 = d.nnz_begin;
    const int cnt = d.nnz_end - d.nnz_begin;
    const int nseg = d.seg_end - d.seg_begin;
    const bool whole = d.npieces == 0;

    // Every load of phase 1 is unconditional, from an index clamped into the
    // tile (lanes past its end repeat its last element and store nothing),
    // so that each group of loads issues back to back and is waited for
    // once; per-element branches would put a wait after every load.
    // 1a. issue the tile's matrix stream (coalesced, non-temporal)
    int jj[kPer];
    MT aa[kPer];
    int pp[kPer];             // where each product goes in LDS (gather-sorted tiles)
    if (cnt > 0) {
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int e = min((int)threadIdx.x + q * kBlock, cnt - 1);
            jj[q] = nt_load(idx + nnz0 + e);
            aa[q] = nt_load(val + nnz0 + e);
        }
        if (pos) {
#pragma unroll
            for (int q = 0; q < kPer; ++q)
                pp[q] = nt_load(pos + nnz0 + min((int)threadIdx.x + q * kBlock, cnt - 1));
        } else {
#pragma unroll
            for (int q = 0; q < kPer; ++q) pp[q] = threadIdx.x + q * kBlock;
        }
    }
    // 1b. segment pointers to LDS and the epilogue's vector loads
    typename Op::Pre pre[kPre];
    if (whole) {
        constexpr int kPtrIt = (kMaxSegs + kBlock) / kBlock;   // covers nseg + 1 <= kMaxSegs + 1
        int sp[kPtrIt];
#pragma unroll
        for (int i = 0; i < kPtrIt; ++i)
            sp[i] = seg_ptr[d.seg_begin + min((int)threadIdx.x + i * kBlock, nseg)];
#pragma unroll
        for (int q = 0; q < kPre; ++q)
            op.prefetch(d.seg_begin + min((int)threadIdx.x + q * kBlock, nseg - 1), pre[q]);
#pragma unroll
        for (int i = 0; i < kPtrIt; ++i) {
            const int s = threadIdx.x + i * kBlock;
            if (s <= nseg) s_ptr[s] = sp[i] - nnz0;
        }
    }
    // 1c. gathers (all issued before the first product is stored), products to LDS
    if (cnt > 0) {
        AT pv[kPer][NR];
#pragma unroll
        for (int q = 0; q < kPer; ++q) op.value(aa[q], jj[q], pv[q]);
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int e = threadIdx.x + q * kBlock;
            if (e < cnt) {
#pragma unroll
                for (int r = 0; r < NR; ++r) s_prod[r][pp[q]] = pv[q][r];
            }
        }
    }
    __syncthreads();

    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0;

    if (whole) {
        // 2. segment reductions by groups of G lanes
        const int G = 1 << d.width_log2;
        const int lane = threadIdx.x & (G - 1);
        const int ngrp = kBlock >> d.width_log2;
        for (int s = threadIdx.x >> d.width_log2; s < nseg; s += ngrp) {
            const int b = s_ptr[s], e = s_ptr[s + 1];
            AT r[NR];
#pragma unroll
            for (int q = 0; q < NR; ++q) r[q] = R::template id<AT>();
            for (int p = b + lane; p < e; p += G) {
#pragma unroll
                for (int q = 0; q < NR; ++q) r[q] = R::comb(r[q], s_prod[q][p]);
            }
#pragma unroll
            for (int q = 0; q < NR; ++q) r[q] = group_reduce<R>(r[q], G);
            if (lane == 0) {
#pragma unroll
                for (int q = 0; q < NR; ++q) s_seg[q][s] = r[q];
            }
        }
        __syncthreads();
        // 3. fused epilogue, one thread per segment (coalesced vector I/O)
#pragma unroll
        for (int q = 0; q < kPre; ++q) {
            const int s = threadIdx.x + q * kBlock;
            if (s < nseg) {
                AT r[NR];
#pragma unroll
                for (int z = 0; z < NR; ++z) r[z] = s_seg[z][s];
                op.epilogue(d.seg_begin + s, r, pre[q], acc);
            }
        }
        for (int s = threadIdx.x + kPre * kBlock; s < nseg; s += kBlock) {
            AT r[NR];
#pragma unroll
            for (int z = 0; z < NR; ++z) r[z] = s_seg[z][s];
            typename Op::Pre p1;
            op.prefetch(d.seg_begin + s, p1);
            op.epilogue(d.seg_begin + s, r, p1, acc);
        }
        if (Op::NQ > 0) {
            block_reduce<SumOp, NQ>(acc, s_red);
            if (threadIdx.x == 0)
                for (int q = 0; q < Op::NQ; ++q) op.partials[(size_t)q * ntiles + t] = acc[q];
        }
        return;
    }

    // Split segment: reduce this piece and publish it; k_split_fix adds the
    // pieces in piece order after this launch (no in-kernel cross-workgroup
    // communication, so no L2-wide fences).
    AT pr[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) pr[q] = R::template id<AT>();
    for (int e = threadIdx.x; e < cnt; e += kBlock) {
#pragma unroll
        for (int q = 0; q < NR; ++q) pr[q] = R::comb(pr[q], s_prod[q][e]);
    }
    block_reduce<R, NR>(pr, s_redp);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NR; ++q) carries[(size_t)q * ntiles + t] = pr[q];
    }
}

// A segment split over npieces consecutive tiles starting at tile t0.
struct SplitSeg {
    int32_t seg, t0, npieces, slice;
};

// Finish split segments: one thread per split segment sums its pieces'
// carries in piece order and runs the epilogue; the segment's partial-sum
// contribution goes to the slot of its first piece (the other pieces' slots
// get zero), so every slot is written exactly once per pass.
template <class Op>
__global__ __launch_bounds__(64) void k_split_fix(Op op0, const SplitSeg *__restrict__ splits,
                                                   int nsplit, int ntiles,
                                                   const typename Op::AT *__restrict__ carries)
{
    using AT = typename Op::AT;
    using R = typename Op::R;
    constexpr int NR = Op::NR;
    constexpr int NQ = Op::NQ > 0 ? Op::NQ : 1;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nsplit) return;
    const SplitSeg sg = splits[i];
    Op op = op0;
    op.slice = sg.slice;
    op.resolve();
    AT r[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        r[q] = R::template id<AT>();
        for (int pc = 0; pc < sg.npieces; ++pc)
            r[q] = R::comb(r[q], carries[(size_t)q * ntiles + sg.t0 + pc]);
    }
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
    typename Op::Pre p1;
    op.prefetch(sg.seg, p1);
    op.epilogue(sg.seg, r, p1, acc);
    if (Op::NQ > 0)
        for (int pc = 0; pc < sg.npieces; ++pc)
            for (int q = 0; q < Op::NQ; ++q)
                op.partials[(size_t)q * ntiles + sg.t0 + pc] = pc == 0 ? acc[q] : 0.0;
}

struct NoPre {};

// Iteration scalars read from device memory by graph-replayed launches:
// the primal / dual step size and the Halpern index of the run's first
// iteration (the launch adds its offset j inside the run).
struct IterDev {
    double tau, sigma;
    long long k0;
};

// ---------------------------------------------------------------------------
// Fused PDHG steps (Sec. 2.2 / Algorithm 1 steps 1-2, with the reflected
// Halpern update of App. A fused in).  T is double (FP64) or float (FP32).

// Primal step over CSC tiles, one segment per column j:
//   g = c~_j - (A~^T y)_j ; xh = clamp(x_j - tau g, l_j, u_j) ; xbar = 2 xh - x_j
//   x_j <- a ((1+gamma) xh - gamma x_j) + b xa_j,  a = (k+1)/(k+2), b = 1/(k+2)
template <typename T>
struct PrimalOp {
    using MT = T; using AT = T; using R = SumOp;
    static constexpr int NR = 1, NQ = 0;
    int slice = 0;
    __device__ void resolve()
    {
        if (!dev) return;
        const double kk = (double)(dev->k0 + j);
        tau = (T)dev->tau;
        a = (T)((kk + 1.0) / (kk + 2.0));
        b = (T)(1.0 / (kk + 2.0));
    }
    const T *__restrict__ y;
    const T *__restrict__ c;
    const T *__restrict__ lo;
    const T *__restrict__ hi;
    const T *__restrict__ xa;
    T *__restrict__ x;
    T *__restrict__ xbar;
    double *__restrict__ xh;      // written when write_hat
    double *__restrict__ dx;      // x_j - xh_j, written when write_hat
    double *partials;
    T tau, a, b, gamma;
    int write_hat;
    const IterDev *dev = nullptr;   // graph replays: tau and k from here
    int j = 0;
    struct Pre { T x, c, lo, hi, xa; };
    __device__ void value(MT v, int j, AT *out) const { out[0] = v * y[j]; }
    __device__ void prefetch(int j, Pre &p) const
    {
        p.x = nt_load(x + j); p.c = nt_load(c + j); p.lo = nt_load(lo + j);
        p.hi = nt_load(hi + j); p.xa = nt_load(xa + j);
    }
    __device__ void epilogue(int j, const AT *r, const Pre &p, double *) const
    {
        const T g = p.c - r[0];
        const T xk = p.x;
        const T xhv = clampv(xk - tau * g, p.lo, p.hi);
        xbar[j] = T(2) * xhv - xk;
        nt_store(x + j, a * ((T(1) + gamma) * xhv - gamma * xk) + b * p.xa);
        if (write_hat) {
            xh[j] = (double)xhv;
            dx[j] = (double)xk - (double)xhv;
        }
    }
};

// Primal step of a QP with diagonal Q (Sec. 6) over CSC tiles: the step
// minimises q x^2 / 2 + g x + (x - x_j)^2 / (2 tau) over the box, separately
// per column, so xh = clamp((x_j - tau g) / (1 + tau q_j), l_j, u_j) (a
// convex one-dimensional quadratic); the rest is the LP step.  q is the
// scaled diagonal D_c Q D_c.  A type of its own, so the LP step's kernel
// arguments and code stay as they are.
template <typename T>
struct PrimalQPOp : PrimalOp<T> {
    using Base = PrimalOp<T>;
    const T *__restrict__ q;
    struct Pre { T x, c, lo, hi, xa, q; };
    __device__ void prefetch(int j, Pre &p) const
    {
        p.x = nt_load(this->x + j); p.c = nt_load(this->c + j); p.lo = nt_load(this->lo + j);
        p.hi = nt_load(this->hi + j); p.xa = nt_load(this->xa + j); p.q = nt_load(q + j);
    }
    __device__ void epilogue(int j, const T *r, const Pre &p, double *) const
    {
        const T g = p.c - r[0];
        const T xk = p.x;
        const T tau = this->tau;
        const T xhv = clampv((xk - tau * g) / (T(1) + tau * p.q), p.lo, p.hi);
        this->xbar[j] = T(2) * xhv - xk;
        nt_store(this->x + j, this->a * ((T(1) + this->gamma) * xhv - this->gamma * xk) + this->b * p.xa);
        if (this->write_hat) {
            this->xh[j] = (double)xhv;
            this->dx[j] = (double)xk - (double)xhv;
        }
    }
};

// Dual step over CSR tiles, one segment per row i:
//   q = (A~ xbar)_i ; w = y_i / sigma - q ; yh = sigma (w - clamp(w, -u_i, -l_i))
//   y_i <- a ((1+gamma) yh - gamma y_i) + b ya_i
template <typename T>
struct DualOp {
    using MT = T; using AT = T; using R = SumOp;
    static constexpr int NR = 1, NQ = 0;
    int slice = 0;
    __device__ void resolve()
    {
        if (!dev) return;
        const double kk = (double)(dev->k0 + j);
        sigma = (T)dev->sigma;
        a = (T)((kk + 1.0) / (kk + 2.0));
        b = (T)(1.0 / (kk + 2.0));
    }
    const T *__restrict__ xbar;
    const T *__restrict__ lo;
    const T *__restrict__ hi;
    const T *__restrict__ ya;
    T *__restrict__ y;
    double *__restrict__ yh;
    double *__restrict__ dy;
    double *partials;
    T sigma, a, b, gamma;
    int write_hat;
    const IterDev *dev = nullptr;
    int j = 0;
    struct Pre { T y, lo, hi, ya; };
    __device__ void value(MT v, int j, AT *out) const { out[0] = v * xbar[j]; }
    __device__ void prefetch(int i, Pre &p) const
    {
        p.y = y[i]; p.lo = nt_load(lo + i); p.hi = nt_load(hi + i); p.ya = nt_load(ya + i);
    }
    __device__ void epilogue(int i, const AT *r, const Pre &p, double *) const
    {
        const T yk = p.y;
        const T w = yk / sigma - r[0];
        const T yhv = sigma * (w - clampv(w, -p.hi, -p.lo));
        y[i] = a * ((T(1) + gamma) * yhv - gamma * yk) + b * p.ya;
        if (write_hat) {
            yh[i] = (double)yhv;
            dy[i] = (double)yk - (double)yhv;
        }
    }
};

// Per-slice segment sums for the XCD-sliced form of the fused steps:
//   partial[slice * nseg + seg] = sum over the slice's nonzeros of a * v[idx]
template <typename T>
struct PartialOp {
    using MT = T; using AT = T; using R = SumOp;
    static constexpr int NR = 1, NQ = 0;
    int slice = 0;
    __device__ void resolve() {}
    const T *__restrict__ v;
    T *__restrict__ partial;        // one value per compact segment
    double *partials;
    using Pre = NoPre;
    __device__ void value(MT a, int j, AT *o) const { o[0] = a * v[j]; }
    __device__ void prefetch(int, Pre &) const {}
    __device__ void epilogue(int g, const AT *r, const Pre &, double *) const
    {
        partial[g] = r[0];
    }
};

// Per-slice segment sums of two right-hand sides (the sliced CSR check
// pass: A~ xh and A~ dx); the second one is stored G entries after the first.
struct PartialOp2 {
    using MT = double; using AT = double; using R = SumOp;
    static constexpr int NR = 2, NQ = 0;
    int slice = 0;
    __device__ void resolve() {}
    const double *__restrict__ v;
    const double *__restrict__ v2;
    double *__restrict__ partial;
    int64_t G;
    double *partials;
    using Pre = NoPre;
    __device__ void value(MT a, int j, AT *o) const
    {
        o[0] = a * v[j];
        o[1] = a * v2[j];
    }
    __device__ void prefetch(int, Pre &) const {}
    __device__ void epilogue(int g, const AT *r, const Pre &, double *) const
    {
        partial[g] = r[0];
        partial[G + g] = r[1];
    }
};

// Adds the slice partials of each segment in slice order and runs a fused
// epilogue (PrimalOp / DualOp, or a check pass) on the sums; one thread per
// segment.  The partials are compact (only the slices where the segment has
// nonzeros): the position of segment j's partial in slice s is
// cbase[block * S + s] plus the number of segments of this block before j
// that have slice s, counted with wave ballots over the mask bits.  With
// Op::NR = 2 the second right-hand side's partials start G entries later.
// Ops with NQ > 0 (check passes) leave per-block partial sums in
// op.partials[q * gridDim.x + block].
template <class Op>
__global__ __launch_bounds__(kBlock) void k_combine(Op op0, int nseg, int S,
                                                    const typename Op::AT *__restrict__ partial,
                                                    const uint8_t *__restrict__ mask,
                                                    const int *__restrict__ cbase, int64_t G)
{
    using AT = typename Op::AT;
    constexpr int NR = Op::NR;
    constexpr int NQ = Op::NQ > 0 ? Op::NQ : 1;
    __shared__ int s_cnt[8][kBlock / 64];
    __shared__ double s_red[NQ][kBlock / 64];
    const int j = blockIdx.x * kBlock + threadIdx.x;
    const bool in = j < nseg;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    Op op = op0;
    op.resolve();
    typename Op::Pre p;
    if (in) op.prefetch(j, p);
    AT r[NR];
#pragma unroll
    for (int z = 0; z < NR; ++z) r[z] = SumOp::template id<AT>();
    const int *cb = cbase + (size_t)blockIdx.x * S;
    for (int pl = 0; pl < S / 8; ++pl) {
        const unsigned mb = in ? (unsigned)mask[(size_t)pl * nseg + j] : 0u;
        unsigned long long bal[8];
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            bal[b] = __ballot((mb >> b) & 1u);
            if (lane == 0) s_cnt[b][wave] = __popcll(bal[b]);
        }
        __syncthreads();
        // positions of all 8 slices first, then all loads (absent slices
        // load partial[0], always allocated, and add nothing), then the sums
        // in slice order
        int off[8];
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            int o = cb[pl * 8 + b] + __popcll(bal[b] & below);
            for (int w = 0; w < wave; ++w) o += s_cnt[b][w];
            off[b] = ((mb >> b) & 1u) ? o : 0;
        }
        AT pv[8][NR];
#pragma unroll
        for (int b = 0; b < 8; ++b)
#pragma unroll
            for (int z = 0; z < NR; ++z) pv[b][z] = partial[(size_t)z * G + off[b]];
#pragma unroll
        for (int b = 0; b < 8; ++b)
            if ((mb >> b) & 1u)
#pragma unroll
                for (int z = 0; z < NR; ++z) r[z] += pv[b][z];
        __syncthreads();
    }
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
    if (in) op.epilogue(j, r, p, acc);
    if (Op::NQ > 0) {
        block_reduce<SumOp, NQ>(acc, s_red);
        if (threadIdx.x == 0)
            for (int q = 0; q < Op::NQ; ++q) op.partials[(size_t)q * gridDim.x + blockIdx.x] = acc[q];
    }
}

// ---------------------------------------------------------------------------
// Check passes (App. B.4 KKT; App. B.2 / D.2.1 fixed-point residual; App. B.3
// distances to the anchor), FP64 on the FP64 matrix.  TA: anchor type.

// CSR pass with two right-hand sides (xh, dx).  Per-tile partial sums:
//   0 sum r_i^2, r = (A x) - proj_S(A x) in the original space
//   1 sum (l_i y_i^+ - u_i y_i^-)          (= -p(-y), original space)
//   2 sum dy_i^2
//   3 sum (A~ dx)_i dy_i                    (the <A dx, dy> coupling term)
//   4 sum (yh_i - ya_i)^2
template <typename TA>
struct CheckRowOp {
    using MT = double; using AT = double; using R = SumOp;
    static constexpr int NR = 2, NQ = 5;
    int slice = 0;
    __device__ void resolve() {}
    const double *__restrict__ xh;
    const double *__restrict__ dx;
    const double *__restrict__ yh;
    const double *__restrict__ dy;
    const TA *__restrict__ ya;
    const double *__restrict__ dr;
    const double *__restrict__ lo0;
    const double *__restrict__ hi0;
    double *partials;
    __device__ void value(MT v, int j, AT *out) const
    {
        out[0] = v * xh[j];
        out[1] = v * dx[j];
    }
    using Pre = NoPre;
    __device__ void prefetch(int, Pre &) const {}
    __device__ void epilogue(int i, const AT *r, const Pre &, double *acc) const
    {
        const double axi = r[0] / dr[i];
        const double res = axi - clampv(axi, lo0[i], hi0[i]);
        acc[0] += res * res;
        const double yi = dr[i] * yh[i];
        if (yi > 0.0) acc[1] += lo0[i] * yi;
        else if (yi < 0.0) acc[1] += hi0[i] * yi;
        const double dyi = dy[i];
        acc[2] += dyi * dyi;
        acc[3] += r[1] * dyi;
        const double an = yh[i] - (double)ya[i];
        acc[4] += an * an;
    }
};

// CSC pass (yh).  Per-tile partial sums:
//   0 sum ((g - s)_j / dc_j)^2, g = c~ - A~^T yh, s from the primal step with tau
//   1 sum c_j x_j   (original space)
//   2 sum s_j x_j   (original space)
//   3 sum dx_j^2
//   4 sum (xh_j - xa_j)^2
template <typename TA>
struct CheckColOp {
    using MT = double; using AT = double; using R = SumOp;
    static constexpr int NR = 1, NQ = 5;
    int slice = 0;
    __device__ void resolve() {}
    const double *__restrict__ yh;
    const double *__restrict__ xh;
    const double *__restrict__ dx;
    const TA *__restrict__ xa;
    const double *__restrict__ c;     // scaled
    const double *__restrict__ c0;    // original
    const double *__restrict__ lo;    // scaled variable bounds
    const double *__restrict__ hi;
    const double *__restrict__ dc;
    const double *__restrict__ q;     // scaled diagonal of Q, or null (an LP)
    double *partials;
    double tau;
    __device__ void value(MT v, int i, AT *out) const { out[0] = v * yh[i]; }
    using Pre = NoPre;
    __device__ void prefetch(int, Pre &) const {}
    __device__ void epilogue(int j, const AT *r, const Pre &, double *acc) const
    {
        // a QP (Sec. 6) adds Q x to the gradient, x^T Q x / 2 to the primal
        // objective and takes it off the dual one; q~ x~ = D_c (Q x) and
        // q~ x~^2 = x^T Q x per column
        const double qx = q ? q[j] * xh[j] : 0.0;
        const double g = c[j] + qx - r[0];
        const double u = xh[j] - tau * g;
        const double s = (clampv(u, lo[j], hi[j]) - u) / tau;
        const double dres = (g - s) / dc[j];
        acc[0] += dres * dres;
        const double xj = dc[j] * xh[j];
        const double half_xqx = 0.5 * qx * xh[j];
        acc[1] += c0[j] * xj + half_xqx;
        acc[2] += (s / dc[j]) * xj - half_xqx;
        const double dxj = dx[j];
        acc[3] += dxj * dxj;
        const double an = xh[j] - (double)xa[j];
        acc[4] += an * an;
    }
};

// Plain product with an optional divisor read from device memory:
//   out_s = sum_p a_p * (in[idx_p] / *div); partial 0 = sum out_s^2.
struct SpmvOp {
    using MT = double; using AT = double; using R = SumOp;
    static constexpr int NR = 1, NQ = 1;
    int slice = 0;
    __device__ void resolve() {}
    const double *__restrict__ in;
    const double *__restrict__ div;   // may be null
    double *__restrict__ out;
    double *partials;
    __device__ void value(MT v, int j, AT *o) const
    {
        o[0] = div ? v * (in[j] / *div) : v * in[j];
    }
    using Pre = NoPre;
    __device__ void prefetch(int, Pre &) const {}
    __device__ void epilogue(int s, const AT *r, const Pre &, double *acc) const
    {
        out[s] = r[0];
        acc[0] += r[0] * r[0];
    }
};

// One half-step of the Golub-Kahan-Lanczos bidiagonalization, with the
// normalisations deferred to the scalars: out <- (A in) / nin - (nin / nprev)
// out (first: no second term); per-tile partials of sum out^2.
struct LanczosOp {
    using MT = double; using AT = double; using R = SumOp;
    static constexpr int NR = 1, NQ = 1;
    int slice = 0;
    __device__ void resolve() {}
    const double *__restrict__ in;
    double *__restrict__ out;
    const double *nin;              // ||in|| (device scalar)
    const double *nprev;            // norm of the previous out (device scalar)
    int first;
    double *partials;
    __device__ void value(MT v, int j, AT *o) const { o[0] = v * in[j]; }
    struct Pre { double o; };
    __device__ void prefetch(int s, Pre &p) const { p.o = first ? 0.0 : out[s]; }
    __device__ void epilogue(int s, const AT *r, const Pre &p, double *acc) const
    {
        const double a = *nin;
        double v = r[0] / a;
        if (!first) v -= (a / *nprev) * p.o;
        out[s] = v;
        acc[0] += v * v;
    }
};

// Rescaling reductions: Ruiz (max |a|) and Pock-Chambolle (sum |a|^p);
// epilogue writes the factor 1/sqrt(.) (1 for an empty / zero segment).
struct AbsMaxOp {
    using MT = double; using AT = double; using R = MaxOp;
    static constexpr int NR = 1, NQ = 0;
    int slice = 0;
    __device__ void resolve() {}
    double *__restrict__ f;
    double *partials;
    __device__ void value(MT v, int, AT *o) const { o[0] = fabs(v); }
    using Pre = NoPre;
    __device__ void prefetch(int, Pre &) const {}
    __device__ void epilogue(int s, const AT *r, const Pre &, double *) const
    {
        f[s] = r[0] > 0.0 ? 1.0 / sqrt(r[0]) : 1.0;
    }
};
struct AbsPowSumOp {
    using MT = double; using AT = double; using R = SumOp;
    static constexpr int NR = 1, NQ = 0;
    int slice = 0;
    __device__ void resolve() {}
    double *__restrict__ f;
    double *partials;
    double p;
    __device__ void value(MT v, int, AT *o) const { o[0] = p == 1.0 ? fabs(v) : pow(fabs(v), p); }
    using Pre = NoPre;
    __device__ void prefetch(int, Pre &) const {}
    __device__ void epilogue(int s, const AT *r, const Pre &, double *) const
    {
        f[s] = r[0] > 0.0 ? 1.0 / sqrt(r[0]) : 1.0;
    }
};

}  // namespace dpdlp
