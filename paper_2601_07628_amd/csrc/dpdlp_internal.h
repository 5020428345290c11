// Internal declarations shared by the host preprocessing (dpdlp_host.cpp)
// and the device solver (dpdlp_solver.hip).
#pragma once
#include <cstdint>
#include <memory>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/dpdlp.h"

namespace dpdlp {

// Tile descriptor: 8 int32 (see dpdlp_build_tiles).
struct Tile {
    int32_t seg_begin, seg_end, nnz_begin, nnz_end;
    int32_t width_log2, piece, npieces, slice;   // slice: gather slice (sliced sets)
};

// Host arrays of matrix size: resize() leaves the elements uninitialised,
// so that the threads that fill them also take their first-touch page
// faults (a zero-filling resize of 40M elements costs about a second).
template <class T>
struct NoInitAlloc : std::allocator<T> {
    template <class U> struct rebind { using other = NoInitAlloc<U>; };
    NoInitAlloc() = default;
    template <class U> NoInitAlloc(const NoInitAlloc<U> &) {}
    template <class U, class... A> void construct(U *p, A &&...a)
    {
        if constexpr (sizeof...(A) == 0) ::new ((void *)p) U;
        else ::new ((void *)p) U(std::forward<A>(a)...);
    }
};
template <class T> using hvec = std::vector<T, NoInitAlloc<T>>;

// The XCD-sliced form of one format (gathered dimension cut into S slices
// of `size` indices) in compact layout: slice s keeps only the segments
// with a nonzero in its index range, numbered globally in slice-major order
// ("compact segments", seg_base[s] .. seg_base[s+1]); ptr has one entry per
// compact segment (+1) into idx/src, and src[q] is the position in the
// unsliced format that sliced nonzero q comes from.  mask holds, per
// original segment, one bit per slice in S/8 byte planes (plane-major);
// cbase[q * S + s] is the compact index of the first segment of slice s at
// or after original segment q * kBlock.  Tiles carry their slice.
struct SlicedHost {
    int32_t S = 0;
    std::vector<int32_t> bounds;     // slice s gathers indices [bounds[s], bounds[s+1])
    int64_t G = 0;
    hvec<int32_t> ptr, idx, src;
    std::vector<int32_t> seg_base, cbase;
    std::vector<uint8_t> mask;
    std::vector<Tile> tiles;
};
// Distinct 128-byte lines of the gathered vector (line_elems indices per
// line) that the tiles' wave instructions touch: each tile's nonzeros in
// groups of 64 consecutive positions (one wave's load of a tile kernel),
// counted in storage order, or (sorted = true) after ordering every tile's
// nonzeros by gathered index.
int64_t tile_gather_lines(const std::vector<Tile> &tiles, const hvec<int32_t> &idx,
                          int32_t line_elems, bool sorted);
// Orders every tile's nonzeros by gathered index (stable), permuting idx
// and src alike; pos[q] receives, for the nonzero now at q, its position
// inside its tile before the sort (the tile kernel stores its product
// there, so the segment sums keep their order).
void sort_tiles_by_gather(const std::vector<Tile> &tiles, hvec<int32_t> &idx,
                          hvec<int32_t> &src, hvec<uint16_t> &pos);

// Slices are S contiguous ranges of the gathered index that hold about
// nnz / S nonzeros each; gptr[nidx + 1] is the gathered dimension's own
// pointer array (its nonzero counts as prefix sums).
void slice_bounds(const hvec<int32_t> &gptr, int32_t nidx, int32_t S,
                  std::vector<int32_t> &bounds);
void slice_format(const hvec<int32_t> &ptr, const hvec<int32_t> &idx, const hvec<int32_t> &gptr,
                  int32_t nseg, int32_t nidx, int32_t S, int32_t tile_nnz, SlicedHost &out);
// Number of compact segments (segment, slice) with a nonzero, for S slices.
int64_t count_compact(const hvec<int32_t> &ptr, const hvec<int32_t> &idx,
                      const hvec<int32_t> &gptr, int32_t nseg, int32_t nidx, int32_t S);
// Bytes of the gathered vector (distinct 128-byte lines of line_elems
// indices) touched by `window` consecutive nonzeros in storage order: the
// median over nsample windows spread over the matrix.
double gather_window_bytes(const hvec<int32_t> &idx, int64_t nnz, int32_t nidx, int64_t window,
                           int32_t line_elems, int nsample);

constexpr int kBlock = 256;          // threads per workgroup (4 wave64)
#ifndef DPDLP_TILE_NNZ_MAX
#define DPDLP_TILE_NNZ_MAX 2048
#endif
#ifndef DPDLP_TILE_SEGS_MAX
#define DPDLP_TILE_SEGS_MAX 1024
#endif
constexpr int kTileNnzMax = DPDLP_TILE_NNZ_MAX;   // products staged in LDS per tile
constexpr int kMaxSegs = DPDLP_TILE_SEGS_MAX;     // segments per tile

void set_error(const std::string &msg);

// The two memory kinds of the C ABI.  Any other value is rejected before a
// pointer is touched (a host pointer read as device memory would fault).
inline bool mem_kind_ok(int32_t k) { return k == DPDLP_MEM_HOST || k == DPDLP_MEM_DEVICE; }
int bad_mem_kind();     // sets the message, returns DPDLP_E_INVALID_ARG

// Host copy of an LP after the block permutation, with both formats.
struct HostMatrix {
    int32_t m = 0, n = 0;
    int64_t nnz = 0;
    hvec<int32_t> rp, ci;             // CSR (permuted)
    hvec<double> v;
    hvec<int32_t> cp, ri;             // CSC (permuted), row order kept
    hvec<double> vt;
    std::vector<int32_t> perm_row, perm_col;   // perm[new] = old
};

// Read-only view of a prepared problem's device data (permuted order), for
// the warm-start network, which runs on the same bipartite graph.
struct ProblemView {
    int32_t m = 0, n = 0;
    int64_t nnz = 0;
    const int32_t *rp = nullptr, *ci = nullptr, *cp = nullptr, *ri = nullptr;
    const double *v = nullptr, *vt = nullptr;        // scaled A~ (CSR, CSC)
    const int32_t *perm_row = nullptr, *perm_col = nullptr;
    const double *dr = nullptr, *dc = nullptr;
    const double *vlo0 = nullptr, *vhi0 = nullptr;   // original variable bounds (permuted)
};
int problem_view(dpdlp_problem *P, ProblemView *out);

int validate_host(const dpdlp_csr_lp *lp);
// Start vector of the Golub-Kahan-Lanczos process: w[j] in [-1, 1) from a
// splitmix64 stream; returns ||w||_2.
double lanczos_start(int32_t n, uint64_t seed, double *w);
// Largest singular value of the k x k upper bidiagonal matrix with diagonal
// alpha[0..k-1] and superdiagonal beta[1..k-1] (beta[0] unused), from the
// largest eigenvalue of B^T B by Sturm-sequence bisection.
double bidiag_sigma_max(const double *alpha, const double *beta, int k);
void block_permutation(int32_t count, int32_t block, uint64_t seed, int32_t *perm);
void build_tiles(const int32_t *seg_ptr, int32_t nseg, int32_t tile_nnz,
                 std::vector<Tile> &out);
// Permute rows/columns of a host CSR LP and build the CSC copy.
void permute_and_transpose(const dpdlp_csr_lp *lp, int32_t block, uint64_t seed,
                           int32_t order, HostMatrix &H);

}  // namespace dpdlp
