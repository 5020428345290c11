// Host check of the compact XCD-sliced format (slice_format, count_compact)
// and of the combine kernel's partial-sum indexing, on random segmented
// matrices with empty, short and very long segments:
//   * the compact segment count equals count_compact;
//   * every compact segment is covered by exactly one tile (or one first
//     piece of a split), tiles stay inside their slice's compact range and
//     their nonzero range matches the pointers;
//   * every sliced nonzero lies in its slice's index range and src points
//     back to the same index in the unsliced format;
//   * the slice ranges tile [0, nidx) and hold equal nonzero counts up to
//     one index's count (slice_bounds);
//   * gather_window_bytes equals a brute-force count of distinct lines on
//     single windows;
//   * the combine's position rule (cbase of the 256-segment block plus the
//     count of earlier segments of the block with that slice bit) stays in
//     range and adds up to the unsliced segment sum;
//   * gather-sorted tiles (sort_tiles_by_gather): per tile a permutation
//     that sends every product back to its unsorted position, ascending
//     indices, and no more touched lines than the storage order
//     (tile_gather_lines).
// Built with g++ (AddressSanitizer, UBSan) by tests/test_host_cpu.py.
#include "dpdlp_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <random>

using namespace dpdlp;

int main()
{
    std::mt19937_64 rng(1);
    int bad = 0;
    for (int trial = 0; trial < 60; ++trial) {
        // the first trials are tiny (fewer indices than slices: empty slices)
        const int nseg = trial < 10 ? 1 + trial % 3 : 1 + (int)(rng() % 3000);
        const int nidx = trial < 10 ? 1 + trial % 5 : 1 + (int)(rng() % 5000);
        const int S = 8 * (1 + (int)(rng() % 3));
        hvec<int32_t> ptr((size_t)nseg + 1), idx;
        ptr[0] = 0;
        for (int g = 0; g < nseg; ++g) {
            int len = (rng() % 10 == 0) ? (int)(rng() % 5000) : (int)(rng() % 12);
            if (rng() % 7 == 0) len = 0;
            std::vector<int> cols;
            for (int q = 0; q < len; ++q) cols.push_back((int)(rng() % nidx));
            std::sort(cols.begin(), cols.end());
            cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
            for (int c : cols) idx.push_back(c);
            ptr[(size_t)g + 1] = (int32_t)idx.size();
        }
        // the gathered dimension's pointers (its nonzero counts as prefix sums)
        hvec<int32_t> gptr((size_t)nidx + 1);
        std::vector<int32_t> gcnt((size_t)nidx, 0);
        for (int32_t c : idx) gcnt[(size_t)c]++;
        gptr[0] = 0;
        for (int i = 0; i < nidx; ++i) gptr[(size_t)i + 1] = gptr[(size_t)i] + gcnt[(size_t)i];
        std::vector<double> val(idx.size()), v((size_t)nidx);
        for (auto &a : val) a = (double)(rng() % 1000) / 7.0;
        for (auto &a : v) a = (double)(rng() % 1000) / 3.0;
        SlicedHost sh;
        const int tile = 64 << (rng() % 6);
        slice_format(ptr, idx, gptr, nseg, nidx, S, tile, sh);
        if (sh.G != count_compact(ptr, idx, gptr, nseg, nidx, S)) { std::printf("G mismatch\n"); ++bad; }
        if ((int)sh.bounds.size() != S + 1 || sh.bounds[0] != 0 || sh.bounds[(size_t)S] != nidx) {
            std::printf("bounds ends\n");
            ++bad;
            continue;
        }
        {
            const int64_t nz = (int64_t)idx.size();
            const int32_t big = *std::max_element(gcnt.begin(), gcnt.end());
            for (int s = 0; s < S; ++s) {
                if (sh.bounds[(size_t)s] > sh.bounds[(size_t)s + 1]) { std::printf("bounds order\n"); ++bad; }
                const int64_t in = gptr[(size_t)sh.bounds[(size_t)s + 1]] - gptr[(size_t)sh.bounds[(size_t)s]];
                if (in > nz / S + 1 + big) { std::printf("slice %d holds %ld of %ld\n", s, (long)in, (long)nz); ++bad; }
            }
        }
        std::vector<int> cover((size_t)sh.G, 0);
        for (const Tile &t : sh.tiles) {
            if (t.seg_begin < sh.seg_base[(size_t)t.slice] || t.seg_end > sh.seg_base[(size_t)t.slice + 1]) {
                std::printf("tile outside its slice\n");
                ++bad;
                continue;
            }
            for (int g = t.seg_begin; g < t.seg_end; ++g) cover[(size_t)g] += t.npieces ? (t.piece == 0) : 1;
            if (t.nnz_begin < sh.ptr[(size_t)t.seg_begin] || t.nnz_end > sh.ptr[(size_t)t.seg_end]) {
                std::printf("tile nonzero range\n");
                ++bad;
            }
        }
        for (int64_t g = 0; g < sh.G; ++g)
            if (cover[(size_t)g] != 1) { std::printf("cover %ld: %d\n", (long)g, cover[(size_t)g]); ++bad; break; }
        std::vector<double> part((size_t)sh.G, 0.0);
        for (int s = 0; s < S; ++s)
            for (int64_t g = sh.seg_base[(size_t)s]; g < sh.seg_base[(size_t)s + 1]; ++g)
                for (int p = sh.ptr[(size_t)g]; p < sh.ptr[(size_t)g + 1]; ++p) {
                    if (sh.idx[(size_t)p] < sh.bounds[(size_t)s] || sh.idx[(size_t)p] >= sh.bounds[(size_t)s + 1]) {
                        std::printf("index outside slice\n");
                        ++bad;
                    }
                    if (idx[(size_t)sh.src[(size_t)p]] != sh.idx[(size_t)p]) { std::printf("src\n"); ++bad; }
                    part[(size_t)g] += val[(size_t)sh.src[(size_t)p]] * v[(size_t)sh.idx[(size_t)p]];
                }
        const int nblk = (nseg + 255) / 256;
        for (int b = 0; b < nblk; ++b)
            for (int t = 0; t < 256; ++t) {
                const int j = b * 256 + t;
                if (j >= nseg) break;
                double r = 0.0, ref = 0.0;
                for (int s = 0; s < S; ++s) {
                    const int pl = s / 8, bit = s % 8;
                    if (!((sh.mask[(size_t)pl * nseg + j] >> bit) & 1)) continue;
                    int off = sh.cbase[(size_t)b * S + s];
                    for (int u = b * 256; u < j; ++u) off += (sh.mask[(size_t)pl * nseg + u] >> bit) & 1;
                    if (off < 0 || off >= sh.G) { std::printf("partial index out of range\n"); ++bad; continue; }
                    r += part[(size_t)off];
                }
                for (int p = ptr[(size_t)j]; p < ptr[(size_t)j + 1]; ++p) ref += val[(size_t)p] * v[(size_t)idx[(size_t)p]];
                if (std::fabs(r - ref) > 1e-9 * (1 + std::fabs(ref))) {
                    if (bad < 5) std::printf("segment %d: %g vs %g\n", j, r, ref);
                    ++bad;
                }
            }
        // gather-sorted tiles: pos is a permutation of each tile's positions,
        // the sorted nonzero at q is the one that was at nnz_begin + pos[q],
        // its indices ascend inside the tile, and its product lands where
        // the unsorted tile kernel put it (so every segment sum is unchanged)
        {
            hvec<int32_t> sidx = sh.idx, ssrc = sh.src;
            hvec<uint16_t> pos;
            const int64_t l0 = tile_gather_lines(sh.tiles, sh.idx, 16, false);
            const int64_t l1 = tile_gather_lines(sh.tiles, sh.idx, 16, true);
            if (l1 > l0) { std::printf("sorting added lines\n"); ++bad; }
            sort_tiles_by_gather(sh.tiles, sidx, ssrc, pos);
            if (pos.size() != sh.idx.size()) { std::printf("pos size\n"); ++bad; continue; }
            if (tile_gather_lines(sh.tiles, sidx, 16, false) != l1) { std::printf("sorted lines\n"); ++bad; }
            for (const Tile &t : sh.tiles) {
                const int cnt = t.nnz_end - t.nnz_begin;
                std::vector<char> hit((size_t)cnt, 0);
                for (int q = t.nnz_begin; q < t.nnz_end; ++q) {
                    const int o = pos[(size_t)q];
                    if (o < 0 || o >= cnt || hit[(size_t)o]) { std::printf("pos not a permutation\n"); ++bad; break; }
                    hit[(size_t)o] = 1;
                    if (sidx[(size_t)q] != sh.idx[(size_t)(t.nnz_begin + o)] ||
                        ssrc[(size_t)q] != sh.src[(size_t)(t.nnz_begin + o)]) {
                        std::printf("sorted entry does not match its origin\n");
                        ++bad;
                        break;
                    }
                    if (q > t.nnz_begin && sidx[(size_t)q] < sidx[(size_t)q - 1]) { std::printf("not sorted\n"); ++bad; break; }
                }
    }
    // gather_window_bytes: one window (nsample = 1 takes the first) against a
    // brute-force set of lines, on random and on clustered indices
    for (int trial = 0; trial < 20; ++trial) {
        const int32_t nidx = 1 + (int32_t)(rng() % 100000);
        const int64_t nnz = 1 + (int64_t)(rng() % 50000);
        hvec<int32_t> idx((size_t)nnz);
        const int32_t span = trial % 2 ? nidx : 1 + nidx / 50;
        for (auto &x : idx) x = (int32_t)(rng() % (uint64_t)span);
        const int64_t window = 1 + (int64_t)(rng() % (uint64_t)nnz);
        const int32_t le = trial % 3 ? 16 : 32;
        std::vector<char> seen((size_t)(nidx / le + 1), 0);
        int64_t cnt = 0;
        for (int64_t p = 0; p < window; ++p)
            if (!seen[(size_t)(idx[(size_t)p] / le)]) { seen[(size_t)(idx[(size_t)p] / le)] = 1; ++cnt; }
        const double got = gather_window_bytes(idx, nnz, nidx, window, le, 1);
        if (got != 128.0 * (double)cnt) { std::printf("window %g vs %g\n", got, 128.0 * cnt); ++bad; }
        // several windows: the median lies between the smallest and largest
        const double med = gather_window_bytes(idx, nnz, nidx, window, le, 7);
        if (med < 128.0 || med > 128.0 * (double)window) { std::printf("window median %g\n", med); ++bad; }
            }
        }
    }
    std::printf(bad ? "FAILED %d\n" : "ok\n", bad);
    return bad != 0;
}
