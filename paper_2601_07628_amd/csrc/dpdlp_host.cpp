// Host preprocessing of the LP: validation, the block-wise random
// permutation (Sec. 4.2 of the D-PDLP paper), the CSC copy (both formats are
// kept so that A^T y needs no atomics, App. E.3) and the nonzero-aware tiles
// that balance nonzeros across workgroups (Sec. 4.3, applied at workgroup
// instead of GPU granularity).  Integer work only; no GPU calls.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <string>
#include <thread>
#include <vector>

#include "dpdlp_internal.h"

namespace dpdlp {

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }

int bad_mem_kind()
{
    set_error("mem_kind must be DPDLP_MEM_HOST (0) or DPDLP_MEM_DEVICE (1)");
    return DPDLP_E_INVALID_ARG;
}

int validate_host(const dpdlp_csr_lp *lp)
{
    if (!lp) { set_error("lp is NULL"); return DPDLP_E_INVALID_ARG; }
    if (lp->m < 1 || lp->n < 1) {
        set_error("m and n must be >= 1");
        return DPDLP_E_INVALID_ARG;
    }
    if (!lp->row_ptr || !lp->c || !lp->con_lo || !lp->con_hi || !lp->var_lo ||
        !lp->var_hi) {
        set_error("a required array is NULL");
        return DPDLP_E_INVALID_ARG;
    }
    const int32_t m = lp->m, n = lp->n;
    if (lp->row_ptr[0] != 0) { set_error("row_ptr[0] != 0"); return DPDLP_E_BAD_CSR; }
    for (int32_t i = 0; i < m; ++i)
        if (lp->row_ptr[i + 1] < lp->row_ptr[i]) {
            set_error("row_ptr not monotone at row " + std::to_string(i));
            return DPDLP_E_BAD_CSR;
        }
    const int64_t nnz = lp->row_ptr[m];
    if (nnz > 0 && (!lp->col_idx || !lp->val)) {
        set_error("col_idx / val is NULL");
        return DPDLP_E_INVALID_ARG;
    }
    std::vector<int32_t> mark((size_t)n, -1);
    for (int32_t i = 0; i < m; ++i)
        for (int64_t p = lp->row_ptr[i]; p < lp->row_ptr[i + 1]; ++p) {
            int32_t j = lp->col_idx[p];
            if (j < 0 || j >= n) {
                set_error("column index out of range at nonzero " + std::to_string(p));
                return DPDLP_E_BAD_CSR;
            }
            if (mark[(size_t)j] == i) {
                set_error("duplicate entry (" + std::to_string(i) + "," +
                          std::to_string(j) + ")");
                return DPDLP_E_BAD_CSR;
            }
            mark[(size_t)j] = i;
            if (!std::isfinite(lp->val[p])) {
                set_error("non-finite matrix value at nonzero " + std::to_string(p));
                return DPDLP_E_BAD_CSR;
            }
        }
    for (int32_t j = 0; j < n; ++j) {
        if (!std::isfinite(lp->c[j])) {
            set_error("non-finite c[" + std::to_string(j) + "]");
            return DPDLP_E_BAD_BOUNDS;
        }
        double lo = lp->var_lo[j], hi = lp->var_hi[j];
        if (std::isnan(lo) || std::isnan(hi) || lo > hi || lo == INFINITY ||
            hi == -INFINITY) {
            set_error("bad variable bounds at column " + std::to_string(j));
            return DPDLP_E_BAD_BOUNDS;
        }
    }
    for (int32_t i = 0; i < m; ++i) {
        double lo = lp->con_lo[i], hi = lp->con_hi[i];
        if (std::isnan(lo) || std::isnan(hi) || lo > hi || lo == INFINITY ||
            hi == -INFINITY) {
            set_error("bad constraint bounds at row " + std::to_string(i));
            return DPDLP_E_BAD_BOUNDS;
        }
    }
    return DPDLP_OK;
}

// splitmix64: a small published counter-based generator (Steele, Lea, Flood).
static inline uint64_t splitmix64(uint64_t &s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Runs f(t) for t = 0 .. n - 1 on n host threads.
template <class F>
static void run_threads(int n, F f)
{
    std::vector<std::thread> th;
    for (int t = 1; t < n; ++t) th.emplace_back(f, t);
    f(0);
    for (auto &x : th) x.join();
}

static int host_threads()
{
    return (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
}

double lanczos_start(int32_t n, uint64_t seed, double *w)
{
    uint64_t s = seed;
    double ss = 0.0;
    for (int32_t j = 0; j < n; ++j) {
        w[j] = 2.0 * (double)(splitmix64(s) >> 11) * 0x1.0p-53 - 1.0;
        ss += w[j] * w[j];
    }
    return std::sqrt(ss);
}

double bidiag_sigma_max(const double *alpha, const double *beta, int k)
{
    if (k <= 0) return 0.0;
    // T = B^T B: T_ii = alpha_i^2 + beta_i^2 (beta_0 = 0), T_i,i+1 = alpha_i beta_i+1
    std::vector<double> d((size_t)k), e((size_t)k, 0.0);
    for (int i = 0; i < k; ++i) {
        const double b = i > 0 ? beta[i] : 0.0;
        d[(size_t)i] = alpha[i] * alpha[i] + b * b;
        if (i + 1 < k) e[(size_t)i] = alpha[i] * beta[i + 1];
    }
    double hi = 0.0;
    for (int i = 0; i < k; ++i)
        hi = std::max(hi, d[(size_t)i] + std::fabs(e[(size_t)i]) + (i > 0 ? std::fabs(e[(size_t)i - 1]) : 0.0));
    if (!(hi > 0.0)) return 0.0;
    // number of eigenvalues of T below x (Sturm sequence of the LDL^T pivots)
    auto below = [&](double x) {
        int cnt = 0;
        double q = 1.0;
        for (int i = 0; i < k; ++i) {
            const double e2 = i > 0 ? e[(size_t)i - 1] * e[(size_t)i - 1] : 0.0;
            q = d[(size_t)i] - x - (i > 0 ? e2 / q : 0.0);
            if (q == 0.0) q = -1e-300 * hi;
            if (q < 0.0) ++cnt;
        }
        return cnt;
    };
    double lo = 0.0;
    for (int it = 0; it < 200 && hi - lo > 1e-15 * hi; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (below(mid) == k) hi = mid; else lo = mid;
    }
    return std::sqrt(0.5 * (lo + hi));
}

void block_permutation(int32_t count, int32_t block, uint64_t seed, int32_t *perm)
{
    if (block <= 0 || count <= block) {
        for (int32_t i = 0; i < count; ++i) perm[i] = i;
        return;
    }
    const int32_t nb = (count + block - 1) / block;
    std::vector<int32_t> order((size_t)nb);
    for (int32_t b = 0; b < nb; ++b) order[(size_t)b] = b;
    uint64_t s = seed;
    for (int32_t b = nb - 1; b > 0; --b) {      // Fisher-Yates over blocks
        uint64_t r = splitmix64(s) % (uint64_t)(b + 1);
        std::swap(order[(size_t)b], order[(size_t)r]);
    }
    int32_t pos = 0;
    for (int32_t q = 0; q < nb; ++q) {
        int32_t b = order[(size_t)q];
        int32_t lo = b * block, hi = std::min(count, lo + block);
        for (int32_t i = lo; i < hi; ++i) perm[pos++] = i;
    }
}

static int32_t ceil_log2(int32_t v)
{
    int32_t l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

void build_tiles(const int32_t *ptr, int32_t nseg, int32_t tile_nnz,
                 std::vector<Tile> &out)
{
    out.clear();
    if (tile_nnz <= 0 || tile_nnz > kTileNnzMax) tile_nnz = kTileNnzMax;
    int32_t s = 0;
    while (s < nseg) {
        int32_t len = ptr[s + 1] - ptr[s];
        if (len > tile_nnz) {                      // long segment: split it
            int32_t np = (len + tile_nnz - 1) / tile_nnz;
            for (int32_t pc = 0; pc < np; ++pc) {
                Tile t{};
                t.seg_begin = s; t.seg_end = s + 1;
                t.nnz_begin = ptr[s] + pc * tile_nnz;
                t.nnz_end = std::min(ptr[s + 1], t.nnz_begin + tile_nnz);
                t.width_log2 = 6; t.piece = pc; t.npieces = np;
                out.push_back(t);
            }
            ++s;
            continue;
        }
        int32_t start = s, nz = 0;
        while (s < nseg && s - start < kMaxSegs) {
            int32_t l = ptr[s + 1] - ptr[s];
            if (l > tile_nnz || nz + l > tile_nnz) break;
            nz += l;
            ++s;
        }
        Tile t{};
        t.seg_begin = start; t.seg_end = s;
        t.nnz_begin = ptr[start]; t.nnz_end = ptr[s];
        int32_t nsg = s - start;
        int32_t avg = (nz + nsg - 1) / nsg;
        t.width_log2 = std::min(6, ceil_log2(std::max(1, avg)));
        t.piece = 0; t.npieces = 0;
        out.push_back(t);
    }
}

void slice_bounds(const hvec<int32_t> &gptr, int32_t nidx, int32_t S,
                  std::vector<int32_t> &bounds)
{
    // slice s starts at the first index whose prefix count reaches s nnz / S;
    // whatever the order of the indices, every slice (and so every XCD) gets
    // about the same number of gathers, and under a random order the ranges
    // come out close to equal
    const int64_t nnz = gptr[(size_t)nidx];
    bounds.assign((size_t)S + 1, 0);
    bounds[(size_t)S] = nidx;
    for (int32_t s = 1; s < S; ++s) {
        const int64_t target = nnz * s / S;
        const int32_t b = (int32_t)(std::lower_bound(gptr.begin(), gptr.begin() + (size_t)nidx + 1,
                                                     target,
                                                     [](int32_t v, int64_t t) { return (int64_t)v < t; }) -
                                    gptr.begin());
        bounds[(size_t)s] = std::min(std::max(b, bounds[(size_t)s - 1]), nidx);
    }
}

// slice of every gathered index
static void slice_map(const std::vector<int32_t> &bounds, int32_t nidx, int32_t S, hvec<uint8_t> &map)
{
    map.resize((size_t)nidx);
    for (int32_t s = 0; s < S; ++s)
        std::fill(map.begin() + bounds[(size_t)s], map.begin() + bounds[(size_t)s + 1], (uint8_t)s);
}

double gather_window_bytes(const hvec<int32_t> &idx, int64_t nnz, int32_t nidx, int64_t window,
                           int32_t line_elems, int nsample)
{
    if (nnz <= 0 || nidx <= 0 || nsample <= 0) return 0.0;
    window = std::max<int64_t>(1, std::min(window, nnz));
    const int64_t nlines = ((int64_t)nidx + line_elems - 1) / line_elems;
    std::vector<uint64_t> bits((size_t)((nlines + 63) / 64), 0);
    std::vector<double> fp((size_t)nsample);
    for (int k = 0; k < nsample; ++k) {
        const int64_t a = nsample > 1 ? (nnz - window) * k / (nsample - 1) : 0;
        int64_t cnt = 0;
        for (int64_t p = a; p < a + window; ++p) {
            const int64_t l = idx[(size_t)p] / line_elems;
            uint64_t &w = bits[(size_t)(l >> 6)];
            const uint64_t b = 1ull << (l & 63);
            if (!(w & b)) { w |= b; ++cnt; }
        }
        for (int64_t p = a; p < a + window; ++p) bits[(size_t)((idx[(size_t)p] / line_elems) >> 6)] = 0;
        fp[(size_t)k] = 128.0 * (double)cnt;
    }
    std::nth_element(fp.begin(), fp.begin() + nsample / 2, fp.end());
    return fp[(size_t)nsample / 2];
}

int64_t count_compact(const hvec<int32_t> &ptr, const hvec<int32_t> &idx,
                      const hvec<int32_t> &gptr, int32_t nseg, int32_t nidx, int32_t S)
{
    std::vector<int32_t> bounds;
    slice_bounds(gptr, nidx, S, bounds);
    hvec<uint8_t> smap;
    slice_map(bounds, nidx, S, smap);
    const int nth = host_threads();
    std::vector<int64_t> part((size_t)nth, 0);
    run_threads(nth, [&](int t) {
        const int32_t g0 = (int32_t)((int64_t)nseg * t / nth), g1 = (int32_t)((int64_t)nseg * (t + 1) / nth);
        std::vector<int32_t> last((size_t)S, -1);
        int64_t G = 0;
        for (int32_t g = g0; g < g1; ++g)
            for (int32_t p = ptr[(size_t)g]; p < ptr[(size_t)g + 1]; ++p) {
                const int32_t s = smap[(size_t)idx[(size_t)p]];
                if (last[(size_t)s] != g) { last[(size_t)s] = g; ++G; }
            }
        part[(size_t)t] = G;
    });
    int64_t G = 0;
    for (int64_t v : part) G += v;
    return G;
}

int64_t tile_gather_lines(const std::vector<Tile> &tiles, const hvec<int32_t> &idx,
                          int32_t line_elems, bool sorted)
{
    const int nth = host_threads();
    const int64_t nt = (int64_t)tiles.size();
    std::vector<int64_t> part((size_t)nth, 0);
    run_threads(nth, [&](int th) {
        std::vector<int32_t> v;
        for (int64_t t = nt * th / nth; t < nt * (th + 1) / nth; ++t) {
            const Tile &d = tiles[(size_t)t];
            v.assign(idx.begin() + d.nnz_begin, idx.begin() + d.nnz_end);
            if (sorted) std::stable_sort(v.begin(), v.end());
            for (size_t g = 0; g < v.size(); g += 64) {
                const size_t e = std::min(v.size(), g + 64);
                std::vector<int32_t> lines;
                for (size_t q = g; q < e; ++q) lines.push_back(v[q] / line_elems);
                std::sort(lines.begin(), lines.end());
                part[(size_t)th] += std::unique(lines.begin(), lines.end()) - lines.begin();
            }
        }
    });
    int64_t tot = 0;
    for (int64_t x : part) tot += x;
    return tot;
}

void sort_tiles_by_gather(const std::vector<Tile> &tiles, hvec<int32_t> &idx,
                          hvec<int32_t> &src, hvec<uint16_t> &pos)
{
    pos.resize(idx.size());                  // every entry written below (tiles cover idx)
    const int nth = host_threads();
    const int64_t nt = (int64_t)tiles.size();
    run_threads(nth, [&](int th) {
        std::vector<int32_t> ord, ti, ts;
        for (int64_t t = nt * th / nth; t < nt * (th + 1) / nth; ++t) {
            const Tile &d = tiles[(size_t)t];
            const int32_t b = d.nnz_begin, cnt = d.nnz_end - d.nnz_begin;
            ord.resize((size_t)cnt);
            for (int32_t q = 0; q < cnt; ++q) ord[(size_t)q] = q;
            std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t c) {
                return idx[(size_t)(b + a)] < idx[(size_t)(b + c)];
            });
            ti.assign(idx.begin() + b, idx.begin() + b + cnt);
            ts.assign(src.begin() + b, src.begin() + b + cnt);
            for (int32_t q = 0; q < cnt; ++q) {
                const int32_t o = ord[(size_t)q];
                idx[(size_t)(b + q)] = ti[(size_t)o];
                src[(size_t)(b + q)] = ts[(size_t)o];
                pos[(size_t)(b + q)] = (uint16_t)o;
            }
        }
    });
}

void slice_format(const hvec<int32_t> &ptr, const hvec<int32_t> &idx, const hvec<int32_t> &gptr,
                  int32_t nseg, int32_t nidx, int32_t S, int32_t tile_nnz, SlicedHost &out)
{
    out.S = S;
    slice_bounds(gptr, nidx, S, out.bounds);
    hvec<uint8_t> smap;
    slice_map(out.bounds, nidx, S, smap);
    const int64_t nnz = ptr[(size_t)nseg];
    const int32_t planes = S / 8;
    const int32_t nblk = (nseg + kBlock - 1) / kBlock;
    // threads own ranges of whole segments; every pass below is O(nnz + S nseg)
    const int nth = host_threads();
    std::vector<int32_t> g0v((size_t)nth + 1);
    for (int t = 0; t <= nth; ++t) g0v[(size_t)t] = (int32_t)((int64_t)nseg * t / nth);
    // 1. per (slice, segment) counts and per (thread, slice) totals
    hvec<int32_t> cnt((size_t)S * (size_t)nseg);      // every entry written below
    std::vector<int64_t> tg((size_t)nth * S, 0), tz((size_t)nth * S, 0);
    run_threads(nth, [&](int t) {
        std::vector<int32_t> c((size_t)S);
        for (int32_t g = g0v[(size_t)t]; g < g0v[(size_t)t + 1]; ++g) {
            std::fill(c.begin(), c.end(), 0);
            for (int32_t p = ptr[(size_t)g]; p < ptr[(size_t)g + 1]; ++p) c[(size_t)smap[(size_t)idx[(size_t)p]]]++;
            for (int32_t s = 0; s < S; ++s) {
                cnt[(size_t)s * nseg + g] = c[(size_t)s];
                tg[(size_t)t * S + s] += c[(size_t)s] > 0;
                tz[(size_t)t * S + s] += c[(size_t)s];
            }
        }
    });
    // 2. compact numbering: slice-major, increasing segment within a slice;
    //    each thread's first compact segment and nonzero position per slice
    out.seg_base.assign((size_t)S + 1, 0);
    std::vector<int64_t> nz_base((size_t)S + 1, 0);
    for (int32_t s = 0; s < S; ++s) {
        int64_t G = 0, Z = 0;
        for (int t = 0; t < nth; ++t) { G += tg[(size_t)t * S + s]; Z += tz[(size_t)t * S + s]; }
        out.seg_base[(size_t)s + 1] = out.seg_base[(size_t)s] + (int32_t)G;
        nz_base[(size_t)s + 1] = nz_base[(size_t)s] + Z;
    }
    std::vector<int64_t> tq((size_t)nth * S), tp((size_t)nth * S);
    for (int32_t s = 0; s < S; ++s) {
        int64_t q = out.seg_base[(size_t)s], z = nz_base[(size_t)s];
        for (int t = 0; t < nth; ++t) {
            tq[(size_t)t * S + s] = q;
            tp[(size_t)t * S + s] = z;
            q += tg[(size_t)t * S + s];
            z += tz[(size_t)t * S + s];
        }
    }
    const int64_t G = out.seg_base[(size_t)S];
    out.G = G;
    out.ptr.resize((size_t)G + 1);          // every entry written below
    out.ptr[(size_t)G] = (int32_t)nnz;
    out.cbase.assign((size_t)nblk * (size_t)S, 0);
    out.mask.assign((size_t)planes * (size_t)nseg, 0);
    out.idx.resize((size_t)nnz);
    out.src.resize((size_t)nnz);
    // 3. pointers, combine bases, masks and the scatter, per segment range
    run_threads(nth, [&](int t) {
        std::vector<int64_t> q(tq.begin() + (size_t)t * S, tq.begin() + (size_t)(t + 1) * S);
        std::vector<int64_t> z(tp.begin() + (size_t)t * S, tp.begin() + (size_t)(t + 1) * S);
        for (int32_t g = g0v[(size_t)t]; g < g0v[(size_t)t + 1]; ++g) {
            for (int32_t s = 0; s < S; ++s) {
                if (g % kBlock == 0) out.cbase[(size_t)(g / kBlock) * S + s] = (int32_t)q[(size_t)s];
                if (cnt[(size_t)s * nseg + g] > 0) {
                    out.ptr[(size_t)q[(size_t)s]++] = (int32_t)z[(size_t)s];
                    out.mask[(size_t)(s / 8) * nseg + g] |= (uint8_t)(1u << (s % 8));
                }
            }
            for (int32_t p = ptr[(size_t)g]; p < ptr[(size_t)g + 1]; ++p) {
                const int32_t s = smap[(size_t)idx[(size_t)p]];
                const int64_t at = z[(size_t)s]++;
                out.idx[(size_t)at] = idx[(size_t)p];
                out.src[(size_t)at] = p;
            }
        }
    });
    // 4. tiles per slice over its compact segments (global segment numbers)
    out.tiles.clear();
    std::vector<Tile> tt;
    for (int32_t s = 0; s < S; ++s) {
        const int32_t b0 = out.seg_base[(size_t)s], ns = out.seg_base[(size_t)s + 1] - b0;
        build_tiles(out.ptr.data() + b0, ns, tile_nnz, tt);
        for (Tile t : tt) {
            t.slice = s;
            t.seg_begin += b0;
            t.seg_end += b0;
            out.tiles.push_back(t);
        }
    }
}

void permute_and_transpose(const dpdlp_csr_lp *lp, int32_t block, uint64_t seed,
                           int32_t order, HostMatrix &H)
{
    const int32_t m = lp->m, n = lp->n;
    H.m = m; H.n = n;
    H.nnz = lp->row_ptr[m];
    H.perm_row.resize((size_t)m);
    H.perm_col.resize((size_t)n);
    block_permutation(m, block, seed, H.perm_row.data());
    block_permutation(n, block, seed ^ 0xC01D5EEDull, H.perm_col.data());
    // hot-first (order bit 0: rows, bit 1: columns): a stable sort of the
    // block-permuted order by decreasing nonzero count, so that the entries
    // gathered most often share cache lines at the front of y (or x); equal
    // counts keep their block-random order
    if (order & 1) {
        std::vector<int32_t> rc((size_t)m);
        for (int32_t i = 0; i < m; ++i) rc[(size_t)i] = lp->row_ptr[i + 1] - lp->row_ptr[i];
        std::stable_sort(H.perm_row.begin(), H.perm_row.end(),
                         [&](int32_t a, int32_t b) { return rc[(size_t)a] > rc[(size_t)b]; });
    }
    if (order & 2) {
        std::vector<int32_t> cc((size_t)n, 0);
        for (int64_t p = 0; p < H.nnz; ++p) cc[(size_t)lp->col_idx[p]]++;
        std::stable_sort(H.perm_col.begin(), H.perm_col.end(),
                         [&](int32_t a, int32_t b) { return cc[(size_t)a] > cc[(size_t)b]; });
    }
    std::vector<int32_t> inv_col((size_t)n);
    for (int32_t j = 0; j < n; ++j) inv_col[(size_t)H.perm_col[(size_t)j]] = j;

    H.rp.assign((size_t)m + 1, 0);
    for (int32_t i = 0; i < m; ++i) {
        int32_t o = H.perm_row[(size_t)i];
        H.rp[(size_t)i + 1] = H.rp[(size_t)i] + (lp->row_ptr[o + 1] - lp->row_ptr[o]);
    }
    H.ci.resize((size_t)H.nnz);
    H.v.resize((size_t)H.nnz);
    // rows are independent: fill them in parallel on the host
    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    auto fill = [&](int32_t i0, int32_t i1) {
        for (int32_t i = i0; i < i1; ++i) {
            int32_t o = H.perm_row[(size_t)i];
            int64_t src = lp->row_ptr[o], dst = H.rp[(size_t)i];
            int32_t len = lp->row_ptr[o + 1] - lp->row_ptr[o];
            for (int32_t q = 0; q < len; ++q) {
                H.ci[(size_t)(dst + q)] = inv_col[(size_t)lp->col_idx[src + q]];
                H.v[(size_t)(dst + q)] = lp->val[src + q];
            }
        }
    };
    std::vector<std::thread> th;
    int32_t chunk = (m + (int32_t)nth - 1) / (int32_t)nth;
    for (unsigned q = 0; q < nth; ++q) {
        int32_t a = (int32_t)q * chunk, b = std::min(m, a + chunk);
        if (a < b) th.emplace_back(fill, a, b);
    }
    for (auto &t : th) t.join();

    // CSC by a stable two-level bucket sort (row order kept inside every
    // column).  Thread t owns rows [r_t, r_t+1) and column range c_t:
    // A. each thread counts its nonzeros per column range;
    // B. each thread copies (row, position) of its nonzeros into the column
    //    range's bucket, rows in order, after the earlier threads' part;
    // C. each thread counts, prefix-sums and scatters its own bucket.
    const int nct = host_threads();
    std::vector<int32_t> c0v((size_t)nct + 1), r0v((size_t)nct + 1);
    for (int t = 0; t <= nct; ++t) {
        c0v[(size_t)t] = (int32_t)((int64_t)n * t / nct);
        r0v[(size_t)t] = (int32_t)((int64_t)m * t / nct);
    }
    // owner of column j: the t with c0v[t] <= j < c0v[t+1]
    auto owner = [&](int32_t j) {
        int t = (int)((int64_t)j * nct / n);
        while (t + 1 < nct && j >= c0v[(size_t)t + 1]) ++t;
        while (t > 0 && j < c0v[(size_t)t]) --t;
        return t;
    };
    std::vector<int64_t> bc((size_t)nct * nct, 0);          // [row thread][bucket]
    run_threads(nct, [&](int t) {
        int64_t *c = bc.data() + (size_t)t * nct;
        for (int64_t p = H.rp[(size_t)r0v[(size_t)t]]; p < H.rp[(size_t)r0v[(size_t)t + 1]]; ++p)
            c[owner(H.ci[(size_t)p])]++;
    });
    std::vector<int64_t> boff((size_t)nct * nct), bstart((size_t)nct + 1, 0);
    for (int b = 0; b < nct; ++b) {
        int64_t o = bstart[(size_t)b];
        for (int t = 0; t < nct; ++t) {
            boff[(size_t)t * nct + b] = o;
            o += bc[(size_t)t * nct + b];
        }
        bstart[(size_t)b + 1] = o;
    }
    hvec<int32_t> brow((size_t)H.nnz), bpos((size_t)H.nnz);
    run_threads(nct, [&](int t) {
        std::vector<int64_t> o(boff.begin() + (size_t)t * nct, boff.begin() + (size_t)(t + 1) * nct);
        for (int32_t i = r0v[(size_t)t]; i < r0v[(size_t)t + 1]; ++i)
            for (int32_t p = H.rp[(size_t)i]; p < H.rp[(size_t)i + 1]; ++p) {
                const int64_t q = o[(size_t)owner(H.ci[(size_t)p])]++;
                brow[(size_t)q] = i;
                bpos[(size_t)q] = p;
            }
    });
    H.cp.assign((size_t)n + 1, 0);
    H.ri.resize((size_t)H.nnz);
    H.vt.resize((size_t)H.nnz);
    run_threads(nct, [&](int b) {
        for (int64_t q = bstart[(size_t)b]; q < bstart[(size_t)b + 1]; ++q)
            H.cp[(size_t)H.ci[(size_t)bpos[(size_t)q]] + 1]++;
    });
    for (int32_t j = 0; j < n; ++j) H.cp[(size_t)j + 1] += H.cp[(size_t)j];
    run_threads(nct, [&](int b) {
        std::vector<int32_t> next(H.cp.begin() + c0v[(size_t)b], H.cp.begin() + c0v[(size_t)b + 1]);
        const int32_t cb = c0v[(size_t)b];
        for (int64_t q = bstart[(size_t)b]; q < bstart[(size_t)b + 1]; ++q) {
            const int32_t p = bpos[(size_t)q];
            const int32_t j = H.ci[(size_t)p];
            const int32_t at = next[(size_t)(j - cb)]++;
            H.ri[(size_t)at] = brow[(size_t)q];
            H.vt[(size_t)at] = H.v[(size_t)p];
        }
    });
}

}  // namespace dpdlp

using namespace dpdlp;

extern "C" {

const char *dpdlp_last_error(void) { return g_err.c_str(); }

int dpdlp_validate(const dpdlp_csr_lp *lp)
{
    if (lp && lp->mem_kind != DPDLP_MEM_HOST) {
        set_error("dpdlp_validate takes host pointers");
        return DPDLP_E_INVALID_ARG;
    }
    return validate_host(lp);
}

int dpdlp_row_bounds(int32_t m, const double *b, const int32_t *row_type, double *con_lo,
                     double *con_hi)
{
    if (m < 0 || (m > 0 && (!b || !row_type || !con_lo || !con_hi))) {
        set_error("dpdlp_row_bounds: bad arguments");
        return DPDLP_E_INVALID_ARG;
    }
    for (int32_t i = 0; i < m; ++i) {
        if (row_type[i] < 0 || row_type[i] > 2) {
            set_error("dpdlp_row_bounds: row type must be 0 (=), 1 (>=) or 2 (<=)");
            return DPDLP_E_INVALID_ARG;
        }
        if (!std::isfinite(b[i])) {
            set_error("dpdlp_row_bounds: right-hand side must be finite");
            return DPDLP_E_INVALID_ARG;
        }
    }
    const double inf = std::numeric_limits<double>::infinity();
    for (int32_t i = 0; i < m; ++i) {
        con_lo[i] = row_type[i] == 2 ? -inf : b[i];
        con_hi[i] = row_type[i] == 1 ? inf : b[i];
    }
    return DPDLP_OK;
}

int dpdlp_block_permutation(int32_t count, int32_t block, uint64_t seed, int32_t *perm)
{
    if (count < 0 || (count > 0 && !perm)) {
        set_error("bad arguments");
        return DPDLP_E_INVALID_ARG;
    }
    block_permutation(count, block, seed, perm);
    return DPDLP_OK;
}

int dpdlp_build_tiles(const int32_t *seg_ptr, int32_t nseg, int32_t tile_nnz,
                      int32_t *tiles, int32_t *ntiles)
{
    if (!seg_ptr || nseg < 0 || !ntiles) {
        set_error("bad arguments");
        return DPDLP_E_INVALID_ARG;
    }
    std::vector<Tile> t;
    build_tiles(seg_ptr, nseg, tile_nnz, t);
    if (tiles) {
        if (*ntiles < (int32_t)t.size()) {
            set_error("tile buffer too small");
            return DPDLP_E_INVALID_ARG;
        }
        std::memcpy(tiles, t.data(), t.size() * sizeof(Tile));
    }
    *ntiles = (int32_t)t.size();
    return DPDLP_OK;
}

void dpdlp_params_default(dpdlp_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->eps = 1e-8;
    p->max_iters = 100000;
    p->time_limit = 0.0;
    p->check_period = 64;
    p->ruiz_iters = 10;
    p->gamma = 1.0;
    p->beta_suf = 0.2; p->beta_nec = 0.8; p->beta_art = 0.36;
    p->kp = 0.99; p->ki = 0.01; p->kd = 0.0;
    p->eta = 0.0; p->omega0 = 0.0; p->eta_safety = 0.998;
    p->power_max_iters = 5000;
    p->use_pc = 1;
    p->power_tol = 1e-6;
    p->pc_alpha = 1.0;
    p->perm_block = 256;
    p->tile_nnz = 0;
    p->perm_seed = 20260107ull;
    p->precision = DPDLP_FP64;
    p->xcd_remap = 1;
    p->fp32_switch_tol = 1e-6;
    p->fp32_stall_checks = 64;
    p->gather_slices = -1;
    p->use_graphs = 1;
    p->perm_order = 0;
    p->gather_sort = -1;
    p->fp32_diverge = 10.0;
}

const char *dpdlp_status_string(int32_t s)
{
    switch (s) {
    case DPDLP_RUNNING: return "running";
    case DPDLP_CONVERGED: return "converged";
    case DPDLP_ITER_LIMIT: return "iteration limit";
    case DPDLP_TIME_LIMIT: return "time limit";
    case DPDLP_NUMERICAL: return "numerical error";
    case DPDLP_E_INVALID_ARG: return "invalid argument";
    case DPDLP_E_BAD_CSR: return "bad CSR";
    case DPDLP_E_BAD_BOUNDS: return "bad bounds";
    case DPDLP_E_HIP: return "HIP error";
    case DPDLP_E_OOM: return "out of device memory";
    case DPDLP_E_NOT_SUPPORTED: return "not supported";
    default: return "unknown";
    }
}

}  // extern "C"
