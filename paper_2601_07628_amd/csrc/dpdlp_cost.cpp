// Per-iteration cost model of the distributed method (Sec. 3.3, derived in
// App. E), the grid choice for a device count (Sec. 4.1) and the automatic
// device count that evaluates the model before a run (Sec. 5.1).  Host code
// only.
//
// T_step(R, C) is the sum of four terms for an R x C device grid (N = R C):
//   matrix stream   c_spmv nnz / (b_mem N)
//   vector traffic  c_vec (n / C + m / R) / b_mem
//   ring payload    c_net (V_row + V_col) / b_net, where the row communicator
//                   (R devices) all-reduces n / C elements and the column
//                   communicator (C devices) m / R elements, each device moving
//                   L (K - 1) / K of a payload L over a ring of K
//   latency         n_hop beta_sync (one per dimension that is split)
#include "dpdlp_internal.h"

#include <cmath>
#include <limits>

namespace {

// The per-device ring volume of the two all-reduces, in elements.  Written
// as the two ring volumes, which add up to (n R + m C - (m + n)) / N.
double ring_volume(double m, double n, int32_t R, int32_t C)
{
    const double v_row = (n / C) * (double)(R - 1) / (double)R;
    const double v_col = (m / R) * (double)(C - 1) / (double)C;
    return v_row + v_col;
}

bool cost_params_ok(const dpdlp_cost_params *p)
{
    return p && p->b_mem > 0 && p->b_net > 0 && p->beta_sync >= 0 && p->n_hop >= 0 &&
           p->c_spmv >= 0 && p->c_vec >= 0 && p->c_net >= 0 && std::isfinite(p->b_mem) &&
           std::isfinite(p->b_net) && std::isfinite(p->beta_sync) && std::isfinite(p->n_hop);
}

}  // namespace

extern "C" {

void dpdlp_cost_params_default(dpdlp_cost_params *p)
{
    if (!p) return;
    p->b_mem = 8.0e12;        // MI355X HBM3E peak
    p->b_net = 153.6e9;       // one xGMI link (a ring moves over one link per hop)
    p->beta_sync = 10e-6;     // the paper's handshake latency; not measurable on one GPU
    p->n_hop = 1.0;           // one node, every GPU linked to every other
    p->c_spmv = 24.0;         // FP64 value + INT32 index, CSR and CSC
    p->c_vec = 90.0;
    p->c_net = 8.0;           // FP64 payload
}

int dpdlp_cost_step(int64_t m, int64_t n, int64_t nnz, int32_t R, int32_t C,
                    const dpdlp_cost_params *p, double *out)
{
    if (m < 0 || n < 0 || nnz < 0 || R < 1 || C < 1 || !out || !cost_params_ok(p)) {
        dpdlp::set_error("dpdlp_cost_step: bad arguments");
        return DPDLP_E_INVALID_ARG;
    }
    const double N = (double)R * (double)C;
    const double md = (double)m, nd = (double)n;
    out[0] = p->c_spmv * (double)nnz / (p->b_mem * N);
    out[1] = p->c_vec * (nd / C + md / R) / p->b_mem;
    out[2] = p->c_net * ring_volume(md, nd, R, C) / p->b_net;
    out[3] = p->n_hop * p->beta_sync * ((R > 1 ? 1.0 : 0.0) + (C > 1 ? 1.0 : 0.0));
    out[4] = out[0] + out[1] + out[2] + out[3];
    return DPDLP_OK;
}

int dpdlp_grid_select(int64_t m, int64_t n, int32_t ndev, int32_t *R, int32_t *C)
{
    if (m < 1 || n < 1 || ndev < 1 || !R || !C) {
        dpdlp::set_error("dpdlp_grid_select: bad arguments");
        return DPDLP_E_INVALID_ARG;
    }
    // the factor pair whose aspect ratio R / C is closest to m / n, measured
    // as a ratio (|log(R / C) - log(m / n)|); ties (equal up to rounding,
    // 1e-12) go to the smaller R
    const double target = std::log((double)m) - std::log((double)n);
    double best = std::numeric_limits<double>::infinity();
    for (int32_t r = 1; r <= ndev; ++r) {
        if (ndev % r) continue;
        const int32_t c = ndev / r;
        const double d = std::fabs(std::log((double)r) - std::log((double)c) - target);
        if (d < best - 1e-12) {
            best = d;
            *R = r;
            *C = c;
        }
    }
    return DPDLP_OK;
}

int dpdlp_auto_devices(int64_t m, int64_t n, int64_t nnz, const int32_t *counts,
                       int32_t ncounts, const dpdlp_cost_params *p, int32_t *ndev,
                       int32_t *R, int32_t *C, double *t_step)
{
    if (m < 1 || n < 1 || nnz < 0 || !counts || ncounts < 1 || !ndev || !R || !C ||
        !cost_params_ok(p)) {
        dpdlp::set_error("dpdlp_auto_devices: bad arguments");
        return DPDLP_E_INVALID_ARG;
    }
    for (int32_t i = 0; i < ncounts; ++i)
        if (counts[i] < 1) {
            dpdlp::set_error("dpdlp_auto_devices: device counts must be positive");
            return DPDLP_E_INVALID_ARG;
        }
    int32_t bn = 0, br = 1, bc = 1;
    double best = 0.0;
    for (int32_t i = 0; i < ncounts; ++i) {
        int32_t r = 1, c = 1;
        double t[5];
        dpdlp_grid_select(m, n, counts[i], &r, &c);
        dpdlp_cost_step(m, n, nnz, r, c, p, t);
        // strictly faster wins; equal times keep the smaller count
        if (i == 0 || t[4] < best || (t[4] == best && counts[i] < bn)) {
            best = t[4];
            bn = counts[i];
            br = r;
            bc = c;
        }
    }
    *ndev = bn;
    *R = br;
    *C = bc;
    if (t_step) *t_step = best;
    return DPDLP_OK;
}

}  // extern "C"
