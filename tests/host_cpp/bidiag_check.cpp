// Host check of the Lanczos helpers: bidiag_sigma_max (largest singular
// value of an upper bidiagonal matrix by Sturm bisection on B^T B) against a
// long power iteration on the dense B^T B, for several sizes; and
// lanczos_start (entries in [-1, 1), returned norm = 2-norm).
// Built with g++ (AddressSanitizer, UBSan) by tests/test_host_cpu.py.
#include "dpdlp_internal.h"

#include <cmath>
#include <cstdio>
#include <random>

using namespace dpdlp;

int main()
{
    std::mt19937_64 rng(3);
    std::uniform_real_distribution<double> U(0.01, 2.0);
    int bad = 0;
    for (int k : {1, 2, 3, 5, 17, 60, 200}) {
        std::vector<double> a((size_t)k), b((size_t)k);
        for (int i = 0; i < k; ++i) { a[(size_t)i] = U(rng); b[(size_t)i] = U(rng); }
        std::vector<double> T((size_t)k * k, 0.0);
        for (int i = 0; i < k; ++i) {
            T[(size_t)i * k + i] = a[(size_t)i] * a[(size_t)i] + (i ? b[(size_t)i] * b[(size_t)i] : 0.0);
            if (i + 1 < k) {
                T[(size_t)i * k + i + 1] = a[(size_t)i] * b[(size_t)i + 1];
                T[(size_t)(i + 1) * k + i] = a[(size_t)i] * b[(size_t)i + 1];
            }
        }
        std::vector<double> v((size_t)k, 1.0), w((size_t)k);
        double lam = 0.0;
        for (int it = 0; it < 20000; ++it) {
            double nn = 0.0;
            for (int i = 0; i < k; ++i) {
                double s = 0.0;
                for (int j = 0; j < k; ++j) s += T[(size_t)i * k + j] * v[(size_t)j];
                w[(size_t)i] = s;
                nn += s * s;
            }
            nn = std::sqrt(nn);
            for (int i = 0; i < k; ++i) v[(size_t)i] = w[(size_t)i] / nn;
            lam = nn;
        }
        const double s1 = std::sqrt(lam), s2 = bidiag_sigma_max(a.data(), b.data(), k);
        std::printf("k=%d power %.15g bisection %.15g\n", k, s1, s2);
        if (std::fabs(s1 - s2) > 1e-10 * s1) ++bad;
    }
    std::vector<double> w(1000);
    const double nrm = lanczos_start(1000, 7, w.data());
    double ss = 0.0;
    for (double x : w) {
        ss += x * x;
        if (x < -1.0 || x >= 1.0) ++bad;
    }
    if (std::fabs(std::sqrt(ss) - nrm) > 1e-12 * nrm) ++bad;
    std::printf(bad ? "FAILED\n" : "ok\n");
    return bad != 0;
}
