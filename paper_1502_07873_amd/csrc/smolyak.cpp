// Sparse quadrature for the prior average of D^_KL (paper Section 3.3.4,
// sparse quadrature; Section 4.3 uses Gauss-Legendre rules on total-degree
// index sets): Smolyak combination technique
//   Q_w = sum_{w-d+1 <= |i-1| <= w} (-1)^{w-|i-1|} C(d-1, w-|i-1|) (x)_n Q_{i_n}
// with the m(i) = i point Gauss-Legendre rule as Q_i, coincident nodes merged.
// Host code; the 1-D rules come from Newton iteration on the Legendre
// three-term recurrence.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/eigseis.h"

namespace eig {
int set_error(int code, const std::string& msg);
}

namespace {

// m-point Gauss-Legendre nodes on [-1, 1], weights for the density 1/2.
void gauss_legendre(int m, std::vector<double>& x, std::vector<double>& w) {
    x.assign(m, 0.0);
    w.assign(m, 0.0);
    for (int i = 0; i < (m + 1) / 2; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (m + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;  // P_0, P_1
            for (int n = 2; n <= m; ++n) {
                const double p2 = ((2.0 * n - 1.0) * z * p1 - (n - 1.0) * p0) / n;
                p0 = p1;
                p1 = p2;
            }
            if (m == 1) { p1 = z; p0 = 1.0; }
            // P_m = p1, P_{m-1} = p0; P'_m = m (z P_m - P_{m-1}) / (z^2 - 1)
            dp = m * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        // recompute the derivative at the converged node
        double p0 = 1.0, p1 = z;
        for (int n = 2; n <= m; ++n) {
            const double p2 = ((2.0 * n - 1.0) * z * p1 - (n - 1.0) * p0) / n;
            p0 = p1;
            p1 = p2;
        }
        if (m == 1) { p1 = z; p0 = 1.0; }
        dp = m * (z * p1 - p0) / (z * z - 1.0);
        const double wt = 2.0 / ((1.0 - z * z) * dp * dp);
        x[i] = -z;
        x[m - 1 - i] = z;
        w[i] = w[m - 1 - i] = 0.5 * wt;
    }
    if (m % 2 == 1) x[m / 2] = 0.0;
}

double binom(int n, int k) {
    if (k < 0 || k > n) return 0.0;
    double r = 1.0;
    for (int j = 1; j <= k; ++j) r = r * (n - k + j) / j;
    return r;
}

}  // namespace

extern "C" int sparse_grid_gl(int32_t dim, int32_t level, const double* lo,
                              const double* hi, int32_t capacity, double* nodes,
                              double* weights, int32_t* count) {
    if (dim < 1 || dim > 16 || level < 0 || level > 40 || !count)
        return eig::set_error(EIG_EINVAL, "sparse_grid_gl: dim in 1..16, level in 0..40");
    const int d = dim, w = level;
    std::vector<std::vector<double>> X(w + 2), W(w + 2);
    for (int i = 1; i <= w + 1; ++i) gauss_legendre(i, X[i], W[i]);
    const double tol = 1e-12;
    std::map<std::vector<long long>, std::pair<std::vector<double>, double>> acc;
    std::vector<int> idx(d, 1);
    // enumerate multi-indices i >= 1 with sum(i - 1) <= w
    while (true) {
        int q = 0;
        for (int n = 0; n < d; ++n) q += idx[n] - 1;
        if (q >= w - d + 1 && q <= w) {
            const double coef = ((w - q) % 2 ? -1.0 : 1.0) * binom(d - 1, w - q);
            std::vector<int> pick(d, 0);
            while (true) {
                std::vector<double> x(d);
                std::vector<long long> key(d);
                double wt = coef;
                for (int n = 0; n < d; ++n) {
                    x[n] = X[idx[n]][pick[n]];
                    wt *= W[idx[n]][pick[n]];
                    key[n] = std::llround(x[n] / tol);
                }
                auto it = acc.find(key);
                if (it == acc.end())
                    acc.emplace(key, std::make_pair(x, wt));
                else
                    it->second.second += wt;
                int n = 0;
                while (n < d && ++pick[n] == idx[n]) pick[n++] = 0;
                if (n == d) break;
            }
        }
        // next multi-index in the total-degree set
        int n = 0;
        while (n < d) {
            ++idx[n];
            int s = 0;
            for (int t = 0; t < d; ++t) s += idx[t] - 1;
            if (s <= w) break;
            idx[n] = 1;
            ++n;
        }
        if (n == d) break;
    }
    *count = (int32_t)acc.size();
    if ((int64_t)acc.size() > capacity || !nodes || !weights)
        return eig::set_error(EIG_EINVAL, "sparse_grid_gl: capacity too small");
    int r = 0;
    for (auto& kv : acc) {
        for (int n = 0; n < d; ++n) {
            const double u = kv.second.first[n];
            nodes[(size_t)r * d + n] =
                (lo && hi) ? lo[n] + 0.5 * (u + 1.0) * (hi[n] - lo[n]) : u;
        }
        weights[r] = kv.second.second;
        ++r;
    }
    return EIG_OK;
}
