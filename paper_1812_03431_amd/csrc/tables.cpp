// Host tables: Gauss-Legendre latitudes and orthonormal associated Legendre
// functions (Section 3), computed in long double.
#include <cfloat>
#include <cmath>

#include "internal.hpp"

namespace rexi {

// Roots of P_nlat by Newton's method from the estimate cos(pi (i + 3/4)/(nlat + 1/2)),
// P_n by k P_k = (2k-1) x P_{k-1} - (k-1) P_{k-2}, P'_n = n (x P_n - P_{n-1})/(x^2-1);
// weights 2 / ((1 - x^2) P'_n(x)^2).  Order: descending x (north to south).
void gauss_legendre(int nlat, std::vector<double>& mu, std::vector<double>& w) {
    mu.resize(nlat);
    w.resize(nlat);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int i = 0; i < nlat; ++i) {
        long double x = cosl(pi * (i + 0.75L) / (nlat + 0.5L));
        long double dp = 1;
        for (int it = 0; it < 100; ++it) {
            long double p0 = 1, p1 = x;
            for (int k = 2; k <= nlat; ++k) {
                const long double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (nlat == 1) { p1 = x; p0 = 1; }
            dp = nlat * (x * p1 - p0) / (x * x - 1);
            const long double dx = p1 / dp;
            x -= dx;
            if (fabsl(dx) < 1e-19L * fmaxl(1.0L, fabsl(x))) break;
        }
        {
            long double p0 = 1, p1 = x;
            for (int k = 2; k <= nlat; ++k) {
                const long double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = nlat * (x * p1 - p0) / (x * x - 1);
        }
        mu[i] = (double)x;
        w[i] = (double)(2.0L / ((1 - x * x) * dp * dp));
    }
}

// P_m^m = (1/sqrt2) prod_{k=1}^{m} sqrt((2k+1)/(2k)) (1-mu^2)^{m/2};
// P_n^m = (mu P_{n-1}^m - e_{n-1} P_{n-2}^m) / e_n,  e_n = sqrt((n^2-m^2)/(4n^2-1)).
// long double's exponent range holds the seeds down to the Gaussian latitude
// nearest a pole at T = 1023; results below 1e-300 are stored as 0.
std::vector<double> legendre_table(int T, const std::vector<double>& mu) {
    const int nlat = (int)mu.size();
    std::vector<double> out((size_t)nspec_of(T) * nlat);
    for (int j = 0; j < nlat; ++j) {
        const long double x = mu[j];
        const long double s = sqrtl(fmaxl(0.0L, 1 - x * x));
        long double pmm = 1.0L / sqrtl(2.0L);
        for (int m = 0; m <= T; ++m) {
            if (m > 0) pmm *= sqrtl((2.0L * m + 1) / (2.0L * m)) * s;
            const size_t base = (size_t)spec_offset(T, m) * nlat;
            long double pm2 = 0, pm1 = pmm;
            auto put = [&](int n, long double v) {
                double d = (double)v;
                if (fabs(d) < 1e-300) d = 0.0;
                out[base + (size_t)(n - m) * nlat + j] = d;
            };
            put(m, pm1);
            for (int n = m + 1; n <= T; ++n) {
                const long double en = sqrtl((long double)(n * n - m * m) / (4.0L * n * n - 1));
                const long double en1 =
                    (n - 1 > m) ? sqrtl((long double)((n - 1) * (n - 1) - m * m) / (4.0L * (n - 1) * (n - 1) - 1)) : 0.0L;
                const long double pn = (x * pm1 - en1 * pm2) / en;
                pm2 = pm1;
                pm1 = pn;
                put(n, pn);
            }
        }
    }
    return out;
}

}  // namespace rexi
