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

// Orthonormal associated Legendre functions by the three-term recurrence in n:
//   P_m^m = (1/sqrt2) prod_{k=1}^{m} sqrt((2k+1)/(2k)) (1-mu^2)^{m/2},
//   P_n^m = (mu P_{n-1}^m - e_{n-1} P_{n-2}^m) / e_n,  e_n = sqrt((n^2-m^2)/(4n^2-1)),
// i.e. P_n = a_n mu P_{n-1} - b_n P_{n-2} with a_n = 1/e_n, b_n = e_{n-1}/e_n
// (e_m = 0).  The device runs this recurrence itself; the host supplies the
// coefficients and, every `run` degrees, exact restart values.

// (a_n, b_n) for n > m in spectral order, [nspec][2] (zeros at n = m).
std::vector<double> legendre_coefs(int T) {
    std::vector<double> out(2 * (size_t)nspec_of(T), 0.0);
    for (int m = 0; m <= T; ++m) {
        const size_t base = (size_t)spec_offset(T, m);
        for (int n = m + 1; n <= T; ++n) {
            const long double en = sqrtl((long double)(n * n - m * m) / (4.0L * n * n - 1));
            const long double en1 =
                (n - 1 > m) ? sqrtl((long double)((n - 1) * (n - 1) - m * m) / (4.0L * (n - 1) * (n - 1) - 1)) : 0.0L;
            out[2 * (base + n - m)] = (double)(1.0L / en);
            out[2 * (base + n - m) + 1] = (double)(en1 / en);
        }
    }
    return out;
}

// Restart rows for runs of `run` degrees: for every order m and run r with
// n0 = m + run r <= T, row (run_base[m] + r) holds P_{n0-1}(mu_j) (0 at n0 = m)
// and P_{n0}(mu_j), layout [row][2][nmu].  Long double (its exponent range
// holds the seeds down to the Gaussian latitude nearest a pole at T = 1023);
// values below 1e-300 are stored as 0.
std::vector<double> legendre_restarts(int T, int run, const std::vector<double>& mu, std::vector<int>& run_base) {
    const int nmu = (int)mu.size();
    run_base.assign(T + 2, 0);
    for (int m = 0; m <= T; ++m) run_base[m + 1] = run_base[m] + (T + 1 - m + run - 1) / run;
    std::vector<double> out((size_t)run_base[T + 1] * 2 * nmu, 0.0);
    auto put = [&](int row, int which, int j, long double v) {
        double d = (double)v;
        if (fabs(d) < 1e-300) d = 0.0;
        out[((size_t)row * 2 + which) * nmu + j] = d;
    };
    for (int j = 0; j < nmu; ++j) {
        const long double x = mu[j];
        const long double s = sqrtl(fmaxl(0.0L, 1 - x * x));
        long double pmm = 1.0L / sqrtl(2.0L);
        for (int m = 0; m <= T; ++m) {
            if (m > 0) pmm *= sqrtl((2.0L * m + 1) / (2.0L * m)) * s;
            long double pm2 = 0, pm1 = pmm;  // P_{n-1}, P_n at n = m
            for (int n = m;; ++n) {
                if ((n - m) % run == 0) {
                    const int row = run_base[m] + (n - m) / run;
                    put(row, 0, j, pm2);
                    put(row, 1, j, pm1);
                }
                if (n == T) break;
                const int n1 = n + 1;
                const long double en = sqrtl((long double)(n1 * n1 - m * m) / (4.0L * n1 * n1 - 1));
                const long double en1 = (n > m) ? sqrtl((long double)(n * n - m * m) / (4.0L * n * n - 1)) : 0.0L;
                const long double pn = (x * pm1 - en1 * pm2) / en;
                pm2 = pm1;
                pm1 = pn;
            }
        }
    }
    return out;
}

}  // namespace rexi
