// REXI poles and weights (Section 4.1; renormalisation of Section 6.1).
//
// The paper takes the Gaussian's rational approximation from Haut et al.,
// Table 1, which is not reproduced in it, so the library fits its own:
//   psi(y) = (4 pi)^{-1/2} exp(-y^2/4) ~ Re sum_{l=-L}^{L} a_l / (i y + mu + i l),
// with a_{-l} = conj(a_l).  For fixed real mu the fit is linear least squares
// in 2L+1 real unknowns (solved by Householder QR in long double on y in
// [0, 96]); mu is chosen by a coarse scan followed by a golden-section search
// that minimises the largest error on y in [0, 240].
#include <cmath>
#include <map>
#include <mutex>

#include "internal.hpp"

namespace rexi {
namespace {

constexpr long double kPi = 3.141592653589793238462643383279502884L;

void basis_row(long double y, long double mu, int L, long double* row) {
    const long double mu2 = mu * mu;
    row[0] = mu / (mu2 + y * y);
    for (int l = 1; l <= L; ++l) {
        const long double yp = y + l, ym = y - l;
        const long double dp = mu2 + yp * yp, dm = mu2 + ym * ym;
        row[2 * l - 1] = mu / dp + mu / dm;
        row[2 * l] = yp / dp - ym / dm;
    }
}

long double target(long double y) { return expl(-0.25L * y * y) / sqrtl(4.0L * kPi); }

// min || A x - b ||_2 by Householder QR; A is rows x cols, row-major.
std::vector<long double> least_squares(std::vector<long double> A, std::vector<long double> b,
                                       int rows, int cols) {
    for (int k = 0; k < cols; ++k) {
        long double norm = 0;
        for (int i = k; i < rows; ++i) norm += A[(size_t)i * cols + k] * A[(size_t)i * cols + k];
        norm = sqrtl(norm);
        const long double akk = A[(size_t)k * cols + k];
        const long double alpha = akk > 0 ? -norm : norm;
        // v = x - alpha e1, stored in place of column k (rows k..)
        A[(size_t)k * cols + k] = akk - alpha;
        long double vnorm2 = 0;
        for (int i = k; i < rows; ++i) vnorm2 += A[(size_t)i * cols + k] * A[(size_t)i * cols + k];
        if (vnorm2 > 0) {
            for (int j = k + 1; j < cols; ++j) {
                long double dot = 0;
                for (int i = k; i < rows; ++i) dot += A[(size_t)i * cols + k] * A[(size_t)i * cols + j];
                const long double f = 2 * dot / vnorm2;
                for (int i = k; i < rows; ++i) A[(size_t)i * cols + j] -= f * A[(size_t)i * cols + k];
            }
            long double dot = 0;
            for (int i = k; i < rows; ++i) dot += A[(size_t)i * cols + k] * b[i];
            const long double f = 2 * dot / vnorm2;
            for (int i = k; i < rows; ++i) b[i] -= f * A[(size_t)i * cols + k];
        }
        A[(size_t)k * cols + k] = alpha;  // R diagonal
    }
    std::vector<long double> x(cols);
    for (int k = cols - 1; k >= 0; --k) {
        long double s = b[k];
        for (int j = k + 1; j < cols; ++j) s -= A[(size_t)k * cols + j] * x[j];
        x[k] = s / A[(size_t)k * cols + k];
    }
    return x;
}

struct Trial {
    long double mu;
    std::vector<long double> c;
    long double err;
};

Trial fit_at(long double mu, int L) {
    const int cols = 2 * L + 1;
    const int rows = 4801;  // y = 0, 0.02, ..., 96
    std::vector<long double> A((size_t)rows * cols), b(rows);
    for (int i = 0; i < rows; ++i) {
        const long double y = 0.02L * i;
        basis_row(y, mu, L, &A[(size_t)i * cols]);
        b[i] = target(y);
    }
    Trial t{mu, least_squares(std::move(A), std::move(b), rows, cols), 0};
    std::vector<long double> row(cols);
    long double err = 0;
    for (int i = 0; i <= 48000; ++i) {  // y = 0, 0.005, ..., 240
        const long double y = 0.005L * i;
        basis_row(y, mu, L, row.data());
        long double s = 0;
        for (int j = 0; j < cols; ++j) s += row[j] * t.c[j];
        err = fmaxl(err, fabsl(s - target(y)));
    }
    t.err = err;
    return t;
}

}  // namespace

GaussFit fit_gaussian(int L) {
    static std::mutex mtx;
    static std::map<int, GaussFit> cache;
    std::lock_guard<std::mutex> lock(mtx);
    auto hit = cache.find(L);
    if (hit != cache.end()) return hit->second;

    Trial best = fit_at(-6.0L, L);
    for (int i = 1; i <= 30; ++i) {
        Trial t = fit_at(-6.0L + 0.1L * i, L);
        if (t.err < best.err) best = t;
    }
    // golden-section refinement in [mu - 0.1, mu + 0.1]
    const long double gr = (sqrtl(5.0L) - 1) / 2;
    long double lo = best.mu - 0.1L, hi = best.mu + 0.1L;
    long double x1 = hi - gr * (hi - lo), x2 = lo + gr * (hi - lo);
    Trial t1 = fit_at(x1, L), t2 = fit_at(x2, L);
    while (hi - lo > 1e-4L) {
        if (t1.err < t2.err) {
            hi = x2; x2 = x1; t2 = t1;
            x1 = hi - gr * (hi - lo); t1 = fit_at(x1, L);
        } else {
            lo = x1; x1 = x2; t1 = t2;
            x2 = lo + gr * (hi - lo); t2 = fit_at(x2, L);
        }
    }
    for (const Trial* t : {&t1, &t2})
        if (t->err < best.err) best = *t;

    GaussFit f;
    f.mu = best.mu;
    f.max_err = (double)best.err;
    f.a.assign(2 * L + 1, cld(0, 0));
    f.a[L] = cld(best.c[0], 0);
    for (int l = 1; l <= L; ++l) {
        f.a[L + l] = cld(best.c[2 * l - 1], best.c[2 * l]);
        f.a[L - l] = std::conj(f.a[L + l]);
    }
    cache[L] = f;
    return f;
}

// b_m = e^{h^2} e^{-i m h} (Gaussian sum of Section 4.1; the value follows from
// Poisson summation with int psi_h(t) e^{-i xi t} dt = h e^{-h^2 xi^2}).
// Poles alpha_n = h (mu + i n); beta^c_n = h sum_{m+l=n} Re(b_m) a_l for the real
// part, beta^s_n likewise with Im(b_m); the real parts of the two rational
// sums add the mirrored poles, giving beta+- = (beta^c +- i beta^s)/2.
Poles make_poles(int M, double h, int L, int normalize) {
    const GaussFit f = fit_gaussian(L);
    const int N = 2 * (M + L) + 1;
    const long double hl = h;
    std::vector<cld> bc(N), bs(N);
    const long double eh2 = expl(hl * hl);
    for (int m = -M; m <= M; ++m) {
        const long double re = eh2 * cosl(m * hl), im = -eh2 * sinl(m * hl);
        for (int l = -L; l <= L; ++l) {
            bc[m + l + M + L] += hl * re * f.a[l + L];
            bs[m + l + M + L] += hl * im * f.a[l + L];
        }
    }
    std::vector<cld> al(N);
    cld g0(0, 0);
    for (int i = 0; i < N; ++i) {
        al[i] = cld(hl * f.mu, hl * (i - (M + L)));
        g0 += bc[i] / al[i];
    }
    Poles p;
    p.alpha.resize(N);
    p.beta_plus.resize(N);
    p.beta_minus.resize(N);
    const cld I(0, 1);
    for (int i = 0; i < N; ++i) {
        cld c = bc[i], s = bs[i];
        if (normalize) { c /= g0; s /= g0; }
        const cld bp = 0.5L * (c + I * s), bm = 0.5L * (c - I * s);
        p.alpha[i] = {(double)al[i].real(), (double)al[i].imag()};
        p.beta_plus[i] = {(double)bp.real(), (double)bp.imag()};
        p.beta_minus[i] = {(double)bm.real(), (double)bm.imag()};
    }
    return p;
}

}  // namespace rexi
