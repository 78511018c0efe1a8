// Spherical-harmonic transforms on gfx950 (Section 3).
//
// Analysis:  xi_n^m = sum_j w_j P_n^m(mu_j) F_j^m,  F_j^m = (1/nlon) sum_k xi(mu_j, lam_k) e^{-i m lam_k}
// Synthesis: xi(mu_j, lam_k) = sum_m c_m Re( sum_n xi_n^m P_n^m(mu_j) e^{i m lam_k} ), c_0 = 1, c_m = 2
// (the m = 0 term uses Re(xi_n^0)).
//
// Longitude: one workgroup per grid row runs a radix-2 FFT of length nlon in
// LDS.  Latitude: per zonal order m the Legendre sum is a small dense
// contraction (T+1-m degrees x nlat/2 latitudes x 2B real columns) and runs
// on FP64 MFMA (v_mfma_f64_16x16x4f64).  Gauss latitudes are symmetric about
// the equator and P_n^m(-mu) = (-1)^{n-m} P_n^m(mu), so only the northern
// half of the table is stored and each sum splits into an even part
// (F_j + F_{j'}) and an odd part (F_j - F_{j'}), j' = nlat-1-j.
//
// Workspace layout of the Fourier coefficients: Fw[m][j][c], c = 2b + {0: re, 1: im}.
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.hpp"

namespace rexi {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int bitrev(int x, int bits) { return (int)(__brev((unsigned)x) >> (32 - bits)); }

// In-place radix-2 decimation-in-time FFT of X[0..n) in LDS (input already
// in bit-reversed order).  tw[k] = exp(-2 pi i k / n), k < n/2; conj for the
// inverse direction.
__device__ void fft_lds(double2* X, const double2* __restrict__ tw, int n, bool inverse) {
    for (int len = 2; len <= n; len <<= 1) {
        const int half = len >> 1;
        const int step = n / len;
        for (int t = threadIdx.x; t < n / 2; t += blockDim.x) {
            const int grp = t / half, pos = t - grp * half;
            const int i = grp * len + pos, j = i + half;
            double2 w = tw[pos * step];
            if (inverse) w.y = -w.y;
            const double2 u = X[i], v0 = X[j];
            const double2 v = make_double2(fma(w.x, v0.x, -w.y * v0.y), fma(w.x, v0.y, w.y * v0.x));
            X[i] = make_double2(u.x + v.x, u.y + v.y);
            X[j] = make_double2(u.x - v.x, u.y - v.y);
        }
        __syncthreads();
    }
}

// grid [B][nlat][nlon] -> Fw[m][j][c] for m <= T.
__global__ void __launch_bounds__(256) k_fft_forward(const double* __restrict__ grid, double* __restrict__ Fw,
                                                     const double2* __restrict__ tw, int nlat, int nlon, int bits,
                                                     int T, int C) {
    extern __shared__ double2 X[];
    const int row = blockIdx.x;  // b * nlat + j
    const int b = row / nlat, j = row - b * nlat;
    const double* src = grid + (long long)row * nlon;
    for (int k = threadIdx.x; k < nlon; k += blockDim.x) X[bitrev(k, bits)] = make_double2(src[k], 0.0);
    __syncthreads();
    fft_lds(X, tw, nlon, false);
    const double inv = 1.0 / nlon;
    for (int m = threadIdx.x; m <= T; m += blockDim.x) {
        const double2 v = X[m];
        double* dst = Fw + ((long long)m * nlat + j) * C + 2 * b;
        dst[0] = v.x * inv;
        dst[1] = v.y * inv;
    }
}

// Fw[m][j][c] -> grid [B][nlat][nlon]
__global__ void __launch_bounds__(256) k_fft_inverse(const double* __restrict__ Fw, double* __restrict__ grid,
                                                     const double2* __restrict__ tw, int nlat, int nlon, int bits,
                                                     int T, int C) {
    extern __shared__ double2 X[];
    const int row = blockIdx.x;
    const int b = row / nlat, j = row - b * nlat;
    for (int k = threadIdx.x; k < nlon; k += blockDim.x) X[k] = make_double2(0.0, 0.0);
    __syncthreads();
    // spectrum of the real field: X[m] += F_m, X[n-m] += conj(F_m), X[0] = Re F_0
    for (int m = threadIdx.x; m <= T; m += blockDim.x) {
        const double* s = Fw + ((long long)m * nlat + j) * C + 2 * b;
        if (m == 0) X[0] = make_double2(s[0], 0.0);
        else X[m % nlon] = make_double2(s[0], s[1]);
    }
    __syncthreads();
    for (int m = 1 + threadIdx.x; m <= T; m += blockDim.x) {
        const double* s = Fw + ((long long)m * nlat + j) * C + 2 * b;
        const int q = (nlon - m % nlon) % nlon;
        X[q] = make_double2(X[q].x + s[0], X[q].y - s[1]);
    }
    __syncthreads();
    // bit-reverse permutation in place
    for (int k = threadIdx.x; k < nlon; k += blockDim.x) {
        const int r = bitrev(k, bits);
        if (r > k) {
            const double2 t = X[k];
            X[k] = X[r];
            X[r] = t;
        }
    }
    __syncthreads();
    fft_lds(X, tw, nlon, true);
    double* dst = grid + (long long)row * nlon;
    for (int k = threadIdx.x; k < nlon; k += blockDim.x) dst[k] = X[k].x;
}

// A tile of the Legendre contraction: order m, parity e (n - m even/odd),
// 16 consecutive degrees of that parity starting at index i0 (forward) or 16
// latitudes starting at j0 (inverse).
struct LegTile {
    int m, e, i0, pad;
};

// Forward: out[b][idx(m, n)] = sum_{j<H} P[m][n][j] w_j (F_j +- F_j')  (+ even, - odd)
__global__ void __launch_bounds__(64) k_legendre_forward(const LegTile* __restrict__ tiles,
                                                         const double* __restrict__ plm,
                                                         const double* __restrict__ wts,
                                                         const double* __restrict__ Fw, double* __restrict__ spec,
                                                         int T, int nlat, int H, int C) {
    const LegTile tl = tiles[blockIdx.x];
    const int lane = threadIdx.x;
    const int m = tl.m, e = tl.e;
    const long long so = spec_offset(T, m);
    const int row = lane & 15, kq = lane >> 4;
    const int n_a = m + e + 2 * (tl.i0 + row);  // degree of this lane's A row
    const bool row_ok = n_a <= T;
    const double* prow = plm + (so + (row_ok ? n_a - m : 0)) * H;
    const double sgn = e ? -1.0 : 1.0;
    for (int c0 = 0; c0 < C; c0 += 16) {
        const int col = c0 + (lane & 15);
        const bool col_ok = col < C;
        v4d acc = {0.0, 0.0, 0.0, 0.0};
        for (int j0 = 0; j0 < H; j0 += 4) {
            const int j = j0 + kq;
            double a = 0.0, bv = 0.0;
            if (j < H) {
                if (row_ok) a = prow[j];
                if (col_ok) {
                    const double f1 = Fw[((long long)m * nlat + j) * C + col];
                    const double f2 = Fw[((long long)m * nlat + (nlat - 1 - j)) * C + col];
                    bv = wts[j] * fma(sgn, f2, f1);
                }
            }
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc, 0, 0, 0);
        }
        // accumulator register r of lane l holds D[4 r + l/16][l % 16]
        if (col_ok) {
            const int b = col >> 1, ri = col & 1;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = 4 * r + kq;
                const int n = m + e + 2 * (tl.i0 + i);
                if (n <= T) spec[((long long)b * nspec_of(T) + so + (n - m)) * 2 + ri] = acc[r];
            }
        }
    }
}

// Inverse: for 16 latitudes j (< H): Fe = sum_{n-m even} P S, Fo = sum_{odd} P S;
// Fw[m][j] = Fe + Fo, Fw[m][j'] = Fe - Fo.
__global__ void __launch_bounds__(64) k_legendre_inverse(const LegTile* __restrict__ tiles,
                                                         const double* __restrict__ plm,
                                                         const double* __restrict__ spec,
                                                         double* __restrict__ Fw, int T, int nlat, int H, int C) {
    const LegTile tl = tiles[blockIdx.x];
    const int lane = threadIdx.x;
    const int m = tl.m;
    const long long so = spec_offset(T, m);
    const long long ns = nspec_of(T);
    const int L = T + 1 - m;
    const int jrow = tl.i0 + (lane & 15);  // A row = latitude
    const int kq = lane >> 4;
    const bool lat_ok = jrow < H;
    for (int c0 = 0; c0 < C; c0 += 16) {
        const int col = c0 + (lane & 15);
        const bool col_ok = col < C;
        const int b = col >> 1, ri = col & 1;
        v4d acc[2] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int cnt = (L - e + 1) / 2;  // degrees n = m + e + 2 i < m + L
            for (int i0 = 0; i0 < cnt; i0 += 4) {
                const int i = i0 + kq;
                double a = 0.0, bv = 0.0;
                if (i < cnt) {
                    const int n = m + e + 2 * i;
                    if (lat_ok) a = plm[(so + (n - m)) * H + jrow];
                    if (col_ok) bv = spec[((long long)b * ns + so + (n - m)) * 2 + ri];
                }
                acc[e] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc[e], 0, 0, 0);
            }
        }
        if (col_ok) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = tl.i0 + 4 * r + kq;
                if (j < H) {
                    Fw[((long long)m * nlat + j) * C + col] = acc[0][r] + acc[1][r];
                    Fw[((long long)m * nlat + (nlat - 1 - j)) * C + col] = acc[0][r] - acc[1][r];
                }
            }
        }
    }
}

}  // namespace

int sh_setup(rexi_plan* pl) {
    const int T = pl->T, nlat = pl->prm.nlat, nlon = pl->prm.nlon;
    if (nlat % 2) return fail(REXI_EUNSUPPORTED, "nlat must be even");
    if ((long long)nlon * 16 > 64 * 1024) return fail(REXI_EUNSUPPORTED, "nlon above 4096");
    pl->nlat = nlat;
    pl->nlon = nlon;
    pl->nhalf = nlat / 2;
    gauss_legendre(nlat, pl->mu, pl->w);
    std::vector<double> north(pl->mu.begin(), pl->mu.begin() + pl->nhalf);
    std::vector<double> plm = legendre_table(T, north);
    std::vector<double> wn(pl->w.begin(), pl->w.begin() + pl->nhalf);
    std::vector<double2> tw(nlon / 2);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int k = 0; k < nlon / 2; ++k) {
        const long double a = -2 * pi * k / nlon;
        tw[k] = make_double2((double)cosl(a), (double)sinl(a));
    }
    // tiles: forward (m, parity, 16 degrees); inverse (m, 16 latitudes)
    std::vector<LegTile> tf, ti;
    for (int m = 0; m <= T; ++m) {
        const int L = T + 1 - m;
        for (int e = 0; e < 2; ++e) {
            const int cnt = (L - e + 1) / 2;
            for (int i0 = 0; i0 < cnt; i0 += 16) tf.push_back(LegTile{m, e, i0, 0});
        }
        for (int j0 = 0; j0 < pl->nhalf; j0 += 16) ti.push_back(LegTile{m, 0, j0, 0});
    }
    // sort forward tiles so that the longest orders go first (roughly even waves)
    auto alloc = [&](void** p, size_t bytes) -> int {
        hipError_t e = hipMalloc(p, bytes ? bytes : 1);
        if (e != hipSuccess) return fail(REXI_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
        return REXI_OK;
    };
    int rc = alloc((void**)&pl->d_plm, plm.size() * sizeof(double));
    if (!rc) rc = alloc((void**)&pl->d_wts, wn.size() * sizeof(double));
    if (!rc) rc = alloc((void**)&pl->d_twiddle, tw.size() * sizeof(double2));
    if (!rc) rc = alloc((void**)&pl->d_four, (size_t)(T + 1) * nlat * 2 * pl->prm.max_fields * sizeof(double));
    if (!rc) rc = alloc((void**)&pl->d_tiles_f, tf.size() * sizeof(LegTile));
    if (!rc) rc = alloc((void**)&pl->d_tiles_i, ti.size() * sizeof(LegTile));
    if (rc) return rc;
    REXI_HIP(hipMemcpy(pl->d_plm, plm.data(), plm.size() * sizeof(double), hipMemcpyHostToDevice));
    REXI_HIP(hipMemcpy(pl->d_wts, wn.data(), wn.size() * sizeof(double), hipMemcpyHostToDevice));
    REXI_HIP(hipMemcpy(pl->d_twiddle, tw.data(), tw.size() * sizeof(double2), hipMemcpyHostToDevice));
    REXI_HIP(hipMemcpy(pl->d_tiles_f, tf.data(), tf.size() * sizeof(LegTile), hipMemcpyHostToDevice));
    REXI_HIP(hipMemcpy(pl->d_tiles_i, ti.data(), ti.size() * sizeof(LegTile), hipMemcpyHostToDevice));
    pl->ntiles_f = (int)tf.size();
    pl->ntiles_i = (int)ti.size();
    return REXI_OK;
}

void sh_release(rexi_plan* pl) {
    void* ptrs[] = {pl->d_plm, pl->d_wts, pl->d_twiddle, pl->d_four, pl->d_tiles_f, pl->d_tiles_i};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    pl->d_plm = nullptr;
    pl->d_wts = nullptr;
    pl->d_twiddle = nullptr;
    pl->d_four = nullptr;
    pl->d_tiles_f = nullptr;
    pl->d_tiles_i = nullptr;
}

int sh_run(rexi_plan* pl, const void* in, void* out, int B, bool forward, hipStream_t s) {
    if (pl->nlat == 0) return fail(REXI_EUNSUPPORTED, "plan was created without a grid (nlat = nlon = 0)");
    if (!in || !out) return fail(REXI_EINVAL, "NULL pointer");
    if (B < 1) return fail(REXI_EINVAL, "B must be >= 1");
    if (B > pl->prm.max_fields) return fail(REXI_EUNSUPPORTED, "B exceeds the plan's max_fields");
    const size_t gbytes = (size_t)B * pl->nlat * pl->nlon * sizeof(double);
    const size_t sbytes = (size_t)B * pl->nspec * 16;
    const char* a = (const char*)in;
    const char* o = (const char*)out;
    const size_t na = forward ? gbytes : sbytes, no = forward ? sbytes : gbytes;
    if (a < o + no && o < a + na) return fail(REXI_EALIAS, "output overlaps input");
    const int C = 2 * B;
    int bits = 0;
    while ((1 << bits) < pl->nlon) ++bits;
    const size_t lds = (size_t)pl->nlon * sizeof(double2);
    if (forward) {
        hipLaunchKernelGGL(k_fft_forward, dim3(B * pl->nlat), dim3(256), lds, s, (const double*)in, pl->d_four,
                           pl->d_twiddle, pl->nlat, pl->nlon, bits, pl->T, C);
        REXI_HIP(hipGetLastError());
        REXI_HIP(timed_begin(pl, REXI_KERNEL_LEGENDRE_FWD, s));
        hipLaunchKernelGGL(k_legendre_forward, dim3(pl->ntiles_f), dim3(64), 0, s, (const LegTile*)pl->d_tiles_f,
                           pl->d_plm, pl->d_wts, pl->d_four, (double*)out, pl->T, pl->nlat, pl->nhalf, C);
        REXI_HIP(hipGetLastError());
        REXI_HIP(timed_end(pl, REXI_KERNEL_LEGENDRE_FWD, s));
    } else {
        REXI_HIP(timed_begin(pl, REXI_KERNEL_LEGENDRE_INV, s));
        hipLaunchKernelGGL(k_legendre_inverse, dim3(pl->ntiles_i), dim3(64), 0, s, (const LegTile*)pl->d_tiles_i,
                           pl->d_plm, (const double*)in, pl->d_four, pl->T, pl->nlat, pl->nhalf, C);
        REXI_HIP(hipGetLastError());
        REXI_HIP(timed_end(pl, REXI_KERNEL_LEGENDRE_INV, s));
        hipLaunchKernelGGL(k_fft_inverse, dim3(B * pl->nlat), dim3(256), lds, s, pl->d_four, (double*)out,
                           pl->d_twiddle, pl->nlat, pl->nlon, bits, pl->T, C);
        REXI_HIP(hipGetLastError());
    }
    return REXI_OK;
}

}  // namespace rexi
