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

#include <algorithm>
#include <cmath>

#include "internal.hpp"

namespace rexi {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr size_t kLdsBytes = 64 * 1024;  // LDS per workgroup used by the Legendre kernels

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

// A run of Legendre tiles of one order m for one workgroup of four waves.
// Forward: tiles [t0, t1) over the even-parity degree tiles followed by the
// odd ones (16 degrees each), two per wave.  Inverse: tiles of 16
// latitudes, one per wave.
struct LegWork {
    int m, t0, t1, pad;
};

// Forward: out[b][idx(m, n)] = sum_{j<H} P[m][n][j] w_j (F_j +- F_j')  (+ even, - odd).
// The weighted even/odd Fourier blocks of m, E and O [H][C], are staged in
// LDS once per workgroup.  MFMA k index: within a block of 16 latitudes J,
// lane group kq at k-step s takes latitude J + 4 kq + s, so each lane reads
// four consecutive table entries of its degree.  Each wave keeps four
// independent accumulators (two degree tiles x two column tiles) in flight.
__global__ void __launch_bounds__(256) k_legendre_forward(const LegWork* __restrict__ work,
                                                          const double* __restrict__ plm,
                                                          const double* __restrict__ wts,
                                                          const double* __restrict__ Fw, double* __restrict__ spec,
                                                          int T, int nlat, int H, int Cs, int c_off, int C) {
    // columns [c_off, c_off + C) of the Fourier block (row stride Cs)
    extern __shared__ double lds[];
    const LegWork wk = work[blockIdx.x];
    const int m = wk.m;
    double* E = lds;            // [H][C]
    double* O = lds + H * C;    // [H][C]
    for (int idx = threadIdx.x; idx < H * C; idx += blockDim.x) {
        const int j = idx / C, c = idx - j * C;
        const double f1 = Fw[((long long)m * nlat + j) * Cs + c_off + c];
        const double f2 = Fw[((long long)m * nlat + (nlat - 1 - j)) * Cs + c_off + c];
        E[idx] = wts[j] * (f1 + f2);
        O[idx] = wts[j] * (f1 - f2);
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long long so = spec_offset(T, m);
    const long long ns = nspec_of(T);
    const int L = T + 1 - m;
    const int ne = ((L + 1) / 2 + 15) / 16;  // even-parity tiles
    const int row = lane & 15, kq = lane >> 4;
    for (int tb = wk.t0 + 2 * wave; tb < wk.t1; tb += 8) {
        int e[2], i0[2], nrow[2];
        bool rok[2];
        const double* prow[2];
        const double* B[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int t = tb + u;
            const bool tile_ok = t < wk.t1;
            e[u] = (tile_ok && t >= ne) ? 1 : 0;
            i0[u] = tile_ok ? (t - (e[u] ? ne : 0)) * 16 : 0;
            nrow[u] = m + e[u] + 2 * (i0[u] + row);
            rok[u] = tile_ok && nrow[u] <= T;
            prow[u] = plm + (so + (rok[u] ? nrow[u] - m : 0)) * H;
            B[u] = e[u] ? O : E;
        }
        for (int c0 = 0; c0 < C; c0 += 32) {
            const int col0 = c0 + (lane & 15), col1 = col0 + 16;
            const bool ok0 = col0 < C, ok1 = col1 < C;
            v4d acc[2][2] = {{{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}},
                             {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}}};
            for (int J = 0; J < H; J += 16) {
                const int jb = J + 4 * kq;
                double a[2][4];
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int s = 0; s < 4; ++s) a[u][s] = (rok[u] && jb + s < H) ? prow[u][jb + s] : 0.0;
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const bool jok = jb + s < H;
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        const double b0 = (ok0 && jok) ? B[u][(jb + s) * C + col0] : 0.0;
                        const double b1 = (ok1 && jok) ? B[u][(jb + s) * C + col1] : 0.0;
                        acc[u][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][s], b0, acc[u][0], 0, 0, 0);
                        acc[u][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][s], b1, acc[u][1], 0, 0, 0);
                    }
                }
            }
            // accumulator register r of lane l holds D[4 r + l/16][l % 16]
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int col = h ? col1 : col0;
                    if (!(h ? ok1 : ok0) || tb + u >= wk.t1) continue;
                    const int b = (c_off + col) >> 1, ri = (c_off + col) & 1;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int n = m + e[u] + 2 * (i0[u] + 4 * r + kq);
                        if (n <= T) spec[((long long)b * ns + so + (n - m)) * 2 + ri] = acc[u][h][r];
                    }
                }
        }
    }
}

// Inverse: for 16 latitudes j (< H): Fe = sum_{n-m even} P S, Fo = sum_{odd} P S;
// Fw[m][j] = Fe + Fo, Fw[m][j'] = Fe - Fo.  The spectral block of m, [L][C],
// is staged in LDS once per workgroup; each wave keeps four independent
// accumulators (two parities x two column tiles) in flight.
__global__ void __launch_bounds__(256) k_legendre_inverse(const LegWork* __restrict__ work,
                                                          const double* __restrict__ plm,
                                                          const double* __restrict__ spec,
                                                          double* __restrict__ Fw, int T, int nlat, int H, int Cs,
                                                          int c_off, int C) {
    extern __shared__ double lds[];
    const LegWork wk = work[blockIdx.x];
    const int m = wk.m;
    const long long so = spec_offset(T, m);
    const long long ns = nspec_of(T);
    const int L = T + 1 - m;
    double* Sm = lds;  // [L][C]
    for (int idx = threadIdx.x; idx < L * C; idx += blockDim.x) {
        const int d = idx / C, c = idx - d * C;
        Sm[idx] = spec[((long long)((c_off + c) >> 1) * ns + so + d) * 2 + ((c_off + c) & 1)];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int kq = lane >> 4;
    const int cnt0 = (L + 1) / 2, cnt1 = L / 2;  // degrees of each parity
    for (int t = wk.t0 + wave; t < wk.t1; t += 4) {
        const int j0 = t * 16;
        const int jrow = j0 + (lane & 15);  // A row = latitude
        const bool lat_ok = jrow < H;
        for (int c0 = 0; c0 < C; c0 += 32) {
            const int col0 = c0 + (lane & 15), col1 = col0 + 16;
            const bool ok0 = col0 < C, ok1 = col1 < C;
            v4d acc[2][2] = {{{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}},
                             {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}}};
            for (int i0 = 0; i0 < cnt0; i0 += 4) {
                const int i = i0 + kq;
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const bool iok = i < (e ? cnt1 : cnt0);
                    const int d = e + 2 * i;
                    const double a = (iok && lat_ok) ? plm[(so + d) * H + jrow] : 0.0;
                    const double b0 = (iok && ok0) ? Sm[d * C + col0] : 0.0;
                    const double b1 = (iok && ok1) ? Sm[d * C + col1] : 0.0;
                    acc[e][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b0, acc[e][0], 0, 0, 0);
                    acc[e][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b1, acc[e][1], 0, 0, 0);
                }
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int col = h ? col1 : col0;
                if (!(h ? ok1 : ok0)) continue;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int j = j0 + 4 * r + kq;
                    if (j < H) {
                        Fw[((long long)m * nlat + j) * Cs + c_off + col] = acc[0][h][r] + acc[1][h][r];
                        Fw[((long long)m * nlat + (nlat - 1 - j)) * Cs + c_off + col] = acc[0][h][r] - acc[1][h][r];
                    }
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
    // work: runs of at most 8 tiles of one order (a workgroup of four waves)
    std::vector<LegWork> tf, ti;
    for (int m = 0; m <= T; ++m) {
        const int L = T + 1 - m;
        const int nt = ((L + 1) / 2 + 15) / 16 + (L / 2 + 15) / 16;
        for (int t0 = 0; t0 < nt; t0 += 8) tf.push_back(LegWork{m, t0, std::min(nt, t0 + 8), 0});
        const int nl = (pl->nhalf + 15) / 16;
        for (int t0 = 0; t0 < nl; t0 += 4) ti.push_back(LegWork{m, t0, std::min(nl, t0 + 4), 0});
    }
    auto alloc = [&](void** p, size_t bytes) -> int {
        hipError_t e = hipMalloc(p, bytes ? bytes : 1);
        if (e != hipSuccess) return fail(REXI_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
        return REXI_OK;
    };
    int rc = alloc((void**)&pl->d_plm, plm.size() * sizeof(double));
    if (!rc) rc = alloc((void**)&pl->d_wts, wn.size() * sizeof(double));
    if (!rc) rc = alloc((void**)&pl->d_twiddle, tw.size() * sizeof(double2));
    if (!rc) rc = alloc((void**)&pl->d_four, (size_t)(T + 1) * nlat * 2 * pl->prm.max_fields * sizeof(double));
    if (!rc) rc = alloc((void**)&pl->d_tiles_f, tf.size() * sizeof(LegWork));
    if (!rc) rc = alloc((void**)&pl->d_tiles_i, ti.size() * sizeof(LegWork));
    if (rc) return rc;
    REXI_HIP(hipMemcpy(pl->d_plm, plm.data(), plm.size() * sizeof(double), hipMemcpyHostToDevice));
    REXI_HIP(hipMemcpy(pl->d_wts, wn.data(), wn.size() * sizeof(double), hipMemcpyHostToDevice));
    REXI_HIP(hipMemcpy(pl->d_twiddle, tw.data(), tw.size() * sizeof(double2), hipMemcpyHostToDevice));
    REXI_HIP(hipMemcpy(pl->d_tiles_f, tf.data(), tf.size() * sizeof(LegWork), hipMemcpyHostToDevice));
    REXI_HIP(hipMemcpy(pl->d_tiles_i, ti.data(), ti.size() * sizeof(LegWork), hipMemcpyHostToDevice));
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
        // column chunks whose E/O blocks fit 64 KB of LDS
        const int cc = std::max(2, std::min(C, (int)(kLdsBytes / (2 * sizeof(double) * pl->nhalf)) & ~1));
        for (int c0 = 0; c0 < C; c0 += cc) {
            const int w = std::min(cc, C - c0);
            const size_t lf = sizeof(double) * 2 * (size_t)pl->nhalf * w;
            hipLaunchKernelGGL(k_legendre_forward, dim3(pl->ntiles_f), dim3(256), lf, s,
                               (const LegWork*)pl->d_tiles_f, pl->d_plm, pl->d_wts, pl->d_four, (double*)out,
                               pl->T, pl->nlat, pl->nhalf, C, c0, w);
            REXI_HIP(hipGetLastError());
        }
        REXI_HIP(timed_end(pl, REXI_KERNEL_LEGENDRE_FWD, s));
    } else {
        REXI_HIP(timed_begin(pl, REXI_KERNEL_LEGENDRE_INV, s));
        const int cc = std::max(2, std::min(C, (int)(kLdsBytes / (sizeof(double) * (pl->T + 1))) & ~1));
        for (int c0 = 0; c0 < C; c0 += cc) {
            const int w = std::min(cc, C - c0);
            const size_t li = sizeof(double) * (size_t)(pl->T + 1) * w;
            hipLaunchKernelGGL(k_legendre_inverse, dim3(pl->ntiles_i), dim3(256), li, s,
                               (const LegWork*)pl->d_tiles_i, pl->d_plm, (const double*)in, pl->d_four, pl->T,
                               pl->nlat, pl->nhalf, C, c0, w);
            REXI_HIP(hipGetLastError());
        }
        REXI_HIP(timed_end(pl, REXI_KERNEL_LEGENDRE_INV, s));
        hipLaunchKernelGGL(k_fft_inverse, dim3(B * pl->nlat), dim3(256), lds, s, pl->d_four, (double*)out,
                           pl->d_twiddle, pl->nlat, pl->nlon, bits, pl->T, C);
        REXI_HIP(hipGetLastError());
    }
    return REXI_OK;
}

}  // namespace rexi
