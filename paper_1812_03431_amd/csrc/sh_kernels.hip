// Spherical-harmonic transforms on gfx950 (Section 3).
//
// Analysis:  xi_n^m = sum_j w_j P_n^m(mu_j) F_j^m,  F_j^m = (1/nlon) sum_k xi(mu_j, lam_k) e^{-i m lam_k}
// Synthesis: xi(mu_j, lam_k) = sum_m c_m Re( sum_n xi_n^m P_n^m(mu_j) e^{i m lam_k} ), c_0 = 1, c_m = 2
// (the m = 0 term uses Re(xi_n^0)).
//
// Longitude: one workgroup per pair of grid rows j, j' = nlat-1-j runs one
// complex FFT of length nlon (radix-2 stages taken in pairs) in LDS for both
// rows.  Latitude: per
// zonal order m the Legendre sum is a small dense contraction (T+1-m degrees
// x nlat/2 latitudes x 2B real columns) and runs on FP64 MFMA
// (v_mfma_f64_16x16x4f64).  Gauss latitudes are symmetric about the equator
// and P_n^m(-mu) = (-1)^{n-m} P_n^m(mu), so only northern latitudes are used
// and each sum splits into an even part (F_j + F_{j'}) and an odd part
// (F_j - F_{j'}).
//
// Fourier workspace (c = 2b + {0: re, 1: im}): the analysis writes the
// weighted even/odd parts EO[m][0|1][j][c], j < nlat/2; the synthesis writes
// partial sums Fw[slot][j][c] of degree segments, which the inverse FFT adds.
// Each (m, parity) plane and each slot is padded by kFourPad doubles.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "internal.hpp"

namespace rexi {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));


__device__ __forceinline__ int bitrev(int x, int bits) { return (int)(__brev((unsigned)x) >> (32 - bits)); }

// Plane strides of the Fourier workspace, in doubles: an EO plane [j][c] of one
// (order, parity) and a partial slot [row][c] are padded by kFourPad so that
// the lines of consecutive planes are not a power of two apart.
constexpr int kFourPad = 32;
__host__ __device__ __forceinline__ long long eo_plane(int H, int C) { return (long long)H * C + kFourPad; }
__host__ __device__ __forceinline__ long long slot_plane(int nlat, int C) { return (long long)nlat * C + kFourPad; }

__device__ __forceinline__ double2 cmul(double2 w, double2 v) {
    return make_double2(fma(w.x, v.x, -w.y * v.y), fma(w.x, v.y, w.y * v.x));
}

__device__ __forceinline__ double2 twiddle(const double2* tw, int k, bool inverse) {
    double2 w = tw[k];
    if (inverse) w.y = -w.y;
    return w;
}

// In-place decimation-in-time FFTs of nb arrays X + f n, f < nb, in LDS (input
// already in bit-reversed order); n = 2^bits.  tw[k] = exp(-2 pi i k / n),
// k < n/2; conj for the inverse direction.  Two radix-2 stages at a time: the
// butterflies of half-lengths h and 2h over the four elements pos + {0, h, 2h,
// 3h} of a block of 4h are one radix-4 step with the same arithmetic and
// twiddles, so a stage pair needs one barrier instead of two.  An odd number of
// stages starts with one radix-2 stage.  The FFTs are bound by the latency of
// their barrier-separated stages (11 -> 6 barriers at n = 2048).
__device__ void fft_lds(double2* X, const double2* tw, int bits, int nb, bool inverse) {
    const int n = 1 << bits, hb = bits - 1;
    int lh = 0;  // half-length 2^lh of the next radix-2 stage
    if (bits & 1) {
        const double2 w = twiddle(tw, 0, inverse);
        for (int t = threadIdx.x; t < (nb << hb); t += blockDim.x) {
            const int i = 2 * t, j = i + 1;
            const double2 u = X[i], v = cmul(w, X[j]);
            X[i] = make_double2(u.x + v.x, u.y + v.y);
            X[j] = make_double2(u.x - v.x, u.y - v.y);
        }
        __syncthreads();
        lh = 1;
    }
    for (; lh + 2 <= bits; lh += 2) {
        const int h = 1 << lh, q = hb - 1;  // n/4 = 2^q radix-4 steps per array
        for (int t = threadIdx.x; t < (nb << q); t += blockDim.x) {
            const int f = t >> q, tt = t & ((1 << q) - 1);
            const int grp = tt >> lh, pos = tt & (h - 1);
            const int i0 = f * n + (grp << (lh + 2)) + pos, i1 = i0 + h, i2 = i1 + h, i3 = i2 + h;
            const double2 w1 = twiddle(tw, pos << (hb - lh), inverse);
            const double2 w2 = twiddle(tw, pos << (q - lh), inverse);
            const double2 w3 = twiddle(tw, (pos + h) << (q - lh), inverse);
            const double2 a0 = X[i0], a2 = X[i2];
            const double2 t1 = cmul(w1, X[i1]), t3 = cmul(w1, X[i3]);
            const double2 c0 = make_double2(a0.x + t1.x, a0.y + t1.y), c1 = make_double2(a0.x - t1.x, a0.y - t1.y);
            const double2 c2 = make_double2(a2.x + t3.x, a2.y + t3.y), c3 = make_double2(a2.x - t3.x, a2.y - t3.y);
            const double2 u = cmul(w2, c2), v = cmul(w3, c3);
            X[i0] = make_double2(c0.x + u.x, c0.y + u.y);
            X[i2] = make_double2(c0.x - u.x, c0.y - u.y);
            X[i1] = make_double2(c1.x + v.x, c1.y + v.y);
            X[i3] = make_double2(c1.x - v.x, c1.y - v.y);
        }
        __syncthreads();
    }
}

// Two real rows share one complex FFT: with z = x + i y,
//   X_m = (Z_m + conj(Z_{N-m})) / 2,  Y_m = (Z_m - conj(Z_{N-m})) / (2 i),
// and for the inverse, Z = X + i Y of two Hermitian spectra transforms back to
// x + i y.  Rows j and j' = nlat-1-j of a field are the pair in both
// directions, which is also what the Legendre kernels' equatorial symmetry
// needs.  A workgroup takes the pair for a group of up to nb fields, so that
// the per-order outputs (forward) and inputs (inverse) of the group are
// contiguous.

// Rows j and j' (j < nlat/2) of fields b0 .. b0+nbr-1 -> the Gauss-weighted
// even and odd parts of their Fourier coefficients, for m <= T (T < nlon):
//   EO[m][0][j][c] = w_j s_j (F_j + F_j')_m,  EO[m][1][j][c] = w_j s_j (F_j - F_j')_m,
// F = (1/nlon) DFT, c = 2b + {0: re, 1: im}, s_j = rs[j] (rs may be NULL; it
// is symmetric about the equator).  These are the B operands of the forward
// Legendre contraction.  Workgroup g H + j takes field group g.
// Block b of a launch over G field groups x H row pairs -> (g, j). Blocks are
// dispatched to the eight XCDs in turn (b mod 8), so when H is a multiple of 8
// all G groups of row pair j get consecutive blocks of XCD j mod 8: the groups
// read (inverse) or write (forward) disjoint 16-byte pieces of the same
// spectral-side lines, which then meet in that XCD's L2 instead of being
// fetched or written back once per group. Otherwise the plain g-major split.
__device__ inline void fft_block(int b, int G, int H, int& g, int& j) {
    if ((H & 7) == 0) {
        const int i = b >> 3, q = i / G;
        g = i - q * G;
        j = q * 8 + (b & 7);
    } else {
        g = b / H;
        j = b - g * H;
    }
}

__global__ void __launch_bounds__(256) k_fft_forward(const double* __restrict__ grid, double* __restrict__ EO,
                                                     const double2* __restrict__ tw, const double* __restrict__ wts,
                                                     const double* __restrict__ rs, int nlat, int nlon, int bits,
                                                     int T, int C, int nb) {
    extern __shared__ double2 X[];  // [nb][nlon] data, then [nlon/2] twiddles
    const int H = nlat >> 1, nf = C >> 1;
    int g, j;
    fft_block(blockIdx.x, (nf + nb - 1) / nb, H, g, j);
    const int b0 = g * nb, nbr = min(nb, nf - b0);
    double2* tws = X + nb * nlon;
    for (int k = threadIdx.x; k < nlon / 2; k += blockDim.x) tws[k] = tw[k];
    constexpr int kU = 8;  // all loads of a thread issued before its stores
    const int tot = nbr * nlon;
    for (int k0 = 0; k0 < tot; k0 += kU * 256) {
        double vx[kU], vy[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int e = min(k0 + u * 256 + threadIdx.x, tot - 1);
            const int f = e >> bits, k = e & (nlon - 1);
            vx[u] = grid[((long long)(b0 + f) * nlat + j) * nlon + k];
            vy[u] = grid[((long long)(b0 + f) * nlat + (nlat - 1 - j)) * nlon + k];
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int e = k0 + u * 256 + threadIdx.x;
            if (e < tot) {
                const int f = e >> bits, k = e & (nlon - 1);
                X[f * nlon + bitrev(k, bits)] = make_double2(vx[u], vy[u]);
            }
        }
    }
    __syncthreads();
    fft_lds(X, tws, bits, nbr, false);
    const double sc = 0.5 * wts[j] * (rs ? rs[j] : 1.0) / nlon;
    for (int m = threadIdx.x; m <= T; m += blockDim.x) {
        double* e = EO + (long long)(m * 2) * eo_plane(H, C) + (long long)j * C + 2 * b0;
        double* o = e + eo_plane(H, C);
        for (int f = 0; f < nbr; ++f) {
            const double2 z = X[f * nlon + m], w = X[f * nlon + (nlon - m) % nlon];
            // 2 X_m = z + conj(w), 2 Y_m = -i (z - conj(w))
            const double xr2 = z.x + w.x, xi2 = z.y - w.y;
            const double yr2 = z.y + w.y, yi2 = w.x - z.x;
            e[2 * f] = sc * (xr2 + yr2);
            e[2 * f + 1] = sc * (xi2 + yi2);
            o[2 * f] = sc * (xr2 - yr2);
            o[2 * f + 1] = sc * (xi2 - yi2);
        }
    }
}

// Fw -> rows j and j' = nlat-1-j (j < nlat/2) of fields b0 .. b0+nbr-1 of the
// grid [B][nlat][nlon], scaled by rs[j] (rs may be NULL).  The Fourier
// coefficient of order m <= T (T < 1024) is the sum of the partial slots
// seg[m] .. seg[m+1]-1 of Fw[slot][row][c] (one per degree segment).
__global__ void __launch_bounds__(256) k_fft_inverse(const double* __restrict__ Fw, const int* __restrict__ seg,
                                                     double* __restrict__ grid, const double2* __restrict__ tw,
                                                     const double* __restrict__ rs, int nlat, int nlon, int bits,
                                                     int T, int C, int nb) {
    extern __shared__ double2 X[];  // [nb][nlon] data, then [nlon/2] twiddles
    const int H = nlat >> 1, nf = C >> 1;
    int g, j;
    fft_block(blockIdx.x, (nf + nb - 1) / nb, H, g, j);
    const int j2 = nlat - 1 - j;
    const int b0 = g * nb, nbr = min(nb, nf - b0);
    double2* tws = X + nb * nlon;
    for (int k = threadIdx.x; k < nb * nlon; k += blockDim.x) X[k] = make_double2(0.0, 0.0);
    for (int k = threadIdx.x; k < nlon / 2; k += blockDim.x) tws[k] = tw[k];
    __syncthreads();
    for (int f = 0; f < nbr; ++f) {
        double2* Xf = X + f * nlon;
        const int cb = 2 * (b0 + f);
        constexpr int kM = 4;  // orders per thread: m = tid + 256 k
        double2 fv[kM], gv[kM];  // coefficients of rows j and j'
#pragma unroll
        for (int k = 0; k < kM; ++k) {
            const int m = threadIdx.x + 256 * k;
            double2 v = make_double2(0.0, 0.0), w = v;
            if (m <= T) {
                for (int sl = seg[m]; sl < seg[m + 1]; ++sl) {
                    const double* p = Fw + sl * slot_plane(nlat, C) + (long long)j * C + cb;
                    const double* q = Fw + sl * slot_plane(nlat, C) + (long long)j2 * C + cb;
                    v.x += p[0];
                    v.y += p[1];
                    w.x += q[0];
                    w.y += q[1];
                }
                if (m == 0) v.y = w.y = 0.0;  // real fields: Re F_0
            }
            fv[k] = v;
            gv[k] = w;
        }
        // Z = X + i Y with X[m] = F_m, X[N-m] = conj(F_m) (and Y alike from G):
        // Z[m] += F_m + i G_m, Z[N-m] += conj(F_m) + i conj(G_m); two passes, as
        // orders past N/2 alias onto the same bins
#pragma unroll
        for (int k = 0; k < kM; ++k) {
            const int m = threadIdx.x + 256 * k;
            if (m <= T) Xf[m % nlon] = make_double2(fv[k].x - gv[k].y, fv[k].y + gv[k].x);
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kM; ++k) {
            const int m = threadIdx.x + 256 * k;
            if (m >= 1 && m <= T) {
                const int q = (nlon - m % nlon) % nlon;
                Xf[q] = make_double2(Xf[q].x + fv[k].x + gv[k].y, Xf[q].y - fv[k].y + gv[k].x);
            }
        }
        __syncthreads();
    }
    // bit-reverse permutation in place
    for (int e = threadIdx.x; e < nbr * nlon; e += blockDim.x) {
        const int f = e >> bits, k = e & (nlon - 1);
        const int r = bitrev(k, bits);
        if (r > k) {
            const double2 t = X[f * nlon + k];
            X[f * nlon + k] = X[f * nlon + r];
            X[f * nlon + r] = t;
        }
    }
    __syncthreads();
    fft_lds(X, tws, bits, nbr, true);
    const double sc = rs ? rs[j] : 1.0;
    // streaming stores for the contiguous output rows (measured 22.3 -> 20.5 us
    // at T256, 12 fields; scattered outputs elsewhere measured slower with them)
    for (int e = threadIdx.x; e < nbr * nlon; e += blockDim.x) {
        const int f = e >> bits, k = e & (nlon - 1);
        const double2 z = X[e];
        __builtin_nontemporal_store(z.x * sc, grid + ((long long)(b0 + f) * nlat + j) * nlon + k);
        __builtin_nontemporal_store(z.y * sc, grid + ((long long)(b0 + f) * nlat + j2) * nlon + k);
    }
}

// Legendre contractions with P_n^m generated on the device.  The table
// itself (34 MB at T256) is never stored: P follows from the three-term
// recurrence P_n = a_n mu P_{n-1} - b_n P_{n-2}, restarted from exact host
// values every kRun degrees (and, on grids of at most 128 northern latitudes,
// also every 8 degrees for the inverse), which keeps the FP64 recurrence
// error at a few ulp.
constexpr int kRun = 32;         // degrees per restart row of the table
constexpr int kInvSeg = 4 * kRun;  // degrees per inverse work item (at most; four parts)
constexpr int kFwdDeg = 32;      // degrees per forward run: two 16-row parity tiles
constexpr int kFwdLat = 128;     // latitudes per generated forward block
constexpr int kPtPitch = kFwdLat + 1;  // LDS row pitch of the generated tile (odd: spreads banks)
constexpr int kFwdGroup = 2;     // runs of one order per forward workgroup

// Forward work: nrun consecutive 32-degree runs of order m from degree n0,
// first restart row `row` (m = -1: an empty slot).  Inverse work: latitude
// tiles [t0, t1) of order m (one wave each) over the degree segment
// m + n0 .. m + n0 + kInvSeg - 1, written to partial slot `slot`.
struct LegRun {
    int m, n0, row, nrun;
};
struct LegWork {
    int m, t0, t1, run0;  // order, latitude tiles [t0, t1), restart row of degree m + n0 (the 8-degree table
                          // on grids of at most 128 northern latitudes, else the 32-degree one)
    int n0, slot;         // first degree (offset from m) of the segment, output slot
};

// value of v in lane l of the wave (l uniform)
__device__ __forceinline__ double readlane_f64(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __hiloint2double(hi, lo);
}

// FP64 MFMA of four independent 4x4x4 blocks (v_mfma_f64_4x4x4f64): with
// lane = 16 q + 4 b + p, block b takes A[i = p][k = q], B[k = q][j = p] and
// returns D[i = q][j = p] (layout checked on the GPU).  On this part it keeps
// the matrix pipe near its FP64 rate with one or two waves per SIMD, where the
// 16x16x4 shape needs about eight; and four-column groups fit any even column
// count with at most two idle columns.
__device__ __forceinline__ double mfma4(double a, double b, double c) {
    return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

// Forward: out[b][idx(m, n)] = sum_{j<H} P_n^m(mu_j) EO[m][r][j][c], r the
// parity of n - m (EO holds the Gauss-weighted even / odd Fourier parts),
// over the runs of one work item.  Per run the first kFwdLat threads generate
// the 32 degrees of their latitude into Pt[d][lat] (pitch kPtPitch), one
// barrier, then every wave contracts.  Wave w = 2 h + r owns degree parity r
// (16 degrees per run, four groups of 4) and the column groups [h NH,
// h NH + NH) of 4 columns.  Its MFMA blocks split the latitude sum: block b
// of k-step s takes latitudes 16 s + 4 b + q, so a lane's B operands are
// EO[16 s + 4 b + q][4 g + p], 8 x NH values per 128 latitudes, held in
// registers for the whole work item (larger grids reload them per block); the
// four blocks' partial sums are added across the row at the end of a run.
// The next run's restart values and recurrence coefficients (lane d holds
// degree n0 + d + 1, broadcast by readlane) are loaded before the MFMAs.
// Columns [c_off, c_off + C) of EO (row stride Cs), C <= 32.
template <int NH>
__global__ void __launch_bounds__(256) k_legendre_forward(const LegRun* __restrict__ runs,
                                                          const double* __restrict__ restart,
                                                          const double2* __restrict__ coef,
                                                          const double* __restrict__ mu,
                                                          const double* __restrict__ EO, double* __restrict__ spec,
                                                          int T, int H, int Cs, int c_off, int C) {
    __shared__ double Pt[kFwdDeg * kPtPitch];
    const LegRun rn = runs[blockIdx.x];
    if (rn.m < 0) return;  // padding slot of the XCD-ordered list
    const int m = rn.m;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int p = lane & 3, bq = (lane >> 2) & 3, q = lane >> 4;
    const int r = wave & 1, h = wave >> 1;  // degree parity and column half of this wave
    const bool busy = h * NH * 4 < C;        // the wave has columns
    const long long so = spec_offset(T, m);
    const long long ns = nspec_of(T);
    const double* Bsrc = EO + (long long)(m * 2 + r) * eo_plane(H, Cs) + c_off;
    int bcol[NH];
#pragma unroll
    for (int g = 0; g < NH; ++g) bcol[g] = min(4 * (h * NH + g) + p, C - 1);
    const int nblk = (H + kFwdLat - 1) / kFwdLat;
    const int nit = rn.nrun * nblk;  // (run, latitude block) iterations
    const bool gen = tid < kFwdLat;
    // prefetched inputs of the next iteration's generation
    auto fetch = [&](int it, double& pm, double& pc, double& x, double2& ab) {
        const int g = it / nblk, lb = (it - g * nblk) * kFwdLat;
        const int j = lb + tid;
        const bool ok = gen && j < H;
        const long long row = rn.row + g;
        pm = ok ? restart[(row * 2) * H + j] : 0.0;
        pc = ok ? restart[(row * 2 + 1) * H + j] : 0.0;
        x = ok ? mu[j] : 0.0;
        const int nc = rn.n0 + kFwdDeg * g + (lane & 31) + 1;
        ab = (nc <= T) ? coef[so + (nc - m)] : make_double2(0.0, 0.0);
    };
    double pm_n, pc_n, x_n;
    double2 ab_n;
    fetch(0, pm_n, pc_n, x_n, ab_n);
    double bf[kFwdLat / 16][NH];
    double acc[4][NH];
#pragma unroll
    for (int d = 0; d < 4; ++d)
#pragma unroll
        for (int g = 0; g < NH; ++g) acc[d][g] = 0.0;
    // A operand of degree group d, k-step s: Pt row 2 (4 d + p) + r, latitude 16 s + 4 bq + q
    const double* Ap = Pt + (2 * p + r) * kPtPitch + 4 * bq + q;
    for (int it = 0; it < nit; ++it) {
        const int g = it / nblk, blk = it - g * nblk;
        const int lb = blk * kFwdLat;
        if (it == 0 || nblk > 1) {
#pragma unroll
            for (int s = 0; s < kFwdLat / 16; ++s) {
                const int j = lb + 16 * s + 4 * bq + q;
#pragma unroll
                for (int c = 0; c < NH; ++c) bf[s][c] = (j < H) ? Bsrc[(long long)j * Cs + bcol[c]] : 0.0;
            }
        }
        if (it > 0) __syncthreads();  // the previous tile is consumed
        if (gen) {
            double pm = pm_n, pc = pc_n;
            const double x = x_n;
            const double2 ab = ab_n;
#pragma unroll
            for (int d = 0; d < kFwdDeg; ++d) {
                Pt[d * kPtPitch + tid] = pc;  // zero beyond T (zero coefficients there) and beyond H
                const double ca = readlane_f64(ab.x, d), cb = readlane_f64(ab.y, d);
                const double nx = fma(ca * x, pc, -cb * pm);
                pm = pc;
                pc = nx;
            }
        }
        if (it + 1 < nit) fetch(it + 1, pm_n, pc_n, x_n, ab_n);
        __syncthreads();
        if (busy) {
#pragma unroll
            for (int s = 0; s < kFwdLat / 16; ++s) {
                double av[4];
#pragma unroll
                for (int d = 0; d < 4; ++d) av[d] = Ap[8 * d * kPtPitch + 16 * s];
#pragma unroll
                for (int d = 0; d < 4; ++d)
#pragma unroll
                    for (int c = 0; c < NH; ++c) acc[d][c] = mfma4(av[d], bf[s][c], acc[d][c]);
            }
        }
        if (blk == nblk - 1) {
            // lane 16 q + 4 bq + p holds block bq's partial D[degree q][column p]
            // of each group; the row's four blocks are added by two exchanges
            const int n0 = rn.n0 + kFwdDeg * g;
#pragma unroll
            for (int d = 0; d < 4; ++d)
#pragma unroll
                for (int c = 0; c < NH; ++c) {
                    double v = acc[d][c];
                    v += __shfl_xor(v, 4);
                    v += __shfl_xor(v, 8);
                    acc[d][c] = 0.0;
                    const int col = 4 * (h * NH + c) + p;
                    const int n = n0 + 2 * (4 * d + q) + r;
                    if (busy && bq == 0 && col < C && n <= T) {
                        const int b = (c_off + col) >> 1, ri = (c_off + col) & 1;
                        spec[((long long)b * ns + so + (n - m)) * 2 + ri] = v;
                    }
                }
        }
    }
}

// Inverse: over one degree segment of order m, Fw[slot][j] = Fe + Fo,
// Fw[slot][j'] = Fe - Fo with Fe / Fo the sums of P_n^m(mu_j) S_n over the
// segment's n with n - m even / odd (the inverse FFT adds the segments of an
// order).  A segment is four parts (the shortest multiple of 8 degrees that
// covers it in four; restart rows every 8 degrees, grids of at most 128
// northern latitudes); a workgroup takes up to four
// 16-latitude tiles (one wave each) and stages in LDS the segment's spectral
// block Sm [Ls][C], its coefficient column and the exact restart values of
// its 64 latitudes at the start of each part.  The parts are the k index of
// the four-block MFMA: lane 16 kq + i (i < 16) runs the recurrence of
// latitude i over part kq from its own restart values, so no two lanes repeat
// a recurrence and no lane selects values, and per k-step s it holds
// A_even = P at part degree 2 s and A_odd = P at 2 s + 1 (parts start an even
// number of degrees from m, so the parity of n - m is that of the part
// degree).
// In the MFMA that lane is A[i & 3][kq] of block i >> 2: latitude i of the
// tile.  The blocks share B, the segment's coefficients
// S[Lp kq + 2 s (+1)][4 g + (lane & 3)] of column group g, and the result
// D[q][p] of lane 16 q + 4 b + p is latitude 4 b + q, column 4 g + p.
// Degrees past the segment need no checks: their coefficients are zero, so P
// is zero there, and the B reads are clamped into the block; parts that start
// past the segment have zero restart values.

// Stage the spectral block of degrees m + n0 .. m + n0 + Ls - 1 ([Ls][C],
// columns c_off..) and its coefficient column ([kInvSeg + 16], cf[k] for
// degree m + n0 + k, zero outside 1 <= k < Ls, so that every run's recurrence
// reads staged values up to its end).  The coefficients of one field form
// a contiguous run of 2 Ls <= 256 doubles: thread k takes double k of every
// field (coalesced), all loads before the stores.
__device__ __forceinline__ void stage_segment(long long so, long long ns, int Ls, int C, int c_off,
                                              const double* __restrict__ spec, const double2* __restrict__ coef,
                                              double* Sm, double2* cf) {
    const int k = threadIdx.x;
    const int nb = C >> 1;  // fields of this column chunk (C even, c_off even), <= 16
    const bool ok = k < 2 * Ls;
    double v[16];
#pragma unroll
    for (int f = 0; f < 16; ++f)
        v[f] = (ok && f < nb) ? spec[((long long)((c_off >> 1) + f) * ns + so) * 2 + k] : 0.0;
#pragma unroll
    for (int f = 0; f < 16; ++f)
        if (ok && f < nb) Sm[(k >> 1) * C + 2 * f + (k & 1)] = v[f];  // degree k/2, column 2f + re/im
    for (int q = threadIdx.x; q < kInvSeg + 16; q += blockDim.x)
        cf[q] = (q >= 1 && q < Ls) ? coef[so + q] : make_double2(0.0, 0.0);
}

template <int NG>
__global__ void __launch_bounds__(256) k_legendre_inverse(const LegWork* __restrict__ work,
                                                          const double* __restrict__ restart8,
                                                          const double2* __restrict__ coef,
                                                          const double* __restrict__ mu,
                                                          const double* __restrict__ spec,
                                                          double* __restrict__ Fw, int T, int nlat, int H, int Cs,
                                                          int c_off, int C) {
    extern __shared__ double lds[];
    const LegWork wk = work[blockIdx.x];
    if (wk.m < 0) return;  // padding slot of the XCD-ordered list
    const int m = wk.m;
    const int Ls = min(kInvSeg, T + 1 - m - wk.n0);  // degrees of this segment
    // part length: the shortest multiple of 8 (the restart rows' spacing)
    // that covers the segment in four parts, so short segments idle few MFMA
    // k slots
    const int Lp = 8 * ((Ls + 31) / 32);
    double* Sm = lds;                                        // [Ls][C]
    double2* cf = reinterpret_cast<double2*>(lds + Ls * C);  // [kInvSeg + 16] (Ls * C is even: C is)
    double* Rs = lds + Ls * C + 2 * (kInvSeg + 16);          // [4][2][64]
    stage_segment(spec_offset(T, m) + wk.n0, nspec_of(T), Ls, C, c_off, spec, coef, Sm, cf);
    const int jw = wk.t0 * 16;  // first latitude of the workgroup
    for (int k = threadIdx.x; k < 4 * 128; k += blockDim.x) {
        const int r = k >> 7, w = (k >> 6) & 1, j = min(jw + (k & 63), H - 1);
        Rs[k] = (r * Lp < Ls) ? restart8[((long long)(wk.run0 + r * (Lp / 8)) * 2 + w) * H + j] : 0.0;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int t = wk.t0 + wave;
    if (t >= wk.t1) return;  // no latitude tile for this wave (no barrier follows)
    const int i = lane & 15, kq = lane >> 4, p = lane & 3;
    const int j = t * 16 + i;
    const double x = (j < H) ? mu[j] : 0.0;
    const int rb = kq * Lp;  // first segment degree of this lane's part
    double pv = Rs[(kq * 2) * 64 + wave * 16 + i];
    double cu = Rs[(kq * 2 + 1) * 64 + wave * 16 + i];
    double ae[NG], ao[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) ae[g] = ao[g] = 0.0;
#pragma unroll 4
    for (int s = 0; s < Lp / 2; ++s) {
        const int d = rb + 2 * s;                          // even part degree (segment-relative)
        const double2 c1 = cf[d + 1], c2 = cf[d + 2];      // d + 2 <= 4 Lp <= kInvSeg
        const double* be = Sm + min(d, Ls - 1) * C + p;
        const double* bo = Sm + min(d + 1, Ls - 1) * C + p;
        const double a_e = cu;
        const double a_o = fma(c1.x * x, cu, -c1.y * pv);
        cu = fma(c2.x * x, a_o, -c2.y * a_e);
        pv = a_o;
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            const int cg = min(4 * g, C - 1 - p);  // column 4 g + p, clamped into the block
            ae[g] = mfma4(a_e, be[cg], ae[g]);
            ao[g] = mfma4(a_o, bo[cg], ao[g]);
        }
    }
    // lane 16 q + 4 b + p holds latitude 4 b + q of the tile, column 4 g + p
    const int jj = t * 16 + 4 * ((lane >> 2) & 3) + kq;
    if (jj < H) {
        double* fn = Fw + wk.slot * slot_plane(nlat, Cs) + (long long)jj * Cs + c_off;
        double* fs = Fw + wk.slot * slot_plane(nlat, Cs) + (long long)(nlat - 1 - jj) * Cs + c_off;
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            const int col = 4 * g + p;
            if (col < C) {
                // streaming stores: the partials go out while the kernel runs
                // instead of as dirty L2 lines written back at its end
                __builtin_nontemporal_store(ae[g] + ao[g], fn + col);
                __builtin_nontemporal_store(ae[g] - ao[g], fs + col);
            }
        }
    }
}

// Inverse for grids of more than 128 northern latitudes, on the 16x16x4
// shape (measured faster there: 674 against 1124 us at T1023 on 2048 x 1024
// with 16 fields; the four-block kernel's replicated operand reads, NG per
// parity per k-step, load the LDS more where the column groups are many).  The
// k index is four consecutive degrees: lanes (i = lane & 15, kq = lane >> 4)
// run the recurrence of latitude i in registers (the four kq lanes alike,
// restarted every kSeqRun degrees) and keep what their MFMA fragment needs:
// per k-step of 8 degrees base .. base + 7, A_even = P_{base + 2 kq},
// A_odd = P_{base + 2 kq + 1}; B is the spectral block of column tile
// (16 columns) and k; accumulator register q of lane l holds latitude row
// 4 q + l/16 of the tile and column l % 16.  Same segments, staging, slots and
// streaming stores as k_legendre_inverse.
constexpr int kSeqRun = 64;  // degrees between the sequential inverse's restarts (a multiple of kRun)

template <int NCT>
__global__ void __launch_bounds__(256) k_legendre_inverse_seq(const LegWork* __restrict__ work,
                                                          const double* __restrict__ restart,
                                                          const double2* __restrict__ coef,
                                                          const double* __restrict__ mu,
                                                          const double* __restrict__ spec,
                                                          double* __restrict__ Fw, int T, int nlat, int H, int Cs,
                                                          int c_off, int C) {
    extern __shared__ double lds[];
    const LegWork wk = work[blockIdx.x];
    if (wk.m < 0) return;  // padding slot of the XCD-ordered list
    const int m = wk.m;
    const int Ls = min(kInvSeg, T + 1 - m - wk.n0);  // degrees of this segment
    const int nr = (Ls + kSeqRun - 1) / kSeqRun;       // restarts of this segment
    double* Sm = lds;                                        // [Ls][C]
    double2* cf = reinterpret_cast<double2*>(lds + Ls * C);  // [kInvSeg + 16] (Ls * C is even: C is)
    double* Rs = lds + Ls * C + 2 * (kInvSeg + 16);          // [nr][2][64]
    stage_segment(spec_offset(T, m) + wk.n0, nspec_of(T), Ls, C, c_off, spec, coef, Sm, cf);
    const int jw = wk.t0 * 16;  // first latitude of the workgroup
    for (int k = threadIdx.x; k < nr * 128; k += blockDim.x) {
        const int r = k >> 7, w = (k >> 6) & 1, j = min(jw + (k & 63), H - 1);
        Rs[k] = restart[((long long)(wk.run0 + r * (kSeqRun / kRun)) * 2 + w) * H + j];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int t = wk.t0 + wave;
    if (t >= wk.t1) return;  // no latitude tile for this wave (no barrier follows)
    const int i = lane & 15, kq = lane >> 4;
    const int j = t * 16 + i;
    const double x = (j < H) ? mu[j] : 0.0;
    const int c0 = min(i, C - 1), c1 = min(16 + i, C - 1);
    v4d ae0 = {0.0, 0.0, 0.0, 0.0}, ao0 = ae0, ae1 = ae0, ao1 = ae0;
    for (int r = 0; r < nr; ++r) {
        double pv = Rs[(r * 2) * 64 + wave * 16 + i];
        double cu = Rs[(r * 2 + 1) * 64 + wave * 16 + i];
        const int kr = r * kSeqRun;
#pragma unroll
        for (int ks = 0; ks < kSeqRun; ks += 8) {
            const int kb = kr + ks;
            if (kb >= Ls) break;
            double2 cv[8];
#pragma unroll
            for (int d = 0; d < 8; ++d) cv[d] = cf[kb + d + 1];  // < Ls + 8 <= kInvSeg + 16
            const int de = min(kb + 2 * kq, Ls - 1), dd = min(kb + 2 * kq + 1, Ls - 1);
            const double b0 = Sm[de * C + c0], b1 = Sm[dd * C + c0];
            const double b2 = Sm[de * C + c1], b3 = Sm[dd * C + c1];
            double a_e = 0.0, a_o = 0.0;
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                if ((d & 1) == 0) a_e = (kq == (d >> 1)) ? cu : a_e;
                else a_o = (kq == (d >> 1)) ? cu : a_o;
                const double nx = fma(cv[d].x * x, cu, -cv[d].y * pv);
                pv = cu;
                cu = nx;
            }
            ae0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a_e, b0, ae0, 0, 0, 0);
            ao0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a_o, b1, ao0, 0, 0, 0);
            if constexpr (NCT > 1) {
                ae1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a_e, b2, ae1, 0, 0, 0);
                ao1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a_o, b3, ao1, 0, 0, 0);
            }
        }
    }
    // accumulator register q of lane l holds D[4 q + l/16][l % 16]: latitude
    // row 4 q + kq of the tile, column l % 16 of the column tile
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
        const int col = hh * 16 + i;
        if (hh >= NCT || col >= C) continue;
        const v4d ae = hh ? ae1 : ae0, ao = hh ? ao1 : ao0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int jj = t * 16 + 4 * q + kq;
            if (jj < H) {
                // streaming stores: the partials go out while the kernel runs
                // instead of as dirty L2 lines written back at its end
                __builtin_nontemporal_store(ae[q] + ao[q], Fw + wk.slot * slot_plane(nlat, Cs) + (long long)jj * Cs + c_off + col);
                __builtin_nontemporal_store(ae[q] - ao[q],
                                            Fw + wk.slot * slot_plane(nlat, Cs) + (long long)(nlat - 1 - jj) * Cs + c_off + col);
            }
        }
    }
}

// Vector transforms (Eq. (1): V = k x grad(psi) + grad(chi), lap psi = zeta,
// lap chi = delta; Section 3's scaled winds U = u cos(lat), V = v cos(lat)).
// On degree n, lap = -n(n+1)/a^2, and with eps_n = sqrt((n^2 - m^2)/(4n^2 - 1))
// the latitude derivative of the orthonormal P_n^m obeys
//   (1 - mu^2) dP_n^m/dmu = (n + 1) eps_n P_{n-1}^m - n eps_{n+1} P_{n+1}^m,

// Vector transforms (Eq. (1): V = k x grad(psi) + grad(chi), lap psi = zeta,
// lap chi = delta; Section 3's scaled winds U = u cos(lat), V = v cos(lat)).
// On degree n, lap = -n(n+1)/a^2, and with eps_n = sqrt((n^2 - m^2)/(4n^2 - 1))
// the latitude derivative of the orthonormal P_n^m obeys
//   (1 - mu^2) dP_n^m/dmu = (n + 1) eps_n P_{n-1}^m - n eps_{n+1} P_{n+1}^m,
// so the derivative moves a coefficient one degree up or down and U, V are
// fields of degree T + 1.  Written through zeta and delta directly:
//   U_n = -a [ eps_n zeta_{n-1} / n - eps_{n+1} zeta_{n+1} / (n+1) + i m delta_n / (n(n+1)) ]
//   V_n = -a [ i m zeta_n / (n(n+1)) - eps_n delta_{n-1} / n + eps_{n+1} delta_{n+1} / (n+1) ]
// over m <= n <= T + 1, terms outside m <= degree <= T dropped (the n = 0
// coefficient carries no wind).  Back: with A, B the analyses (degree T + 1)
// of u / cos(lat), v / cos(lat), integration by parts in mu gives
//   zeta_n  = (1/a) [ i m B_n - n eps_{n+1} A_{n+1} + (n+1) eps_n A_{n-1} ]
//   delta_n = (1/a) [ i m A_n + n eps_{n+1} B_{n+1} - (n+1) eps_n B_{n-1} ].
// Layouts: vd pair b at vd + b * stride (zeta, then delta at + nspec(T));
// uvs / ab fields 2b (U or A) and 2b + 1 (V or B) of nspec(T + 1) each.
__device__ __forceinline__ double eps_nm(int n, int m) {
    return sqrt((double)(n * n - m * m) / (4.0 * n * n - 1.0));
}

__global__ void __launch_bounds__(256) k_vd_to_uv_spec(const double2* __restrict__ vd, long long stride,
                                                      double2* __restrict__ uvs, int T, double a) {
    const int m = blockIdx.y, b = blockIdx.z;
    const int n = m + blockIdx.x * blockDim.x + threadIdx.x;
    if (n > T + 1) return;
    const double2* z = vd + b * stride + spec_offset(T, m) - m;  // z[k] = zeta_k^m, m <= k <= T
    const double2* d = z + nspec_of(T);
    double ur = 0.0, ui = 0.0, vr = 0.0, vi = 0.0;
    if (n - 1 >= max(m, 1)) {
        const double e = eps_nm(n, m) / n;
        const double2 zl = z[n - 1], dl = d[n - 1];
        ur += e * zl.x, ui += e * zl.y;
        vr -= e * dl.x, vi -= e * dl.y;
    }
    if (n + 1 <= T) {
        const double e = eps_nm(n + 1, m) / (n + 1);
        const double2 zh = z[n + 1], dh = d[n + 1];
        ur -= e * zh.x, ui -= e * zh.y;
        vr += e * dh.x, vi += e * dh.y;
    }
    if (m > 0 && n <= T) {
        const double f = (double)m / ((double)n * (n + 1));
        const double2 zc = z[n], dc = d[n];
        ur -= f * dc.y, ui += f * dc.x;
        vr -= f * zc.y, vi += f * zc.x;
    }
    const long long ns1 = nspec_of(T + 1), o = spec_offset(T + 1, m) + (n - m);
    uvs[(2LL * b) * ns1 + o] = make_double2(-a * ur, -a * ui);
    uvs[(2LL * b + 1) * ns1 + o] = make_double2(-a * vr, -a * vi);
}

__global__ void __launch_bounds__(256) k_uv_spec_to_vd(const double2* __restrict__ ab, double2* __restrict__ vd,
                                                      long long stride, int T, double a) {
    const int m = blockIdx.y, b = blockIdx.z;
    const int n = m + blockIdx.x * blockDim.x + threadIdx.x;
    if (n > T) return;
    const long long ns1 = nspec_of(T + 1);
    const double2* A = ab + (2LL * b) * ns1 + spec_offset(T + 1, m) - m;  // A[k], m <= k <= T + 1
    const double2* Bv = A + ns1;
    const double2 ac = A[n], bc = Bv[n], ah = A[n + 1], bh = Bv[n + 1];
    const double eh = n * eps_nm(n + 1, m);
    double zr = -m * bc.y - eh * ah.x, zi = m * bc.x - eh * ah.y;
    double dr = -m * ac.y + eh * bh.x, di = m * ac.x + eh * bh.y;
    if (n - 1 >= m) {
        const double el = (n + 1) * eps_nm(n, m);
        const double2 al = A[n - 1], bl = Bv[n - 1];
        zr += el * al.x, zi += el * al.y;
        dr -= el * bl.x, di -= el * bl.y;
    }
    const double ia = 1.0 / a;
    double2* z = vd + b * stride + spec_offset(T, m) + (n - m);
    z[0] = make_double2(zr * ia, zi * ia);
    z[nspec_of(T)] = make_double2(dr * ia, di * ia);
}


// Inverse LDS: a segment's block [kInvSeg][w], coefficient column and restart
// values (2 x 64 latitudes per run).
// Restart rows every 8 degrees (besides every kRun) for grids of at most 128
// northern latitudes, where the table stays small (9 MB at T256): the
// inverse's four parts then shrink with short segments.
bool restart8_rows(int H) { return H <= 128; }

size_t inverse_lds(int w) {
    return sizeof(double) * ((size_t)kInvSeg * w + 2 * (size_t)(kInvSeg + 16) + (size_t)(kInvSeg / kRun) * 128);
}

}  // namespace

namespace {

int device_alloc(void** p, size_t bytes) {
    hipError_t e = hipMalloc(p, bytes ? bytes : 1);
    if (e != hipSuccess) return fail(REXI_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    return REXI_OK;
}

// Restart rows, coefficients and work lists of the Legendre kernels for
// degrees 0..Tt over orders m <= the plan's T.
int leg_build(rexi_plan* pl, LegTables& t, int Tt, const std::vector<double>& north) {
    const int T = pl->T, H = pl->nhalf;
    std::vector<int> run_base, run_base8;
    std::vector<double> restart = legendre_restarts(Tt, kRun, north, run_base);
    std::vector<double> lcoef = legendre_coefs(Tt);
    const bool reg = restart8_rows(H);
    std::vector<double> restart8;
    if (reg) restart8 = legendre_restarts(Tt, 8, north, run_base8);
    // forward: one workgroup per kFwdGroup consecutive 32-degree runs of an
    // order.  Workgroups go to the eight
    // XCDs round-robin by index, so slot s is filled from the queue of XCD
    // s % 8, which holds the runs of the orders m = s (mod 8), longest orders
    // first: all runs of an order share one XCD and its L2, where the order's
    // Fourier block is read from HBM once.  Queues that run out early are
    // padded with empty slots (m = -1).
    // inverse: four latitude tiles (one per wave) of one degree segment of one
    // order.  One order per workgroup: pairing m with T - m evens the work per
    // wave but halves the waves in flight, which measured slower (30 vs 26 us
    // at T256)
    constexpr int kXcd = 8;
    std::vector<std::vector<LegRun>> q(kXcd);
    for (int m = 0; m <= T; ++m) {
        const int nr = (Tt - m) / kFwdDeg + 1;
        for (int r = 0; r < nr; r += kFwdGroup)
            q[m % kXcd].push_back(LegRun{m, m + kFwdDeg * r, run_base[m] + r * (kFwdDeg / kRun),
                                         std::min(kFwdGroup, nr - r)});
    }
    // within a queue, two-run items before one-run items (the longest
    // orders still first among equals): the short items fill in at the end
    for (auto& v : q)
        std::stable_sort(v.begin(), v.end(), [](const LegRun& a, const LegRun& b) { return a.nrun > b.nrun; });
    size_t qmax = 0;
    for (auto& v : q) qmax = std::max(qmax, v.size());
    std::vector<LegRun> tf;
    for (size_t k = 0; k < qmax; ++k)
        for (int x = 0; x < kXcd; ++x) tf.push_back(k < q[x].size() ? q[x][k] : LegRun{-1, 0, 0, 0});
    while (!tf.empty() && tf.back().m < 0) tf.pop_back();
    std::vector<LegWork> ti;
    const int nl = (H + 15) / 16;
    // inverse: degree segments of kInvSeg, partial slot seg[m] + s; full
    // segments first (the longest work), each with its latitude tile groups.
    // All tile groups of a segment stage the same spectral block, so they go
    // to one XCD: the k-th segment in this order to the queue of XCD k % 8,
    // and the queues are interleaved like the forward list (padding m = -1).
    // Spread over the XCDs, each group read the block from HBM again (9x the
    // spectral bytes at T1023 on 1024 latitudes).
    std::vector<int> seg(T + 2, 0);
    for (int m = 0; m <= T; ++m) seg[m + 1] = seg[m] + (Tt - m) / kInvSeg + 1;
    std::vector<std::vector<LegWork>> qi(kXcd);
    int kseg = 0;
    for (int full = 1; full >= 0; --full)
        for (int m = 0; m <= T; ++m)
            for (int n0 = 0; m + n0 <= Tt; n0 += kInvSeg) {
                if ((m + n0 + kInvSeg - 1 <= Tt) != (full == 1)) continue;
                std::vector<LegWork>& dst = qi[kseg++ % kXcd];
                for (int t0 = 0; t0 < nl; t0 += 4)
                    dst.push_back(LegWork{m, t0, std::min(nl, t0 + 4),
                                          reg ? run_base8[m] + n0 / 8 : run_base[m] + n0 / kRun, n0,
                                          seg[m] + n0 / kInvSeg});
            }
    size_t qimax = 0;
    for (auto& v : qi) qimax = std::max(qimax, v.size());
    for (size_t k = 0; k < qimax; ++k)
        for (int x = 0; x < kXcd; ++x) ti.push_back(k < qi[x].size() ? qi[x][k] : LegWork{-1, 0, 0, 0, 0, 0});
    while (!ti.empty() && ti.back().m < 0) ti.pop_back();
    t.nslots = seg[T + 1];
    t.T = Tt;
    int rc = device_alloc((void**)&t.d_restart, restart.size() * sizeof(double));
    if (!rc && reg) rc = device_alloc((void**)&t.d_restart8, restart8.size() * sizeof(double));
    if (!rc) rc = device_alloc((void**)&t.d_lcoef, lcoef.size() * sizeof(double));
    if (!rc) rc = device_alloc((void**)&t.d_tiles_f, tf.size() * sizeof(LegRun));
    if (!rc) rc = device_alloc((void**)&t.d_tiles_i, ti.size() * sizeof(LegWork));
    if (!rc) rc = device_alloc((void**)&t.d_seg, seg.size() * sizeof(int));
    if (rc) return rc;
    REXI_HIP(hipMemcpy(t.d_restart, restart.data(), restart.size() * sizeof(double), hipMemcpyHostToDevice));
    if (reg)
        REXI_HIP(hipMemcpy(t.d_restart8, restart8.data(), restart8.size() * sizeof(double), hipMemcpyHostToDevice));
    REXI_HIP(hipMemcpy(t.d_lcoef, lcoef.data(), lcoef.size() * sizeof(double), hipMemcpyHostToDevice));
    REXI_HIP(hipMemcpy(t.d_tiles_f, tf.data(), tf.size() * sizeof(LegRun), hipMemcpyHostToDevice));
    REXI_HIP(hipMemcpy(t.d_tiles_i, ti.data(), ti.size() * sizeof(LegWork), hipMemcpyHostToDevice));
    REXI_HIP(hipMemcpy(t.d_seg, seg.data(), seg.size() * sizeof(int), hipMemcpyHostToDevice));
    t.ntiles_f = (int)tf.size();
    t.ntiles_i = (int)ti.size();
    return REXI_OK;
}

void leg_release(LegTables& t) {
    void* ptrs[] = {t.d_restart, t.d_restart8, t.d_lcoef, t.d_tiles_f, t.d_tiles_i, t.d_seg};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    t = LegTables{};
}

constexpr size_t kFftLds = 96 * 1024;  // LDS allowance of the FFT kernels (nlon = 4096 needs 96 KB)

int fft_bits(int nlon) {
    int bits = 0;
    while ((1 << bits) < nlon) ++bits;
    return bits;
}

// grid rows [nf][nlat][nlon] -> Fw (C = 2 nf columns), row scale rs or NULL
// Fields per FFT workgroup.  One: the FFTs are latency-bound per workgroup,
// and four fields per workgroup (contiguous per-order writes, a quarter of the
// workgroups) measured slower at T256, 12 fields (22.4 / 30.7 us against
// 16.5 / 20.9 us forward / inverse).
int fft_group(const rexi_plan*, int) { return 1; }

int fft_forward(rexi_plan* pl, const double* grid, int nf, const double* rs, hipStream_t s) {
    const int nb = fft_group(pl, nf);
    const size_t lds = (size_t)(nb * pl->nlon + pl->nlon / 2) * sizeof(double2);
    hipLaunchKernelGGL(k_fft_forward, dim3(((nf + nb - 1) / nb) * pl->nhalf), dim3(256), lds, s, grid, pl->d_four,
                       pl->d_twiddle, pl->d_wts, rs, pl->nlat, pl->nlon, fft_bits(pl->nlon), pl->T, 2 * nf, nb);
    REXI_HIP(hipGetLastError());
    return REXI_OK;
}

int fft_inverse(rexi_plan* pl, const LegTables& t, double* grid, int nf, const double* rs, hipStream_t s) {
    const int nb = fft_group(pl, nf);
    const size_t lds = (size_t)(nb * pl->nlon + pl->nlon / 2) * sizeof(double2);
    hipLaunchKernelGGL(k_fft_inverse, dim3(((nf + nb - 1) / nb) * pl->nhalf), dim3(256), lds, s, pl->d_four, t.d_seg,
                       grid, pl->d_twiddle, rs, pl->nlat, pl->nlon, fft_bits(pl->nlon), pl->T, 2 * nf, nb);
    REXI_HIP(hipGetLastError());
    return REXI_OK;
}

// EO (C columns) -> spec [C/2][nspec(t.T)], in launches of at most 32 columns;
// each wave takes half of a launch's four-column groups
int leg_forward(rexi_plan* pl, const LegTables& t, double* spec, int C, hipStream_t s) {
    const double2* coef = reinterpret_cast<const double2*>(t.d_lcoef);
    for (int c0 = 0; c0 < C; c0 += 32) {
        const int w = std::min(32, C - c0);
        const int nh = ((w + 3) / 4 + 1) / 2;  // column groups per wave, 1..4
        const dim3 g(t.ntiles_f), b(256);
        const LegRun* rl = (const LegRun*)t.d_tiles_f;
#define REXI_FWD(NH_)                                                                                           \
    if (nh == NH_)                                                                                              \
    hipLaunchKernelGGL(k_legendre_forward<NH_>, g, b, 0, s, rl, t.d_restart, coef, pl->d_mu, pl->d_four, spec, \
                       t.T, pl->nhalf, C, c0, w)
        REXI_FWD(1);
        REXI_FWD(2);
        REXI_FWD(3);
        REXI_FWD(4);
#undef REXI_FWD
        REXI_HIP(hipGetLastError());
    }
    return REXI_OK;
}

// spec [C/2][nspec(t.T)] -> partial slots of Fw (C columns), in launches of
// at most 32 columns (up to eight four-column groups)
int leg_inverse(rexi_plan* pl, const LegTables& t, const double* spec, int C, hipStream_t s) {
    const int H = pl->nhalf;
    const double2* coef = reinterpret_cast<const double2*>(t.d_lcoef);
    for (int c0 = 0; c0 < C; c0 += 32) {
        const int w = std::min(32, C - c0);
        const int ng = (w + 3) / 4;
        const size_t li = inverse_lds(w);
        const LegWork* wl = (const LegWork*)t.d_tiles_i;
        const dim3 g(t.ntiles_i), b(256);
        const bool reg = restart8_rows(H);  // the plan holds restart rows every 8 degrees
        if (!reg) {
            if (w > 16)
                hipLaunchKernelGGL(k_legendre_inverse_seq<2>, g, b, li, s, wl, t.d_restart, coef, pl->d_mu, spec,
                                   pl->d_four, t.T, pl->nlat, H, C, c0, w);
            else
                hipLaunchKernelGGL(k_legendre_inverse_seq<1>, g, b, li, s, wl, t.d_restart, coef, pl->d_mu, spec,
                                   pl->d_four, t.T, pl->nlat, H, C, c0, w);
            REXI_HIP(hipGetLastError());
            continue;
        }

#define REXI_INV(NG_)                                                                                        \
    if (ng == NG_)                                                                                           \
    hipLaunchKernelGGL(k_legendre_inverse<NG_>, g, b, li, s, wl, t.d_restart8, coef, pl->d_mu, spec, pl->d_four, \
                       t.T, pl->nlat, H, C, c0, w)
        REXI_INV(1);
        REXI_INV(2);
        REXI_INV(3);
        REXI_INV(4);
        REXI_INV(5);
        REXI_INV(6);
        REXI_INV(7);
        REXI_INV(8);
#undef REXI_INV
        REXI_HIP(hipGetLastError());
    }
    return REXI_OK;
}

}  // namespace

int sh_setup(rexi_plan* pl) {
    const int T = pl->T, nlat = pl->prm.nlat, nlon = pl->prm.nlon;
    // the plan's parameter check has already refused these (before allocating)
    if (nlat % 2 || nlat > 2048 || nlon > 4096) return fail(REXI_EINVAL, "grid outside the supported range");
    pl->nlat = nlat;
    pl->nlon = nlon;
    pl->nhalf = nlat / 2;
    const int H = pl->nhalf;
    gauss_legendre(nlat, pl->mu, pl->w);
    std::vector<double> north(pl->mu.begin(), pl->mu.begin() + H);
    std::vector<double> wn(pl->w.begin(), pl->w.begin() + H);
    std::vector<double> rcos(nlat);
    for (int j = 0; j < nlat; ++j) {
        const long double x = pl->mu[j];
        rcos[j] = (double)(1.0L / sqrtl((1.0L - x) * (1.0L + x)));
    }
    std::vector<double2> tw(nlon / 2);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int k = 0; k < nlon / 2; ++k) {
        const long double a = -2 * pi * k / nlon;
        tw[k] = make_double2((double)cosl(a), (double)sinl(a));
    }
    int rc = leg_build(pl, pl->leg, T, north);
    if (!rc) rc = leg_build(pl, pl->legv, T + 1, north);
    if (!rc) rc = device_alloc((void**)&pl->d_mu, north.size() * sizeof(double));
    if (!rc) rc = device_alloc((void**)&pl->d_wts, wn.size() * sizeof(double));
    if (!rc) rc = device_alloc((void**)&pl->d_rcos, rcos.size() * sizeof(double));
    if (!rc) rc = device_alloc((void**)&pl->d_twiddle, tw.size() * sizeof(double2));
    // Fourier workspace: the forward's even/odd parts of T + 1 orders, or the
    // inverse's partial slots
    const size_t nsl = std::max<size_t>(T + 1, std::max(pl->leg.nslots, pl->legv.nslots));
    // (T + 1) x 2 EO planes or nslots slots, each padded by kFourPad
    if (!rc) rc = device_alloc((void**)&pl->d_four, nsl * (nlat * 2 * pl->prm.max_fields + 2 * kFourPad) * sizeof(double));
    if (!rc && pl->prm.max_fields >= 2)
        rc = device_alloc((void**)&pl->d_vspec, (size_t)pl->prm.max_fields * nspec_of(T + 1) * sizeof(double2));
    if (rc) return rc;
    REXI_HIP(hipMemcpy(pl->d_mu, north.data(), north.size() * sizeof(double), hipMemcpyHostToDevice));
    REXI_HIP(hipMemcpy(pl->d_wts, wn.data(), wn.size() * sizeof(double), hipMemcpyHostToDevice));
    REXI_HIP(hipMemcpy(pl->d_rcos, rcos.data(), rcos.size() * sizeof(double), hipMemcpyHostToDevice));
    REXI_HIP(hipMemcpy(pl->d_twiddle, tw.data(), tw.size() * sizeof(double2), hipMemcpyHostToDevice));
    // dynamic LDS above 64 KB per workgroup
    REXI_HIP(hipFuncSetAttribute((const void*)k_fft_forward, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kFftLds));
    REXI_HIP(hipFuncSetAttribute((const void*)k_fft_inverse, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kFftLds));

    return REXI_OK;
}

void sh_release(rexi_plan* pl) {
    leg_release(pl->leg);
    leg_release(pl->legv);
    void* ptrs[] = {pl->d_mu, pl->d_wts, pl->d_rcos, pl->d_twiddle, pl->d_four, pl->d_vspec};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    pl->d_mu = nullptr;
    pl->d_wts = nullptr;
    pl->d_rcos = nullptr;
    pl->d_twiddle = nullptr;
    pl->d_four = nullptr;
    pl->d_vspec = nullptr;
}

static bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
    const char* x = (const char*)a;
    const char* y = (const char*)b;
    return x < y + nb && y < x + na;
}

int sh_run(rexi_plan* pl, const void* in, void* out, int B, bool forward, hipStream_t s) {
    if (pl->nlat == 0) return fail(REXI_EUNSUPPORTED, "plan was created without a grid (nlat = nlon = 0)");
    if (!in || !out) return fail(REXI_EINVAL, "NULL pointer");
    if (B < 1) return fail(REXI_EINVAL, "B must be >= 1");
    if (B > pl->prm.max_fields) return fail(REXI_EUNSUPPORTED, "B exceeds the plan's max_fields");
    const size_t gbytes = (size_t)B * pl->nlat * pl->nlon * sizeof(double);
    const size_t sbytes = (size_t)B * pl->nspec * 16;
    if (overlaps(in, forward ? gbytes : sbytes, out, forward ? sbytes : gbytes))
        return fail(REXI_EALIAS, "output overlaps input");
    const int C = 2 * B;
    int rc;
    if (forward) {
        if ((rc = fft_forward(pl, (const double*)in, B, nullptr, s))) return rc;
        REXI_HIP(timed_begin(pl, REXI_KERNEL_LEGENDRE_FWD, s));
        if ((rc = leg_forward(pl, pl->leg, (double*)out, C, s))) return rc;
        REXI_HIP(timed_end(pl, REXI_KERNEL_LEGENDRE_FWD, s));
    } else {
        REXI_HIP(timed_begin(pl, REXI_KERNEL_LEGENDRE_INV, s));
        if ((rc = leg_inverse(pl, pl->leg, (const double*)in, C, s))) return rc;
        REXI_HIP(timed_end(pl, REXI_KERNEL_LEGENDRE_INV, s));
        if ((rc = fft_inverse(pl, pl->leg, (double*)out, B, nullptr, s))) return rc;
    }
    return REXI_OK;
}

// Vector transforms: vd pairs (zeta, delta) at stride `stride` complex entries
// <-> winds uv [B][2][nlat][nlon].  Through the degree-(T+1) fields of
// u / cos(lat), v / cos(lat) (forward) or u cos(lat), v cos(lat) (inverse) in
// d_vspec; the 1 / cos(lat) row scale is applied inside the FFT kernels.
int sh_vec_run(rexi_plan* pl, const void* in, void* out, long long stride, int B, bool to_uv, hipStream_t s) {
    if (pl->nlat == 0) return fail(REXI_EUNSUPPORTED, "plan was created without a grid (nlat = nlon = 0)");
    if (!in || !out) return fail(REXI_EINVAL, "NULL pointer");
    if (B < 1) return fail(REXI_EINVAL, "B must be >= 1");
    if (stride < 2 * pl->nspec) return fail(REXI_EINVAL, "stride must be at least 2 nspec");
    if (2LL * B > pl->prm.max_fields) return fail(REXI_EUNSUPPORTED, "2 B exceeds the plan's max_fields");
    const size_t gbytes = (size_t)2 * B * pl->nlat * pl->nlon * sizeof(double);
    const size_t sbytes = ((size_t)(B - 1) * stride + 2 * (size_t)pl->nspec) * 16;
    if (overlaps(in, to_uv ? sbytes : gbytes, out, to_uv ? gbytes : sbytes))
        return fail(REXI_EALIAS, "output overlaps input");
    const int T = pl->T;
    const int C = 4 * B;
    const dim3 grid((T + 2 + 255) / 256, T + 1, B);
    int rc;
    if (to_uv) {
        hipLaunchKernelGGL(k_vd_to_uv_spec, grid, dim3(256), 0, s, (const double2*)in, stride, pl->d_vspec, T,
                           pl->prm.radius);
        REXI_HIP(hipGetLastError());
        if ((rc = leg_inverse(pl, pl->legv, (const double*)pl->d_vspec, C, s))) return rc;
        if ((rc = fft_inverse(pl, pl->legv, (double*)out, 2 * B, pl->d_rcos, s))) return rc;
    } else {
        if ((rc = fft_forward(pl, (const double*)in, 2 * B, pl->d_rcos, s))) return rc;
        if ((rc = leg_forward(pl, pl->legv, (double*)pl->d_vspec, C, s))) return rc;
        hipLaunchKernelGGL(k_uv_spec_to_vd, grid, dim3(256), 0, s, (const double2*)pl->d_vspec, (double2*)out,
                           stride, T, pl->prm.radius);
        REXI_HIP(hipGetLastError());
    }
    return REXI_OK;
}

}  // namespace rexi
