// Fused T-REXI step kernels for gfx950.
//
// One step (Section 4.2; Algorithm 1's sum over terms and its reduction) is
//   u1 = D^{-1} [ sum_k beta+_k (alpha_k + dt L^)^{-1} + sum_k beta-_k (alpha_k - dt L^)^{-1} ] D u0
// per zonal order m (the operator is block diagonal in m, Section 5), where L^
// is the operator of Eq. (1) in energy variables (vorticity and divergence
// scaled by s_n = a sqrt(Phibar/(n(n+1))), which makes L^ skew-Hermitian).
//
// Structure used here (not the paper's Phi-only band of Fig. 1):
//  * Coriolis couples vorticity at degree n only to divergence at n +- 1 and
//    vice versa; Phi_n couples only to divergence at n.  Eliminating Phi_n,
//    Phi_n = (r^Phi_n + dt w_n delta_n)/alpha, leaves two independent
//    tridiagonal chains per (pole, m): chain p holds vorticity at n == p
//    (mod 2) and divergence elsewhere.  Divergence elements get the diagonal
//    alpha + i dt theta + (dt w_n)^2/alpha and the right-hand side
//    r^delta - (dt w_n/alpha) r^Phi.
//  * The minus-sign solves reuse the plus-sign factorisation: with
//    J = diag((-1)^n (1, -1, -1)), J conj(L^) J = -L^, so
//    (alpha - dt L^)^{-1} v = J conj[(conj(alpha) + dt L^)^{-1} conj(J v)],
//    and conj(alpha_k) = alpha_{-k} is again a pole.  Every pole therefore
//    gets two right-hand sides per state, u and conj(J u), and the weights
//    wx_k = beta+_k and wy_k = conj(beta-_{-k}) (adjoint: swapped roles).
//  * The sum over poles of Phi needs no per-pole Phi: sum_k w_k Phi_k =
//    r^Phi sum_k w_k/alpha_k + dt w_n sum_k (w_k/alpha_k) delta_k.
//
// Parallel layout: a wavefront owns one (m, chain, state tile, pole range)
// work item.  Within the wave, P lanes share one chain (P a power of two,
// 64/P poles in flight), each lane holding s consecutive elements in
// registers.  Per pole, each lane eliminates its interior elements
// (Thomas-like sweep plus two spike vectors for the neighbours' interface
// unknowns), the interface unknowns (one per lane) form a tridiagonal system
// solved by parallel cyclic reduction across the P lanes with cross-lane
// shuffles, and the interior is recovered.  Without pivoting: the Hermitian
// part of alpha + dt L^ is Re(alpha) I = h mu I with h mu < 0, and Schur
// complements keep it definite, so every pivot has |Re| >= h |mu|.
// The beta-weighted sums over the item's poles stay in registers (FP64);
// items write partial sums that a second kernel adds in a fixed order, so
// results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace rexi {
namespace {

struct cd {
    double r, i;
};

__device__ __forceinline__ cd mk(double r, double i) { return cd{r, i}; }
__device__ __forceinline__ cd ld2(const double2* p, long long k) {
    const double2 v = p[k];
    return cd{v.x, v.y};
}
__device__ __forceinline__ void st2(double2* p, long long k, cd v) { p[k] = make_double2(v.r, v.i); }
__device__ __forceinline__ cd cadd(cd a, cd b) { return cd{a.r + b.r, a.i + b.i}; }
__device__ __forceinline__ cd csub(cd a, cd b) { return cd{a.r - b.r, a.i - b.i}; }
__device__ __forceinline__ cd cneg(cd a) { return cd{-a.r, -a.i}; }
__device__ __forceinline__ cd cconj(cd a) { return cd{a.r, -a.i}; }
__device__ __forceinline__ cd cscale(cd a, double s) { return cd{a.r * s, a.i * s}; }
__device__ __forceinline__ cd cmul(cd a, cd b) {
    return cd{fma(a.r, b.r, -a.i * b.i), fma(a.r, b.i, a.i * b.r)};
}
// a - b * c
__device__ __forceinline__ cd cfms(cd a, cd b, cd c) {
    return cd{fma(-b.r, c.r, fma(b.i, c.i, a.r)), fma(-b.r, c.i, fma(-b.i, c.r, a.i))};
}
// a - s * b, s real
__device__ __forceinline__ cd csubs(cd a, double s, cd b) { return cd{fma(-s, b.r, a.r), fma(-s, b.i, a.i)}; }
// acc + w * x
__device__ __forceinline__ cd cfma(cd acc, cd w, cd x) {
    return cd{fma(w.r, x.r, fma(-w.i, x.i, acc.r)), fma(w.r, x.i, fma(w.i, x.r, acc.i))};
}
// acc + j * conj(w * x), j = +-1
__device__ __forceinline__ cd cfma_conj(cd acc, double j, cd w, cd x) {
    const double pr = fma(w.r, x.r, -w.i * x.i);
    const double pi = fma(w.r, x.i, w.i * x.r);
    return cd{fma(j, pr, acc.r), fma(-j, pi, acc.i)};
}
__device__ __forceinline__ cd crcp(cd a) {
    const double d = fma(a.r, a.r, a.i * a.i);
    const double s = 1.0 / d;
    return cd{a.r * s, -a.i * s};
}
__device__ __forceinline__ cd shfl(cd v, int src) { return cd{__shfl(v.r, src, 64), __shfl(v.i, src, 64)}; }

struct SolveArgs {
    const Item* items;
    const MInfo* minfo;
    const double* th;   // dt theta_{n,m}
    const double* om;   // dt w_n
    const double* cc;   // 2 Omega dt kappa_{n,m}: coupling of degrees n-1 and n
    const double2* alpha;
    const double2* ainv;
    const double2* wx;
    const double2* wy;
    const double2* wxa;
    const double2* wya;
    const double2* ch_var;  // [S][nslots + 2]
    const double2* ch_phi;  // [S][nspec]
    double2* part;
    int T, S;
    long long var_stride, nspec;
};

// ACCUM = true: add into part (per-term form, one launch per pole) instead of storing.
template <int SM, int ST, bool ACCUM>
__global__ void __launch_bounds__(64) k_solve(const SolveArgs A) {
    const Item it = A.items[blockIdx.x];
    const MInfo mi = A.minfo[it.m];
    const int lane = threadIdx.x;
    const int P = mi.P, s = mi.s, L = mi.L, n0 = mi.n0, p = it.p, m = it.m;
    const int G = 64 / P;
    const int g = lane / P;
    const int l = lane - g * P;
    const int S0 = it.tile * ST;
    const int nst = min(ST, A.S - S0);

    // ---- per-element constants and (pole-independent) right-hand sides
    double th[SM], om[SM], ca[SM], cb[SM], jv[SM];
    bool dl[SM], vd[SM];
    cd rv[ST][SM], rp[ST][SM];
#pragma unroll
    for (int t = 0; t < SM; ++t) {
        const int j = l * s + t;
        const int n = n0 + j;
        vd[t] = (t < s) && (j < L);
        th[t] = om[t] = ca[t] = cb[t] = 0.0;
        jv[t] = 1.0;
        dl[t] = false;
#pragma unroll
        for (int q = 0; q < ST; ++q) rv[q][t] = rp[q][t] = mk(0, 0);
        if (vd[t]) {
            const long long i = mi.spec_off + (n - m);
            th[t] = A.th[i];
            om[t] = A.om[i];
            dl[t] = ((n + p) & 1) != 0;
            const double sg = dl[t] ? 1.0 : -1.0;
            ca[t] = (j > 0) ? sg * A.cc[i] : 0.0;
            cb[t] = (n < A.T) ? sg * A.cc[i + 1] : 0.0;
            jv[t] = (n & 1) ? 1.0 : -1.0;
            const long long slot = mi.slot_base + (long long)p * L + j;
#pragma unroll
            for (int q = 0; q < ST; ++q) {
                if (q < nst) {
                    rv[q][t] = ld2(A.ch_var, (S0 + q) * A.var_stride + slot);
                    if (dl[t]) rp[q][t] = ld2(A.ch_phi, (S0 + q) * A.nspec + i);
                }
            }
        }
    }

    cd av[ST][SM], ap[ST][SM];
#pragma unroll
    for (int q = 0; q < ST; ++q)
#pragma unroll
        for (int t = 0; t < SM; ++t) av[q][t] = ap[q][t] = mk(0, 0);

    const int src_dn = (lane + 1) & 63;
    const int src_up = (lane + 63) & 63;

    for (int kb = it.k0; kb < it.k1; kb += G) {
        const int k = kb + g;
        const bool act = k < it.k1;
        const int kk = act ? k : kb;
        const cd al = ld2(A.alpha, kk), ai = ld2(A.ainv, kk);
        const cd wx = act ? ld2(A.wx, kk) : mk(0, 0);
        const cd wy = act ? ld2(A.wy, kk) : mk(0, 0);
        const cd wxa = act ? ld2(A.wxa, kk) : mk(0, 0);
        const cd wya = act ? ld2(A.wya, kk) : mk(0, 0);

        // diagonal b and Phi-elimination factor f = dt w_n / alpha
        cd b[SM], f[SM];
#pragma unroll
        for (int t = 0; t < SM; ++t) {
            f[t] = mk(0, 0);
            b[t] = mk(1, 0);
            if (vd[t]) {
                if (dl[t]) f[t] = cscale(ai, om[t]);
                b[t] = mk(al.r + om[t] * f[t].r, al.i + th[t] + om[t] * f[t].i);
            }
        }

        // interior factorisation (t = 0 .. s-2) and spikes v (left), w (right)
        cd q[SM], e[SM], v[SM], w[SM];
#pragma unroll
        for (int t = 0; t < SM; ++t) q[t] = e[t] = v[t] = w[t] = mk(0, 0);
#pragma unroll
        for (int t = 0; t < SM - 1; ++t) {
            if (t < s - 1) {
                cd bp = b[t];
                if (t > 0) bp = csubs(bp, ca[t] * cb[t - 1], q[t - 1]);
                q[t] = crcp(bp);
                e[t] = cscale(q[t], cb[t]);
                v[t] = (t == 0) ? cscale(q[0], ca[0]) : cmul(q[t], cscale(v[t - 1], -ca[t]));
            }
        }
#pragma unroll
        for (int t = SM - 3; t >= 0; --t)
            if (t < s - 2) v[t] = cfms(v[t], e[t], v[t + 1]);
#pragma unroll
        for (int t = SM - 2; t >= 0; --t) {
            if (t == s - 2) w[t] = e[t];
            else if (t < s - 2) w[t] = cneg(cmul(e[t], w[t + 1]));
        }

        // interface row (t = s-1) reduced to the lanes' interface unknowns X
        double aI = 0.0, cI = 0.0;
        cd bI = mk(1, 0), vL = mk(0, 0), wL = mk(0, 0);
#pragma unroll
        for (int t = 0; t < SM; ++t)
            if (t == s - 1) { aI = ca[t]; cI = cb[t]; bI = b[t]; }
#pragma unroll
        for (int t = 0; t < SM - 1; ++t)
            if (t == s - 2) { vL = v[t]; wL = w[t]; }
        const bool last = (l == P - 1);
        const bool first = (l == 0);
        cd vN = shfl(v[0], src_dn), wN = shfl(w[0], src_dn);
        if (last) vN = wN = mk(0, 0);
        cd Ac = cneg(cscale(vL, aI));
        cd Bc = csubs(csubs(bI, aI, wL), cI, vN);
        cd Cc = cneg(cscale(wN, cI));

        // right-hand sides: r = 2 q + kind, kind 0: u, kind 1: conj(J u)
        cd x[2 * ST][SM];
        cd D[2 * ST];
#pragma unroll
        for (int r = 0; r < 2 * ST; ++r) {
            const int qs = r >> 1;
#pragma unroll
            for (int t = 0; t < SM; ++t) {
                if (r & 1) {
                    const cd z = cadd(cconj(rv[qs][t]), cmul(f[t], cconj(rp[qs][t])));
                    x[r][t] = cscale(z, jv[t]);
                } else {
                    x[r][t] = cfms(rv[qs][t], f[t], rp[qs][t]);
                }
            }
#pragma unroll
            for (int t = 0; t < SM - 1; ++t) {
                if (t < s - 1) {
                    const cd y = (t == 0) ? x[r][0] : csubs(x[r][t], ca[t], x[r][t - 1]);
                    x[r][t] = cmul(q[t], y);
                }
            }
#pragma unroll
            for (int t = SM - 3; t >= 0; --t)
                if (t < s - 2) x[r][t] = cfms(x[r][t], e[t], x[r][t + 1]);
            cd dI = mk(0, 0), gL = mk(0, 0);
#pragma unroll
            for (int t = 0; t < SM; ++t)
                if (t == s - 1) dI = x[r][t];
#pragma unroll
            for (int t = 0; t < SM - 1; ++t)
                if (t == s - 2) gL = x[r][t];
            cd gN = shfl(x[r][0], src_dn);
            if (last) gN = mk(0, 0);
            D[r] = csubs(csubs(dI, aI, gL), cI, gN);
        }

        // parallel cyclic reduction over the P interface unknowns of a chain
        for (int d = 1; d < P; d <<= 1) {
            const cd ib = crcp(Bc);
            const int sl = (lane - d) & 63, sr = (lane + d) & 63;
            const bool hl = l >= d, hr = l + d < P;
            cd AL = shfl(Ac, sl), CL = shfl(Cc, sl), IL = shfl(ib, sl);
            cd AR = shfl(Ac, sr), CR = shfl(Cc, sr), IR = shfl(ib, sr);
            if (!hl) AL = CL = IL = mk(0, 0);
            if (!hr) AR = CR = IR = mk(0, 0);
            const cd k1 = cmul(Ac, IL), k2 = cmul(Cc, IR);
#pragma unroll
            for (int r = 0; r < 2 * ST; ++r) {
                cd DL = shfl(D[r], sl), DR = shfl(D[r], sr);
                if (!hl) DL = mk(0, 0);
                if (!hr) DR = mk(0, 0);
                D[r] = cfms(cfms(D[r], k1, DL), k2, DR);
            }
            Bc = cfms(cfms(Bc, k1, CL), k2, AR);
            Ac = cneg(cmul(k1, AL));
            Cc = cneg(cmul(k2, CR));
        }
        const cd iB = crcp(Bc);

        // recovery and beta-weighted accumulation
#pragma unroll
        for (int r = 0; r < 2 * ST; ++r) {
            const int qs = r >> 1;
            const cd X = cmul(D[r], iB);
            cd XL = shfl(X, src_up);
            if (first) XL = mk(0, 0);
#pragma unroll
            for (int t = 0; t < SM; ++t) {
                if (t < s) {
                    const cd xv = (t == s - 1) ? X : cfms(cfms(x[r][t], v[t], XL), w[t], X);
                    if (vd[t]) {
                        if (r & 1) {
                            av[qs][t] = cfma_conj(av[qs][t], jv[t], wy, xv);
                            if (dl[t]) ap[qs][t] = cfma_conj(ap[qs][t], -jv[t], wya, xv);
                        } else {
                            av[qs][t] = cfma(av[qs][t], wx, xv);
                            if (dl[t]) ap[qs][t] = cfma(ap[qs][t], wxa, xv);
                        }
                    }
                }
            }
        }
    }

    // add the G groups' sums (same chain positions) in a fixed tree order
    for (int off = 32; off >= P; off >>= 1) {
        const int src = (lane + off) & 63;
#pragma unroll
        for (int qq = 0; qq < ST; ++qq)
#pragma unroll
            for (int t = 0; t < SM; ++t) {
                av[qq][t] = cadd(av[qq][t], shfl(av[qq][t], src));
                ap[qq][t] = cadd(ap[qq][t], shfl(ap[qq][t], src));
            }
    }
    if (g == 0) {
#pragma unroll
        for (int qq = 0; qq < ST; ++qq) {
            if (qq >= nst) continue;
#pragma unroll
            for (int t = 0; t < SM; ++t) {
                if (!vd[t]) continue;
                const int j = l * s + t;
                const long long o0 = it.part_off + ((long long)(qq * 2 + 0) * L + j);
                const long long o1 = it.part_off + ((long long)(qq * 2 + 1) * L + j);
                if (ACCUM) {
                    st2(A.part, o0, cadd(ld2(A.part, o0), av[qq][t]));
                    st2(A.part, o1, cadd(ld2(A.part, o1), ap[qq][t]));
                } else {
                    st2(A.part, o0, av[qq][t]);
                    st2(A.part, o1, ap[qq][t]);
                }
            }
        }
    }
}

// Layout conversion: physical state [S][3][nspec] -> chain layout, scaled.
__global__ void k_prep(const double2* __restrict__ u, double2* __restrict__ ch_var,
                       double2* __restrict__ ch_phi, const MInfo* __restrict__ minfo,
                       const int* __restrict__ idx_n, const int* __restrict__ idx_m,
                       const double* __restrict__ sc, int invert_scale, int S, long long nspec,
                       long long var_stride, long long nslots) {
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (long long)S * nspec) return;
    const int st = (int)(gid / nspec);
    const long long i = gid - (long long)st * nspec;
    const double2* us = u + (long long)st * 3 * nspec;
    ch_phi[st * nspec + i] = us[i];
    if (i == 0) {
        ch_var[st * var_stride + nslots + 0] = us[nspec];
        ch_var[st * var_stride + nslots + 1] = us[2 * nspec];
        return;
    }
    const int n = idx_n[i], m = idx_m[i];
    const MInfo mi = minfo[m];
    const double f = invert_scale ? 1.0 / sc[i] : sc[i];
    const long long pz = n & 1, pd = (n + 1) & 1;
    const double2 z = us[nspec + i], dv = us[2 * nspec + i];
    ch_var[st * var_stride + mi.slot_base + pz * mi.L + (n - mi.n0)] = make_double2(z.x * f, z.y * f);
    ch_var[st * var_stride + mi.slot_base + pd * mi.L + (n - mi.n0)] = make_double2(dv.x * f, dv.y * f);
}

struct ReduceArgs {
    const MInfo* minfo;
    const Group* groups;
    const int* slot_m;
    const double* om;
    const double* sc;
    const double2* part;
    const double2* ch_var_in;
    const double2* ch_phi_in;
    double2* ch_var_out;  // chain layout (next step), or null
    double2* ch_phi_out;
    double2* u_out;       // physical layout (last step), or null
    int ST, ntiles, S, invert_scale;
    long long nspec, var_stride, nslots;
    cd g00, gphi;
};

// Sum an item group's partials in order; finish Phi; write the next chain
// state or the unscaled physical state.
__global__ void k_reduce(const ReduceArgs R) {
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long per_state = R.nslots + 1;
    if (gid >= (long long)R.S * per_state) return;
    const int st = (int)(gid / per_state);
    const long long q = gid - (long long)st * per_state;
    if (q == R.nslots) {  // (n=0, m=0): the operator is zero there
        const cd phi = ld2(R.ch_phi_in, st * R.nspec);
        const cd z = ld2(R.ch_var_in, st * R.var_stride + R.nslots);
        const cd dv = ld2(R.ch_var_in, st * R.var_stride + R.nslots + 1);
        const cd a = cmul(R.g00, phi), b = cmul(R.g00, z), c = cmul(R.g00, dv);
        if (R.u_out) {
            double2* us = R.u_out + (long long)st * 3 * R.nspec;
            st2(us, 0, a);
            st2(us, R.nspec, b);
            st2(us, 2 * R.nspec, c);
        } else {
            st2(R.ch_phi_out, st * R.nspec, a);
            st2(R.ch_var_out, st * R.var_stride + R.nslots, b);
            st2(R.ch_var_out, st * R.var_stride + R.nslots + 1, c);
        }
        return;
    }
    const int m = R.slot_m[q];
    const MInfo mi = R.minfo[m];
    const long long rel = q - mi.slot_base;
    const int p = (int)(rel / mi.L);
    const int j = (int)(rel - (long long)p * mi.L);
    const int n = mi.n0 + j;
    const int tile = st / R.ST, qs = st - tile * R.ST;
    const Group gr = R.groups[((long long)m * 2 + p) * R.ntiles + tile];
    cd av = mk(0, 0), ap = mk(0, 0);
    const long long stride = (long long)R.ST * 2 * mi.L;
    for (int r = 0; r < gr.nr; ++r) {
        const long long o = gr.part_off + r * stride + (long long)(qs * 2) * mi.L + j;
        av = cadd(av, ld2(R.part, o));
        ap = cadd(ap, ld2(R.part, o + mi.L));
    }
    const long long i = mi.spec_off + (n - m);
    const bool isdiv = ((n + p) & 1) != 0;
    cd phi = mk(0, 0);
    if (isdiv) {
        const cd rphi = ld2(R.ch_phi_in, st * R.nspec + i);
        phi = cadd(cmul(rphi, R.gphi), cscale(ap, R.om[i]));
    }
    if (R.u_out) {
        const double f = R.invert_scale ? R.sc[i] : 1.0 / R.sc[i];
        double2* us = R.u_out + (long long)st * 3 * R.nspec;
        st2(us, (isdiv ? 2 : 1) * R.nspec + i, cscale(av, f));
        if (isdiv) st2(us, i, phi);
    } else {
        st2(R.ch_var_out, st * R.var_stride + q, av);
        if (isdiv) st2(R.ch_phi_out, st * R.nspec + i, phi);
    }
}

__global__ void k_zero(double2* p, long long n) {
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid < n) p[gid] = make_double2(0.0, 0.0);
}

template <int SM, int ST, bool ACC>
hipError_t launch_solve_t(const SolveArgs& a, int nitems, hipStream_t s) {
    hipLaunchKernelGGL((k_solve<SM, ST, ACC>), dim3(nitems), dim3(64), 0, s, a);
    return hipGetLastError();
}

template <bool ACC>
hipError_t launch_solve(int SM, int ST, const SolveArgs& a, int nitems, hipStream_t s) {
    if (SM == 4 && ST == 1) return launch_solve_t<4, 1, ACC>(a, nitems, s);
    if (SM == 4 && ST == 2) return launch_solve_t<4, 2, ACC>(a, nitems, s);
    if (SM == 8 && ST == 1) return launch_solve_t<8, 1, ACC>(a, nitems, s);
    return hipErrorInvalidValue;
}

}  // namespace

// Tilings compiled into the library (elements per lane x states per wave).
// Larger tiles exceed the register file and spill to scratch memory.
bool solve_variant_supported(int SM, int ST) { return (SM == 4 && (ST == 1 || ST == 2)) || (SM == 8 && ST == 1); }

// Internal launchers used by the C ABI (plan.cpp).
hipError_t enqueue_prep(rexi_plan* pl, const void* u, int buf, int S, int adjoint, const MInfo* d_layout,
                        hipStream_t s) {
    const long long n = (long long)S * pl->nspec;
    const int bs = 256;
    hipLaunchKernelGGL(k_prep, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s, (const double2*)u,
                       pl->d_ch_var[buf], pl->d_ch_phi[buf], d_layout, pl->d_idx_n, pl->d_idx_m, pl->d_sc,
                       adjoint, S, pl->nspec, pl->nslots + 2, pl->nslots);
    return hipGetLastError();
}

hipError_t enqueue_solve(rexi_plan* pl, const Schedule& sc, int buf, int S, int adjoint, hipStream_t s) {
    SolveArgs a;
    a.items = sc.d_items;
    a.minfo = sc.d_minfo;
    a.th = pl->d_th;
    a.om = pl->d_om;
    a.cc = pl->d_cc;
    a.alpha = pl->d_alpha;
    a.ainv = pl->d_ainv;
    a.wx = pl->d_wx[adjoint];
    a.wy = pl->d_wy[adjoint];
    a.wxa = pl->d_wxa[adjoint];
    a.wya = pl->d_wya[adjoint];
    a.ch_var = pl->d_ch_var[buf];
    a.ch_phi = pl->d_ch_phi[buf];
    a.part = pl->d_part;
    a.T = pl->T;
    a.S = S;
    a.var_stride = pl->nslots + 2;
    a.nspec = pl->nspec;
    return launch_solve<false>(sc.SM, sc.ST, a, (int)sc.items.size(), s);
}

hipError_t enqueue_reduce(rexi_plan* pl, const Schedule& sc, const double2* part, int buf_in, int buf_out,
                          void* u_out, int S, int adjoint, const int* d_slot_m, hipStream_t s) {
    ReduceArgs r;
    r.minfo = sc.d_minfo;
    r.groups = sc.d_groups;
    r.slot_m = d_slot_m;
    r.om = pl->d_om;
    r.sc = pl->d_sc;
    r.part = part;
    r.ch_var_in = pl->d_ch_var[buf_in];
    r.ch_phi_in = pl->d_ch_phi[buf_in];
    r.ch_var_out = u_out ? nullptr : pl->d_ch_var[buf_out];
    r.ch_phi_out = u_out ? nullptr : pl->d_ch_phi[buf_out];
    r.u_out = (double2*)u_out;
    r.ST = sc.ST;
    r.ntiles = (S + sc.ST - 1) / sc.ST;
    r.S = S;
    r.invert_scale = adjoint;
    r.nspec = pl->nspec;
    r.var_stride = pl->nslots + 2;
    r.nslots = pl->nslots;
    const std::complex<double> g00 = adjoint ? pl->g00_adj : pl->g00_fwd;
    const std::complex<double> gp = adjoint ? pl->gphi_adj : pl->gphi_fwd;
    r.g00 = cd{g00.real(), g00.imag()};
    r.gphi = cd{gp.real(), gp.imag()};
    const long long n = (long long)S * (pl->nslots + 1);
    const int bs = 256;
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s, r);
    return hipGetLastError();
}

hipError_t enqueue_zero(double2* p, long long n, hipStream_t s) {
    const int bs = 256;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s, p, n);
    return hipGetLastError();
}

// Per-term form: one launch per pole over all (m, p, tile) items, each adding
// its pole's weighted solution into the accumulator (fixed pole order).
hipError_t enqueue_per_term_pole(rexi_plan* pl, const Schedule& sc, int k, int buf, int S, hipStream_t s) {
    SolveArgs a;
    a.items = sc.d_items;
    a.minfo = sc.d_minfo;
    a.th = pl->d_th;
    a.om = pl->d_om;
    a.cc = pl->d_cc;
    a.alpha = pl->d_alpha + k;
    a.ainv = pl->d_ainv + k;
    a.wx = pl->d_wx[0] + k;
    a.wy = pl->d_wy[0] + k;
    a.wxa = pl->d_wxa[0] + k;
    a.wya = pl->d_wya[0] + k;
    a.ch_var = pl->d_ch_var[buf];
    a.ch_phi = pl->d_ch_phi[buf];
    a.part = pl->d_acc;
    a.T = pl->T;
    a.S = S;
    a.var_stride = pl->nslots + 2;
    a.nspec = pl->nspec;
    return launch_solve<true>(sc.SM, sc.ST, a, (int)sc.items.size(), s);
}

}  // namespace rexi
