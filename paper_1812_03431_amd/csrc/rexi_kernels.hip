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

#include <algorithm>

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

// Per-pole data: pole, its reciprocal and the four weights (see top).
struct __align__(16) PoleData {
    double2 al, ai, wx, wy, wxa, wya;
};

struct SolveArgs {
    const Item* items;
    const MInfo* minfo;
    const double* th;   // dt theta_{n,m}
    const double* om;   // dt w_n
    const double* cc;   // 2 Omega dt kappa_{n,m}: coupling of degrees n-1 and n
    const PoleData* poles;
    const double2* ch_var;  // [S][nslots + 2]
    const double2* ch_phi;  // [S][nspec]
    double2* part;
    int T, S;
    long long var_stride, nspec;
};

constexpr int kWaves = 4;   // waves per workgroup; they share one item's staged data

__device__ __forceinline__ cd crcp_newton(cd a) {
    // 1/(x + i y) = (x - i y)/(x^2 + y^2).  The real reciprocal r of v_rcp_f64
    // (relative error ~5e-8 here) is refined with one third-order step,
    // r <- r (1 + e + e^2), e = 1 - d r: the error becomes ~e^3 plus rounding,
    // one fma fewer than two Newton steps.
    const double d = fma(a.r, a.r, a.i * a.i);
    const double r0 = __builtin_amdgcn_rcp(d);
    const double e = fma(-d, r0, 1.0);
    const double r = fma(r0, fma(e, e, e), r0);
    return cd{a.r * r, -a.i * r};
}

// acc + conj(w x)
__device__ __forceinline__ cd cfma_cj(cd acc, cd w, cd x) {
    return cd{fma(w.r, x.r, fma(-w.i, x.i, acc.r)), fma(-w.r, x.i, fma(-w.i, x.r, acc.i))};
}

// Cross-lane moves of the interface solve.  The P lanes of one chain form a
// group; "lo" receives the value of chain lane l - D, "hi" that of l + D
// (finite but meaningless where that lane lies outside the group: the callers
// multiply it by zero there).
//   kind 0: group = lanes [g P, g P + P), any P <= 64, ds_bpermute.
//   kind 1: the same with P <= 16, so a group lies inside one 16-lane row and
//           moves are DPP row shifts (row_shr:D gives lane i the value of lane
//           i - D, row_shl:D that of lane i + D, zero outside the row).
//   kind 2: P = 32 over the row pair (2g, 2g + 1) with chain lane l = 2 j + r
//           for row-local lane j and row r of the pair.  Strides D >= 2 stay
//           inside the row (a shift by D/2); stride 1 crosses rows:
//           v_permlane16_swap hands each row its partner row's value, and a
//           one-lane row shift applied to one row of the pair completes it.
constexpr int kMoveBperm = 0, kMoveRow = 1, kMovePair = 2;

template <int CTRL>
__device__ __forceinline__ double dpp_zero(double x) {
    const long long v = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)v, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// kind 2, stride 1, on one 32-bit word.  After the swap, s[0] holds in the
// odd row of each pair the even row's value and s[1] in the even row the odd
// row's value (same row-local lane).  Even rows (r = 0, l = 2j) take l - 1 =
// (j - 1, odd row) and keep l + 1 = (j, odd row); odd rows (l = 2j + 1) keep
// l - 1 = (j, even row) and take l + 1 = (j + 1, even row).
__device__ __forceinline__ void pair_step(int w, int& lo, int& hi) {
    const auto s = __builtin_amdgcn_permlane16_swap(w, w, false, false);
    lo = __builtin_amdgcn_update_dpp((int)s[0], (int)s[1], 0x111, 0x5, 0xF, false);  // row_shr:1, even rows
    hi = __builtin_amdgcn_update_dpp((int)s[1], (int)s[0], 0x101, 0xA, 0xF, false);  // row_shl:1, odd rows
}
__device__ __forceinline__ void pair_step(double x, double& lo, double& hi) {
    const long long v = __double_as_longlong(x);
    int l0, h0, l1, h1;
    pair_step((int)(unsigned)v, l0, h0);
    pair_step((int)(v >> 32), l1, h1);
    lo = __longlong_as_double(((long long)l1 << 32) | (long long)(unsigned)l0);
    hi = __longlong_as_double(((long long)h1 << 32) | (long long)(unsigned)h0);
}

template <int KIND, int D>
struct Mover {
    __device__ static __forceinline__ void both(cd x, int lane, cd& lo, cd& hi) {
        if constexpr (KIND == kMoveBperm) {
            lo = shfl(x, (lane - D) & 63);
            hi = shfl(x, (lane + D) & 63);
        } else if constexpr (KIND == kMoveRow) {
            lo = cd{dpp_zero<0x110 + D>(x.r), dpp_zero<0x110 + D>(x.i)};
            hi = cd{dpp_zero<0x100 + D>(x.r), dpp_zero<0x100 + D>(x.i)};
        } else if constexpr (D == 1) {
            pair_step(x.r, lo.r, hi.r);
            pair_step(x.i, lo.i, hi.i);
        } else {
            lo = cd{dpp_zero<0x110 + D / 2>(x.r), dpp_zero<0x110 + D / 2>(x.i)};
            hi = cd{dpp_zero<0x100 + D / 2>(x.r), dpp_zero<0x100 + D / 2>(x.i)};
        }
    }
    __device__ static __forceinline__ cd below(cd x, int lane) {
        cd lo, hi;
        both(x, lane, lo, hi);
        return lo;
    }
    __device__ static __forceinline__ cd above(cd x, int lane) {
        cd lo, hi;
        both(x, lane, lo, hi);
        return hi;
    }
};

// One cyclic-reduction level with stride D, split into the matrix part (the
// row (A, B, C) of every lane and the multipliers k1, k2 of the level, which
// depend on the pole only) and the right-hand-side part (both right-hand
// sides of one state, with the level's multipliers).
template <int KIND, int D>
__device__ __forceinline__ void pcr_matrix(cd& Ac, cd& Bc, cd& Cc, cd& k1, cd& k2, int l, int P, int lane) {
    typedef Mover<KIND, D> Mv;
    // neighbours outside the chain's group: multipliers are zero.  Each moved
    // value is consumed before the next move (keeps few values live).
    cd lo, hi;
    Mv::both(crcp_newton(Bc), lane, lo, hi);
    k1 = (l >= D) ? cmul(Ac, lo) : mk(0, 0);
    k2 = (l + D < P) ? cmul(Cc, hi) : mk(0, 0);
    Mv::both(Cc, lane, lo, hi);
    Bc = cfms(Bc, k1, lo);
    Cc = cneg(cmul(k2, hi));
    Mv::both(Ac, lane, lo, hi);
    Bc = cfms(Bc, k2, hi);
    Ac = cneg(cmul(k1, lo));
}
template <int KIND, int D>
__device__ __forceinline__ void pcr_rhs(cd k1, cd k2, cd& Du, cd& Dw, int lane) {
    typedef Mover<KIND, D> Mv;
    cd lo, hi;
    Mv::both(Du, lane, lo, hi);
    Du = cfms(cfms(Du, k1, lo), k2, hi);
    Mv::both(Dw, lane, lo, hi);
    Dw = cfms(cfms(Dw, k1, lo), k2, hi);
}

// LDS of a work item.  Staged per chain position, as planes of doubles
// [t][plane][slot]: th, om, c_left, c_right, then Re/Im of the chain variable
// and of Phi for each of the item's R states (each state's block of four
// planes SBLK doubles long).  With R > 1 every wave also
// owns a factorisation region: per interior element t and wave lane the
// pivot reciprocal q_t and, where LDS allows, the running product pi_t
// (NQ >= 4) and the left spike gv_t (NQ = 6), [t][quantity][64]; then per
// cyclic-reduction level the multipliers k1, k2 [level][4][64] and the
// interface pivot's reciprocal [2][64].
template <int SE, int KIND, int W, int R>
struct SolveLds {
    static constexpr int PS = (KIND == kMoveRow) ? 16 : (KIND == kMovePair) ? 32 : 64;  // slots per position
    static constexpr int NI = SE - 1;
    static constexpr int LV = (KIND == kMoveRow) ? 4 : (KIND == kMovePair) ? 5 : 6;    // levels for P <= PS
    static constexpr int SPAD = 0;                                                      // state block pad
    static constexpr int SBLK = 4 * PS + SPAD;                                          // state block
    static constexpr int POS = 4 * PS + R * SBLK;                                       // per position
    static constexpr int kStaged = POS * SE;                                            // doubles
    // two waves per SIMD (two workgroups of four waves per CU) where the
    // registers allow it: tiles of up to 6 elements, and 8 with one state per
    // item; the others take a CU's whole LDS (160 KB)
    static constexpr int kWavesPerSimd = (SE <= 6 || (SE == 8 && R == 1)) ? 2 : 1;
    static constexpr int kMaxDoubles = ((kWavesPerSimd == 2 ? 80 : 160) * 1024 - 64) / 8;
    static constexpr int region(int nq) { return 64 * (NI * nq + 4 * LV + 2); }
    static constexpr int total(int nq) { return kStaged + (R > 1 ? W * region(nq) : 0); }
    // the reuse passes recompute the spike and the running product from the
    // pivots (12 VALU instructions per element), which measured faster than
    // reading them (LDS reads, not VALU issue, bound those passes)
    static constexpr int NQ = 2;
    static constexpr int kRegion = R > 1 ? region(NQ) : 0;
    static constexpr int kDoubles = total(NQ);
    static_assert(kDoubles <= kMaxDoubles, "work item does not fit in LDS");
};

// One work item: chain p of order m, the R states [tile R, tile R + R), a
// pole range.  SE elements per lane (even, compile time); PH fixes the
// element types: element t of every lane is a divergence element iff
// (t + PH) is odd.
//
// Per pole each lane runs one forward sweep over its interior elements
// t = 0..SE-2 that at once forms the pivots q, multipliers e = q c, the
// forward part gv of the left spike and the forward parts G of both
// right-hand sides, and accumulates, with the running product
// pi_t = prod_{s<t} (-e_s), the back-substituted first elements
// (y_0 = sum_t pi_t Y_t) that the left neighbour's interface row needs.  The
// interface rows (one per lane) are solved by cyclic reduction across the
// chain's P lanes, matrix and both right-hand sides in the same levels, and a
// reverse sweep recovers the interior with both interface values.
//
// States (R > 1): the factorisation (q, e, gv, pi, and the reduction's
// multipliers) depends on the pole and the chain only.  Group g of a wave
// keeps state g mod R for the whole item, and the groups form blocks of R.
// For each batch of the wave's G poles, pass 0 has every group solve its own
// pole for its own state, computing the factorisation and publishing it in
// the wave's LDS region; passes 1..R-1 have group g solve the pole of group
// blk R + (g + j) mod R of its block for its own state, reading that
// factorisation instead of recomputing it.  Each pole is so solved for all R
// states with one factorisation.
//
// Mirrored right-hand side: with jv = -(-1)^n the J sign of vorticity and
// divergence, the staged chain data v gives conj(J v) = jv conj(v) on the
// chain and -jv conj(r^Phi) on Phi.  Since SE is even, jv = j0 (-1)^t with one
// sign j0 per item; the solve is linear, so j0 is dropped from the right-hand
// side and cancels against the same factor of J on the output.  What remains
// is (-1)^t on input and output.
template <int SE, int PH, bool ACCUM, int KIND, int W, int R>
__device__ __forceinline__ void solve_item(const SolveArgs& A, const Item& it, const MInfo& mi, double* sm) {
    static_assert(SE % 2 == 0, "elements per lane must be even");
    static_assert(R == 1 || R == 2 || R == 4, "states per item");
    typedef SolveLds<SE, KIND, W, R> Lds;
    constexpr int NI = SE - 1;  // interior elements 0 .. SE-2; interface SE-1
    constexpr int PS = Lds::PS, POS = Lds::POS, NQ = Lds::NQ;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int P = (KIND == kMovePair) ? 32 : mi.P;
    const int L = mi.L, n0 = mi.n0, m = it.m, p = it.p;
    const int G = 64 / P;
    int g, l;
    if constexpr (KIND == kMovePair) {
        g = lane >> 5;
        l = 2 * (lane & 15) + ((lane >> 4) & 1);
    } else {
        g = lane / P;
        l = lane - g * P;
    }
    // LDS slot of chain lane l: its lane within the group (kind 2: j + 16 r);
    // slots per chunk fixed at compile time so that every LDS offset below is
    // an immediate
    const int slot = (KIND == kMovePair) ? (lane & 31) : l;
    const int st0 = it.tile * R;
    const int npos = P * SE;
    const int sg_state = g & (R - 1);   // this group's state within the item
    const int blk = g / R;              // its block of R groups

    // ---- stage the item's constants and right-hand sides in LDS as planes of
    // doubles per position, [t][plane][slot], so that the lanes of a row read
    // consecutive 8-byte words (8-byte reads issue far faster here than
    // 16-byte ones)
    double2* c = reinterpret_cast<double2*>(sm);
    for (int j = tid; j < npos; j += blockDim.x) {
        const int l2 = j / SE, t2 = j - l2 * SE;
        const int s2 = (KIND == kMovePair) ? ((l2 >> 1) + 16 * (l2 & 1)) : l2;
        const int n = n0 + j;
        double2 v0 = make_double2(0.0, 0.0), v1 = v0;
        const bool in = j < L;
        const long long i = mi.spec_off + (n - m);
        if (in) {
            v0 = make_double2(A.th[i], A.om[i]);
            v1 = make_double2((j > 0) ? A.cc[i] : 0.0, (n < A.T) ? A.cc[i + 1] : 0.0);
        }
        double* o = sm + (size_t)t2 * POS + s2;
        o[0] = v0.x;
        o[PS] = v0.y;
        o[2 * PS] = v1.x;
        o[3 * PS] = v1.y;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            double2 v2 = make_double2(0.0, 0.0), v3 = v2;
            if (in) {
                v2 = A.ch_var[(st0 + q) * A.var_stride + mi.slot_base + (long long)p * L + j];
                if ((n + p) & 1) v3 = A.ch_phi[(st0 + q) * A.nspec + i];
            }
            double* os = o + 4 * PS + q * Lds::SBLK;
            os[0] = v2.x;
            os[PS] = v2.y;
            os[2 * PS] = v3.x;
            os[3 * PS] = v3.y;
        }
    }
    __syncthreads();

    bool vd[SE];
#pragma unroll
    for (int t = 0; t < SE; ++t) vd[t] = (l * SE + t) < L;

    cd av[SE], ap[SE];
#pragma unroll
    for (int t = 0; t < SE; ++t) av[t] = ap[t] = mk(0, 0);

    const int stride = W * G;

    // staged data of position t of this lane.  om and r_Phi exist only on
    // divergence positions; the right coupling of position t is the left one
    // of t + 1, so it is read only where that position is not read anyway.
    struct Pos {
        double th, om, cl, cr;
        cd rv, rp;
    };
    const double* cbase = sm + slot;                                   // planes 0..3
    const double* sbase = sm + slot + 4 * PS + sg_state * Lds::SBLK;   // this group's state
    auto fetch = [&](int t, bool with_cr) {
        const double* o = cbase + (size_t)t * POS;
        const double* os = sbase + (size_t)t * POS;
        Pos x;
        x.th = o[0];
        x.cl = o[2 * PS];
        x.cr = with_cr ? o[3 * PS] : 0.0;
        x.rv = cd{os[0], os[PS]};
        if ((PH + t) & 1) {
            x.om = o[PS];
            x.rp = cd{os[2 * PS], os[3 * PS]};
        } else {
            x.om = 0.0;
            x.rp = mk(0, 0);
        }
        return x;
    };
    // the wave's factorisation region (R > 1)
    double* reg = sm + Lds::kStaged + wave * Lds::kRegion;
    constexpr int kPcr = 64 * NI * NQ;        // start of the reduction's multipliers
    constexpr int kIb = kPcr + 64 * 4 * Lds::LV;

    // Latency hiding where registers allow (row groups): the pole and its
    // reciprocal are fetched one iteration ahead, the staged data of position
    // t + 1 before the work on t, and scheduling barriers keep these reads
    // where they are.  The row-pair kind has no registers to spare for it.
    constexpr bool kAhead = (KIND == kMoveRow) || (KIND == kMovePair && Lds::kWavesPerSimd == 1 && R > 1);
    // pole solved by this group in pass j of the batch starting at kb
    auto pole_of = [&](int kb, int j) { return kb + wave * G + blk * R + ((sg_state + j) & (R - 1)); };
    cd al_n = mk(0, 0), ai_n = mk(0, 0);
    if constexpr (kAhead) {
        const int k = pole_of(it.k0, 0);
        const PoleData& pn = A.poles[k < it.k1 ? k : it.k0];
        al_n = cd{pn.al.x, pn.al.y};
        ai_n = cd{pn.ai.x, pn.ai.y};
    }

    // element of position t: couplings and both right-hand sides (the
    // mirrored one as described above); f = om / alpha on divergence rows
    auto element_rhs = [&](int t, const Pos& x, const cd& ai, double& ca, double& cb, cd& du, cd& dw, cd& f) {
        const double sg = ((PH + t) & 1) ? 1.0 : -1.0;  // divergence rows +, vorticity rows -
        const double ts = (t & 1) ? -1.0 : 1.0;         // (-1)^t
        ca = sg * x.cl;
        cb = sg * x.cr;
        if ((PH + t) & 1) {
            // divergence element, Phi eliminated: right-hand side r_div - (om/alpha) r_Phi
            f = cscale(ai, x.om);
            du = cfms(x.rv, f, x.rp);
            const double wr = fma(f.r, x.rp.r, fma(f.i, x.rp.i, x.rv.r));
            const double wi = fma(f.i, x.rp.r, fma(-f.r, x.rp.i, -x.rv.i));
            dw = cd{ts * wr, ts * wi};
        } else {
            f = mk(0, 0);
            du = x.rv;
            dw = cd{ts * x.rv.r, -ts * x.rv.i};
        }
    };

    // reverse sweep with both interface values and the weighted sums.  The
    // mirrored solution enters conjugated with (-1)^t on the chain variable
    // and -(-1)^t on Phi.
    auto back_and_accumulate = [&](const cd* e, const cd* gv, const cd* Gu, const cd* Gw, cd Xu, cd Xw, cd XLu,
                                   cd XLw, cd wx, cd wxa, cd wyE, cd wyaE, bool act) {
        wyaE = cneg(wyaE);
        if (!act) wx = wxa = wyE = wyaE = mk(0, 0);
        cd xu = Xu, xw = Xw;
#pragma unroll
        for (int t = SE - 1; t >= 0; --t) {
            if (t < NI) {
                xu = cfms(cfms(Gu[t], XLu, gv[t]), e[t], xu);
                xw = cfms(cfms(Gw[t], XLw, gv[t]), e[t], xw);
            }
            if (vd[t]) {
                const cd wy = (t & 1) ? cneg(wyE) : wyE;
                av[t] = cfma_cj(cfma(av[t], wx, xu), wy, xw);
                if ((PH + t) & 1) {
                    const cd wya = (t & 1) ? cneg(wyaE) : wyaE;
                    ap[t] = cfma_cj(cfma(ap[t], wxa, xu), wya, xw);
                }
            }
        }
    };
    typedef Mover<KIND, 1> M1;

    for (int kb = it.k0; kb < it.k1; kb += stride) {
        if (kb + wave * G >= it.k1) continue;  // this wave has no pole left (uniform)
        // ================= pass 0: own pole, factorisation computed (and published)
        {
            const int k = pole_of(kb, 0);
            const bool act = k < it.k1;
            const PoleData& pd = A.poles[act ? k : it.k0];
            cd al, ai;
            if constexpr (kAhead) {
                al = al_n;
                ai = ai_n;
                const int kn = (R > 1) ? pole_of(kb, 1) : pole_of(kb + stride, 0);
                const PoleData& pn = A.poles[kn < it.k1 ? kn : it.k0];
                al_n = cd{pn.al.x, pn.al.y};
                ai_n = cd{pn.ai.x, pn.ai.y};
                __builtin_amdgcn_sched_barrier(0);
            } else {
                al = cd{pd.al.x, pd.al.y};
                ai = cd{pd.ai.x, pd.ai.y};
            }

            cd e[NI], gv[NI], Gu[NI], Gw[NI];
            cd pi = mk(1, 0), v0 = mk(0, 0), w0 = mk(0, 0), g0u = mk(0, 0), g0w = mk(0, 0);
            cd qprev = mk(0, 0);
            double cbprev = 0.0;
            // element of position t: diagonal b, couplings, right-hand sides
            auto element = [&](int t, const Pos& x, cd& b, double& ca, double& cb, cd& du, cd& dw) {
                cd f;
                element_rhs(t, x, ai, ca, cb, du, dw, f);
                if ((PH + t) & 1) {
                    // divergence element: diagonal alpha + i th + om^2/alpha
                    b = mk(fma(x.om, f.r, al.r), al.i + fma(x.om, f.i, x.th));
                } else {
                    b = mk(al.r, al.i + x.th);
                }
            };
            Pos cur;
            if constexpr (kAhead) cur = fetch(0, false);
#pragma unroll
            for (int t = 0; t < NI; ++t) {
                Pos nxt;
                if constexpr (kAhead) {
                    nxt = fetch(t + 1, t + 1 == SE - 1);
                    __builtin_amdgcn_sched_barrier(0);
                    cur.cr = nxt.cl;
                } else {
                    cur = fetch(t, true);
                }
                cd b, du, dw;
                double ca, cb;
                element(t, cur, b, ca, cb, du, dw);
                if (t > 0) b = csubs(b, ca * cbprev, qprev);
                const cd q = crcp_newton(b);
                e[t] = cscale(q, cb);
                if (t == 0) {
                    gv[0] = cscale(q, ca);
                    Gu[0] = cmul(q, du);
                    Gw[0] = cmul(q, dw);
                } else {
                    gv[t] = cmul(q, cscale(gv[t - 1], -ca));
                    Gu[t] = cmul(q, csubs(du, ca, Gu[t - 1]));
                    Gw[t] = cmul(q, csubs(dw, ca, Gw[t - 1]));
                }
                if constexpr (R > 1) {
                    double* r = reg + (t * NQ) * 64 + lane;
                    r[0] = q.r;
                    r[64] = q.i;
                    if constexpr (NQ >= 4) {
                        r[128] = pi.r;
                        r[192] = pi.i;
                    }
                    if constexpr (NQ >= 6) {
                        r[256] = gv[t].r;
                        r[320] = gv[t].i;
                    }
                }
                v0 = cfma(v0, pi, gv[t]);
                g0u = cfma(g0u, pi, Gu[t]);
                g0w = cfma(g0w, pi, Gw[t]);
                if (t == NI - 1) w0 = cmul(pi, e[t]);
                pi = cneg(cmul(pi, e[t]));
                qprev = q;
                cbprev = cb;
                if constexpr (kAhead) cur = nxt;
            }

            // this pole's weights: read here, used after the interface solve
            cd wx = cd{pd.wx.x, pd.wx.y}, wxa = cd{pd.wxa.x, pd.wxa.y};
            cd wyE = cd{pd.wy.x, pd.wy.y}, wyaE = cd{pd.wya.x, pd.wya.y};
            if constexpr (kAhead) __builtin_amdgcn_sched_barrier(0);

            // interface row -> tridiagonal system over the P lanes of the chain;
            // the right neighbour's values enter with cI, which is zero at a chain end
            cd bI, dIu, dIw;
            double aI, cI;
            if constexpr (!kAhead) cur = fetch(SE - 1, true);
            element(SE - 1, cur, bI, aI, cI, dIu, dIw);
            const cd vN = M1::above(v0, lane), wN = M1::above(w0, lane);
            const cd guN = M1::above(g0u, lane), gwN = M1::above(g0w, lane);
            cd Ac = cneg(cscale(gv[NI - 1], aI));
            cd Bc = csubs(csubs(bI, aI, e[NI - 1]), cI, vN);
            cd Cc = cneg(cscale(wN, cI));
            cd Du = csubs(csubs(dIu, aI, Gu[NI - 1]), cI, guN);
            cd Dw = csubs(csubs(dIw, aI, Gw[NI - 1]), cI, gwN);

            // cyclic reduction over the lanes of the chain
            auto level = [&](auto dconst, int lev) {
                constexpr int D = decltype(dconst)::value;
                cd k1, k2;
                pcr_matrix<KIND, D>(Ac, Bc, Cc, k1, k2, l, P, lane);
                pcr_rhs<KIND, D>(k1, k2, Du, Dw, lane);
                if constexpr (R > 1) {
                    double* r = reg + kPcr + (lev * 4) * 64 + lane;
                    r[0] = k1.r;
                    r[64] = k1.i;
                    r[128] = k2.r;
                    r[192] = k2.i;
                }
            };
            typedef std::integral_constant<int, 1> D1;
            typedef std::integral_constant<int, 2> D2;
            typedef std::integral_constant<int, 4> D4;
            typedef std::integral_constant<int, 8> D8;
            typedef std::integral_constant<int, 16> D16;
            typedef std::integral_constant<int, 32> D32;
            if constexpr (KIND == kMovePair) {
                level(D1{}, 0);
                level(D2{}, 1);
                level(D4{}, 2);
                level(D8{}, 3);
                level(D16{}, 4);
            } else {
                if (1 < P) level(D1{}, 0);
                if (2 < P) level(D2{}, 1);
                if (4 < P) level(D4{}, 2);
                if (8 < P) level(D8{}, 3);
                if constexpr (KIND == kMoveBperm) {
                    if (16 < P) level(D16{}, 4);
                    if (32 < P) level(D32{}, 5);
                }
            }
            const cd iB = crcp_newton(Bc);
            if constexpr (R > 1) {
                double* r = reg + kIb + lane;
                r[0] = iB.r;
                r[64] = iB.i;
            }
            const cd Xu = cmul(Du, iB), Xw = cmul(Dw, iB);
            // the left neighbour's interface values (enter through gv, zero at a chain start)
            const cd XLu = M1::below(Xu, lane), XLw = M1::below(Xw, lane);
            back_and_accumulate(e, gv, Gu, Gw, Xu, Xw, XLu, XLw, wx, wxa, wyE, wyaE, act);
        }

        // ================= passes 1..R-1: the block's other poles, factorisation read
        if constexpr (R > 1) {
#pragma unroll 1
            for (int j = 1; j < R; ++j) {
                const int src = blk * R + ((sg_state + j) & (R - 1));   // group that factorised this pole
                const int k = kb + wave * G + src;
                const bool act = k < it.k1;
                const PoleData& pd = A.poles[act ? k : it.k0];
                cd ai;
                if constexpr (kAhead) {
                    ai = ai_n;
                    const int kn = (j + 1 < R) ? pole_of(kb, j + 1) : pole_of(kb + stride, 0);
                    const PoleData& pn = A.poles[kn < it.k1 ? kn : it.k0];
                    al_n = cd{pn.al.x, pn.al.y};
                    ai_n = cd{pn.ai.x, pn.ai.y};
                    __builtin_amdgcn_sched_barrier(0);
                } else {
                    ai = cd{pd.ai.x, pd.ai.y};
                }
                const double* rs = reg + lane + (src - g) * P;   // the source group's lane for chain lane l

                cd e[NI], gv[NI], Gu[NI], Gw[NI];
                cd pi = mk(1, 0), g0u = mk(0, 0), g0w = mk(0, 0);
                // published factorisation of element t: pivot, and where
                // stored, running product and spike
                struct Fac {
                    cd q, pi, gv;
                };
                auto ffetch = [&](int t) {
                    const double* r = rs + (t * NQ) * 64;
                    Fac x;
                    x.q = cd{r[0], r[64]};
                    if constexpr (NQ >= 4) x.pi = cd{r[128], r[192]};
                    if constexpr (NQ >= 6) x.gv = cd{r[256], r[320]};
                    return x;
                };
                Pos cur;
                Fac fcur;
                if constexpr (kAhead) {
                    cur = fetch(0, false);
                    fcur = ffetch(0);
                }
#pragma unroll
                for (int t = 0; t < NI; ++t) {
                    Pos nxt;
                    Fac fnxt;
                    if constexpr (kAhead) {
                        nxt = fetch(t + 1, t + 1 == SE - 1);
                        if (t + 1 < NI) fnxt = ffetch(t + 1);
                        __builtin_amdgcn_sched_barrier(0);
                        cur.cr = nxt.cl;
                    } else {
                        cur = fetch(t, true);
                        fcur = ffetch(t);
                    }
                    const cd q = fcur.q;
                    cd du, dw, f;
                    double ca, cb;
                    element_rhs(t, cur, ai, ca, cb, du, dw, f);
                    e[t] = cscale(q, cb);
                    if constexpr (NQ >= 6) {
                        gv[t] = fcur.gv;
                    } else {
                        gv[t] = (t == 0) ? cscale(q, ca) : cmul(q, cscale(gv[t - 1], -ca));
                    }
                    if constexpr (NQ >= 4) pi = fcur.pi;
                    if (t == 0) {
                        Gu[0] = cmul(q, du);
                        Gw[0] = cmul(q, dw);
                    } else {
                        Gu[t] = cmul(q, csubs(du, ca, Gu[t - 1]));
                        Gw[t] = cmul(q, csubs(dw, ca, Gw[t - 1]));
                    }
                    g0u = cfma(g0u, pi, Gu[t]);
                    g0w = cfma(g0w, pi, Gw[t]);
                    if constexpr (NQ < 4) pi = cneg(cmul(pi, e[t]));
                    if constexpr (kAhead) {
                        cur = nxt;
                        fcur = fnxt;
                    }
                }
                // first level's multipliers, read ahead of their use
                cd k1n = cd{rs[kPcr], rs[kPcr + 64]}, k2n = cd{rs[kPcr + 128], rs[kPcr + 192]};
                cd wx = cd{pd.wx.x, pd.wx.y}, wxa = cd{pd.wxa.x, pd.wxa.y};
                cd wyE = cd{pd.wy.x, pd.wy.y}, wyaE = cd{pd.wya.x, pd.wya.y};
                if constexpr (kAhead) __builtin_amdgcn_sched_barrier(0);

                cd dIu, dIw, fI;
                double aI, cI;
                if constexpr (!kAhead) cur = fetch(SE - 1, true);
                element_rhs(SE - 1, cur, ai, aI, cI, dIu, dIw, fI);
                const cd guN = M1::above(g0u, lane), gwN = M1::above(g0w, lane);
                cd Du = csubs(csubs(dIu, aI, Gu[NI - 1]), cI, guN);
                cd Dw = csubs(csubs(dIw, aI, Gw[NI - 1]), cI, gwN);
                auto level = [&](auto dconst, int lev) {
                    constexpr int D = decltype(dconst)::value;
                    const cd k1 = k1n, k2 = k2n;
                    // the next level's (the last level reads its own again)
                    const int ln = (lev + 1 < Lds::LV) ? lev + 1 : lev;
                    const double* r = rs + kPcr + (ln * 4) * 64;
                    k1n = cd{r[0], r[64]};
                    k2n = cd{r[128], r[192]};
                    pcr_rhs<KIND, D>(k1, k2, Du, Dw, lane);
                };
                typedef std::integral_constant<int, 1> D1;
                typedef std::integral_constant<int, 2> D2;
                typedef std::integral_constant<int, 4> D4;
                typedef std::integral_constant<int, 8> D8;
                typedef std::integral_constant<int, 16> D16;
                if constexpr (KIND == kMovePair) {
                    level(D1{}, 0);
                    level(D2{}, 1);
                    level(D4{}, 2);
                    level(D8{}, 3);
                    level(D16{}, 4);
                } else {
                    static_assert(KIND == kMoveRow, "states share factorisations only in row and row-pair tilings");
                    if (1 < P) level(D1{}, 0);
                    if (2 < P) level(D2{}, 1);
                    if (4 < P) level(D4{}, 2);
                    if (8 < P) level(D8{}, 3);
                }
                const cd iB = cd{rs[kIb], rs[kIb + 64]};
                const cd Xu = cmul(Du, iB), Xw = cmul(Dw, iB);
                const cd XLu = M1::below(Xu, lane), XLw = M1::below(Xw, lane);
                back_and_accumulate(e, gv, Gu, Gw, Xu, Xw, XLu, XLw, wx, wxa, wyE, wyaE, act);
            }
        }
    }

    // sum the groups of each wave that hold the same state (same chain lanes,
    // groups g and g + R, g + 2R, ...) in a fixed tree order
    for (int off = 32; off >= R * P; off >>= 1) {
        const int src = (lane + off) & 63;
#pragma unroll
        for (int t = 0; t < SE; ++t) {
            av[t] = cadd(av[t], shfl(av[t], src));
            if ((PH + t) & 1) ap[t] = cadd(ap[t], shfl(ap[t], src));
        }
    }
    // then the waves, in order, through LDS (reusing the staging area):
    // acc[state][2][SE][P], groups 0..R-1 of each wave hold states 0..R-1
    __syncthreads();
    double2* acc = c;
    for (int wv = 0; wv < W; ++wv) {
        if (wave == wv && g < R) {
#pragma unroll
            for (int t = 0; t < SE; ++t) {
                const int o0 = ((g * 2 + 0) * SE + t) * P + l, o1 = ((g * 2 + 1) * SE + t) * P + l;
                double2 a0 = make_double2(av[t].r, av[t].i);
                double2 a1 = make_double2(ap[t].r, ap[t].i);
                if (wv > 0) {
                    a0.x += acc[o0].x;
                    a0.y += acc[o0].y;
                    a1.x += acc[o1].x;
                    a1.y += acc[o1].y;
                }
                acc[o0] = a0;
                acc[o1] = a1;
            }
        }
        __syncthreads();
    }
    for (int idx = tid; idx < 2 * R * L; idx += blockDim.x) {
        const int sp = idx / L;            // state * 2 + plane
        const int plane = sp & 1;
        const int j = idx - sp * L;
        const int l2 = j / SE, t2 = j - l2 * SE;
        if (plane == 1 && !(((PH + t2) & 1) != 0)) continue;
        const double2 v = acc[(sp * SE + t2) * P + l2];
        const long long o = it.part_off + ((long long)sp * L + j);
        if (ACCUM) {
            const double2 old = A.part[o];
            A.part[o] = make_double2(old.x + v.x, old.y + v.y);
        } else {
            A.part[o] = v;
        }
    }
}

template <int SE, bool ACCUM, int KIND, int W, int R>
__device__ __forceinline__ void run_item(const SolveArgs& A, int idx, double* sm) {
    const Item it = A.items[idx];
    const MInfo mi = A.minfo[it.m];
    if ((mi.n0 + it.p) & 1) solve_item<SE, 1, ACCUM, KIND, W, R>(A, it, mi, sm);
    else solve_item<SE, 0, ACCUM, KIND, W, R>(A, it, mi, sm);
}

// One workgroup per item (counter == null), or persistent: a grid of resident
// workgroups takes items [item0, item0 + nitems) from an atomic counter that
// starts at zero, until none is left (every workgroup then leaves the loop).
// Small tiles are held to 256 registers (two waves per SIMD); larger ones use
// the whole register file (10 elements would spill at 256).
template <int SE, bool ACCUM, int KIND, int W, int R>
__global__ void __launch_bounds__(64 * W)
    __attribute__((amdgpu_waves_per_eu(SolveLds<SE, KIND, W, R>::kWavesPerSimd)))
k_solve(const SolveArgs A, int item0, int nitems, int* counter) {
    extern __shared__ double sm[];
    if (counter == nullptr) {
        run_item<SE, ACCUM, KIND, W, R>(A, item0 + blockIdx.x, sm);
        return;
    }
    __shared__ int next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(counter, 1);
        __syncthreads();
        const int i = next;
        __syncthreads();
        if (i < 0 || i >= nitems) break;
        run_item<SE, ACCUM, KIND, W, R>(A, item0 + i, sm);
    }
}

__global__ void k_reset_counters(int* c, int n) {
    if ((int)threadIdx.x < n) c[threadIdx.x] = 0;
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
    int S, invert_scale;
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
    const Group gr = R.groups[((long long)m * 2 + p) * R.S + st];
    cd av = mk(0, 0), ap = mk(0, 0);
    const long long stride = (long long)gr.st * 2 * mi.L;
    for (int r = 0; r < gr.nr; ++r) {
        const long long o = gr.part_off + r * stride + j;
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

// Chain layout (scaled) -> physical state [S][3][nspec].
__global__ void k_finish(const double2* __restrict__ ch_var, const double2* __restrict__ ch_phi,
                         double2* __restrict__ u, const MInfo* __restrict__ minfo, const int* __restrict__ idx_n,
                         const int* __restrict__ idx_m, const double* __restrict__ sc, int invert_scale, int S,
                         long long nspec, long long var_stride, long long nslots) {
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (long long)S * nspec) return;
    const int st = (int)(gid / nspec);
    const long long i = gid - (long long)st * nspec;
    double2* us = u + (long long)st * 3 * nspec;
    us[i] = ch_phi[st * nspec + i];
    if (i == 0) {
        us[nspec] = ch_var[st * var_stride + nslots];
        us[2 * nspec] = ch_var[st * var_stride + nslots + 1];
        return;
    }
    const int n = idx_n[i], m = idx_m[i];
    const MInfo mi = minfo[m];
    const double f = invert_scale ? sc[i] : 1.0 / sc[i];
    const long long pz = n & 1, pd = (n + 1) & 1;
    const double2 z = ch_var[st * var_stride + mi.slot_base + pz * mi.L + (n - mi.n0)];
    const double2 dv = ch_var[st * var_stride + mi.slot_base + pd * mi.L + (n - mi.n0)];
    us[nspec + i] = make_double2(z.x * f, z.y * f);
    us[2 * nspec + i] = make_double2(dv.x * f, dv.y * f);
}

__global__ void k_zero(double2* p, long long n) {
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid < n) p[gid] = make_double2(0.0, 0.0);
}

// f-sphere variant (Section 4.3): with a constant Coriolis parameter f0 the
// operator couples (Phi, zeta, delta) only at the same (n, m).  In energy
// variables Phi_t = -w delta, zeta_t = -f0 delta, delta_t = f0 zeta + w Phi, so
// with p = dt w_n and q = dt f0 the shifted system (a + dt L^) x = r has the
// closed-form solution
//   delta = (a r_d - q r_z - p r_P) / (a^2 + p^2 + q^2),
//   Phi = (r_P + p delta) / a,  zeta = (r_z + q delta) / a,
// and (a - dt L^) flips the signs of p and q.  One thread per (state, n, m)
// sums over the poles; the adjoint uses conj(beta), conj(alpha) and
// L^H = -L^ with the inverse scaling.  (n, m) = (0, 0): the operator is zero.
__device__ __forceinline__ cd cdiv(cd a, cd b) {
    const double d = fma(b.r, b.r, b.i * b.i);
    return cd{fma(a.r, b.r, a.i * b.i) / d, fma(a.i, b.r, -a.r * b.i) / d};
}
__device__ __forceinline__ void fsphere_solve(cd a, double p, double q, cd rP, cd rz, cd rd, cd& xP, cd& xz,
                                              cd& xd) {
    const cd den = cd{fma(a.r, a.r, -a.i * a.i) + p * p + q * q, 2.0 * a.r * a.i};
    const cd num = cd{a.r * rd.r - a.i * rd.i - q * rz.r - p * rP.r, a.r * rd.i + a.i * rd.r - q * rz.i - p * rP.i};
    xd = cdiv(num, den);
    xP = cdiv(cd{rP.r + p * xd.r, rP.i + p * xd.i}, a);
    xz = cdiv(cd{rz.r + q * xd.r, rz.i + q * xd.i}, a);
}

__global__ void k_fsphere_step(const double2* __restrict__ in, double2* __restrict__ out,
                               const double2* __restrict__ poles, int N, const double* __restrict__ om,
                               const double* __restrict__ sc, const int* __restrict__ idx_n, double qf, int S,
                               long long nspec, int adjoint) {
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (long long)S * nspec) return;
    const int st = (int)(gid / nspec);
    const long long i = gid - (long long)st * nspec;
    const long long base = (long long)st * 3 * nspec + i;
    const int n = idx_n[i];
    const double p = n > 0 ? om[i] : 0.0, q = n > 0 ? qf : 0.0;
    const double f = adjoint ? 1.0 / sc[i] : sc[i];  // into energy variables
    const cd rP = ld2(in, base), rz = cscale(ld2(in, base + nspec), f), rd = cscale(ld2(in, base + 2 * nspec), f);
    const double sg = adjoint ? -1.0 : 1.0;  // L^H = -L^
    cd aP = mk(0, 0), az = mk(0, 0), ad = mk(0, 0);
    for (int k = 0; k < N; ++k) {
        cd a = ld2(poles, 3LL * k), bp = ld2(poles, 3LL * k + 1), bm = ld2(poles, 3LL * k + 2);
        if (adjoint) {
            a = cconj(a);
            bp = cconj(bp);
            bm = cconj(bm);
        }
        cd xP, xz, xd;
        fsphere_solve(a, sg * p, sg * q, rP, rz, rd, xP, xz, xd);
        aP = cfma(aP, bp, xP);
        az = cfma(az, bp, xz);
        ad = cfma(ad, bp, xd);
        fsphere_solve(a, -sg * p, -sg * q, rP, rz, rd, xP, xz, xd);
        aP = cfma(aP, bm, xP);
        az = cfma(az, bm, xz);
        ad = cfma(ad, bm, xd);
    }
    st2(out, base, aP);
    st2(out, base + nspec, cscale(az, 1.0 / f));
    st2(out, base + 2 * nspec, cscale(ad, 1.0 / f));
}

// LDS of one workgroup: the staged positions of the largest chain group.
// The batched form runs kWaves waves per workgroup (sharing the staged data of
// an item); the per-term form (ACC) one wave per chain.
template <int SE, bool ACC, int KIND, int R>
hipError_t launch_solve_t(const SolveArgs& a, int item0, int nitems, int* counter, hipStream_t s) {
    constexpr int W = ACC ? 1 : kWaves;
    const size_t lds = sizeof(double) * (size_t)SolveLds<SE, KIND, W, R>::kDoubles;
    int grid = nitems;
    if (counter) {
        // resident workgroups of this kernel on the whole device
        int dev = 0, ncu = 0, per_cu = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_solve<SE, ACC, KIND, W, R>, 64 * W, lds);
        if (e != hipSuccess) return e;
        grid = std::max(1, std::min(nitems, std::max(1, per_cu) * ncu));
    }
    hipLaunchKernelGGL((k_solve<SE, ACC, KIND, W, R>), dim3(grid), dim3(64 * W), lds, s, a, item0, nitems, counter);
    return hipGetLastError();
}

// Compiled variants: (elements per lane, move kind, states per item).  States
// share a pole's factorisation when a wave holds at least that many chain
// groups (row and row-pair tilings).  The per-term form needs only the
// tilings of the default policy, one state per item.
constexpr int kVariants[][3] = {
    {4, kMoveRow, 1},  {6, kMoveRow, 1},  {8, kMoveRow, 1},  {10, kMoveRow, 1}, {12, kMoveRow, 1},
    {14, kMoveRow, 1}, {16, kMoveRow, 1}, {4, kMovePair, 1}, {8, kMovePair, 1}, {16, kMoveBperm, 1},
    {4, kMoveRow, 2},  {6, kMoveRow, 2},  {8, kMoveRow, 2},  {10, kMoveRow, 2}, {12, kMoveRow, 2},
    {14, kMoveRow, 2}, {16, kMoveRow, 2}, {4, kMovePair, 2}, {8, kMovePair, 2},
    {4, kMoveRow, 4},  {6, kMoveRow, 4},  {8, kMoveRow, 4},  {10, kMoveRow, 4}, {12, kMoveRow, 4},
    {14, kMoveRow, 4}, {16, kMoveRow, 4}};
constexpr int kPerTermVariants[][3] = {{8, kMoveRow, 1}, {8, kMovePair, 1}, {16, kMoveBperm, 1}};

template <bool ACC>
hipError_t launch_solve(const Launch& L, const SolveArgs& a, int* counter, hipStream_t s) {
    if (L.nitems <= 0) return hipSuccess;
    const int pcap = L.kind == kMoveRow ? 16 : L.kind == kMovePair ? 32 : 64;
    if (L.pmax > pcap) return hipErrorInvalidValue;
    if (L.rot < 1 || L.pmax * L.rot > 64) return hipErrorInvalidValue;  // a wave holds R groups or more
#define REXI_CASE(SE_, K_, R_) \
    if (L.SE == SE_ && L.kind == K_ && L.rot == R_) return launch_solve_t<SE_, ACC, K_, R_>(a, L.item0, L.nitems, counter, s)
    REXI_CASE(8, kMoveRow, 1);
    REXI_CASE(8, kMovePair, 1);
    REXI_CASE(16, kMoveBperm, 1);
    if constexpr (!ACC) {
        REXI_CASE(4, kMoveRow, 1);
        REXI_CASE(6, kMoveRow, 1);
        REXI_CASE(10, kMoveRow, 1);
        REXI_CASE(12, kMoveRow, 1);
        REXI_CASE(14, kMoveRow, 1);
        REXI_CASE(16, kMoveRow, 1);
        REXI_CASE(4, kMovePair, 1);
        REXI_CASE(4, kMoveRow, 2);
        REXI_CASE(6, kMoveRow, 2);
        REXI_CASE(8, kMoveRow, 2);
        REXI_CASE(10, kMoveRow, 2);
        REXI_CASE(12, kMoveRow, 2);
        REXI_CASE(14, kMoveRow, 2);
        REXI_CASE(16, kMoveRow, 2);
        REXI_CASE(4, kMovePair, 2);
        REXI_CASE(8, kMovePair, 2);
        REXI_CASE(4, kMoveRow, 4);
        REXI_CASE(6, kMoveRow, 4);
        REXI_CASE(8, kMoveRow, 4);
        REXI_CASE(10, kMoveRow, 4);
        REXI_CASE(12, kMoveRow, 4);
        REXI_CASE(14, kMoveRow, 4);
        REXI_CASE(16, kMoveRow, 4);
    }
#undef REXI_CASE
    return hipErrorInvalidValue;
}

}  // namespace

bool solve_variant_supported(int SE, int kind, int rot, bool per_term) {
    if (per_term) {
        for (const auto& v : kPerTermVariants)
            if (v[0] == SE && v[1] == kind && v[2] == rot) return true;
        return false;
    }
    for (const auto& v : kVariants)
        if (v[0] == SE && v[1] == kind && v[2] == rot) return true;
    return false;
}
int solve_waves_per_item() { return kWaves; }

int solve_variant_list(bool per_term, int* se, int* kind, int* st, int cap) {
    int n = 0;
    auto put = [&](int a, int b, int c) {
        if (n < cap) {
            if (se) se[n] = a;
            if (kind) kind[n] = b;
            if (st) st[n] = c;
        }
        ++n;
    };
    if (per_term) {
        for (const auto& v : kPerTermVariants) put(v[0], v[1], v[2]);
    } else {
        for (const auto& v : kVariants) put(v[0], v[1], v[2]);
    }
    return n;
}

// Internal launchers used by the C ABI (plan.cpp).
hipError_t enqueue_prep(rexi_plan* pl, const Workspace& ws, const void* u, int buf, int S, int adjoint,
                        const MInfo* d_layout, hipStream_t s) {
    const long long n = (long long)S * pl->nspec;
    const int bs = 256;
    hipLaunchKernelGGL(k_prep, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s, (const double2*)u,
                       ws.ch_var[buf], ws.ch_phi[buf], d_layout, pl->d_idx_n, pl->d_idx_m, pl->d_sc,
                       adjoint, S, pl->nspec, pl->nslots + 2, pl->nslots);
    return hipGetLastError();
}

hipError_t enqueue_solve(rexi_plan* pl, const Workspace& ws, const Schedule& sc, int buf, int S, int adjoint,
                         hipStream_t s) {
    SolveArgs a;
    a.items = sc.d_items;
    a.minfo = sc.d_minfo;
    a.th = pl->d_th;
    a.om = pl->d_om;
    a.cc = pl->d_cc;
    a.poles = reinterpret_cast<const PoleData*>(pl->d_poles[adjoint]);
    a.ch_var = ws.ch_var[buf];
    a.ch_phi = ws.ch_phi[buf];
    a.part = ws.part;
    a.T = pl->T;
    a.S = S;
    a.var_stride = pl->nslots + 2;
    a.nspec = pl->nspec;
    if (sc.persistent) {
        const int n = (int)sc.launches.size();
        if (n > kMaxLaunches) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, s, ws.counters, n);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int nl = (int)sc.launches.size();
    if (!pl->concurrent || nl < 2) {
        for (int c = 0; c < nl; ++c) {
            hipError_t e = launch_solve<false>(sc.launches[c], a, sc.persistent ? ws.counters + c : nullptr, s);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    // fork: every class on its own side stream after the work already on s;
    // join: s waits for all of them (each class writes its own partials)
    hipError_t e = hipEventRecord(pl->fork_ev, s);
    for (int c = 0; c < nl && e == hipSuccess; ++c) {
        e = hipStreamWaitEvent(pl->side[c], pl->fork_ev, 0);
        if (e == hipSuccess)
            e = launch_solve<false>(sc.launches[c], a, sc.persistent ? ws.counters + c : nullptr, pl->side[c]);
        if (e == hipSuccess) e = hipEventRecord(pl->join_ev[c], pl->side[c]);
    }
    for (int c = 0; c < nl && e == hipSuccess; ++c) e = hipStreamWaitEvent(s, pl->join_ev[c], 0);
    return e;
}

hipError_t enqueue_reduce(rexi_plan* pl, const Workspace& ws, const Schedule& sc, const double2* part, int buf_in,
                          int buf_out, void* u_out, int S, int adjoint, const int* d_slot_m, hipStream_t s) {
    ReduceArgs r;
    r.minfo = sc.d_minfo;
    r.groups = sc.d_groups;
    r.slot_m = d_slot_m;
    r.om = pl->d_om;
    r.sc = pl->d_sc;
    r.part = part;
    r.ch_var_in = ws.ch_var[buf_in];
    r.ch_phi_in = ws.ch_phi[buf_in];
    r.ch_var_out = u_out ? nullptr : ws.ch_var[buf_out];
    r.ch_phi_out = u_out ? nullptr : ws.ch_phi[buf_out];
    r.u_out = (double2*)u_out;
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

hipError_t enqueue_finish(rexi_plan* pl, const Workspace& ws, int buf, void* u, int S, int adjoint,
                          const MInfo* d_layout, hipStream_t s) {
    const long long n = (long long)S * pl->nspec;
    const int bs = 256;
    hipLaunchKernelGGL(k_finish, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s, ws.ch_var[buf],
                       ws.ch_phi[buf], (double2*)u, d_layout, pl->d_idx_n, pl->d_idx_m, pl->d_sc, adjoint, S,
                       pl->nspec, pl->nslots + 2, pl->nslots);
    return hipGetLastError();
}

hipError_t enqueue_fsphere_step(rexi_plan* pl, const void* in, void* out, int S, int adjoint, hipStream_t s) {
    const long long n = (long long)S * pl->nspec;
    const int bs = 256;
    hipLaunchKernelGGL(k_fsphere_step, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s, (const double2*)in,
                       (double2*)out, pl->d_fs_poles, pl->N, pl->d_om, pl->d_sc, pl->d_idx_n, pl->f0dt, S,
                       pl->nspec, adjoint);
    return hipGetLastError();
}

hipError_t enqueue_zero(double2* p, long long n, hipStream_t s) {
    const int bs = 256;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s, p, n);
    return hipGetLastError();
}

// Per-term form: one launch per pole over all (m, p, tile) items, each adding
// its pole's weighted solution into the accumulator (fixed pole order).
hipError_t enqueue_per_term_pole(rexi_plan* pl, const Workspace& ws, const Schedule& sc, int k, int buf, int S,
                                 hipStream_t s) {
    SolveArgs a;
    a.items = sc.d_items;
    a.minfo = sc.d_minfo;
    a.th = pl->d_th;
    a.om = pl->d_om;
    a.cc = pl->d_cc;
    a.poles = reinterpret_cast<const PoleData*>(pl->d_poles[0]) + k;
    a.ch_var = ws.ch_var[buf];
    a.ch_phi = ws.ch_phi[buf];
    a.part = pl->d_acc;
    a.T = pl->T;
    a.S = S;
    a.var_stride = pl->nslots + 2;
    a.nspec = pl->nspec;
    for (const Launch& L : sc.launches) {
        hipError_t e = launch_solve<true>(L, a, nullptr, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace rexi
