// C ABI of the T-REXI library: argument checking, plans, schedules, step
// drivers and the schedule autotuner.  The arithmetic runs in the HIP kernels
// (rexi_kernels.hip, sh_kernels.hip); this file only prepares tables and
// enqueues work.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "internal.hpp"

namespace rexi {


namespace {
thread_local std::string g_err;
}

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(REXI_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

hipError_t timed_begin(rexi_plan* pl, int kind, hipStream_t s) {
    if (!pl->timing) return hipSuccess;
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e != hipSuccess) return e;
    e = hipEventCreate(&b);
    if (e != hipSuccess) { (void)hipEventDestroy(a); return e; }
    pl->events[kind].push_back({a, b});
    return hipEventRecord(a, s);
}

hipError_t timed_end(rexi_plan* pl, int kind, hipStream_t s) {
    if (!pl->timing || pl->events[kind].empty()) return hipSuccess;
    return hipEventRecord(pl->events[kind].back().second, s);
}

namespace {

template <class T>
int dev_alloc(T** p, size_t count) {
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void**)p, count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(REXI_ENOMEM, std::string("hipMalloc of ") + std::to_string(count * sizeof(T)) +
                                     " bytes failed: " + hipGetErrorString(e));
    }
    return REXI_OK;
}

template <class T>
int upload(T** p, const std::vector<T>& v) {
    int rc = dev_alloc(p, v.size());
    if (rc) return rc;
    REXI_HIP(hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return REXI_OK;
}

template <class T>
void dev_free(T*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

int check_params(const rexi_params* p) {
    if (!p) return fail(REXI_EINVAL, "params is NULL");
    if (p->T < 1 || p->T > 1023) return fail(REXI_EINVAL, "T must be in [1, 1023]");
    if (!(p->dt > 0) || !std::isfinite(p->dt)) return fail(REXI_EINVAL, "dt must be positive and finite");
    if (!(p->radius > 0) || !(p->gravity > 0) || !(p->mean_depth > 0) || !std::isfinite(p->omega))
        return fail(REXI_EINVAL, "radius, gravity and mean_depth must be positive, omega finite");
    if (p->M < 1 || p->M > 1 << 20) return fail(REXI_EINVAL, "M must be in [1, 2^20]");
    if (!(p->h > 0) || !std::isfinite(p->h)) return fail(REXI_EINVAL, "h must be positive");
    if (p->L < 1 || p->L > 32) return fail(REXI_EINVAL, "L must be in [1, 32]");
    if (p->max_states < 1 || p->max_states > 64) return fail(REXI_EINVAL, "max_states must be in [1, 64]");
    if (p->fsphere != 0 && p->fsphere != 1) return fail(REXI_EINVAL, "fsphere must be 0 or 1");
    if (p->fsphere && !std::isfinite(p->f0)) return fail(REXI_EINVAL, "f0 must be finite");
    if (p->nlat != 0 || p->nlon != 0) {
        if (p->nlat < 2 || p->nlat > 2048 || (p->nlat & 1))
            return fail(REXI_EINVAL, "nlat must be even and in [2, 2048]");
        if (p->nlon < 4 || p->nlon > 4096 || (p->nlon & (p->nlon - 1)))
            return fail(REXI_EINVAL, "nlon must be a power of two in [4, 4096]");
        if (p->T >= p->nlon) return fail(REXI_EINVAL, "T must be below nlon");
        if (p->max_fields < 1 || p->max_fields > 1024) return fail(REXI_EINVAL, "max_fields must be in [1, 1024]");
    }
    return REXI_OK;
}

long double eps_nm(int n, int m) {
    if (n <= 0 || n < m) return 0.0L;
    return sqrtl((long double)((long long)n * n - (long long)m * m) / (4.0L * n * n - 1.0L));
}

// Layout of the chain slots (independent of the lane tiling).
std::vector<MInfo> chain_layout(int T) {
    std::vector<MInfo> mi(T + 1);
    long long slot = 0;
    for (int m = 0; m <= T; ++m) {
        MInfo x{};
        x.n0 = std::max(m, 1);
        x.L = T + 1 - x.n0;
        x.spec_off = (int)spec_offset(T, m);
        x.slot_base = (int)slot;
        slot += 2LL * x.L;
        mi[m] = x;
    }
    return mi;
}

// Elements-per-lane class SE and cross-lane move kind of a chain of L
// elements under a policy.  Kinds: 0 ds_bpermute (groups up to 64 lanes),
// 1 DPP row shifts (groups inside one 16-lane row), 2 DPP over a pair of rows
// (groups of exactly 32 lanes).
//   0 "8":       8 (L <= 128, rows), 8 (L <= 256, row pairs)
//   1 "8/16":    8 (L <= 128), 16 (<= 256), rows
//   2 "16":      16 (L <= 256), rows
//   3 "8/12/16": 8 (L <= 128), 12 (<= 192), 16 (<= 256), rows
//   4 "4/8":     4 (L <= 64, rows), 4 (L <= 128, row pairs), 8 (L <= 256, row pairs)
//   5 "fine":    8 (L <= 64), 6 (<= 96), 8 (<= 128), 10 (<= 160), 12 (<= 192),
//                14 (<= 224), 16 (<= 256), rows: padding at most 2 elements per lane
// Beyond 256 elements every policy uses 16 with ds_bpermute (L <= 1024).
void tile_class(int policy, int L, int& SE, int& kind) {
    kind = 1;
    switch (policy) {
        case 0:
            if (L <= 128) { SE = 8; return; }
            if (L <= 256) { SE = 8; kind = 2; return; }
            break;
        case 1:
            if (L <= 128) { SE = 8; return; }
            if (L <= 256) { SE = 16; return; }
            break;
        case 2:
            if (L <= 256) { SE = 16; return; }
            break;
        case 3:
            if (L <= 128) { SE = 8; return; }
            if (L <= 192) { SE = 12; return; }
            if (L <= 256) { SE = 16; return; }
            break;
        case 4:
            if (L <= 64) { SE = 4; return; }
            if (L <= 128) { SE = 4; kind = 2; return; }
            if (L <= 256) { SE = 8; kind = 2; return; }
            break;
        default:
            if (L <= 64) { SE = 8; return; }
            if (L <= 256) { SE = 2 * ((L + 31) / 32); return; }  // 16 lanes x SE >= L
            break;
    }
    kind = 0;
    SE = 16;
}

const char* kPolicyName[] = {"8", "8/16", "16", "8/12/16", "4/8", "fine"};
constexpr int kPolicies = 6;

// Work split of one candidate schedule.  Items are (m, chain, state tile,
// pole range).  Per order the tile holds R states, the largest of 4, 2, 1
// that is at most the mode's limit, divides S, fits the chain groups of a wave
// (P R <= 64) and is compiled; the item's waves then factorise each pole
// once for its R states.  Modes: 0 one state per item; 1 the most states per
// item in every class; 2 the same only for tiles of at most 6 or at least 14
// elements per lane (measured at T256: sharing gains 14-20% there, while
// the 8-element tile loses its second wave per SIMD to the factorisation's
// LDS and the 10- and 12-element tiles gain nothing).  The number of items per (m, chain, tile) follows a
// cost model per wave iteration (elements x sweep work + log2(P) reduction
// levels, the factorising pass and R - 1 passes that reuse it, scaled by the
// waves a SIMD can hold for the class).  One launch per (SE, kind, R) class;
// items in a launch run longest first.
int build_schedule(rexi_plan* pl, int S, int policy, long long target_items, bool per_term, int rot_mode,
                   Schedule& out) {
    const int rot_max = rot_mode == 0 ? 1 : 4;
    const int T = pl->T, N = per_term ? 1 : pl->N;
    out = Schedule();
    out.rot_max = rot_max;
    out.S = S;
    out.minfo = chain_layout(T);
    struct Unit { int m, p, tile, rot; double cost; int iters; int G; int cls; };
    std::vector<Unit> units;
    struct Cls { int SE, kind, rot; };
    std::vector<Cls> classes;
    double total = 0;
    for (int m = 0; m <= T; ++m) {
        MInfo& mi = out.minfo[m];
        int SE, kind;
        tile_class(policy, mi.L, SE, kind);
        int P = 1;
        while (P * SE < mi.L) P *= 2;
        if (kind == 1 ? P > 16 : kind == 2 ? P != 32 : P > 64)
            return fail(REXI_EUNSUPPORTED, "chain length does not fit this tiling");
        int rot = 1;
        const bool share = rot_mode == 1 || (rot_mode == 2 && (SE <= 6 || SE >= 14));
        for (int r : {4, 2})
            if (share && r <= rot_max && S % r == 0 && P * r <= 64 && solve_variant_supported(SE, kind, r, per_term)) {
                rot = r;
                break;
            }
        if (!solve_variant_supported(SE, kind, rot, per_term)) return fail(REXI_EUNSUPPORTED, "tile class not compiled");
        mi.P = P;
        mi.s = SE;
        out.SM = std::max(out.SM, SE);
        int cls = -1;
        for (int c = 0; c < (int)classes.size(); ++c)
            if (classes[c].SE == SE && classes[c].kind == kind && classes[c].rot == rot) cls = c;
        if (cls < 0) { cls = (int)classes.size(); classes.push_back({SE, kind, rot}); }
        const int G = 64 / P * (per_term ? 1 : solve_waves_per_item());  // poles per workgroup iteration
        int lg = 0;
        while ((1 << lg) < P) ++lg;
        const double occ = (SE <= 8 && rot == 1) ? 2.0 : 1.0;
        const double lvl = kind == 0 ? 160.0 : kind == 2 ? 100.0 : 90.0;
        const double fused = SE * 100.0 + lg * lvl + 60.0;
        const double reuse = SE * 65.0 + lg * 0.5 * lvl + 40.0;
        const double it_cost = (fused + (rot - 1) * reuse) / occ;
        const int iters = (N + G - 1) / G;
        for (int p = 0; p < 2; ++p)
            for (int t = 0; t < S / rot; ++t) {
                units.push_back({m, p, t, rot, it_cost * iters, iters, G, cls});
                total += it_cost * iters;
            }
    }
    const double target = per_term ? 1e300 : total / (double)std::max<long long>(1, target_items);
    out.groups.assign((size_t)(T + 1) * 2 * S, Group{0, 0, 0});
    long long off = 0;
    std::vector<std::vector<std::pair<double, Item>>> by_class(classes.size());
    for (const Unit& u : units) {
        int nr = (int)std::lround(u.cost / target);
        nr = std::max(1, std::min(nr, u.iters));
        const long long L2 = 2LL * out.minfo[u.m].L;
        for (int q = 0; q < u.rot; ++q) {
            Group& gr = out.groups[((size_t)u.m * 2 + u.p) * S + u.tile * u.rot + q];
            gr.part_off = off + q * L2;
            gr.nr = nr;
            gr.st = u.rot;
        }
        for (int r = 0; r < nr; ++r) {
            const int i0 = (int)((long long)u.iters * r / nr), i1 = (int)((long long)u.iters * (r + 1) / nr);
            Item it;
            it.m = u.m;
            it.p = u.p;
            it.tile = u.tile;
            it.k0 = i0 * u.G;
            it.k1 = std::min(N, i1 * u.G);
            it.part_off = off;
            off += u.rot * L2;
            by_class[u.cls].push_back({u.cost * (i1 - i0) / u.iters, it});
        }
    }
    for (int c = 0; c < (int)classes.size(); ++c) {
        auto& v = by_class[c];
        std::stable_sort(v.begin(), v.end(), [](const std::pair<double, Item>& a, const std::pair<double, Item>& b) {
            return a.first > b.first;
        });
        int pmax = 1;
        for (auto& x : v) pmax = std::max(pmax, out.minfo[x.second.m].P);
        Launch L{classes[c].SE, classes[c].kind, (int)out.items.size(), (int)v.size(), pmax, classes[c].rot};
        for (auto& x : v) out.items.push_back(x.second);
        out.launches.push_back(L);
    }
    out.part_size = off;
    // "_shared": every class shares factorisations among states, "_mixed": some do
    int nshare = 0;
    for (const Cls& c : classes) nshare += c.rot > 1;
    const char* share_tag = nshare == 0 ? "" : nshare == (int)classes.size() ? "_shared" : "_mixed";
    char buf[96];
    std::snprintf(buf, sizeof buf, "%s_items%lld%s%s", kPolicyName[policy], (long long)out.items.size(), share_tag,
                  per_term ? "_perterm" : "");
    out.name = buf;
    int rc = upload(&out.d_minfo, out.minfo);
    if (!rc) rc = upload(&out.d_items, out.items);
    if (!rc) rc = upload(&out.d_groups, out.groups);
    return rc;
}

void free_schedule(Schedule& s) {
    dev_free(s.d_minfo);
    dev_free(s.d_items);
    dev_free(s.d_groups);
}

// Each graph is destroyed only after its last launch has completed (its
// buffers may be freed or reused right after: ensure_part, schedule and
// stream changes).
void drop_graphs(rexi_plan* pl) {
    for (auto& g : pl->graphs) {
        if (g.done) {
            (void)hipEventSynchronize(g.done);
            (void)hipEventDestroy(g.done);
        }
        (void)hipGraphExecDestroy(g.exec);
    }
    pl->graphs.clear();
    ++pl->graph_gen;
}

int ensure_part(rexi_plan* pl, long long n) {
    if (n <= pl->part_capacity) return REXI_OK;
    drop_graphs(pl);
    dev_free(pl->d_part);
    pl->part_capacity = 0;
    int rc = dev_alloc(&pl->d_part, (size_t)n);
    if (rc) return rc;
    pl->part_capacity = n;
    return REXI_OK;
}

// Candidate schedules for S states (built on first use).
int schedules_for(rexi_plan* pl, int S, std::vector<Schedule>** out) {
    if ((int)pl->sched.size() <= S) {
        pl->sched.resize(S + 1);
        pl->chosen.resize(S + 1, -1);
    }
    std::vector<Schedule>& c = pl->sched[S];
    if (c.empty()) {
        // item targets: ~2816 measured fastest at T256 (four states per
        // item, concurrent classes), by 3% over ~4096, with ~2048 and ~3072
        // on either side slower
        const long long tg[] = {2048, 2816, 4096, 8192};
        // states per item (see build_schedule): one (each state factorises
        // its own poles), and for an even number of states up to four sharing
        // each factorisation, in every tile class or in some
        std::vector<int> rots = {0};
        if (S % 2 == 0) {
            rots.push_back(1);
            rots.push_back(2);
        }
        int dflt = -1;
        for (int rot : rots)
        for (int persistent = 0; persistent < 2; ++persistent)
            for (int policy = 0; policy < kPolicies; ++policy)
                for (long long t : tg) {
                    Schedule sc;
                    int rc = build_schedule(pl, S, policy, t, false, rot, sc);
                    if (rc == REXI_EUNSUPPORTED) { free_schedule(sc); continue; }
                    if (rc) { free_schedule(sc); return rc; }
                    if ((int)sc.launches.size() > kMaxLaunches) { free_schedule(sc); continue; }
                    sc.persistent = persistent != 0;
                    if (sc.persistent) sc.name = "persistent_" + sc.name;
                    rc = ensure_part(pl, sc.part_size);
                    if (rc) { free_schedule(sc); return rc; }
                    // until autotuned: "fine", ~2816 items, one launch per item,
                    // states sharing factorisations where that measured faster
                    if (!persistent && policy == 5 && t == 2816 && rot == rots.back()) dflt = (int)c.size();
                    c.push_back(sc);
                }
        if (c.empty()) return fail(REXI_EUNSUPPORTED, "no schedule fits this truncation");
        pl->chosen[S] = dflt >= 0 ? dflt : 0;
    }
    *out = &c;
    return REXI_OK;
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
    const char* x = (const char*)a;
    const char* y = (const char*)b;
    return x < y + nb && y < x + na;
}


// The graph of one step for (S, direction, input buffer): solve launches and
// the reduction into the other chain buffer, captured on the plan's stream.
int step_graph(rexi_plan* pl, const Schedule& sc, int S, int adjoint, int buf, hipGraphExec_t* out,
               hipEvent_t* done) {
    for (auto& g : pl->graphs)
        if (g.sched == &sc && g.S == S && g.adjoint == adjoint && g.buf == buf && g.gen == pl->graph_gen) {
            *out = g.exec;
            *done = g.done;
            return REXI_OK;
        }
    hipGraph_t graph = nullptr;
    REXI_HIP(hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal));
    const Workspace ws = plan_workspace(pl);
    hipError_t e1 = enqueue_solve(pl, ws, sc, buf, S, adjoint, pl->cap_stream);
    hipError_t e2 = hipSuccess;
    if (e1 == hipSuccess)
        e2 = enqueue_reduce(pl, ws, sc, ws.part, buf, buf ^ 1, nullptr, S, adjoint, pl->d_slot_m, pl->cap_stream);
    hipError_t e3 = hipStreamEndCapture(pl->cap_stream, &graph);
    if (e1 != hipSuccess) { if (graph) (void)hipGraphDestroy(graph); return hip_fail(e1, "capture solve"); }
    if (e2 != hipSuccess) { if (graph) (void)hipGraphDestroy(graph); return hip_fail(e2, "capture reduce"); }
    if (e3 != hipSuccess) return hip_fail(e3, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    hipError_t e4 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e4 != hipSuccess) return hip_fail(e4, "hipGraphInstantiate");
    hipEvent_t ev = nullptr;
    hipError_t e5 = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e5 != hipSuccess) {
        (void)hipGraphExecDestroy(exec);
        return hip_fail(e5, "hipEventCreateWithFlags");
    }
    pl->graphs.push_back({&sc, S, adjoint, buf, pl->graph_gen, exec, ev});
    *out = exec;
    *done = ev;
    return REXI_OK;
}

int run_steps(rexi_plan* pl, const Schedule& sc, const void* u0, void* u1, int S, int nsteps, int adjoint,
              hipStream_t s) {
    const size_t bytes = (size_t)S * 3 * pl->nspec * 16;
    if (nsteps == 0) {
        REXI_HIP(hipMemcpyAsync(u1, u0, bytes, hipMemcpyDeviceToDevice, s));
        return REXI_OK;
    }
    const Workspace ws = plan_workspace(pl);
    REXI_HIP(enqueue_prep(pl, ws, u0, 0, S, adjoint, pl->sched_layout, s));
    int cur = 0;
    if (pl->use_graphs) {
        // captured step graphs (solve + reduction), then the final layout
        // change; with timing on, each replay is bracketed by an event pair
        for (int k = 0; k < nsteps; ++k) {
            hipGraphExec_t exec = nullptr;
            hipEvent_t done = nullptr;
            int rc = step_graph(pl, sc, S, adjoint, cur, &exec, &done);
            if (rc) return rc;
            REXI_HIP(timed_begin(pl, REXI_KERNEL_SOLVE, s));
            REXI_HIP(hipGraphLaunch(exec, s));
            REXI_HIP(timed_end(pl, REXI_KERNEL_SOLVE, s));
            REXI_HIP(hipEventRecord(done, s));
            cur ^= 1;
        }
        REXI_HIP(enqueue_finish(pl, ws, cur, u1, S, adjoint, pl->sched_layout, s));
        return REXI_OK;
    }
    for (int k = 0; k < nsteps; ++k) {
        const bool last = (k == nsteps - 1);
        REXI_HIP(timed_begin(pl, REXI_KERNEL_SOLVE, s));
        REXI_HIP(enqueue_solve(pl, ws, sc, cur, S, adjoint, s));
        REXI_HIP(timed_end(pl, REXI_KERNEL_SOLVE, s));
        REXI_HIP(enqueue_reduce(pl, ws, sc, ws.part, cur, cur ^ 1, last ? u1 : nullptr, S, adjoint, pl->d_slot_m, s));
        cur ^= 1;
    }
    return REXI_OK;
}

}  // namespace

int check_state_call(rexi_plan* pl, const void* in, const void* out, int S, int nsteps) {
    if (!pl) return fail(REXI_EINVAL, "plan is NULL");
    if (!in || !out) return fail(REXI_EINVAL, "state pointer is NULL");
    if (S < 1) return fail(REXI_EINVAL, "S must be >= 1");
    if (S > pl->prm.max_states) return fail(REXI_EUNSUPPORTED, "S exceeds the plan's max_states");
    if (nsteps < 0) return fail(REXI_EINVAL, "nsteps must be >= 0");
    const size_t bytes = (size_t)S * 3 * pl->nspec * 16;
    if (overlaps(in, bytes, out, bytes)) return fail(REXI_EALIAS, "output overlaps input");
    return REXI_OK;
}

}  // namespace rexi

using namespace rexi;

namespace {

// f-sphere steps: the closed-form kernel, alternating between u1 and the work
// buffer so that the last step lands in u1.
int run_fsphere(rexi_plan* pl, const void* u0, void* u1, int S, int nsteps, int adjoint, hipStream_t s) {
    const size_t bytes = (size_t)S * 3 * pl->nspec * 16;
    if (nsteps == 0) {
        REXI_HIP(hipMemcpyAsync(u1, u0, bytes, hipMemcpyDeviceToDevice, s));
        return REXI_OK;
    }
    const void* src = u0;
    for (int k = 0; k < nsteps; ++k) {
        void* dst = ((nsteps - 1 - k) % 2 == 0) ? u1 : (void*)pl->d_fs_work;
        REXI_HIP(enqueue_fsphere_step(pl, src, dst, S, adjoint, s));
        src = dst;
    }
    return REXI_OK;
}

int do_step(rexi_plan* pl, const void* u0, void* u1, int S, int nsteps, int adjoint, void* stream) {
    int rc = check_state_call(pl, u0, u1, S, nsteps);
    if (rc) return rc;
    if (pl->prm.fsphere) return run_fsphere(pl, u0, u1, S, nsteps, adjoint, (hipStream_t)stream);
    std::vector<Schedule>* c = nullptr;
    rc = schedules_for(pl, S, &c);
    if (rc) return rc;
    return run_steps(pl, (*c)[pl->chosen[S]], u0, u1, S, nsteps, adjoint, (hipStream_t)stream);
}

void drop_events(rexi_plan* pl) {
    for (auto& v : pl->events) {
        for (auto& ab : v) {
            (void)hipEventDestroy(ab.first);
            (void)hipEventDestroy(ab.second);
        }
        v.clear();
    }
}

void release(rexi_plan* pl) {
    drop_events(pl);
    drop_graphs(pl);
    dev_free(pl->d_counters);
    if (pl->cap_stream) (void)hipStreamDestroy(pl->cap_stream);
    pl->cap_stream = nullptr;
    for (int c = 0; c < kMaxLaunches; ++c) {
        if (pl->side[c]) (void)hipStreamDestroy(pl->side[c]);
        if (pl->join_ev[c]) (void)hipEventDestroy(pl->join_ev[c]);
        pl->side[c] = nullptr;
        pl->join_ev[c] = nullptr;
    }
    if (pl->fork_ev) (void)hipEventDestroy(pl->fork_ev);
    pl->fork_ev = nullptr;
    for (auto& c : pl->sched)
        for (auto& s : c) free_schedule(s);
    for (auto& s : pl->per_term) free_schedule(s);
    dev_free(pl->d_th);
    dev_free(pl->d_om);
    dev_free(pl->d_cc);
    dev_free(pl->d_sc);
    dev_free(pl->d_idx_n);
    dev_free(pl->d_idx_m);
    for (int d = 0; d < 2; ++d) {
        dev_free(pl->d_poles[d]);
        dev_free(pl->d_ch_var[d]);
        dev_free(pl->d_ch_phi[d]);
    }
    dev_free(pl->d_part);
    dev_free(pl->d_acc);
    dev_free(pl->d_fs_poles);
    dev_free(pl->d_fs_work);
    dev_free(pl->sched_layout);
    dev_free(pl->d_slot_m);
    sh_release(pl);
}

std::vector<double2> to_d2(const std::vector<std::complex<double>>& v) {
    std::vector<double2> o(v.size());
    for (size_t i = 0; i < v.size(); ++i) o[i] = make_double2(v[i].real(), v[i].imag());
    return o;
}

int create(const rexi_params* p, rexi_plan** out) {
    int rc = check_params(p);
    if (rc) return rc;
    rexi_plan* pl = new rexi_plan();
    pl->prm = *p;
    const int T = p->T;
    pl->T = T;
    pl->N = 2 * (p->M + p->L) + 1;
    pl->nspec = nspec_of(T);
    pl->nslots = 2 * (pl->nspec - 1);
    pl->phibar = p->gravity * p->mean_depth;
    pl->poles = make_poles(p->M, p->h, p->L, p->normalize);
    const int N = pl->N;
    typedef std::complex<double> C;
    std::vector<C> ainv(N), wx[2], wy[2], wxa[2], wya[2];
    for (int d = 0; d < 2; ++d) {
        wx[d].resize(N);
        wy[d].resize(N);
        wxa[d].resize(N);
        wya[d].resize(N);
    }
    C g00(0, 0), gx[2] = {C(0, 0), C(0, 0)}, gy[2] = {C(0, 0), C(0, 0)};
    for (int k = 0; k < N; ++k) {
        const C a = pl->poles.alpha[k];
        ainv[k] = 1.0 / a;
        const C bp = pl->poles.beta_plus[k];
        const C bm_mirror = std::conj(pl->poles.beta_minus[N - 1 - k]);  // conj(beta-_{-k})
        wx[0][k] = bp;
        wy[0][k] = bm_mirror;
        wx[1][k] = bm_mirror;
        wy[1][k] = bp;
        for (int d = 0; d < 2; ++d) {
            wxa[d][k] = wx[d][k] / a;
            wya[d][k] = wy[d][k] / a;
            gx[d] += wxa[d][k];
            gy[d] += wya[d][k];
        }
        g00 += (pl->poles.beta_plus[k] + pl->poles.beta_minus[k]) / a;
    }
    pl->g00_fwd = g00;
    pl->g00_adj = std::conj(g00);
    pl->gphi_fwd = gx[0] + std::conj(gy[0]);
    pl->gphi_adj = gx[1] + std::conj(gy[1]);

    // per-(n, m) constants of the energy-scaled operator (times dt)
    const long long ns = pl->nspec;
    std::vector<double> th(ns), om(ns), cc(ns), sc(ns);
    std::vector<int> in(ns), im(ns);
    const long double a = p->radius, Om = p->omega, pb = pl->phibar, dt = p->dt;
    for (int m = 0; m <= T; ++m)
        for (int n = m; n <= T; ++n) {
            const long long i = spec_offset(T, m) + (n - m);
            in[i] = n;
            im[i] = m;
            if (n == 0) {
                th[i] = om[i] = cc[i] = 0.0;
                sc[i] = 1.0;
                continue;
            }
            const long double nn = (long double)n * (n + 1);
            th[i] = (double)(2 * Om * m / nn * dt);
            om[i] = (double)(sqrtl(pb * nn) / a * dt);
            const long double kap = eps_nm(n, m) * sqrtl((long double)n * n - 1) / n;
            cc[i] = (double)(2 * Om * dt * kap);
            sc[i] = (double)(a * sqrtl(pb / nn));
        }
    std::vector<MInfo> lay = chain_layout(T);
    std::vector<int> slot_m(pl->nslots);
    for (int m = 0; m <= T; ++m)
        for (int q = 0; q < 2 * lay[m].L; ++q) slot_m[lay[m].slot_base + q] = m;

    rc = upload(&pl->d_th, th);
    if (!rc) rc = upload(&pl->d_om, om);
    if (!rc) rc = upload(&pl->d_cc, cc);
    if (!rc) rc = upload(&pl->d_sc, sc);
    if (!rc) rc = upload(&pl->d_idx_n, in);
    if (!rc) rc = upload(&pl->d_idx_m, im);
    for (int d = 0; d < 2 && !rc; ++d) {
        std::vector<std::complex<double>> pd;
        pd.reserve(6 * (size_t)N);
        for (int k = 0; k < N; ++k) {
            pd.push_back(pl->poles.alpha[k]);
            pd.push_back(ainv[k]);
            pd.push_back(wx[d][k]);
            pd.push_back(wy[d][k]);
            pd.push_back(wxa[d][k]);
            pd.push_back(wya[d][k]);
        }
        rc = upload(&pl->d_poles[d], to_d2(pd));
    }
    if (!rc) rc = upload(&pl->sched_layout, lay);
    if (!rc) rc = upload(&pl->d_slot_m, slot_m);
    for (int d = 0; d < 2 && !rc; ++d) {
        rc = dev_alloc(&pl->d_ch_var[d], (size_t)p->max_states * (pl->nslots + 2));
        if (!rc) rc = dev_alloc(&pl->d_ch_phi[d], (size_t)p->max_states * pl->nspec);
    }
    if (!rc && p->fsphere) {
        pl->f0dt = p->f0 * p->dt;
        std::vector<std::complex<double>> fp;
        fp.reserve(3 * (size_t)N);
        for (int k = 0; k < N; ++k) {
            fp.push_back(pl->poles.alpha[k]);
            fp.push_back(pl->poles.beta_plus[k]);
            fp.push_back(pl->poles.beta_minus[k]);
        }
        rc = upload(&pl->d_fs_poles, to_d2(fp));
        if (!rc) rc = dev_alloc(&pl->d_fs_work, (size_t)p->max_states * 3 * pl->nspec);
    }
    if (!rc) rc = dev_alloc(&pl->d_counters, kMaxLaunches);
    if (!rc) {
        hipError_t e = hipMemset(pl->d_counters, 0, kMaxLaunches * sizeof(int));
        if (e != hipSuccess) rc = hip_fail(e, "hipMemset");
    }
    if (!rc) {
        hipError_t e = hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) rc = hip_fail(e, "hipStreamCreateWithFlags");
    }
    for (int c = 0; c < kMaxLaunches && !rc; ++c) {
        hipError_t e = hipStreamCreateWithFlags(&pl->side[c], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->join_ev[c], hipEventDisableTiming);
        if (e != hipSuccess) rc = hip_fail(e, "side stream / event");
    }
    if (!rc) {
        hipError_t e = hipEventCreateWithFlags(&pl->fork_ev, hipEventDisableTiming);
        if (e != hipSuccess) rc = hip_fail(e, "hipEventCreateWithFlags");
    }
    if (!rc) {
        hipError_t e = hipGetDevice(&pl->device);
        if (e != hipSuccess) rc = hip_fail(e, "hipGetDevice");
    }
    // the no-allocation step's workspace on this device (looked up once per device)
    if (!rc) rc = scratch_setup(&pl->scratch, &pl->scratch_bytes);
    if (!rc && p->nlat > 0) rc = sh_setup(pl);
    if (rc) {
        release(pl);
        delete pl;
        return rc;
    }
    *out = pl;
    return REXI_OK;
}

}  // namespace

extern "C" {

const char* rexi_last_error(void) { return g_err.c_str(); }

int rexi_coeffs(int M, double h, int L, int normalize, int capacity, double* alpha, double* beta_plus,
                double* beta_minus, int* n_poles) {
    try {
        g_err.clear();
        if (M < 1 || M > 1 << 20) return fail(REXI_EINVAL, "M must be in [1, 2^20]");
        if (!(h > 0) || !std::isfinite(h)) return fail(REXI_EINVAL, "h must be positive");
        if (L < 1 || L > 32) return fail(REXI_EINVAL, "L must be in [1, 32]");
        if (capacity < 0) return fail(REXI_EINVAL, "capacity must be >= 0");
        const int N = 2 * (M + L) + 1;
        if (n_poles) *n_poles = N;
        if (capacity == 0) return REXI_OK;
        if (capacity < N) return fail(REXI_EINVAL, "capacity below the number of poles");
        if (!alpha || !beta_plus || !beta_minus) return fail(REXI_EINVAL, "output array is NULL");
        const Poles P = make_poles(M, h, L, normalize);
        for (int k = 0; k < N; ++k) {
            alpha[2 * k] = P.alpha[k].real();
            alpha[2 * k + 1] = P.alpha[k].imag();
            beta_plus[2 * k] = P.beta_plus[k].real();
            beta_plus[2 * k + 1] = P.beta_plus[k].imag();
            beta_minus[2 * k] = P.beta_minus[k].real();
            beta_minus[2 * k + 1] = P.beta_minus[k].imag();
        }
        return REXI_OK;
    } catch (const std::bad_alloc&) {
        return fail(REXI_ENOMEM, "host allocation failed");
    }
}

int rexi_plan_create(const rexi_params* p, rexi_plan** out) {
    if (!out) return fail(REXI_EINVAL, "out is NULL");
    *out = nullptr;
    try {
        return create(p, out);
    } catch (const std::bad_alloc&) {
        return fail(REXI_ENOMEM, "host allocation failed");
    }
}

int rexi_plan_destroy(rexi_plan* plan) {
    if (!plan) return fail(REXI_EINVAL, "plan is NULL");
    release(plan);
    delete plan;
    return REXI_OK;
}

int rexi_plan_info(const rexi_plan* plan, int* n_poles, int* nspec, long long* blocks) {
    if (!plan) return fail(REXI_EINVAL, "plan is NULL");
    if (n_poles) *n_poles = plan->N;
    if (nspec) *nspec = (int)plan->nspec;
    if (blocks) *blocks = (long long)plan->N * (plan->T + 1);
    return REXI_OK;
}

int rexi_plan_coeffs(const rexi_plan* plan, double* alpha, double* beta_plus, double* beta_minus) {
    if (!plan || !alpha || !beta_plus || !beta_minus) return fail(REXI_EINVAL, "NULL argument");
    for (int k = 0; k < plan->N; ++k) {
        alpha[2 * k] = plan->poles.alpha[k].real();
        alpha[2 * k + 1] = plan->poles.alpha[k].imag();
        beta_plus[2 * k] = plan->poles.beta_plus[k].real();
        beta_plus[2 * k + 1] = plan->poles.beta_plus[k].imag();
        beta_minus[2 * k] = plan->poles.beta_minus[k].real();
        beta_minus[2 * k + 1] = plan->poles.beta_minus[k].imag();
    }
    return REXI_OK;
}

int rexi_step(rexi_plan* plan, const void* u0, void* u1, int S, int nsteps, void* stream) {
    try {
        return do_step(plan, u0, u1, S, nsteps, 0, stream);
    } catch (const std::bad_alloc&) {
        return fail(REXI_ENOMEM, "host allocation failed");
    }
}

int rexi_step_adjoint(rexi_plan* plan, const void* g1, void* g0, int S, int nsteps, void* stream) {
    try {
        return do_step(plan, g1, g0, S, nsteps, 1, stream);
    } catch (const std::bad_alloc&) {
        return fail(REXI_ENOMEM, "host allocation failed");
    }
}

int rexi_step_per_term(rexi_plan* plan, const void* u0, void* u1, int S, void* stream) {
    int rc = check_state_call(plan, u0, u1, S, 1);
    if (rc) return rc;
    if (plan->prm.fsphere) return fail(REXI_EUNSUPPORTED, "the per-term form is not built for f-sphere plans");
    try {
        if ((int)plan->per_term.size() <= S) plan->per_term.resize(S + 1);
        Schedule& sc = plan->per_term[S];
        if (sc.items.empty()) {
            rc = build_schedule(plan, S, 0, 0, true, 0, sc);  // 8 elements per lane, one wave per chain
            if (rc) { free_schedule(sc); sc = Schedule(); return rc; }
        }
        if (sc.part_size > plan->acc_capacity) {
            dev_free(plan->d_acc);
            plan->acc_capacity = 0;
            rc = dev_alloc(&plan->d_acc, (size_t)sc.part_size);
            if (rc) return rc;
            plan->acc_capacity = sc.part_size;
        }
        hipStream_t s = (hipStream_t)stream;
        const Workspace ws = plan_workspace(plan);
        REXI_HIP(enqueue_prep(plan, ws, u0, 0, S, 0, plan->sched_layout, s));
        REXI_HIP(enqueue_zero(plan->d_acc, sc.part_size, s));
        for (int k = 0; k < plan->N; ++k) REXI_HIP(enqueue_per_term_pole(plan, ws, sc, k, 0, S, s));
        REXI_HIP(enqueue_reduce(plan, ws, sc, plan->d_acc, 0, 1, u1, S, 0, plan->d_slot_m, s));
        return REXI_OK;
    } catch (const std::bad_alloc&) {
        return fail(REXI_ENOMEM, "host allocation failed");
    }
}

int rexi_plan_set_schedule(rexi_plan* plan, int S, int index, int* count) {
    if (!plan) return fail(REXI_EINVAL, "plan is NULL");
    if (plan->prm.fsphere) return fail(REXI_EUNSUPPORTED, "f-sphere plans have no schedules");
    if (S < 1 || S > plan->prm.max_states) return fail(REXI_EINVAL, "S out of range");
    std::vector<Schedule>* c = nullptr;
    int rc = schedules_for(plan, S, &c);
    if (rc) return rc;
    if (count) *count = (int)c->size();
    if (index < 0) return REXI_OK;
    if (index >= (int)c->size()) return fail(REXI_EINVAL, "schedule index out of range");
    if (plan->chosen[S] != index) drop_graphs(plan);
    plan->chosen[S] = index;
    return REXI_OK;
}

int rexi_plan_get_schedule(rexi_plan* plan, int S, int* index) {
    if (!plan || !index) return fail(REXI_EINVAL, "NULL argument");
    if (plan->prm.fsphere) return fail(REXI_EUNSUPPORTED, "f-sphere plans have no schedules");
    if (S < 1 || S > plan->prm.max_states) return fail(REXI_EINVAL, "S out of range");
    std::vector<Schedule>* c = nullptr;
    int rc = schedules_for(plan, S, &c);
    if (rc) return rc;
    *index = plan->chosen[S];
    return REXI_OK;
}

int rexi_plan_autotune(rexi_plan* plan, int S, void* stream, int* chosen) {
    if (!plan) return fail(REXI_EINVAL, "plan is NULL");
    if (plan->prm.fsphere) return fail(REXI_EUNSUPPORTED, "f-sphere plans have no schedules");
    if (S < 1 || S > plan->prm.max_states) return fail(REXI_EINVAL, "S out of range");
    std::vector<Schedule>* c = nullptr;
    int rc = schedules_for(plan, S, &c);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const size_t bytes = (size_t)S * 3 * plan->nspec * 16;
    void *u0 = nullptr, *u1 = nullptr;
    REXI_HIP(hipMalloc(&u0, bytes));
    hipError_t e = hipMalloc(&u1, bytes);
    if (e != hipSuccess) { (void)hipFree(u0); return hip_fail(e, "hipMalloc"); }
    hipEvent_t a = nullptr, b = nullptr;
    int best = -1;
    float best_ms = 0;
    rc = REXI_OK;
    do {
        if ((e = hipMemsetAsync(u0, 0, bytes, s)) != hipSuccess) { rc = hip_fail(e, "hipMemsetAsync"); break; }
        if ((e = hipEventCreate(&a)) != hipSuccess || (e = hipEventCreate(&b)) != hipSuccess) {
            rc = hip_fail(e, "hipEventCreate");
            break;
        }
        for (int i = 0; i < (int)c->size() && !rc; ++i) {
            const Schedule& sc = (*c)[i];
            rc = run_steps(plan, sc, u0, u1, S, 1, 0, s);
            if (rc) break;
            if ((e = hipEventRecord(a, s)) != hipSuccess) { rc = hip_fail(e, "hipEventRecord"); break; }
            rc = run_steps(plan, sc, u0, u1, S, 3, 0, s);
            if (rc) break;
            if ((e = hipEventRecord(b, s)) != hipSuccess) { rc = hip_fail(e, "hipEventRecord"); break; }
            if ((e = hipEventSynchronize(b)) != hipSuccess) { rc = hip_fail(e, "hipEventSynchronize"); break; }
            float ms = 0;
            if ((e = hipEventElapsedTime(&ms, a, b)) != hipSuccess) { rc = hip_fail(e, "hipEventElapsedTime"); break; }
            if (best < 0 || ms < best_ms) { best = i; best_ms = ms; }
        }
    } while (0);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    (void)hipStreamSynchronize(s);
    (void)hipFree(u0);
    (void)hipFree(u1);
    if (rc) return rc;
    if (plan->chosen[S] != best) drop_graphs(plan);
    plan->chosen[S] = best;
    if (chosen) *chosen = best;
    return REXI_OK;
}

int rexi_solve_variants(int per_term, int capacity, int* se, int* kind, int* states_per_item, int* count) {
    if (capacity < 0) return fail(REXI_EINVAL, "capacity must be >= 0");
    const int n = solve_variant_list(per_term != 0, se, kind, states_per_item, capacity);
    if (count) *count = n;
    return REXI_OK;
}

int rexi_plan_schedule_classes(rexi_plan* plan, int S, int index, int capacity, int* se, int* kind,
                               int* states_per_item, int* count) {
    if (!plan) return fail(REXI_EINVAL, "plan is NULL");
    if (plan->prm.fsphere) return fail(REXI_EUNSUPPORTED, "f-sphere plans have no schedules");
    if (S < 1 || S > plan->prm.max_states) return fail(REXI_EINVAL, "S out of range");
    if (capacity < 0) return fail(REXI_EINVAL, "capacity must be >= 0");
    const Schedule* sc = nullptr;
    if (index == -1) {
        if ((int)plan->per_term.size() <= S || plan->per_term[S].items.empty())
            return fail(REXI_EINVAL, "the per-term schedule for S is built by the first rexi_step_per_term call");
        sc = &plan->per_term[S];
    } else {
        std::vector<Schedule>* c = nullptr;
        int rc = schedules_for(plan, S, &c);
        if (rc) return rc;
        if (index < -1 || index >= (int)c->size()) return fail(REXI_EINVAL, "schedule index out of range");
        sc = &(*c)[index];
    }
    const int n = (int)sc->launches.size();
    for (int i = 0; i < n && i < capacity; ++i) {
        if (se) se[i] = sc->launches[i].SE;
        if (kind) kind[i] = sc->launches[i].kind;
        if (states_per_item) states_per_item[i] = sc->launches[i].rot;
    }
    if (count) *count = n;
    return REXI_OK;
}

int rexi_plan_schedule_name(rexi_plan* plan, int S, int index, char* buf, int capacity) {
    if (!plan) return fail(REXI_EINVAL, "plan is NULL");
    if (!buf || capacity < 1) return fail(REXI_EINVAL, "buf is NULL or capacity < 1");
    buf[0] = 0;
    if (plan->prm.fsphere) return fail(REXI_EUNSUPPORTED, "f-sphere plans have no schedules");
    if (S < 1 || S > plan->prm.max_states) return fail(REXI_EINVAL, "S out of range");
    const Schedule* sc = nullptr;
    if (index == -1) {
        if ((int)plan->per_term.size() <= S || plan->per_term[S].items.empty())
            return fail(REXI_EINVAL, "the per-term schedule for S is built by the first rexi_step_per_term call");
        sc = &plan->per_term[S];
    } else {
        std::vector<Schedule>* c = nullptr;
        int rc = schedules_for(plan, S, &c);
        if (rc) return rc;
        if (index < -1 || index >= (int)c->size()) return fail(REXI_EINVAL, "schedule index out of range");
        sc = &(*c)[index];
    }
    std::snprintf(buf, (size_t)capacity, "%s", sc->name.c_str());
    return REXI_OK;
}

int rexi_plan_set_streams(rexi_plan* plan, int enable) {
    if (!plan) return fail(REXI_EINVAL, "plan is NULL");
    const bool on = enable != 0;
    if (on != plan->concurrent) drop_graphs(plan);
    plan->concurrent = on;
    return REXI_OK;
}

int rexi_plan_set_graphs(rexi_plan* plan, int enable) {
    if (!plan) return fail(REXI_EINVAL, "plan is NULL");
    plan->use_graphs = enable != 0;
    return REXI_OK;
}

int rexi_plan_set_timing(rexi_plan* plan, int enable) {
    if (!plan) return fail(REXI_EINVAL, "plan is NULL");
    plan->timing = enable != 0;
    return REXI_OK;
}

int rexi_plan_kernel_time(rexi_plan* plan, int kernel, double* total_ms, long long* launches) {
    if (!plan) return fail(REXI_EINVAL, "plan is NULL");
    if (kernel < 0 || kernel > 2) return fail(REXI_EINVAL, "unknown kernel");
    double tot = 0;
    long long n = 0;
    for (auto& ab : plan->events[kernel]) {
        REXI_HIP(hipEventSynchronize(ab.second));
        float ms = 0;
        REXI_HIP(hipEventElapsedTime(&ms, ab.first, ab.second));
        tot += ms;
        ++n;
        (void)hipEventDestroy(ab.first);
        (void)hipEventDestroy(ab.second);
    }
    plan->events[kernel].clear();
    if (total_ms) *total_ms = tot;
    if (launches) *launches = n;
    return REXI_OK;
}

int sh_forward(rexi_plan* plan, const double* grid, void* spec, int B, void* stream) {
    if (!plan) return fail(REXI_EINVAL, "plan is NULL");
    return sh_run(plan, grid, spec, B, true, (hipStream_t)stream);
}

int sh_inverse(rexi_plan* plan, const void* spec, double* grid, int B, void* stream) {
    if (!plan) return fail(REXI_EINVAL, "plan is NULL");
    return sh_run(plan, spec, grid, B, false, (hipStream_t)stream);
}

int sh_vortdiv_to_uv(rexi_plan* plan, const void* vd, long long stride, double* uv, int B, void* stream) {
    if (!plan) return fail(REXI_EINVAL, "plan is NULL");
    return sh_vec_run(plan, vd, uv, stride, B, true, (hipStream_t)stream);
}

int sh_uv_to_vortdiv(rexi_plan* plan, const double* uv, void* vd, long long stride, int B, void* stream) {
    if (!plan) return fail(REXI_EINVAL, "plan is NULL");
    return sh_vec_run(plan, uv, vd, stride, B, false, (hipStream_t)stream);
}

}  // extern "C"
