// The step entry point that allocates nothing: rexi_step_noalloc.
//
// For callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid it).  It runs the same
// kernels as rexi_step with the plan's current schedule, but its workspace
// (the states in chain layout, the solve's partial sums and the persistent
// launches' work counters) lives in one fixed device array defined here
// instead of the plan's allocations, and it launches the kernels one by one
// (no graph is instantiated, no event is created).  The array is part of the
// library's code object: every GPU the library runs on holds its own copy, at
// its own address, until the process ends.  Calls that overlap on one GPU
// share that copy and race.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "internal.hpp"

namespace rexi {
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per GPU
constexpr int kMaxDevices = 64;

// In host code this name is a host-side stand-in, not a device address: the
// kernels receive the address hipGetSymbolAddress returns for it.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

// Address of this device's copy of the array (the current device), looked
// up with the device current on the first call for that device.
int scratch_setup(void** ptr, size_t* bytes) {
    int dev = 0;
    REXI_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(REXI_EUNSUPPORTED, "device ordinal above 63");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress of the no-allocation workspace");
        if (!p) return fail(REXI_EHIP, "hipGetSymbolAddress returned no address for the workspace");
        g_ptr[dev] = p;
    }
    *ptr = g_ptr[dev];
    *bytes = kScratchBytes;
    return REXI_OK;
}

}  // namespace rexi

using namespace rexi;

extern "C" int rexi_step_noalloc(rexi_plan* plan, const void* u0, void* u1, int S, int nsteps, void* stream) {
    int rc = check_state_call(plan, u0, u1, S, nsteps);
    if (rc) return rc;
    if (plan->prm.fsphere) return fail(REXI_EUNSUPPORTED, "the no-allocation step is built for the rotating sphere only");
    if (!plan->scratch) return fail(REXI_EUNSUPPORTED, "no workspace on the plan's device");
    if ((int)plan->sched.size() <= S || plan->sched[S].empty() || plan->chosen[S] < 0)
        return fail(REXI_EINVAL,
                    "no schedule for this S yet: one call of rexi_step, rexi_plan_set_schedule or "
                    "rexi_plan_autotune with S builds them (and allocates); call it before the no-allocation step");
    const Schedule& sc = plan->sched[S][plan->chosen[S]];
    // switched off: persistent schedules launched outside a graph (a first
    // run of this step over every T256 candidate went silent there)
    if (sc.persistent)
        return fail(REXI_EUNSUPPORTED, "the no-allocation step does not run persistent schedules; select a "
                                       "one-workgroup-per-item schedule with rexi_plan_set_schedule");
    // carve the workspace out of the array, every piece 256-byte aligned
    size_t off = 0;
    auto take = [&off](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~size_t(255);
        return o;
    };
    const size_t var_bytes = (size_t)S * (plan->nslots + 2) * 16, phi_bytes = (size_t)S * plan->nspec * 16;
    const size_t o_v0 = take(var_bytes), o_v1 = take(var_bytes), o_p0 = take(phi_bytes), o_p1 = take(phi_bytes);
    const size_t o_part = take((size_t)sc.part_size * 16), o_cnt = take(kMaxLaunches * sizeof(int));
    if (off > plan->scratch_bytes)
        return fail(REXI_EUNSUPPORTED, "this step needs " + std::to_string(off) + " bytes of workspace, above the "
                                       "no-allocation limit of " + std::to_string(plan->scratch_bytes) +
                                       " bytes (a schedule with fewer work items needs less)");
    char* base = static_cast<char*>(plan->scratch);
    const Workspace ws{{reinterpret_cast<double2*>(base + o_v0), reinterpret_cast<double2*>(base + o_v1)},
                       {reinterpret_cast<double2*>(base + o_p0), reinterpret_cast<double2*>(base + o_p1)},
                       reinterpret_cast<double2*>(base + o_part), reinterpret_cast<int*>(base + o_cnt)};
    hipStream_t s = (hipStream_t)stream;
    if (nsteps == 0) {
        REXI_HIP(hipMemcpyAsync(u1, u0, (size_t)S * 3 * plan->nspec * 16, hipMemcpyDeviceToDevice, s));
        return REXI_OK;
    }
    // the chain-layout states are written by the layout kernel, the partial
    // sums by every work item and the counters by the persistent launches' own
    // reset kernel, so nothing of an earlier call's contents is read
    REXI_HIP(enqueue_prep(plan, ws, u0, 0, S, 0, plan->sched_layout, s));
    int cur = 0;
    for (int k = 0; k < nsteps; ++k) {
        const bool last = (k == nsteps - 1);
        REXI_HIP(enqueue_solve(plan, ws, sc, cur, S, 0, s));
        REXI_HIP(enqueue_reduce(plan, ws, sc, ws.part, cur, cur ^ 1, last ? u1 : nullptr, S, 0, plan->d_slot_m, s));
        cur ^= 1;
    }
    return REXI_OK;
}
