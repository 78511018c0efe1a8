// Internal declarations shared by the library's host and device sources.
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <string>
#include <vector>

#include "../../include/rexi.h"

namespace rexi {

using cld = std::complex<long double>;

// ---------------------------------------------------------------- errors
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);
#define REXI_HIP(call)                                            \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) return ::rexi::hip_fail(e_, #call); \
    } while (0)

// ---------------------------------------------------------------- host math
// Gaussian rational fit (Section 4.1): mu and a_l, l = -L..L.
struct GaussFit {
    long double mu;
    std::vector<cld> a;  // size 2L+1, index l + L
    double max_err;
};
GaussFit fit_gaussian(int L);

// Two-sided REXI list (see rexi.h).  Index k + M + L for k = -(M+L)..(M+L).
struct Poles {
    std::vector<std::complex<double>> alpha, beta_plus, beta_minus;
};
Poles make_poles(int M, double h, int L, int normalize);

// Gauss-Legendre nodes (descending, north to south) and weights.
void gauss_legendre(int nlat, std::vector<double>& mu, std::vector<double>& w);

// Recurrence coefficients (a_n, b_n) of the orthonormal P_n^m, [nspec][2], and
// exact restart rows (P_{n0-1}, P_{n0}) at n0 = m + run r, [row][2][nmu] with
// row = run_base[m] + r (run_base has T + 2 entries).
std::vector<double> legendre_coefs(int T);
std::vector<double> legendre_restarts(int T, int run, const std::vector<double>& mu, std::vector<int>& run_base);

// Device tables of the Legendre kernels for degrees 0..T (orders m <= the
// plan's truncation): restart rows, recurrence coefficients and work lists.
struct LegTables {
    int T = 0;
    double* d_restart = nullptr;  // [row][2][nhalf], rows every 32 degrees
    double* d_restart8 = nullptr; // [row][2][nhalf], rows every 8 degrees (grids of <= 128 northern latitudes; inverse)
    double* d_lcoef = nullptr;    // [nspec(T)][2]
    void* d_tiles_f = nullptr;    // forward runs
    void* d_tiles_i = nullptr;    // inverse work
    int* d_seg = nullptr;         // inverse partial slots of order m: d_seg[m] .. d_seg[m+1]-1
    int ntiles_f = 0, ntiles_i = 0, nslots = 0;
};

__host__ __device__ inline long long spec_offset(int T, int m) {
    return (long long)m * (T + 1) - (long long)m * (m - 1) / 2;
}
__host__ __device__ inline long long nspec_of(int T) { return (long long)(T + 1) * (T + 2) / 2; }

// ---------------------------------------------------------------- device-side structs
// Per zonal order m: the two parity chains of the Phi-eliminated block.
//   chain p holds vorticity at degrees n == p (mod 2) and divergence at the
//   others; Phi_n is carried with the divergence element of degree n.
//   n0 = max(m, 1) (the (0,0) mode is handled on its own), L = T + 1 - n0.
//   P lanes per chain problem (a power of two), s elements per lane.
struct MInfo {
    int n0, L, P, s;
    int spec_off;   // idx(m, m)
    int slot_base;  // first chain slot of this m (chain p at slot_base + p L)
};

// One work item of the fused solve: chain p of order m, the R states
// [tile*R, tile*R + R) (R = the launch's states per item), poles [k0, k1).
// Its partial sums go to part + part_off (complex units), layout [R][2][L].
struct Item {
    int m, p, tile, k0, k1;
    long long part_off;
};

// Per (m, p, state): where the partial sums of that state start in the
// first of its nr consecutive items, and the states per item st of those
// items (successive items are st * 2L complex entries apart).
struct Group {
    long long part_off;
    int nr;
    int st;
};

// One launch of the solve kernel: items [item0, item0 + nitems) share the
// elements-per-lane class SE, the cross-lane move kind and the number of
// states per item (rot), whose solves share each pole's factorisation.
struct Launch {
    int SE;
    int kind;  // cross-lane moves: 0 ds_bpermute, 1 DPP within 16-lane rows, 2 DPP over row pairs
    int item0, nitems;
    int pmax;  // largest lane group of the launch (sizes its LDS)
    int rot;   // states per work item
};

constexpr int kMaxLaunches = 8;  // solve launches per step (tile classes)

// Device workspace of a step: the states in chain layout (double buffered
// between steps), the solve's partial sums and the work counters of
// persistent launches.  A plan owns one; the no-allocation step carves one
// out of a fixed device array.
struct Workspace {
    double2* ch_var[2];  // [S][nslots + 2]
    double2* ch_phi[2];  // [S][nspec]
    double2* part;       // partial sums, the schedule's part_size entries
    int* counters;       // kMaxLaunches
};

struct Schedule {
    bool persistent = false;  // resident grid + atomic work counter per launch
    int SM = 4;       // largest elements-per-lane class used
    int rot_max = 1;  // largest states-per-item the schedule may use
    int S = 0;        // states this schedule serves
    std::vector<Launch> launches;
    std::vector<MInfo> minfo;
    std::vector<Item> items;
    std::vector<Group> groups;  // index ((m * 2 + p) * S + state)
    long long part_size = 0;    // complex entries
    // device copies
    MInfo* d_minfo = nullptr;
    Item* d_items = nullptr;
    Group* d_groups = nullptr;
    std::string name;
};

}  // namespace rexi

// ---------------------------------------------------------------- the plan
struct rexi_plan {
    rexi_params prm;
    int T = 0, N = 0;
    long long nspec = 0, nslots = 0;
    double phibar = 0;
    rexi::Poles poles;
    std::complex<double> g00_fwd, g00_adj, gphi_fwd, gphi_adj;

    // per-(n, m) constants in spectral order (device)
    double *d_th = nullptr, *d_om = nullptr, *d_cc = nullptr, *d_sc = nullptr;
    int *d_idx_n = nullptr, *d_idx_m = nullptr;
    // per pole, forward [0] and adjoint [1]: alpha, 1/alpha, wx, wy, wx/alpha,
    // wy/alpha (6 complex, see rexi_kernels.hip)
    double2* d_poles[2] = {nullptr, nullptr};
    // workspace (sized for max_states)
    double2 *d_ch_var[2] = {nullptr, nullptr};  // [S][nslots + 2]
    double2 *d_ch_phi[2] = {nullptr, nullptr};  // [S][nspec]
    double2 *d_part = nullptr;
    long long part_capacity = 0;
    double2 *d_acc = nullptr;                    // per-term form accumulator [S][2][nslots]
    // chain-slot layout (device) and slot -> m table
    rexi::MInfo* sched_layout = nullptr;
    int* d_slot_m = nullptr;
    // schedules: candidates per S, chosen index per S; per-term form per S
    std::vector<std::vector<rexi::Schedule>> sched;  // [S] -> candidates
    std::vector<int> chosen;
    std::vector<rexi::Schedule> per_term;             // [S]
    long long acc_capacity = 0;

    // transforms
    int nlat = 0, nlon = 0, nhalf = 0;
    std::vector<double> mu, w;
    rexi::LegTables leg;          // degrees 0..T (scalar transforms)
    rexi::LegTables legv;         // degrees 0..T+1 (vector transforms)
    double* d_mu = nullptr;       // northern Gauss nodes [nhalf]
    double* d_wts = nullptr;      // Gauss weights
    double* d_rcos = nullptr;     // 1 / cos(lat_j) [nlat]
    double* d_four = nullptr;     // Fourier workspace [slots][nlat][2B] + padding per plane (slots >= T+1)
    double2* d_twiddle = nullptr; // FFT twiddles
    double2* d_vspec = nullptr;   // vector transforms: [max_fields][nspec(T+1)]

    // f-sphere variant: constant Coriolis parameter times dt, poles
    // [N][3] (alpha, beta+, beta-), one state-sized work buffer
    double f0dt = 0.0;
    double2* d_fs_poles = nullptr;
    double2* d_fs_work = nullptr;

    // persistent launches: one work counter per solve launch
    int* d_counters = nullptr;
    // captured step graphs: key (S, adjoint, input buffer), valid for `graph_gen`
    struct StepGraph {
        const rexi::Schedule* sched;
        int S, adjoint, buf;
        long long gen;
        hipGraphExec_t exec;
        hipEvent_t done;  // recorded after each launch of exec
    };
    std::vector<StepGraph> graphs;
    long long graph_gen = 0;
    bool use_graphs = true;
    hipStream_t cap_stream = nullptr;
    // concurrent tile-class launches: side streams, fork and join events
    bool concurrent = true;
    hipStream_t side[rexi::kMaxLaunches] = {};
    hipEvent_t fork_ev = nullptr;
    hipEvent_t join_ev[rexi::kMaxLaunches] = {};

    // the device the plan was created on, and the no-allocation step's fixed
    // workspace there (see rexi_step_noalloc)
    int device = 0;
    void* scratch = nullptr;
    size_t scratch_bytes = 0;

    // measurement: event pairs around timed launches, per kernel kind
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events[3];
};

namespace rexi {
// Launchers (rexi_kernels.hip, sh_kernels.hip) and library internals used
// across the sources.
bool solve_variant_supported(int SE, int kind, int rot, bool per_term);
int solve_waves_per_item();
int solve_variant_list(bool per_term, int* se, int* kind, int* st, int cap);
hipError_t enqueue_prep(rexi_plan* pl, const Workspace& ws, const void* u, int buf, int S, int adjoint,
                        const MInfo* d_layout, hipStream_t s);
hipError_t enqueue_solve(rexi_plan* pl, const Workspace& ws, const Schedule& sc, int buf, int S, int adjoint,
                         hipStream_t s);
hipError_t enqueue_reduce(rexi_plan* pl, const Workspace& ws, const Schedule& sc, const double2* part, int buf_in,
                          int buf_out, void* u_out, int S, int adjoint, const int* d_slot_m, hipStream_t s);
hipError_t enqueue_zero(double2* p, long long n, hipStream_t s);
hipError_t enqueue_fsphere_step(rexi_plan* pl, const void* in, void* out, int S, int adjoint, hipStream_t s);
hipError_t enqueue_finish(rexi_plan* pl, const Workspace& ws, int buf, void* u, int S, int adjoint,
                          const MInfo* d_layout, hipStream_t s);
hipError_t enqueue_per_term_pole(rexi_plan* pl, const Workspace& ws, const Schedule& sc, int k, int buf, int S,
                                 hipStream_t s);
int sh_setup(rexi_plan* pl);
void sh_release(rexi_plan* pl);
int sh_run(rexi_plan* pl, const void* in, void* out, int B, bool forward, hipStream_t s);
int sh_vec_run(rexi_plan* pl, const void* in, void* out, long long stride, int B, bool to_uv, hipStream_t s);
int check_state_call(rexi_plan* pl, const void* in, const void* out, int S, int nsteps);
// The no-allocation step's fixed device array: its address on the current
// device, looked up once per device (noalloc.hip).
int scratch_setup(void** ptr, size_t* bytes);

// The plan's own workspace.
inline Workspace plan_workspace(const rexi_plan* pl) {
    return Workspace{{pl->d_ch_var[0], pl->d_ch_var[1]}, {pl->d_ch_phi[0], pl->d_ch_phi[1]}, pl->d_part,
                     pl->d_counters};
}
// Record an event before / after a timed launch when timing is on.
hipError_t timed_begin(rexi_plan* pl, int kind, hipStream_t s);
hipError_t timed_end(rexi_plan* pl, int kind, hipStream_t s);
}  // namespace rexi
