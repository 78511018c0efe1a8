/*
 * rexi.h - C ABI of the MI355X (gfx950) T-REXI library for the linearised
 * shallow-water equations on the rotating sphere.
 *
 * Method: Schreiber & Loft, "A Parallel Time-Integrator for Solving the
 * Linearized Shallow Water Equations on the Rotating Sphere".  One time step
 * applies the rational approximation of the exponential integrator
 * (Section 4.2),
 *     U_{n+1} ~ sum_k beta_k (alpha_k I + dt L)^{-1} U_n,
 * to the linear operator L of Eq. (1) in spherical-harmonic space
 * (Section 3), where L is block diagonal in the zonal order m (Section 5,
 * Fig. 1) and every block is banded in the degree n.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Spectral layout.  Triangular truncation 0 <= m <= n <= T, only m >= 0
 *   stored (m = 0 coefficients describe real fields).  Coefficients are
 *   complex128 (interleaved re, im doubles) in m-major order,
 *   idx(m, n) = m (T+1) - m (m-1)/2 + (n - m),  nspec = (T+1)(T+2)/2.
 *   A state is [S][3][nspec] with the variables (Phi, vorticity, divergence)
 *   in physical units (m^2/s^2, 1/s, 1/s).
 * Basis.  Y_n^m = P_n^m(mu) e^{i m lam}, P_n^m orthonormal on [-1, 1]
 *   (int P^2 dmu = 1), no Condon-Shortley phase, mu = sin(latitude)
 *   (Section 3).
 * Grid layout.  Real float64 [B][nlat][nlon]; latitude row 0 is the
 *   northernmost Gauss-Legendre latitude, lam_k = 2 pi k / nlon.
 * REXI sign convention.  The pole list alpha_k = h (mu + i k),
 *   k = -(M+L)..(M+L), and the two weight lists beta+_k, beta-_k satisfy
 *       e^{z} ~ sum_k beta+_k / (z + alpha_k) + sum_k beta-_k / (alpha_k - z)
 *   for z = i x on the covered range (Section 4.1), so one step is
 *       u1 = sum_k beta+_k (alpha_k + dt L)^{-1} u0 + sum_k beta-_k (alpha_k - dt L)^{-1} u0.
 *   (The same list written as (alpha'_k I - dt L) u_k = u0 uses
 *   alpha' in {-alpha_k} u {alpha_k} with beta' in {-beta+_k} u {beta-_k}.)
 * Memory.  Pointers documented "device" must be device memory of the
 *   current HIP device (e.g. torch tensors), contiguous; "host" pointers are
 *   plain host memory.  The caller owns every buffer it passes; the plan owns
 *   its tables, workspace and captured graphs.  Outputs must not overlap
 *   inputs (REXI_EALIAS).
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = the null
 *   stream).  Calls enqueue work and return; argument errors are reported
 *   synchronously, errors of enqueued work by the next call or at
 *   synchronisation.
 * Threads.  A plan may be used from one thread at a time.  Calls on one plan
 *   share its workspace: calls that overlap on different streams race.
 * Errors.  Every int-returning call returns REXI_OK (0) or a negative code;
 *   rexi_last_error() then describes the failure (thread-local string).
 */
#ifndef REXI_H
#define REXI_H

#ifdef __cplusplus
extern "C" {
#endif

enum {
    REXI_OK = 0,
    REXI_EINVAL = -1,        /* bad argument (size, pointer, parameter range) */
    REXI_ENOMEM = -2,        /* device or host allocation failed */
    REXI_EHIP = -3,          /* a HIP runtime call failed */
    REXI_EUNSUPPORTED = -4,  /* valid but not supported (e.g. size above plan limits) */
    REXI_EALIAS = -5         /* output overlaps input */
};

/* Opaque plan: tables, schedule, workspace and graphs for one configuration. */
typedef struct rexi_plan rexi_plan;

/* Parameters of a plan.
 *   T                 truncation (1 <= T <= 1023)
 *   nlat, nlon        Gaussian grid of the transforms: nlat even, 2 <= nlat <= 2048
 *                     (the transforms pair latitude j with nlat-1-j); nlon a power
 *                     of two, 4 <= nlon <= 4096, T < nlon; 0, 0 = no transforms.
 *                     Outside these ranges rexi_plan_create returns REXI_EINVAL
 *                     before it allocates anything.
 *   radius, omega, gravity, mean_depth
 *                     planet radius a (m), rotation rate Omega (1/s), g (m/s^2),
 *                     mean depth H (m); Phibar = g H (Eq. (1), Section 6)
 *   dt                time step (s), > 0
 *   M, h, L           REXI: Gaussians per side, Gaussian width, half-width K of
 *                     the rational basis (Section 4.1); M >= 1, 0 < h, 1 <= L <= 32
 *   normalize         1: divide beta by the x = 0 response (Section 6.1), 0: raw
 *   max_states        largest S accepted by rexi_step / rexi_step_adjoint (<= 64)
 *   max_fields        largest B accepted by sh_forward / sh_inverse
 *   fsphere, f0       fsphere = 1: the f-sphere variant (Section 4.3), a constant
 *                     Coriolis parameter f0 (1/s) in place of 2 Omega sin(lat);
 *                     then every (n, m) is a 3x3 system of (Phi, zeta, delta)
 *                     (Phi_t = -Phibar delta, zeta_t = -f0 delta,
 *                     delta_t = f0 zeta - lap Phi), whose eigenvalues are 0 and
 *                     +-i sqrt(f0^2 + Phibar n(n+1)/a^2).  Such a plan supports
 *                     rexi_step, rexi_step_adjoint and the transforms; the
 *                     schedule, autotune and per-term calls return
 *                     REXI_EUNSUPPORTED.  fsphere = 0: the rotating sphere (f0
 *                     ignored). */
typedef struct rexi_params {
    int T;
    int nlat, nlon;
    double radius, omega, gravity, mean_depth;
    double dt;
    int M;
    double h;
    int L;
    int normalize;
    int max_states;
    int max_fields;
    int fsphere;
    double f0;
} rexi_params;

/* REXI poles and weights (Section 4.1; renormalisation of Section 6.1).
 * Fits the Gaussian psi(y) = (4 pi)^{-1/2} e^{-y^2/4} by
 * Re sum_{l=-L}^{L} a_l / (i y + mu + i l) with a_{-l} = conj(a_l)
 * (least squares, mu chosen by a scan), forms the Gaussian sum
 * b_m = e^{h^2} e^{-i m h}, m = -M..M, and merges both into the two-sided
 * list described above.  Host only; no GPU needed.
 *   capacity   number of complex entries the three output arrays can hold;
 *              0 = only report the count in *n_poles (arrays may be NULL)
 *   alpha, beta_plus, beta_minus
 *              host, 2*capacity doubles each (re, im interleaved), pole index
 *              k = -(M+L)..(M+L) stored at position k + M + L
 *   n_poles    host, receives N = 2 (M + L) + 1
 * Returns REXI_EINVAL for M < 1, h <= 0, L < 1 or L > 32, or
 * capacity in (0, N); REXI_OK otherwise. */
int rexi_coeffs(int M, double h, int L, int normalize, int capacity,
                double *alpha, double *beta_plus, double *beta_minus, int *n_poles);

/* Build a plan: coefficients, per-(n, m) operator constants in energy
 * variables, Gauss-Legendre nodes and Legendre tables, work schedule and
 * device workspace for up to max_states states / max_fields fields.
 * p: host; *out receives the plan.  Uses the current HIP device. */
int rexi_plan_create(const rexi_params *p, rexi_plan **out);

/* Release a plan and everything it owns (synchronises the device first). */
int rexi_plan_destroy(rexi_plan *plan);

/* Plan facts: N (poles), nspec, and the number of (pole, m) blocks per step,
 * N (T+1).  Any pointer may be NULL. */
int rexi_plan_info(const rexi_plan *plan, int *n_poles, int *nspec, long long *blocks_per_step);

/* Copy the plan's pole list to host arrays of 2N doubles each (same layout
 * as rexi_coeffs). */
int rexi_plan_coeffs(const rexi_plan *plan, double *alpha, double *beta_plus, double *beta_minus);

/* Spherical-harmonic analysis (Section 3): grid -> spectral.
 * xi_n^m = sum_j w_j P_n^m(mu_j) (1/nlon) sum_k xi(mu_j, lam_k) e^{-i m lam_k}
 *   grid  device float64 [B][nlat][nlon]
 *   spec  device complex128 [B][nspec]
 *   1 <= B <= max_fields.  Exact inverse of sh_inverse for n < nlat and
 *   m < nlon/2; beyond that the quadrature / Nyquist limits apply. */
int sh_forward(rexi_plan *plan, const double *grid, void *spec, int B, void *stream);

/* Spherical-harmonic synthesis (Section 3): spectral -> grid.
 * xi = sum_n Re(xi_n^0) P_n^0 + 2 Re sum_{m>0} sum_n xi_n^m P_n^m e^{i m lam}
 *   spec  device complex128 [B][nspec];  grid  device float64 [B][nlat][nlon] */
int sh_inverse(rexi_plan *plan, const void *spec, double *grid, int B, void *stream);

/* Winds from vorticity and divergence (Eq. (1): V = k x grad(psi) + grad(chi)
 * with lap psi = zeta, lap chi = delta; Section 3's scaled winds
 * U = u cos(lat), V = v cos(lat)).  The latitude derivative raises the degree
 * by one, so U and V are synthesised at degree T + 1 (orders m <= T) and
 * divided by cos(lat) on the grid; the n = 0 coefficients carry no wind.
 *   vd      device complex128; pair b: zeta [nspec] at vd + b * stride, delta
 *           [nspec] right after it (stride in complex entries, >= 2 nspec;
 *           stride 3 nspec with vd = u + nspec reads the (zeta, delta) of the
 *           states [S][3][nspec] of rexi_step)
 *   uv      device float64 [B][2][nlat][nlon]: u (eastward), v (northward), in
 *           the units of radius * zeta
 *   1 <= 2 B <= max_fields (REXI_EUNSUPPORTED above).  Exact (to rounding)
 *   inverse of sh_uv_to_vortdiv on such winds when nlat >= T + 1 and
 *   nlon > 2 T.  Needs a plan with a grid; no allocation. */
int sh_vortdiv_to_uv(rexi_plan *plan, const void *vd, long long stride, double *uv, int B, void *stream);

/* Vorticity and divergence of winds (Eq. (1)): zeta = k . curl V,
 * delta = div V, analysed on the Gaussian grid (Section 3).  The integral of
 * the latitude derivative is taken by parts, so the quadrature acts on
 * u / cos(lat) and v / cos(lat) at degree T + 1 (no pole values are needed).
 *   uv      device float64 [B][2][nlat][nlon] (u, v)
 *   vd      device complex128, layout as for sh_vortdiv_to_uv; only the zeta
 *           and delta entries of each pair are written (a state's Phi between
 *           them is left as it is)
 *   1 <= 2 B <= max_fields; output and input must not overlap. */
int sh_uv_to_vortdiv(rexi_plan *plan, const double *uv, void *vd, long long stride, int B, void *stream);

/* nsteps T-REXI steps (Section 4.2, Algorithm 1's sum and reduction) of S
 * states: u1 = R^nsteps u0 with
 *   R = sum_k beta+_k (alpha_k + dt L)^{-1} + sum_k beta-_k (alpha_k - dt L)^{-1}.
 *   u0, u1  device complex128 [S][3][nspec] (must not overlap)
 *   1 <= S <= max_states, nsteps >= 0 (0 copies u0 to u1). */
int rexi_step(rexi_plan *plan, const void *u0, void *u1, int S, int nsteps, void *stream);

/* Adjoint of rexi_step: g0 = (R^H)^nsteps g1, the conjugate-transposed
 * shifted solves with conjugated weights.  For a real loss of u1 with
 * gradient g1 = dL/dRe(u1) + i dL/dIm(u1), g0 is the same gradient for u0.
 * Arguments as rexi_step. */
int rexi_step_adjoint(rexi_plan *plan, const void *g1, void *g0, int S, int nsteps, void *stream);

/* rexi_step for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same kernels and the plan's current schedule for S, with the workspace
 * (states in chain layout, partial sums, work counters) in one fixed 64 MiB
 * device array of the library instead of the plan's allocations; kernels
 * launched one by one, no graph, no event.  Calls no hipMalloc, hipFree or
 * other allocating routine.
 *   Arguments as rexi_step.  The schedules for S must exist: one earlier
 *   rexi_step, rexi_plan_set_schedule or rexi_plan_autotune call with S
 *   builds them (and allocates); otherwise REXI_EINVAL.  A step whose
 *   workspace exceeds 64 MiB returns REXI_EUNSUPPORTED (a schedule with fewer
 *   work items, rexi_plan_set_schedule, needs less; T256 with 4 states fits
 *   with about 2048 items).  Persistent schedules (a resident grid taking
 *   items from a counter) return REXI_EUNSUPPORTED.
 *   The array is per GPU and lives until the process ends; every call on a
 *   GPU uses it, so calls that overlap on one GPU (on different streams or
 *   from different threads) race. */
int rexi_step_noalloc(rexi_plan *plan, const void *u0, void *u1, int S, int nsteps, void *stream);

/* One forward step in the plain per-term form: one launch per pole k that
 * solves every m-block of (alpha_k +- dt L) and accumulates into a device
 * accumulator, then a final conversion.  Same arithmetic and result as
 * rexi_step with nsteps = 1 (to rounding); kept as the comparison point for
 * the batched form.  Arguments as rexi_step. */
int rexi_step_per_term(rexi_plan *plan, const void *u0, void *u1, int S, void *stream);

/* Time the candidate tile/wave schedules for S states on `stream` (runs
 * steps on internal buffers) and keep the fastest for later calls with S.
 * *chosen (may be NULL) receives the index of the chosen candidate. */
int rexi_plan_autotune(rexi_plan *plan, int S, void *stream, int *chosen);

/* Select schedule candidate `index` (as reported by rexi_plan_autotune) for
 * S states; REXI_EINVAL if out of range.  *count (may be NULL) receives the
 * number of candidates. */
int rexi_plan_set_schedule(rexi_plan *plan, int S, int index, int *count);

/* *index receives the schedule candidate that steps with S states use now
 * (the default until rexi_plan_autotune or rexi_plan_set_schedule). */
int rexi_plan_get_schedule(rexi_plan *plan, int S, int *index);

/* Compiled variants of the fused solve kernel (the batched step, or with
 * per_term = 1 the per-term form): variant i tiles a chain with se[i]
 * elements per lane, moves values between the lanes of a chain with
 * kind[i] (0 ds_bpermute, 1 DPP within 16-lane rows, 2 DPP and
 * permlane16_swap over row pairs) and solves states_per_item[i] states per
 * work item, sharing each pole's factorisation among them.  Host only.
 *   capacity  entries the three arrays can hold (0 = only *count)
 *   se, kind, states_per_item  host int arrays or NULL
 *   count     receives the number of variants (may exceed capacity) */
int rexi_solve_variants(int per_term, int capacity, int *se, int *kind, int *states_per_item, int *count);

/* The solve launches of one schedule candidate for S states (index as for
 * rexi_plan_set_schedule; -1 = the per-term schedule, which the first
 * rexi_step_per_term call with S builds): per launch the variant's (se,
 * kind, states_per_item), as rexi_solve_variants reports them. */
int rexi_plan_schedule_classes(rexi_plan *plan, int S, int index, int capacity, int *se, int *kind,
                               int *states_per_item, int *count);

/* The name of schedule candidate `index` for S states (-1 = the per-term
 * schedule, once built): tile policy, work-item count, "persistent_" for a
 * grid of resident workgroups pulling items from a counter, and "_shared" /
 * "_mixed" where states share each pole's factorisation in every / some of
 * its tile classes (no suffix: in none).  Written NUL-terminated into buf (host, capacity bytes, truncated
 * to fit); REXI_EINVAL for a NULL buf or capacity < 1. */
int rexi_plan_schedule_name(rexi_plan *plan, int S, int index, char *buf, int capacity);

/* Step graphs.  By default every step is replayed as a captured HIP graph
 * (solve launches + reduction), built on first use per (S, direction, buffer)
 * and rebuilt after a schedule change; enable = 0 makes the plan launch the
 * kernels one by one instead.  Results are identical either way. */
int rexi_plan_set_graphs(rexi_plan *plan, int enable);

/* Tile-class launches.  A step launches one solve kernel per tile class; by
 * default they run concurrently on side streams of the plan (default
 * priority), forked from and joined back into the caller's stream, so that
 * the tail of one class overlaps the others.  enable = 0 launches them one
 * after another on the caller's stream.  Results are identical either way. */
int rexi_plan_set_streams(rexi_plan *plan, int enable);

/* Kernel timing for measurement.  rexi_plan_set_timing(plan, 1) makes the plan
 * bracket every later launch of the timed kernels with a HIP event pair on the
 * launch stream; 0 stops recording.  A solve timing covers one step: with step
 * graphs on (the default) the replay of the step's graph, i.e. the solve
 * launches and the reduction of their partial sums; with graphs off the solve
 * launches alone.  rexi_plan_kernel_time synchronises on the recorded events
 * and returns the summed elapsed time (ms) and the number of launches of one
 * kernel since the last query, then forgets them.
 *   kernel  REXI_KERNEL_SOLVE (fused banded solve), REXI_KERNEL_LEGENDRE_FWD,
 *           REXI_KERNEL_LEGENDRE_INV */
enum { REXI_KERNEL_SOLVE = 0, REXI_KERNEL_LEGENDRE_FWD = 1, REXI_KERNEL_LEGENDRE_INV = 2 };
int rexi_plan_set_timing(rexi_plan *plan, int enable);
int rexi_plan_kernel_time(rexi_plan *plan, int kernel, double *total_ms, long long *launches);

/* Description of the last non-zero return on this thread ("" if none). */
const char *rexi_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* REXI_H */
