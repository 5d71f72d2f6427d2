/*
 * Ensemble DNS of plane Couette and plane Poiseuille flow on one MI355X GPU.
 *
 * C ABI of the HIP library libdns_ensemble.so.  The solver advances an ensemble
 * of independent flow realisations of the incompressible Navier-Stokes
 * equations between two parallel walls (arXiv 2306.12739, Sec. 2, Eqs. (1)-(3)),
 * written for the wall-normal velocity v and vorticity eta with the mean
 * profiles U00, W00 (Eqs. (Dv), (eta), (U00), (W00)), discretised with Fourier
 * modes in x and z and Chebyshev collocation in y (Sec. 2), and integrated with
 * the CN/RK3 scheme of Sec. 3.1 using pre-inverted per-(kx,kz) operators
 * (Sec. 3.2, Eqs. (CN1)-(CN4)).  All ensemble members share the grid, box,
 * Reynolds number and time step; members are independent (Sec. 3.2, last
 * paragraph: members are extra columns of every operator application).
 *
 * Conventions shared by all calls
 *   - Walls at y = -1 and y = +1 (half width h = 1); Re = U h / nu with U the
 *     Couette wall speed or the laminar channel centreline speed (Sec. 2).
 *   - Nx, Nz: even Fourier sizes; stored modes n_x = 0..Nx/2-1 and
 *     |n_z| <= Nz/2-1 (2/3-rule de-aliasing, Sec. 3.2, done as 3/2 padding:
 *     the physical grid has 3Nx/2 x 3Nz/2 points).  Ny: Chebyshev-Gauss-Lobatto
 *     points y_j = -cos(pi j/(Ny-1)), j = 0..Ny-1, walls included.
 *   - Spectral normalisation: f_hat(k) = 1/(Mx Mz) sum f e^{-i(kx x + kz z)},
 *     so f_hat(0,0) is the plane mean.
 *   - Every call returns DNS_OK (0) or a negative DNS_E_* code and records a
 *     message retrievable with dns_last_error().
 *   - Handles are not thread-safe: calls on one handle must not overlap.
 */
#ifndef DNS_ENSEMBLE_H
#define DNS_ENSEMBLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define DNS_OK 0
#define DNS_E_INVALID (-1)     /* bad argument or unsupported combination       */
#define DNS_E_NOMEM (-2)       /* device or host allocation failed              */
#define DNS_E_HIP (-3)         /* a HIP runtime call failed                     */
#define DNS_E_NONFINITE (-4)   /* at least one member produced NaN/Inf          */
#define DNS_E_UNSUPPORTED (-5) /* valid but not built (grid size, precision)    */
#define DNS_E_STATE (-6)       /* call-order misuse (e.g. NULL handle)          */

#define DNS_FLOW_COUETTE 0
#define DNS_FLOW_POISEUILLE 1

typedef struct dns_handle dns_handle;

/* Problem statement of Sec. 2: box and wall forcing.
 *   flow : DNS_FLOW_COUETTE (walls at y = -1/+1 move at -Uw/+Uw, gamma = 0) or
 *          DNS_FLOW_POISEUILLE (walls at rest, gamma(t) holds the bulk flux).
 *   Lx, Lz : periodic box lengths (k_x = 2 pi n / Lx, k_z = 2 pi m / Lz).
 *   Uw   : Couette wall speed (default 1 when <= 0).
 *   flux : channel bulk flux target int_{-1}^{1} U dy (4/3 when <= 0, the
 *          laminar parabola U = 1 - y^2). */
typedef struct {
  int flow;
  double Lx, Lz;
  double Uw;
  double flux;
} dns_geometry;

/* Create an ensemble solver (Sec. 3.2: operators are built once per (kx,kz) and
 * h in {1/2, 1}, on the host in extended precision, then uploaded).
 *   Nx, Nz : 16, 32, 48, 64, 72 or 96 with Nx == Nz, or (Nx, Nz) = (64, 32)
 *            or (32, 64) (advective form only: DNS_OPT_ADVECTION and
 *            DNS_OPT_QUASILINEAR then return DNS_E_UNSUPPORTED);
 *            Ny : 5..254 (odd or even);
 *   ensemble >= 1; dt > 0; Re > 0.
 * The state is initialised to the laminar profile (Couette U = Uw y, channel
 * U = 1 - y^2) with zero perturbations.  Device memory is owned by the handle.
 * On failure *out is set to NULL.  Errors: DNS_E_INVALID, DNS_E_UNSUPPORTED,
 * DNS_E_NOMEM, DNS_E_HIP. */
int dns_create(const dns_geometry* g, double Re, int Nx, int Ny, int Nz, int ensemble, double dt,
               dns_handle** out);

/* Several ensembles advanced together (Sec. 3.2 batches members of one
 * configuration; here independent configurations -- different Re, grid, box,
 * dt or flow -- share one dns_step).  Each group is a full ensemble as made by
 * dns_create, with its own operators and buffers.  Each sub-step runs the
 * groups' advection kernels on streams of their own (forked from and joined
 * back into the grouped handle's stream) and then one per-mode launch over
 * every group (DNS_OPT_GROUP_STREAMS selects per-group streams for the whole
 * step instead).  Grouped steps run eagerly: DNS_OPT_GRAPH = 1 on a grouped
 * handle returns DNS_E_UNSUPPORTED.  Members are numbered group-major: group g
 * holds members [sum of earlier groups' members, + members).
 *   groups  : ngroups descriptions, 1 <= ngroups <= DNS_MAX_GROUPS; read only
 *             during the call.
 * On a grouped handle: dns_set_state / dns_get_state take member ranges inside
 * one group (in that group's state layout); dns_stats fills the per-member
 * arrays (group-major) and requires every profile pointer to be NULL (profiles
 * differ per group: read them from the group's handle); DNS_OPT_PRECISION and
 * DNS_OPT_STATS apply to every group; dns_debug_stage0 and dns_kernel_times
 * need a group's handle.  Errors as dns_create, the message naming the group. */
#define DNS_MAX_GROUPS 16
typedef struct {
  dns_geometry g;
  double Re;
  int Nx, Ny, Nz;
  int members;
  double dt;
} dns_group;
int dns_create_grouped(const dns_group* groups, int ngroups, dns_handle** out);

/* Handle of group `group` of a grouped handle, for the per-group calls
 * (statistics with profiles, state I/O in local member numbers, kernel times).
 * The grouped handle owns it: dns_destroy on it does nothing, and it is freed
 * with the grouped handle.  Calls on it wait for the grouped handle's queued
 * work first.  Errors: DNS_E_INVALID (not grouped, group out of range). */
int dns_group_handle(dns_handle* h, int group, dns_handle** out);

/* Options (dns_set_option keys) */
#define DNS_OPT_PRECISION 1   /* value: DNS_PREC_*                                */
#define DNS_OPT_STREAM 2      /* value: hipStream_t cast to integer (0 = default) */
#define DNS_OPT_GRAPH 3       /* value: 1 capture one step as a hipGraph, 0 eager;
                                 DNS_E_UNSUPPORTED for 1 on a grouped handle     */
#define DNS_OPT_STATS 4       /* value: 1 accumulate one-point statistics each step */
#define DNS_OPT_PLANE_ROWS 5  /* value: advection-kernel variant, one of the built
                                 ones (DNS_E_UNSUPPORTED otherwise), for the current
                                 precision and advection form: the physical z rows
                                 per chunk of the general kernel, or, for the
                                 advective form on grids with Nx = Nz = 32 or 64,
                                 100 + rows (+ 50 when its forward-z sums are kept
                                 in the output buffer instead of registers) for
                                 the lane-parallel x-transform kernel, which is
                                 the default there                              */
#define DNS_OPT_MODE_TILE 6   /* value: members per workgroup of the per-mode kernel,
                                 1, 2, 4 or 8, fitting 160 KB of LDS; the tile
                                 runs in workgroups of 512 threads when two fit
                                 a CU, else of 1024 when one does.  Default: the
                                 largest tile of which two 512-thread workgroups
                                 fit a CU, else the largest in one of 1024     */
#define DNS_OPT_CHAINS 7      /* value: 1..DNS_MAX_CHAINS (<= ensemble): the members
                                 are advanced in this many contiguous chains, each
                                 on a stream of its own forked from and joined
                                 into the handle's stream, so that one chain's
                                 advection kernel overlaps another's per-mode
                                 kernel.  Results do not depend on it.  Default:
                                 1.                                             */
#define DNS_OPT_ADVECTION 8   /* value: DNS_ADV_*, the form of the advection term;
                                 DNS_E_UNSUPPORTED if no variant of that form is
                                 built for the grid at the current precision   */
#define DNS_OPT_SHARED_MEAN 9 /* value: 1 the members share one streamwise-mean flow
                                 (approximate S3T ensemble, Sec. 4: the n_x = 0
                                 modes of v and eta and the profiles U00, W00),
                                 advanced by the member averages of the members'
                                 forcing terms of those modes, i.e. by the mean's
                                 own advection plus the perturbation Reynolds
                                 stresses averaged over the members.  Turning it
                                 on replaces each member's mean by the member
                                 average (so does dns_set_state while it is on)
                                 and sets DNS_OPT_CHAINS to 1 (larger values are
                                 then rejected).  Default 0.                    */
#define DNS_OPT_QUASILINEAR 10 /* value: 1 the advection of the perturbations
                                 (n_x >= 1) is linearised about the streamwise
                                 mean, U_m . grad u' + u' . grad U_m, while the
                                 mean keeps the full advection including the
                                 streamwise average of u' . grad u' (the second-
                                 cumulant closure of S3T); 2 the adjoint of that
                                 linearised advection, -(U_m . grad) l' +
                                 (grad U_m)^T l' (App. B, integrated forward in
                                 the reversed time; use with a frozen mean).
                                 Advective form only (DNS_E_INVALID with
                                 DNS_ADV_ROTATIONAL).  Fewer plane-kernel
                                 chunk-row variants fit its LDS.  Default 0.    */
#define DNS_OPT_FROZEN_MEAN 11 /* value: 1 steps leave the n_x = 0 modes and U00,
                                 W00 as they are (a base flow for linearised or
                                 adjoint perturbation dynamics, App. B).
                                 Default 0.                                     */
#define DNS_OPT_V_DISCRETIZATION 12 /* value: DNS_VDISC_*; rebuilds the v operators
                                 on the host (long double) and reloads them   */
#define DNS_OPT_GROUP_STREAMS 13 /* grouped handles only.  value 0 (default):
                                 each sub-step runs every group's per-mode work
                                 (right-hand sides, solves, velocities) in one
                                 launch, a descriptor per group, after the
                                 groups' advection kernels ran on their own
                                 streams; 1: each group's whole step runs on a
                                 stream of its own (used anyway while a group
                                 has an external forcing or the groups'
                                 precisions differ).  Results do not depend on
                                 it.                                            */

/* Wall-normal discretizations of the v equation (Eq. (CN1)).  The paper uses
 * the fourth derivative of the clamped interpolant (Sec. 2).  The alternative
 * writes the CN step for phi = Lap v as a Helmholtz problem and Lap v = phi as
 * a Poisson problem, both collocated at the interior nodes, with phi's wall
 * values fixed by the clamped conditions v = dv/dy = 0 (the influence-matrix
 * method of Kim, Moin and Moser); both are spectral discretizations of the
 * same equation and converge to each other as Ny grows. */
#define DNS_VDISC_CLAMPED 0   /* clamped fourth-derivative operator (default)     */
#define DNS_VDISC_KMM 1       /* Helmholtz-Poisson with an influence matrix       */
#define DNS_MAX_CHAINS 4

/* Advection forms.  The paper advances the momentum equation (Sec. 2) with the
 * advective term u . grad u (Sec. 3.2).  Its rotational form omega x u differs
 * from it by the gradient of |u|^2 / 2, which the curl operators of the v-eta
 * equations remove, so both forms solve the same equations; discretely they
 * agree exactly for fields whose squared velocity the Chebyshev grid resolves
 * and differ by collocation error otherwise.  The rotational form needs 6
 * inverse x-z transforms per plane instead of 11.  With it, the dissipation
 * of dns_stats is the enstrophy form 1/(Re V) int |omega|^2 (equal to the
 * gradient form between no-slip walls). */
#define DNS_ADV_ADVECTIVE 0   /* u . grad u (the paper's form; default)          */
#define DNS_ADV_ROTATIONAL 1  /* omega x u                                       */

#define DNS_PREC_FP64 0        /* every stage in FP64                               */
#define DNS_PREC_MIXED_FP32 1  /* x-z FFTs and advection products in FP32, FP32
                                  stage buffers; y-derivative products, implicit
                                  solves, mean flow and flux update in FP64       */
#define DNS_PREC_MIXED_3XBF16 2 /* as DNS_PREC_MIXED_FP32, with the y-derivative
                                  products (D1 and the clamped D1c) on BF16
                                  matrix cores as three split products
                                  (hi*hi + hi*lo + lo*hi, FP32 accumulation)       */
#define DNS_PREC_MIXED_FP32MM 3 /* as DNS_PREC_MIXED_FP32, with the y-derivative
                                  products on FP32 matrix cores (FP32 operators
                                  and operands, FP32 accumulation): FFTs and
                                  derivative products in FP32, solves in FP64      */

/* Set an option.  Precision may be changed between steps (the stage buffers
 * are re-derived from the FP64 state).  Errors: DNS_E_INVALID. */
int dns_set_option(dns_handle* h, int key, long long value);

/* Host or device view of ensemble states.
 *   v_hat, eta_hat : interleaved complex double,
 *                    [member][n_x 0..Nx/2-1][n_z FFT order][j 1..Ny-2]
 *                    where FFT order is n_z = 0..Nz/2-1 then -(Nz/2-1)..-1
 *                    (Nz-1 entries); interior Chebyshev nodes only (v = eta = 0
 *                    at the walls, Eq. (b_ve)).  The n_x = 0 column must be
 *                    Hermitian (f(0,-n_z) = conj f(0,n_z)); (0,0) must be 0.
 *   U00, W00       : double [member][j 0..Ny-1], walls included.
 *   on_device      : 0 host pointers, 1 device pointers (same layout).
 * The caller owns the buffers; the library copies. */
typedef struct {
  double* v_hat;
  double* eta_hat;
  double* U00;
  double* W00;
  int on_device;
} dns_state_view;

/* Load members [member0, member0+count) from s.  Every member must satisfy the
 * rules of dns_check_state (checked on the host; device views have their
 * profiles and n_x = 0 columns copied back for it); the state is left as it
 * was when a member does not.  Clears the members' failure flags.
 * Errors: DNS_E_INVALID (the message names the member and the rule). */
int dns_set_state(dns_handle* h, int member0, int count, const dns_state_view* s);

/* Host-side check of `count` members of a host state view (on_device = 0)
 * against what dns_set_state requires for an ensemble of flow g->flow, wall
 * speed g->Uw and grid Nx x Ny x Nz; needs no handle and no GPU.
 *   - U00/W00 wall values match the boundary conditions (Sec. 2: Couette
 *     U00(-1) = -Uw, U00(1) = Uw; channel 0; W00 = 0) within 1e-12;
 *   - the (0,0) mode of v_hat and of eta_hat is zero, and their n_x = 0
 *     column is Hermitian, f(0,-n_z) = conj f(0,n_z) (Appendix A: only half
 *     of the conjugate pairs is stored), both within 1e-12 of the largest
 *     |f| of that member's column.
 * NaN or Inf in a wall value or in the n_x = 0 column fails the check (other
 * entries may hold anything: a non-finite member is accepted and flagged by
 * the step).  Returns DNS_OK, or DNS_E_INVALID with a message naming the
 * member and the rule (dns_last_error(NULL)). */
int dns_check_state(const dns_geometry* g, int Nx, int Ny, int Nz, int count, const dns_state_view* s);

/* Additive forcing of the (Lap v, eta) equations of members [member0,
 * member0+count): d(Lap v)/dt and d(eta)/dt gain f_lapv and f_eta, held
 * constant over each step until replaced (Sec. 4: the stochastic forcing of an
 * S3T ensemble is a mixture of eigenvectors of the diffusion operator acting
 * on a (Lap v, eta) state; the caller draws the mixture for each step and
 * calls this before the step).  Layout as dns_state_view's v_hat/eta_hat:
 * [member][n_x][n_z FFT order][j 1..Ny-2] interleaved complex doubles, host or
 * device memory (on_device), read during the call; a NULL field counts as
 * zero.  Both NULL: forcing off (the default).  With DNS_OPT_SHARED_MEAN the
 * n_x = 0 modes of the forcing are replaced by their member average.  The
 * first call allocates two state-sized device buffers; later calls reuse
 * them, so a captured step graph stays valid while the forcing changes.
 * Errors: DNS_E_INVALID (member range). */
int dns_set_forcing(dns_handle* h, int member0, int count, const double* f_lapv, const double* f_eta,
                    int on_device);

/* Kinetic energy density E = 1/(2V) int |u'|^2 of each member's perturbation
 * (its n_x >= 1 modes), from the FP64 state; out has `ensemble` entries
 * (App. B: the growth G(T) = E(T) / E(0)).  Synchronises the stream.
 * Errors: DNS_E_INVALID (NULL output, grouped handle). */
int dns_perturbation_energy(dns_handle* h, double* out);

/* Modified Gram-Schmidt of the members, in member order, over their n_x >= 1
 * modes in the kinetic-energy inner product, each normalised to energy density
 * 1; the n_x = 0 modes and U00, W00 are left as they are (App. B: the
 * orthonormalisation step of the forward-adjoint iteration that yields the
 * leading optimal disturbances).  Runs on the host in FP64 over a copy of the
 * state.  Errors: DNS_E_INVALID (a member without an independent
 * perturbation, grouped handle). */
int dns_orthonormalize(dns_handle* h);

/* Copy members [member0, member0+count) into s (synchronises the stream). */
int dns_get_state(dns_handle* h, int member0, int count, dns_state_view* s);

/* Advance every member by nsteps CN/RK3 time steps (Sec. 3.1), asynchronously
 * on the handle's stream.  A member that produces NaN/Inf is flagged
 * (sticky) and reported by dns_stats / dns_sync as DNS_E_NONFINITE; the other
 * members are unaffected (members never exchange data).  Errors: DNS_E_HIP. */
int dns_step(dns_handle* h, int nsteps);

/* Per-member diagnostics of the current state and time/ensemble-averaged
 * one-point statistics (Sec. 4: mean profile U(y), rms u', v', w' about it,
 * Reynolds stress u'v').  Any pointer may be NULL.  Arrays of length
 * `ensemble` (per member) or Ny (profiles) are owned by the caller.
 * Volume averages use Clenshaw-Curtis weights over y and divide by Ly = 2.
 *   energy      E = 1/(2V) int |u|^2 (mean flow included)
 *   dissipation eps = 1/(Re V) int |grad u|^2 (|omega|^2 with DNS_ADV_ROTATIONAL)
 *   power       Couette Uw (U'(1) + U'(-1)) / (Re Ly); channel gamma Q / Ly
 *   flux        Q = int U dy;  gamma: pressure gradient of the last sub-step
 *   div_max     max over modes/nodes of |i kx u + dv/dy + i kz w|
 *   tau_lower/upper  U'(-1)/Re and U'(+1)/Re;  failed: sticky NaN/Inf flag
 *   profiles    averaged over members and the samples since the last reset;
 *   tau_w       Couette mean |U'| at the walls / Re, channel (U'(-1)-U'(1))/(2Re)
 *   re_tau      Re sqrt(tau_w)
 *   member_profiles  [member][8][Ny]: each member's time averages since the
 *               last reset of U00, W00, U00^2, W00^2 and of the x-z plane
 *               means of u^2, v^2, w^2 and u v (mean flow included: the plane
 *               mean of u^2 is U00^2 + sum over k != 0 of m_k |u_k|^2, m_k = 1
 *               for n_x = 0, else 2), in that order.  The pooled statistics
 *               above are, per node, U = <U00>, u'^2 = <u^2> - U^2,
 *               v'^2 = <v^2>, w'^2 = <w^2> - W^2, u'v' = <u v> with <.> the
 *               mean over members of these arrays, so resampling members (a
 *               bootstrap) needs only them.  Zero before the first sample.
 *               Must be NULL on grouped handles.
 *   member_tau  [member][2]: each member's time averages of U'(-1)/Re and
 *               U'(+1)/Re since the last reset (group-major on grouped handles)
 * Synchronises.  Returns DNS_E_NONFINITE if any member failed, else DNS_OK. */
typedef struct {
  double* energy;
  double* dissipation;
  double* power;
  double* flux;
  double* gamma;
  double* div_max;
  double* tau_lower;
  double* tau_upper;
  int* failed;
  double* U;
  double* W;
  double* urms;
  double* vrms;
  double* wrms;
  double* uv;
  double tau_w;
  double re_tau;
  long long samples;
  long long steps;
  double* member_profiles;
  double* member_tau;
} dns_stats_out;
int dns_stats(dns_handle* h, dns_stats_out* o);

/* Restart the time averages of dns_stats. */
int dns_stats_reset(dns_handle* h);

/* Wait for all queued work; DNS_E_NONFINITE if a member has failed. */
int dns_sync(dns_handle* h);

/* Free every resource of the handle.  NULL-safe. */
void dns_destroy(dns_handle* h);

/* Message of the last error on h (or of the calling thread when h is NULL). */
const char* dns_last_error(const dns_handle* h);

/* Tile-shape tuner.  Times every built chunk-row variant of the advection
 * kernel and every admissible member tile of the per-mode kernel on the current
 * state (HIP events on the handle's stream, 5 launches each, the per-mode
 * kernel at its second sub-step; the state does not advance) and keeps the
 * fastest of each for the current precision; the current member tile stays
 * unless another is more than 2 % faster.  Tile shapes change the order of
 * floating-point operations in the FFTs, never the method.
 *   cache_path : optional text file (NULL: none).  A line "<precision> <Nx>
 *                <Ny> <Nz> <members> <plane_rows> <mode_members> <plane_ms>
 *                <mode_ms>" with this handle's key is applied without timing
 *                (the last such line wins); new results are appended.
 *   out        : NULL, or one dns_tuning per group (1 for a plain handle).
 * Synchronises.  Errors: DNS_E_HIP, DNS_E_INVALID (cache not writable or its
 * entry not applicable). */
typedef struct {
  int plane_rows;     /* chosen chunk rows of the advection kernel   */
  int mode_members;   /* chosen members per per-mode workgroup       */
  double plane_ms;    /* its time per launch (from the cache if so)  */
  double mode_ms;
  int from_cache;     /* 1 if read from cache_path                   */
} dns_tuning;
int dns_tune(dns_handle* h, const char* cache_path, dns_tuning* out);

/* Stage intermediates for verification (not needed for time stepping).
 * From the current state, without advancing it, computes the first RK3
 * sub-step's inputs and copies them to host buffers (NULL skips):
 *   vel   : complex double [5][member][Ny][Nx/2][Nz-1]: u, v, w, du/dy, dw/dy
 *           (Sec. 3.2 u/w recovery and y derivatives);
 *   nl    : complex double [3][member][Ny][Nx/2][Nz-1]: de-aliased advection
 *           terms u.grad u, u.grad v, u.grad w (Sec. 3.1);
 *   means : double [2][member][Ny]: plane means <uv>, <wv> (Eqs. (U00), (W00)).
 * Synchronises.  Errors: DNS_E_HIP. */
int dns_debug_stage0(dns_handle* h, double* vel, double* nl, double* means);

/* Average device time of one launch of each hot kernel, measured with HIP
 * events on the handle's stream over nreps back-to-back launches at the
 * current precision (Sec. 4.4 times the same operation classes of one step).
 * Does not advance the state: the second RK3 sub-step's kernels are timed
 * against the current stage buffers and the next dns_step re-derives them.
 * Outputs, milliseconds per launch (NULL skips):
 *   plane_ms : de-aliased advection kernel (x-z FFTs and products, Sec. 3.1);
 *   mode_ms  : per-(kx,kz) right-hand side, CN solve and velocity kernel
 *              (Eqs. (CN1)-(CN4)).
 * Synchronises.  Errors: DNS_E_INVALID (nreps < 1), DNS_E_HIP. */
int dns_kernel_times(dns_handle* h, int nreps, double* plane_ms, double* mode_ms);

/* Host-side operator construction for verification; needs no GPU.
 * Builds on the host, in extended precision, exactly the operators dns_create
 * uploads for one sub-step fraction (h_index 0: h = 1/2, 1: h = 1) and v
 * discretization (DNS_VDISC_*; A_v, B_v only depend on it), with
 * c = h dt / (2 Re) (Sec. 3.2, Eqs. (CN1)-(CN4), Listings 1 and 3):
 *   ops      : double [Nx/2 * Nz/2][4][Ny-2][Ny-2], row-major; per group
 *              g = n_x*(Nz/2) + |n_z| the folded A_v, B_v, A_eta, B_eta with
 *              v_new = A_v v0 - h dt B_v F and eta_new = A_eta eta0 - h dt B_eta G;
 *              group 0 (the mean) is zero;
 *   mean_ops : double [2][Ny-2][Ny-2]: A_U, B_U of the mean profiles;
 *   lift     : double [Ny-2]: Couette wall-velocity contribution to U;
 *   green    : double [Ny-2]: response of U to a unit pressure gradient gamma;
 *   D1       : double [Ny][Ny] Chebyshev first derivative (ascending nodes);
 *   D1c      : double [Ny][Ny-2] first derivative of the clamped interpolant;
 *   ccw      : double [Ny] Clenshaw-Curtis weights.
 * NULL outputs are skipped.  Errors: DNS_E_INVALID, DNS_E_UNSUPPORTED. */
int dns_host_operators(const dns_geometry* g, double Re, int Nx, int Ny, int Nz, double dt,
                       int h_index, int v_discretization, double* ops, double* mean_ops, double* lift,
                       double* green, double* D1, double* D1c, double* ccw);

#ifdef __cplusplus
}
#endif

#endif /* DNS_ENSEMBLE_H */
