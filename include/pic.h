/*
 * pic.h -- C interface of the MI355X (gfx950) quasi-cylindrical, arbitrary-order
 * PSATD particle-in-cell cycle.
 *
 * Method: Jalas et al., "Accurate modeling of plasma acceleration with arbitrary
 * order pseudo-spectral particle-in-cell methods".  One PIC cycle per azimuthal
 * mode m is
 *   (a) linear-shape deposit of rho and J onto the (r, z) grid of each mode,
 *   (b) FFT along z and discrete Hankel transform along r
 *       (Sec. "Finite order pseudo-spectral solvers", the quasi-cylindrical
 *       decomposition into spectral +, -, z components),
 *   (c) PSATD update of E and B, Eqs. (1a)-(1b) with the operators of
 *       Eqs. (2a)-(2b) and k_z replaced by the modified wavenumber [k_z] of
 *       Eq. (5) everywhere, including inside |k|, C and S,
 *   (d) inverse transforms,
 *   (e) field gather and Boris push.
 *
 * Units: normalized plasma units (lengths 1/k_p, time 1/omega_p, u = gamma*beta,
 * densities n0, charge e, mass m_e; c = 1).
 *
 * Conventions shared by every entry point
 *   - Fields of mode m are complex; the real field is
 *     F = sum_{m=-M..M} F_m exp(-i m theta) with F_{-m} = conj(F_m).
 *     Vector fields are stored as F_+ = (F_r - i F_theta)/2, F_- = (F_r + i F_theta)/2
 *     and F_z; their Hankel orders in mode m are m+1, m-1 and m.
 *   - Grid nodes: z_j = z_min + j dz (periodic in z, j = 0..nz-1),
 *     r_i = (i + 1/2) dr (i = 0..nr-1).  Host field buffers are [nr][nz]
 *     complex float32 (interleaved re, im; z fastest).  Spectral buffers are
 *     [nr (k_perp index)][nz (FFT order along k_z)].
 *   - Every call returns a status (PIC_OK = 0 or a negative pic_status); no
 *     exception or abort crosses the interface.  Work is enqueued on the stream
 *     given to pic_init; errors of asynchronous GPU work surface at the next
 *     synchronizing call (pic_diagnostics, pic_get_*, pic_set_field, pic_sync,
 *     pic_free) as PIC_EHIP.
 *   - Memory: the caller owns one device workspace of pic_workspace_bytes()
 *     bytes (any device allocation, e.g. a torch uint8 tensor) that must stay
 *     alive and untouched until pic_free; the library allocates no device
 *     memory of its own.  Host pointers passed in are only read during the call.
 *   - Calls on one context must not overlap (one host thread at a time).
 */
#ifndef PIC_H
#define PIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PIC_OK = 0,
  PIC_EINVAL = -1,    /* invalid configuration, species or pointer */
  PIC_ENOSPC = -2,    /* workspace too small, or particle capacity exceeded */
  PIC_EHIP = -3,      /* HIP runtime error (launch or asynchronous fault) */
  PIC_ESTATE = -4,    /* call out of order (see the step order below) */
  PIC_ENUMERIC = -5   /* NaN or Inf found by pic_diagnostics, or produced by a split-precision
                         Hankel product (an operand beyond the range of its halves: FP16
                         65504), reported by the next synchronizing call */
} pic_status;

/* Radial wavenumber grid of the discrete Hankel transform.  In mode m the
   components F_-, F_z and F_+ are synthesised with Bessel functions of order
   m - 1, m and m + 1 at the same wavenumbers; the forward transform is the
   pseudo-inverse of that synthesis matrix (singular values below 1e-4 of
   the largest dropped). */
typedef enum {
  PIC_KPERP_J0_ZEROS = 0, /* k_i = j_{0,i} / R for every mode.  Well conditioned, but in
                             mode 1 the order-2 basis is neither orthogonal nor of equal
                             norm, and mode 1 grows without bound in beam-plasma runs */
  PIC_KPERP_SINE = 1,     /* k_i = (i + 1) pi / R (comparison only) */
  PIC_KPERP_JM_ZEROS = 2  /* k_i = j_{m,i} / R for mode m (recommended): the three
                             orders share one norm and are orthogonal, so the field
                             energy the spectral update conserves is the one the
                             particles see */
} pic_kperp_grid;

/* Arithmetic of the Hankel-transform matrix products. */
typedef enum {
  PIC_H_FP32 = 0,   /* FP32 MFMA, FP32 operands */
  PIC_H_BF16X3 = 1, /* split hi+lo bfloat16 operands, 3 MFMA products, FP32 accumulate */
  PIC_H_FP16X3 = 2  /* split hi+lo float16 operands, 3 MFMA products, FP32 accumulate */
} pic_hankel_prec;

/* Field components addressed by pic_get_field / pic_set_field. */
typedef enum {
  PIC_E_PLUS = 0, PIC_E_MINUS = 1, PIC_E_Z = 2,
  PIC_B_PLUS = 3, PIC_B_MINUS = 4, PIC_B_Z = 5,
  PIC_J_PLUS = 6, PIC_J_MINUS = 7, PIC_J_Z = 8,
  PIC_RHO_OLD = 9,   /* rho^n   (deposited at x^n)      */
  PIC_RHO_NEW = 10,  /* rho^{n+1} (deposited at x^{n+1}) */
  PIC_N_COMP = 11
} pic_comp;

typedef struct pic_ctx pic_ctx;

typedef struct {
  int32_t nz;          /* cells along z: power of two, 64 <= nz <= 4096 */
  int32_t nr;          /* radial cells: multiple of 32, 32 <= nr <= 1024 */
  int32_t n_modes;     /* azimuthal modes m = 0..n_modes-1, 1 <= n_modes <= 4 */
  int32_t order;       /* stencil order p = 2n (even, >= 2); 0 = infinite order */
  double dz, dr, dt;   /* > 0; dt <= 2 min(dz, dr) (particles cross at most two cells per step) */
  double z_min;        /* position of node j = 0 at step 0 */
  int32_t moving_window;      /* 1: z_min advances by dz after every step (needs dt == dz) */
  int32_t kperp_grid;         /* pic_kperp_grid */
  int32_t hankel_prec;        /* pic_hankel_prec */
  int32_t current_correction; /* 1 (default); 0 disables the spectral correction */
  int32_t filter;             /* binomial smoothing of J and rho before the field update:
                                 0 = none (default); n = 1..4 passes of the 1-2-1 average along
                                 z and along r, applied in spectral space as the factor
                                 [cos^2(k_z dz / 2) cos^2(k_perp dr / 2)]^n (zero at the z Nyquist
                                 wavenumber, where a beam at dt = dz / c drives the numerical
                                 Cherenkov instability of the infinite-order solver) */
  int32_t damp_cells;         /* absorbing layers at the z ends of the grid: 0 = none (default);
                                 N in 1..nz/4: after every step the real-space E and B at the N
                                 nodes nearest each z end are multiplied by sin^2(pi s / (2 N)),
                                 s = 0..N-1 the node's distance in cells from the end node (the
                                 end node is zeroed), and the next step transforms E and B from
                                 real space again, so the field state is the damped one.  Keeps
                                 what leaves the grid at one end from re-entering at the other
                                 through the periodic z transform */
  int32_t galilean;           /* 1 (needs moving_window): Galilean PSATD (the scheme the paper
                                 names as intrinsically stable for drifting plasmas, Sec. "Finite
                                 order pseudo-spectral solvers"): the fields live in coordinates
                                 moving with the window, v = dz / dt, where Maxwell's equations
                                 gain the advection term i [k_z] v F; the update is their exact
                                 solution with J constant over the step, the current correction
                                 enforces the moving-frame continuity equation, rho^{n+1} and J
                                 are carried onto the grids of t^{n+1} and t^{n+1/2} (exact
                                 periodic one- and half-node moves; the half move is zero at the
                                 z Nyquist wavenumber) and E, B are not shifted by the window
                                 move.  0 (default): the lab-frame update of Eqs. (1a)-(1b) */
  int32_t shape_order;        /* particle shape of the deposit and the gather: 1 (or 0, the
                                 default) linear; 3 cubic B-spline over the four nearest nodes
                                 along z and along r (ghost nodes at -dr/2 and -3dr/2 stand for
                                 nodes 0 and 1 across the axis with the factor (-1)^nu of the
                                 Hankel order).  Cubic shapes deposit every particle straight
                                 into the tile blocks (no register runs): a slower option */
} pic_config;

typedef struct {
  int64_t n;          /* macro-particles (may be 0) */
  double q, m;        /* charge (units of e, nonzero) and mass (units of m_e, > 0) */
  int32_t mobile;     /* 0: immobile background, deposited into rho only.  With a
                         moving window an immobile species must be uniform in z
                         (a lattice with a one-cell period), else PIC_EINVAL */
  int32_t inject;     /* 1: a cold lattice column is injected at the head at every
                         window move (ppc_z x ppc_r x ppc_t particles per cell at
                         z = (j + (a+1/2)/ppc_z) dz, r = (i + (b+1/2)/ppc_r) dr,
                         theta = 2 pi l / ppc_t, weight density * r dr dz 2pi/(ppc_z ppc_r ppc_t)) */
  int32_t ppc_z, ppc_r, ppc_t;
  double density;     /* injected lattice density (units of n0) */
  int32_t diag;       /* 1: species selectable by pic_diagnostics */
  int32_t self_field; /* 1 (mobile, cold, monoenergetic beams): pic_init adds the beam's
                         own field, the field of its charge moving rigidly at its mean
                         velocity along z: phi = rho / (k_perp^2 + [k_z]^2 / gamma^2),
                         E = -grad phi with E_z scaled by 1/gamma^2, B_+ = -i beta E_+,
                         B_- = +i beta E_-, B_z = 0 (spectral operators of Eqs. (2a)-(2b));
                         it satisfies the discrete Gauss law.  0: the species starts with
                         no field of its own */
  const double *x, *y, *z;            /* host, length n */
  const float *ux, *uy, *uz, *w;      /* host, length n; u = gamma beta (u_z is widened
                                         to FP64 on the device); w = macro-particle weight */
} pic_species;

/* Bytes of device workspace needed for cfg, the species and a particle capacity
 * of max_particles mobile macro-particles (0 = total mobile count + 12.5 %).
 * Errors: PIC_EINVAL (bad cfg / species / null pointer). */
int pic_workspace_bytes(const pic_config* cfg, const pic_species* species, int n_species,
                        int64_t max_particles, size_t* bytes);

/* Builds a context: validates, carves the workspace, builds in FP64 on the GPU
 * the [k_z] table (Eq. (5)), the k_perp grid and the Hankel matrices of each
 * mode m and order nu = m-1, m, m+1 (the quasi-cylindrical spectral
 * representation of Sec. "Finite order pseudo-spectral solvers"):
 *   backward B_nu[i_r][i_k] = J_nu(k_{i_k} r_{i_r});
 *   forward  F_nu = Moore-Penrose pseudo-inverse of B_nu, from a one-sided
 *            Jacobi SVD in FP64 (B_nu = U S V^T, F_nu = sum over the singular
 *            values s_j >= 1e-4 s_max of v_j u_j^T / s_j; directions below the
 *            cut-off are projected out, not amplified; on the J_m-zero grid
 *            this drops the one near-null direction of order 0 in mode 1),
 * both rounded to FP32 for the products; uploads the particles (host arrays
 * are read during the call only), deposits the immobile background once
 * and adds the own fields of self_field species; E, B start at zero
 * otherwise.  `hip_stream` is a hipStream_t (NULL = default stream); the
 * context keeps it.  Synchronizes once.
 * Errors: PIC_EINVAL (bad cfg or species; the Jacobi SVD of a Hankel matrix
 * did not converge within 60 sweeps; an immobile species that is not uniform
 * in z with a moving window; the deposit tile block exceeds the device's
 * LDS), PIC_ENOSPC (workspace smaller than pic_workspace_bytes, or more
 * mobile particles than the capacity), PIC_EHIP.  On error *out is NULL and
 * nothing needs freeing. */
int pic_init(const pic_config* cfg, const pic_species* species, int n_species,
             int64_t max_particles, void* workspace, size_t bytes, void* hip_stream,
             pic_ctx** out);

/* Step order: gather_push -> deposit -> spectral_push, repeated.  Any other
 * order returns PIC_ESTATE.  Particle storage order changes at every deposit. */

/* Gathers E^n, B^n at x^n (linear shapes, 4 nodes per mode; 16 with
 * shape_order = 3), Boris-pushes
 * u^{n-1/2} -> u^{n+1/2} and moves x^{n+1} = x^n + dt u^{n+1/2}/gamma.
 * Fields live at integer steps and momenta at half steps, the staggering the
 * PSATD update (1a)-(1b) assumes when it takes J at n+1/2 and rho at n, n+1
 * (Sec. "Finite order pseudo-spectral solvers").  Asynchronous; computes each
 * particle's new cell key for the sort.  Errors: PIC_EINVAL (null ctx),
 * PIC_ESTATE (not at the start of a step), PIC_EHIP (launch failure). */
int pic_gather_push(pic_ctx* ctx);

/* Sorts the particles by cell, then deposits rho^n at x^n, J^{n+1/2} at
 * x^{n+1/2} = x^{n+1} - dt v^{n+1/2}/2 with v^{n+1/2} and rho^{n+1} at x^{n+1}:
 * the three source time levels of the E update (1a) and of the current
 * correction (Sec. "Finite order pseudo-spectral solvers").  Linear shapes
 * (cubic B-splines with shape_order = 3); mode m of a density carries exp(i m theta_p) and is divided by the ring
 * volume 2 pi r_i dr dz; below the first radial node the inner shape node is
 * the ghost node -dr/2, folded onto node 0 with the sign (-1)^nu of the
 * component's Hankel order.  The immobile background density is added node by
 * node to both densities.  Atomic-free at global scope: each grid tile is
 * written once by the workgroup that owns it.  Asynchronous.  Errors:
 * PIC_EINVAL (null ctx), PIC_ESTATE (gather_push not done), PIC_EHIP; a
 * deposit work list larger than the launch sets a device flag reported as
 * PIC_ENOSPC by the next synchronizing call. */
int pic_deposit(pic_ctx* ctx);

/* Forward FFT along z and Hankel transform of J, rho^n, rho^{n+1}; spectral
 * current correction (J += grad F, F = (div J + (rho^{n+1}-rho^n)/dt)/k^2);
 * PSATD update of the spectral E, B; inverse transforms to real space; then,
 * with a moving window, shifts the fields one cell toward the tail (head column
 * zeroed), advances z_min, drops particles behind it and injects lattice columns
 * at the head. */
int pic_spectral_push(pic_ctx* ctx);

/* n x (gather_push, deposit, spectral_push). */
int pic_step(pic_ctx* ctx, int n);

/* Waits for all enqueued work; reports asynchronous errors as PIC_EHIP. */
int pic_sync(pic_ctx* ctx);

typedef struct {
  int32_t species;        /* index into the pic_init species array (must have diag = 1) */
  double slice_len;       /* slice length (1/k_p) */
  double n_sigma;         /* slices cover |z - <z>| <= n_sigma * sigma_z */
  int32_t min_per_slice;  /* slices with fewer macro-particles are skipped */
} pic_diag_req;

typedef struct {
  double eps_nx, eps_ny;          /* normalized rms emittances sqrt(<x^2><ux^2> - <x ux>^2) */
  double mean_gamma, sigma_gamma; /* weighted mean and rms of gamma */
  double mean_slice_sigma_gamma;  /* average over kept slices of the slice rms gamma */
  double z_mean, sigma_z;
  int64_t n;                      /* macro-particles of the species inside the window */
  int32_t n_slices, nan_flag;
} pic_diag_out;

/* Beam diagnostics of one species (weighted, central moments accumulated in
 * FP64): the quantities behind the paper's Err_eps and Err_sigma_gamma,
 * Eqs. (11)-(12).  Synchronizes.  Returns PIC_ENUMERIC (with out filled and
 * nan_flag = 1) if a position or momentum of the species is not finite. */
int pic_diagnostics(pic_ctx* ctx, const pic_diag_req* req, pic_diag_out* out);

/* pic_diagnostics plus the per-slice values behind Err_sigma_gamma, Eq. (11):
 * slice k (0 <= k < n_total) covers xi = z - <z> in [(k - n_total/2) L,
 * (k - n_total/2 + 1) L), L = slice_len, n_total = 2 ceil(n_sigma sigma_z / L);
 * sigma_gamma[k] is its weighted rms gamma (0 when the slice has fewer than
 * min_per_slice macro-particles) and count[k] its macro-particle count.  The
 * first min(cap, n_total) slices are written to the host arrays; *n_total is
 * always set (0 when sigma_z = 0).  Synchronizes.  Errors as pic_diagnostics. */
int pic_diagnostics_slices(pic_ctx* ctx, const pic_diag_req* req, pic_diag_out* out, double* sigma_gamma,
                           double* count, int32_t cap, int32_t* n_total);

/* pic_diagnostics_slices for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  Same arguments, results and errors as pic_diagnostics_slices,
 * except:
 *   - its partial sums and per-slice accumulators live in one static device
 *     array of the library (168 KB on each GPU it runs on, held until the
 *     process ends) instead of the context's workspace; it calls no hipMalloc
 *     or hipFree and allocates no host memory;
 *   - at most 4096 slices: a request needing more returns PIC_ENOSPC with
 *     *n_total set to the number needed and the moments in *out filled;
 *   - every call on a GPU shares that GPU's array, which keeps the last call's
 *     contents (each call clears what it accumulates); calls that overlap on
 *     one GPU, from any context, race and must be serialized by the caller.
 * Synchronizes.  Errors: PIC_EINVAL (null pointers, bad request), PIC_ENOSPC,
 * PIC_EHIP (also when the array's device address could not be looked up at
 * pic_init), PIC_ENUMERIC. */
int pic_diagnostics_slices_noalloc(pic_ctx* ctx, const pic_diag_req* req, pic_diag_out* out,
                                   double* sigma_gamma, double* count, int32_t cap, int32_t* n_total);

/* Copies one field component of one mode to host memory ([nr][nz] complex
 * float32, 8*nr*nz bytes).  spectral = 0: real space; 1: spectral.  E, B are
 * the current fields; J, rho are those of the last deposit (spectral J is after
 * the current correction; the spectral transform keeps rho^{n+1} - rho^n rather
 * than rho^n, and spectral rho^n is returned as rho^{n+1} minus it).
 * Synchronizes.  Errors: PIC_EINVAL, PIC_EHIP. */
int pic_get_field(pic_ctx* ctx, int mode, int comp, int spectral, void* host_dst);

/* Overwrites one real-space field component of one mode from host memory
 * ([nr][nz] complex float32).  Setting E or B makes the next spectral_push
 * re-transform the real-space E, B; setting all five source components
 * (J_+, J_-, J_z, rho^n, rho^{n+1}) of every mode allows spectral_push without a
 * deposit.  Synchronizes.  Errors: PIC_EINVAL. */
int pic_set_field(pic_ctx* ctx, int mode, int comp, const void* host_src);

/* Number of live mobile macro-particles (inside the window).  Synchronizes. */
int pic_num_particles(pic_ctx* ctx, int64_t* n);

/* Copies the live mobile particles of one species (index into the pic_init
 * array) to host: xyz = n*3 doubles (x, y, z per particle), uvw = n*3 doubles
 * (u_x, u_y, u_z: the library keeps u_x, u_y in FP32 and u_z in FP64),
 * w = n floats (may be NULL); at most `cap` particles, count in *n.
 * Order is the library's current storage order.  Synchronizes.
 * Errors: PIC_EINVAL (null pointer, bad species), PIC_ENOSPC (more than cap
 * particles: the first cap are copied), PIC_EHIP. */
int pic_get_particles(pic_ctx* ctx, int species, int64_t cap, double* xyz, double* uvw,
                      float* w, int64_t* n);

/* Current window position z_min and number of completed steps. */
int pic_get_state(pic_ctx* ctx, double* z_min, int64_t* steps);

/* Frees the host-side context (the workspace stays the caller's).  Synchronizes. */
int pic_free(pic_ctx* ctx);

/* Static description of a status code. */
const char* pic_strerror(int status);

/* --------------------------------------------------------------------------
 * Kernel timing (measurement support): when enabled, HIP events are recorded
 * on the context's stream around each phase of the cycle; pic_timing_read
 * synchronizes and returns the summed GPU time and launch count of a phase
 * since the last pic_timing_enable.
 * ------------------------------------------------------------------------ */
typedef enum {
  PIC_T_GATHER_PUSH = 0, /* gather + Boris push kernel */
  PIC_T_SORT = 1,        /* particle scatter into cell order */
  PIC_T_DEPOSIT = 2,     /* tile deposit kernel (LDS accumulation of one tile or chunk) */
  PIC_T_FFT_FWD = 3,     /* forward z-FFT of the sources (and of E, B when re-transformed) */
  PIC_T_DHT_FWD = 4,     /* forward Hankel-transform products */
  PIC_T_PSATD = 5,       /* window shift + current correction + PSATD update */
  PIC_T_DHT_INV = 6,     /* inverse Hankel-transform products of E, B */
  PIC_T_FFT_INV = 7,     /* inverse z-FFT of E, B (+ window shift) */
  PIC_T_WINDOW = 8,      /* departed-column transform, window advance, injection,
                            absorbing layers */
  PIC_T_SCAN = 9,        /* exclusive scan of the per-cell particle counts */
  PIC_T_DEP_PLAN = 10,   /* deposit work list: particles per tile, chunk offsets */
  PIC_T_DEP_COMBINE = 11,/* node-parallel sum of the tile blocks into the grid */
  PIC_T_PACK = 12,       /* node-interleaved copy of E, B for the gather */
  PIC_T_N = 13
} pic_timer;

/* enable != 0 clears previous records and starts recording; 0 stops. */
int pic_timing_enable(pic_ctx* ctx, int enable);
/* Errors: PIC_EINVAL (bad timer), PIC_EHIP. */
int pic_timing_read(pic_ctx* ctx, int timer, double* total_ms, int64_t* launches);

/* --------------------------------------------------------------------------
 * Repeated steps without host launch overhead, batches of independent runs,
 * and performance tunables (used by parameter scans: many instances of the
 * cycle with different grids, orders and beams run side by side).
 * ------------------------------------------------------------------------ */

/* Launch parameters that change speed only (results agree to rounding). */
typedef struct {
  int32_t gemm_tile_m;     /* output rows per Hankel-product workgroup tile: 32, 64 or 128
                              (must divide nr), or 0 (the default): per product the
                              largest tile whose workgroups fill the compute units in
                              nearly whole rounds */
  int32_t deposit_chunk;   /* particles per deposit work item of a dense tile: 2048, 4096
                              or 8192 (tiles above 3x this are cut into such chunks) */
} pic_tuning;

/* Read / set the tunables.  Errors: PIC_EINVAL (null or unsupported values). */
int pic_get_tuning(pic_ctx* ctx, pic_tuning* t);
int pic_set_tuning(pic_ctx* ctx, const pic_tuning* t);

/* n whole steps, enqueued as replays of a HIP graph that holds two steps of
 * this context (captured at the first call and again whenever a tunable or
 * the pending window shift changed; a first step after pic_init or
 * pic_set_field runs eagerly).  The context's stream must not be the legacy
 * null stream, timing must be off and the call must start a step (PIC_ESTATE
 * otherwise).  Asynchronous like pic_step; same results to rounding. */
int pic_step_graph(pic_ctx* ctx, int n);

/* A batch of independent contexts (parameter scans: many instances with
 * different grids, orders and beams, Sec. "Accurate modeling of plasma
 * accelerators in finite order PSATD") advanced by ONE HIP graph: two steps of
 * every context, each on the context's own stream, forked from and joined
 * into the batch's lead stream, so that one graph launch advances the whole
 * batch by two steps and the GPU overlaps the instances' kernels.
 *
 * pic_batch_create: ctxs holds n_ctx >= 1 distinct contexts of the current
 * device, each with its own non-null stream; the batch keeps the pointers
 * (the contexts must outlive it) and owns a lead stream and events.  Nothing
 * is captured yet.  Errors: PIC_EINVAL (null or repeated context, legacy
 * stream), PIC_EHIP.
 *
 * pic_batch_run: n steps of every context.  A first step after pic_init or
 * pic_set_field of any context runs eagerly on every context; the graph is
 * captured at the first run and again when a context's tunables or pending
 * window shift differ from those it was captured with; an odd last step runs
 * eagerly.  Each context's later work on its own stream is ordered after the
 * replays.  Asynchronous.  Every context must be at the start of a step with
 * timing off.  Same results as pic_step to rounding.  Errors: PIC_ESTATE,
 * PIC_EINVAL, PIC_EHIP (steps already enqueued stay enqueued).
 *
 * pic_batch_free: waits for the batch's replays and for the work queued on
 * every context's stream, then releases the graph, events and lead stream
 * (not the contexts).  Errors: PIC_EINVAL, PIC_EHIP. */
typedef struct pic_batch pic_batch;
int pic_batch_create(pic_ctx* const* ctxs, int n_ctx, pic_batch** out);
int pic_batch_run(pic_batch* batch, int n);
int pic_batch_free(pic_batch* batch);

/* n steps of each of n_ctx independent contexts: pic_batch_create, then
 * pic_batch_run(n), then pic_batch_free (so it returns once the replays are
 * done).  n_ctx = 0 or n = 0 does nothing.  Errors as those calls. */
int pic_batch_step(pic_ctx* const* ctxs, int n_ctx, int n);

/* Autotuner: for every supported (gemm_tile_m, deposit_chunk) pair, runs two
 * untimed and then steps_per_trial timed graph steps (HIP events on the
 * context's stream), keeps the fastest pair and returns it with its time per
 * step in ms.  The simulation advances by all these steps.  Synchronizes.
 * Errors: PIC_EINVAL (steps_per_trial < 2, null stream, timing on). */
int pic_autotune(pic_ctx* ctx, int steps_per_trial, pic_tuning* best, double* best_ms);

/* --------------------------------------------------------------------------
 * Kernel-level entry points used by parity tests and benchmarks.  Each runs
 * one step of the cycle on caller-provided device buffers (no context), on
 * `hip_stream`, asynchronously.  Pointers are device pointers.
 * ------------------------------------------------------------------------ */

/* Batched complex FFT along the contiguous axis: `rows` rows of nz complex
 * float32, in place.  inverse = 0: X_k = sum_j x_j exp(-2 pi i j k / nz);
 * inverse = 1: x_j = (1/nz) sum_k X_k exp(+2 pi i j k / nz).  nz is a power of
 * two in [16, 4096].  Errors: PIC_EINVAL. */
int pic_fft_z(void* data, int64_t rows, int nz, int inverse, void* hip_stream);

/* Batched real matrix product Y_b = A_b X_b of `batch` pairs: A_b is n x n
 * float32 stored TRANSPOSED (at[k][m] = A[m][k]), X_b and Y_b are n x ncols
 * float32 row-major (a complex [n][nz] field is the real n x 2nz matrix).
 * a_t[b], x[b], y[b] are device arrays of `batch` device pointers, each
 * 16-byte aligned (operands are read as 16-byte vectors; any hipMalloc'd
 * buffer at an offset of a multiple of 4 floats qualifies).
 * prec = pic_hankel_prec.  n is a multiple of 32, ncols a multiple of 128.
 * Errors: PIC_EINVAL. */
int pic_dht_gemm(const void* const* a_t, const void* const* x, void* const* y, int batch,
                 int n, int ncols, int prec, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* PIC_H */
