/*
 * ep.h -- C ABI of the MI355X cardiac electrophysiology voxel time-stepper.
 *
 * The library advances the operator-split, matrix-free finite-volume
 * monodomain / bidomain equations on a voxel grid (thesis "Computational
 * Tools for Cardiac Simulation", Algorithm Details chapter, section
 * "Electrophysiology"): a pointwise Mitchell-Schaeffer update by explicit
 * Euler (Reaction subsection; eqn:ms1, eqn:ms2), then diffusion through the
 * conductivity tensor field (eqn:sigma1) either explicitly or by implicit
 * Euler solved with Jacobi-preconditioned CG (Discretization and Solver
 * chapter, Linear Solver section, "Implicit Euler"), and for the bidomain
 * model the elliptic extracellular equation (second line of
 * eqn:bidomain1) by FP32 PCG inside FP64 iterative refinement.
 *
 * Conventions shared by every call:
 *  - Every call returns an ep_status; EP_OK is 0.  No C++ exception crosses
 *    the ABI.  ep_last_error(g) gives a message for the last failure on g;
 *    ep_last_error(NULL) gives the calling thread's last failed
 *    ep_create_grid message.
 *  - Box layout: flat index (x*ny + y)*nz + z, z fastest, n = {nx, ny, nz}.
 *  - Units: lengths mm, times ms, diffusivities mm^2/ms, v dimensionless.
 *    chi_m*C_m = 1; the monodomain factor lambda/(1+lambda) is folded into
 *    the conductivities the caller passes.
 *  - Host pointers are borrowed for the duration of a call and copied.
 *    Device memory belongs to the grid.
 *  - A handle is not thread-safe; distinct handles may run concurrently on
 *    distinct streams.  All work of a handle is ordered on its stream.
 */
#ifndef EP_H_
#define EP_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EP_API __attribute__((visibility("default")))

typedef struct ep_grid_s* ep_grid;

typedef enum {
  EP_OK = 0,
  EP_ERR_ARG = 1,         /* invalid argument: sizes, NULL, non-unit fibre,
                             negative conductivity, unstable explicit dt, ... */
  EP_ERR_OOM = 2,         /* device allocation failed */
  EP_ERR_HIP = 3,         /* a HIP runtime call failed */
  EP_ERR_NOCONV = 4,      /* a CG / refinement solve hit its iteration limit;
                             the state was still advanced with the last iterate */
  EP_ERR_NONFINITE = 5,   /* a non-finite potential appeared; sticky until
                             ep_write_state */
  EP_ERR_STATE = 6,       /* call out of order (e.g. ep_step before
                             ep_set_conductivity_fibres) */
  EP_ERR_UNSUPPORTED = 7  /* combination not implemented */
} ep_status;

typedef enum { EP_F64 = 0, EP_F32 = 1 } ep_prec;       /* bulk state + stencil */
typedef enum { EP_MONO = 0, EP_BIDO = 1 } ep_model;
/* Monodomain diffusion: explicit Euler; implicit Euler by Jacobi-PCG to
 * pcg_rtol; or implicit Euler by the thesis's own fixed number of Jacobi
 * sweeps from the current potential (Linear Solver section, "Implicit
 * Euler", eqn:iejac1), jacobi_sweeps per step, with no stopping test.
 * EP_DIFF_EXPLICIT27: explicit Euler with the thesis's own corner-gradient
 * operator (Matrix-Free Assembly section, eqn:ass1 - eqn:ass3, with the
 * conductivity block of the Algorithm Details chapter's Diffusion
 * subsection): gradients at the 8 corners of each voxel from the 2x2x2
 * blocks meeting there, the corner tensor the mean of the block's 8 voxel
 * tensors, fluxes averaged to the face midpoints and summed through the
 * faces; a corner whose block holds non-tissue carries no flux.  It reads
 * the same 3x3x3 neighbourhood and the same 24 B (FP32) of coefficients
 * per voxel as the 19-point operator, is symmetric and negative
 * semidefinite, but has hourglass null modes ((-1)^(i+j), (-1)^(i+k),
 * (-1)^(j+k), (-1)^(i+j+k)), so it is offered for the explicit monodomain
 * step only (not for the implicit solvers, the bidomain, the adjoint or
 * batched serving).  ep_set_conductivity_fibres rejects dt unless
 * dt * 4 max_p(s_p) max(sigma_l, sigma_t) / h^2 < 2, a bound on
 * dt * lambda_max(-A27) that uniform tissue nearly reaches. */
typedef enum {
  EP_DIFF_EXPLICIT = 0,
  EP_DIFF_BE_PCG = 1,
  EP_DIFF_BE_JACOBI = 2,
  EP_DIFF_EXPLICIT27 = 3
} ep_diff;
typedef enum { EP_V = 0, EP_W = 1, EP_PHIE = 2, EP_TACT = 3 } ep_field;

/* Mitchell-Schaeffer constants (eqn:ms1, eqn:ms2).  exc multiplies J_in
 * (ionic excitability).  Above v_gate the gate relaxes as -w/tau_close. */
typedef struct {
  double tau_in, tau_out, tau_open, tau_close, v_gate, exc;
} ep_ionic;

/* Stimulus current amp (1/ms) added to dv/dt (J_stim of eqn:ms1) on tissue
 * voxels p with lo <= p < hi per axis and, when radius > 0, whose centre
 * ((p + 0.5) h, mm) lies within radius of center: dx*dx + dy*dy + dz*dz <=
 * radius*radius evaluated in FP64 in that order.  Active at step n when
 * t_on <= n*dt < t_off (FP64). */
typedef struct {
  int32_t lo[3], hi[3];
  double center[3];
  double radius;
  double amp, t_on, t_off;
} ep_stim;

typedef struct {
  int32_t n[3];              /* voxels per axis, each >= 1 */
  double h;                  /* voxel width (mm), > 0 */
  const uint8_t* mask;       /* host, n0*n1*n2 box layout, nonzero = tissue;
                                NULL = all tissue */
  ep_model model;
  ep_prec prec;
  ep_diff diff;              /* monodomain diffusion; bidomain is explicit */
  double dt;                 /* ms, > 0 */
  ep_ionic ionic;
  const ep_stim* stim;       /* host array of n_stim entries (may be NULL if 0) */
  int32_t n_stim;
  double act_threshold;      /* activation threshold theta (0 < theta < 1) */
  double pcg_rtol;           /* implicit-Euler PCG: stop at ||r|| <= rtol ||b|| */
  int32_t pcg_maxit;
  int32_t jacobi_sweeps;     /* EP_DIFF_BE_JACOBI: sweeps per step (>= 1) */
  double ell_rtol;           /* bidomain elliptic refinement tolerance */
  int32_t ell_max_outer;     /* max refinement (outer) iterations */
  int32_t ell_inner_maxit;   /* max inner FP32 PCG iterations per outer */
  void* stream;              /* hipStream_t (e.g. a torch stream) or NULL for
                                the library's own stream */
  void* arena;               /* optional caller-owned device memory (e.g. a
                                torch tensor): when not NULL every device
                                array of the grid, the adjoint work block
                                included, is carved from it and nothing is
                                allocated; the caller keeps it alive until
                                ep_destroy_grid.  NULL: the grid allocates */
  int64_t arena_bytes;       /* size of arena; too small -> EP_ERR_OOM (a grid
                                created without an arena reports its size in
                                ep_grid_stats' device_bytes).  Ignored by
                                ep_batch_submit */
  const uint8_t* bath;       /* bidomain only (else EP_ERR_UNSUPPORTED): NULL,
                                or host n0*n1*n2 box layout, nonzero on
                                conducting body-tissue (bath / torso) voxels
                                around the heart (Bidomain Model subsection,
                                Boundary Conditions of eqn:bidomain1).  It
                                must not overlap mask (EP_ERR_ARG).  The
                                extracellular potential is then solved on
                                heart + bath with the operator
                                -(A_i + A_e): A_i the intracellular operator
                                on the heart only (no intracellular current
                                crosses the heart's boundary), A_e over heart
                                + bath with D_e on heart voxels and
                                sig_bath I on bath voxels, faces that
                                straddle the two taking the mean of their
                                tensors (phi and the extracellular normal
                                current are continuous across the heart's
                                boundary; no current leaves heart + bath).
                                v, w and T_act live on the heart only.
                                Heart + bath must be one face-connected
                                component; the gauge is sum phi = 0 over it */
  double sig_bath;           /* bath conductivity (mm^2/ms), > 0 with a bath */
  int32_t ell_precond;       /* bidomain inner-solve preconditioner: 0 (default)
                                Jacobi plus the coarse correction over
                                aggregates of 8x8x8 bricks, whose dense
                                inverse is kept in FP16; 1 Jacobi only (no
                                coarse inverse is built).  If an inner
                                solve breaks down ((r, M r) or the step's
                                curvature not positive: the rounded
                                preconditioner is not positive definite on
                                this grid), the grid drops the coarse
                                correction for good, repeats that pass with
                                Jacobi alone and reports precond 1 in
                                ep_solve_info.  Other values: EP_ERR_ARG */
  int32_t persistent_blocks; /* cap on the workgroups of the persistent CG
                                launches (implicit-Euler PCG, elliptic
                                inner solve), a positive multiple of 8 (one
                                share per XCD), e.g. to leave compute units
                                to other work on the GPU; each block then
                                walks more bricks.  0: as many as stay
                                resident (512 or 768 on MI355X).  Other
                                values: EP_ERR_ARG */
  int32_t steps_per_launch;  /* EP_MONO + EP_DIFF_EXPLICIT on a grid of at
                                most 128 8x8x8 bricks (ep_grid_stats'
                                n_bricks; beyond that one launch per step is
                                faster) whose bricks all fit on the device at
                                once: a stretch of steps under one stimulus
                                state runs in one cooperative launch (v*
                                exchanged through global memory, one
                                grid-wide barrier per step), with bitwise the
                                results of one launch per step.  0
                                (default): at most 4096 steps per launch; 1:
                                one launch per step; k > 1: at most k steps
                                per launch.  Ignored by other grids and by
                                ep_batch_submit.  Negative: EP_ERR_ARG */
} ep_grid_desc;

typedef struct {
  int64_t steps;             /* steps advanced by the call */
  int64_t step;              /* global step counter after the call */
  double t;                  /* step * dt (ms) */
  int64_t cg_iters;          /* PCG / inner iterations over the call */
  int32_t cg_max;            /* largest iteration count of one solve */
  int32_t ell_outer;         /* refinement iterations over the call */
  double q_stim;             /* injected charge dt*h^3*sum J_stim over the call (FP64) */
  double mass;               /* h^3 * sum over tissue of v after the call (FP64) */
  double relres;             /* last relative residual of a solve */
} ep_step_info;

typedef struct {
  int32_t outer;             /* refinement iterations */
  int64_t inner_iters;       /* FP32 PCG iterations in total */
  double relres;             /* final ||b - K phi|| / ||b|| in FP64 */
  int32_t precond;           /* inner preconditioner in use after the call
                                (0: Jacobi + coarse correction, 1: Jacobi) */
} ep_solve_info;

/* Create a grid.  Validates the description, builds the brick map of the
 * tissue mask (at most 2^29 voxels in the 8x8x8 bricks holding tissue, else
 * EP_ERR_UNSUPPORTED) (voxel geometry as in the Geometry section: tissue voxels are
 * the volume pass of the SDF encoding), allocates device state (v = 0,
 * w = 1 on tissue, phi = 0, T_act = +inf) and copies stimuli.  On failure
 * *out is NULL.  Errors: EP_ERR_ARG (bad sizes/values, NULL desc or out,
 * no tissue, bidomain tissue not one face-connected component),
 * EP_ERR_OOM, EP_ERR_HIP. */
EP_API ep_status ep_create_grid(const ep_grid_desc* d, ep_grid* out);

/* Set the conductivity from a unit fibre field (eqn:sigma1):
 *   D_p = s_p * (sig_t I + (sig_l - sig_t) f_p f_p^T),
 * fibre: host FP64, 3 per voxel, box layout; must be unit (| |f| - 1 | <=
 * 1e-6) on tissue.  scale: host FP64 per voxel (> 0 on tissue) or NULL for 1.
 * sig_el, sig_et: extracellular pair for EP_BIDO (ignored for EP_MONO).
 * Builds the face / edge coefficients of the 19-point operator on the
 * device (face tensor = mean of the two voxel tensors, edge tensor = mean
 * of the four voxel tensors of the 2x2 block; terms touching non-tissue are
 * dropped: no-flux) and the Jacobi diagonal.  For explicit diffusion it
 * checks dt * lambda_max(-A) < 2 (EP_ERR_ARG otherwise).
 * Errors: EP_ERR_ARG, EP_ERR_HIP. */
EP_API ep_status ep_set_conductivity_fibres(ep_grid g, const double* fibre,
                                            const double* scale, double sig_l,
                                            double sig_t, double sig_el,
                                            double sig_et);

/* ep_set_conductivity_fibres for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops such as a parameter
 * sweep that resets the scale field between runs, harnesses that forbid
 * hipMalloc).  Same arguments, result and errors as
 * ep_set_conductivity_fibres, bit for bit, but the call's device
 * temporaries (fibres and scale in brick layout, voxel tensors, FP64
 * weight scratch, the power-iteration vectors of the explicit stability
 * check and, for EP_BIDO, the coarse operator's set-up) are carved from one
 * fixed scratch array the library holds per GPU (64 MiB, held from the first
 * such call on a device until the process ends) instead of being allocated:
 * no hipMalloc, hipFree or other allocating routine is called.  A grid
 * whose set-up needs more than the scratch holds (about 128 bytes per
 * padded voxel with an FP64 weight copy, so up to ~0.5M padded voxels; plus
 * the dense coarse operator for EP_BIDO) is refused with EP_ERR_ARG before
 * anything runs.  Every call on one GPU shares that GPU's scratch: calls
 * that overlap on one GPU (from several threads, on any grids) race; calls
 * in sequence are safe (the call synchronises the grid's stream before it
 * returns, and clears what must start at zero). */
EP_API ep_status ep_set_conductivity_fibres_noalloc(ep_grid g, const double* fibre,
                                                    const double* scale, double sig_l,
                                                    double sig_t, double sig_el,
                                                    double sig_et);

/* Advance nsteps operator-split steps (reaction, then diffusion; bidomain:
 * reaction, elliptic solve for phi_e from v*, parabolic update).  Activation
 * times are recorded at the first step with v_n < theta <= v_{n+1}, linearly
 * interpolated.  info may be NULL.  Synchronises the stream once at the end.
 * Errors: EP_ERR_STATE (no conductivity yet), EP_ERR_NONFINITE,
 * EP_ERR_NOCONV (state still advanced), EP_ERR_HIP. */
EP_API ep_status ep_step(ep_grid g, int32_t nsteps, ep_step_info* info);

/* Solve the bidomain elliptic equation -(A_i + A_e) phi = A_i v for the
 * current v (second line of eqn:bidomain1, no-flux on the domain's
 * boundary): on the heart, gauge sum_tissue phi = 0; with a bath, on heart
 * + bath as described at ep_grid_desc.bath, gauge sum phi = 0 over both.
 * FP32 PCG inner solves (Jacobi plus an aggregate coarse correction) inside
 * FP64 iterative refinement until ||b - K phi|| <= rel_tol ||b|| (FP64),
 * warm-started from the stored phi.  EP_BIDO grids only
 * (EP_ERR_UNSUPPORTED otherwise); EP_ERR_NOCONV when max_outer refinement
 * iterations do not reach rel_tol (phi holds the last iterate). */
EP_API ep_status ep_solve_elliptic(ep_grid g, double rel_tol, int32_t max_outer,
                                   ep_solve_info* info);

/* Gradient of an activation-time misfit with respect to the per-voxel
 * conductivity scale s (the `scale` of ep_set_conductivity_fibres, D = s D0),
 * by the discrete adjoint of the explicit monodomain step.  The thesis offers
 * the simulation as the objective function of parameter estimation and
 * patient fitting (Abstract; Cardiac Simulation chapter, Results,
 * "Electrophysiology"); this call differentiates that objective:
 *   L = sum over tissue voxels activated during the run with a finite
 *       target of (T_act - T*)^2,
 * T_act as ep_step records it (first crossing of act_threshold, linear
 * interpolation inside the step).
 *  - Runs nsteps explicit steps from the current state, with T_act reset to
 *    +inf at the start; the grid ends in the run's final state (v, w, T_act,
 *    step), as ep_step would leave it.
 *  - tstar: host, box layout, n0*n1*n2 entries in ms; non-finite = no target.
 *  - grad: host output, box layout, dL/ds per voxel (0 off tissue), in the
 *    state precision of the grid, accumulated in FP64; NULL computes the
 *    loss only (the forward run, no checkpoints and no backward pass).
 *  - loss, n_used: L and the number of voxels in the sum.
 *  - ckpt_every K >= 1: the forward run keeps (v, w) every K steps; the
 *    backward pass recomputes one K-step segment at a time.  Device memory:
 *    about (3 ceil(nsteps / K) + 2 K + 7) state-precision fields of the
 *    padded grid.  K = 0 picks K = round(sqrt(1.5 nsteps)).
 *  - The gate-switch derivative at v = v_gate (a Dirac) is dropped: the
 *    gradient is that of the piecewise-smooth map with the branch held.
 * Errors: EP_ERR_UNSUPPORTED (not explicit monodomain), EP_ERR_STATE (no
 * conductivity), EP_ERR_ARG (NULL tstar / loss / n_used, nsteps < 1,
 * ckpt_every < 0), EP_ERR_OOM
 * (work block does not fit), EP_ERR_NONFINITE, EP_ERR_HIP. */
EP_API ep_status ep_adjoint_scale(ep_grid g, int32_t nsteps, int32_t ckpt_every,
                                  const double* tstar, double* loss, double* grad,
                                  int64_t* n_used);

/* Copy a field to host FP64 in box layout (n0*n1*n2 entries); non-tissue
 * voxels read 0 (v, w, phi) or +inf (T_act).  With a bath, phi is read
 * (and written by ep_write_state) on heart + bath.  Synchronises the stream.
 * Errors: EP_ERR_ARG (NULL, n too small, bad field), EP_ERR_HIP. */
EP_API ep_status ep_read_state(ep_grid g, ep_field f, double* host_out, size_t n);

/* Copy a field into caller-owned device memory in box layout (n0*n1*n2
 * entries, z fastest) as FP64 (dtype 0) or FP32 (dtype 1); non-tissue
 * voxels read 0 (v, w, phi) or +inf (T_act).  The state stays on the GPU:
 * the thesis keeps all allocation and arithmetic on the device and moves
 * buffers only to produce output (GPU Computation chapter, PCI Bus
 * subsection); this hands a field to device-side consumers (e.g. a torch
 * tensor) without the host round trip.  dptr must be device memory of this
 * GPU holding n0*n1*n2 elements of the dtype; it is borrowed for the call.
 * The copy is enqueued on the grid's stream and the call returns without
 * waiting: order later reads after that stream (or create the grid on the
 * consumer's stream).  Errors: EP_ERR_ARG (NULL, bad field or dtype),
 * EP_ERR_HIP. */
EP_API ep_status ep_read_state_device(ep_grid g, ep_field f, void* dptr, int32_t dtype);

/* The six limb leads of the electrocardiogram from the extracellular
 * potential (Cardiac Simulation chapter, Results, ECG subsection): with
 * RA, LA, LL the potential at the right-arm, left-arm and left-leg
 * electrodes, out[0..5] = I = LA - RA, II = LL - RA, III = LL - LA,
 * aVR = RA - (LA + LL)/2, aVL = LA - (RA + LL)/2, aVF = LL - (RA + LA)/2.
 * electrodes: host, 9 int32, the (x, y, z) voxel of RA, LA, LL; each must
 * lie in the elliptic domain (heart, or bath with one).  phi is the one the
 * last ep_step (or ep_solve_elliptic) left.  Synchronises the grid's
 * stream.  Errors: EP_ERR_ARG (NULL, electrode outside the box or the
 * domain), EP_ERR_UNSUPPORTED (monodomain grid), EP_ERR_HIP. */
EP_API ep_status ep_ecg_leads(ep_grid g, const int32_t* electrodes, double* out);

/* Overwrite a field from host FP64 in box layout; values at non-tissue
 * voxels are ignored.  Clears the sticky non-finite flag.  For EP_TACT,
 * +inf marks "not yet activated". */
EP_API ep_status ep_write_state(ep_grid g, ep_field f, const double* host_in, size_t n);

/* Global step counter (t_n = step * dt); settable to restart a run. */
EP_API ep_status ep_get_step(ep_grid g, int64_t* step);
EP_API ep_status ep_set_step(ep_grid g, int64_t step);

/* Counts: tissue voxels, active 8x8x8 bricks, and device_bytes: the most
 * device memory the grid has held at once, the temporaries of earlier calls
 * (conductivity encoding, adjoint work block) included -- an arena of that
 * size serves the same sequence of calls. */
EP_API ep_status ep_grid_stats(ep_grid g, int64_t* n_tissue, int64_t* n_bricks,
                               int64_t* device_bytes);

/* Kernel timing for measurement: `enable` is a bit mask of kernel ids
 * (bit k times kernel id k; -1 times all, 0 none).  The library records HIP
 * events on the grid's stream around every launch of the selected kernels;
 * ep_kernel_time returns the summed milliseconds and the launch count since
 * the last ep_kernel_timing call.  Events between launches cost time, so
 * timing only the kernel of interest disturbs a run least.  kernel_id 0: the
 * fused explicit step, one implicit-Euler PCG iteration (x / r update, new
 * direction and operator apply in one launch), or the apply launch of an
 * elliptic inner iteration (z = M^-1 r, w = K z); 1: the first launch of an
 * implicit-Euler PCG solve (p0 = z0, q0 = K p0); 2: the bidomain parabolic
 * stencil; 3: the FP64 elliptic residual; 4: launches that only found the
 * solve done (recorded under a timed id 0 or 1 and moved here); 5: the
 * adjoint step of ep_adjoint_scale (its forward and recompute launches count
 * as 0); 6: the reaction + initial-residual launch of an implicit-Euler
 * step; 7: the implicit-Euler solve's last launch, which only applies the
 * last x update, or the update launch of an elliptic inner iteration (x, r,
 * p, s and the brick sums of r); 8: the coarse correction of an elliptic
 * inner iteration (aggregate sums and the GEMV with the coarse inverse);
 * 9: a multi-step explicit launch (several steps, see steps_per_launch;
 * explicit steps that run one per launch count under 0). */
EP_API ep_status ep_kernel_timing(ep_grid g, int32_t enable);
/* Time only the launches of the steps whose index (ep_get_step) is a
 * multiple of `steps` (1, the default: every step), so that a long run can
 * be timed on a sample of its steps without an event pair around every
 * launch (each pair delays the launch that follows by several us).  Kept
 * across ep_kernel_timing calls.  Errors: EP_ERR_ARG (steps < 1). */
EP_API ep_status ep_kernel_timing_period(ep_grid g, int32_t steps);
EP_API ep_status ep_kernel_time(ep_grid g, int32_t kernel_id, double* total_ms,
                                int64_t* launches);

/* Streaming-bandwidth probe for measurement: the practical HBM ceiling on
 * this GPU, taken with plain HIP kernels of the kind the stencil kernels
 * are (16-byte loads and stores per lane, a grid-stride loop, 8 blocks of
 * 256 threads per CU).  Allocates two buffers of `bytes` on the current
 * device (give well above the 256 MB last-level cache, e.g. 1 GiB), then
 * times a copy (bytes read + bytes written) and a read-only sum over one
 * buffer, each the fastest of `reps` runs after a warm-up, with HIP events
 * on a stream of its own; frees everything.  Outputs in GB/s (1e9 B/s).
 * Errors: EP_ERR_ARG (bytes < 1 MiB, reps < 1, NULL), EP_ERR_OOM,
 * EP_ERR_HIP. */
EP_API ep_status ep_stream_bandwidth(int64_t bytes, int32_t reps, double* copy_gbs,
                                     double* read_gbs);

EP_API ep_status ep_destroy_grid(ep_grid g);
EP_API const char* ep_status_string(ep_status s);
EP_API const char* ep_last_error(ep_grid g);

/* ---- batched serving ----------------------------------------------------
 * Many independent simulations (different grids, conductivities, ionic
 * parameters and step counts) advanced together on one GPU.  The thesis
 * proposes running many independent simulations in parallel (parameter
 * estimation, patient fitting) instead of splitting one across devices
 * (Abstract; Review & Outlook chapter, Assessment, "GPU Processing"); this
 * is that mode, as continuous batching:
 *  - ep_batch_submit queues a request (FP32, monodomain, explicit diffusion,
 *    all stimuli of a request sharing one time window); host data is copied.
 *  - ep_batch_advance admits queued requests in FIFO order while their
 *    device memory fits the HBM budget and a slot is free (their grids,
 *    coefficients and state are built on the device while the previous
 *    launch runs), then launches one captured graph of K steps in which every
 *    admitted request advances by up to K steps (a request never steps past
 *    its own count), and detects the requests that have finished.  Requests admitted later join running
 *    ones at the next graph boundary; their work shares each launch.
 *  - finished requests stay resident until ep_batch_release; read their
 *    fields with ep_batch_read (same layout and conventions as
 *    ep_read_state).
 * Each request's arithmetic is independent of the mix: a request gives the
 * same bits alone, in any mix and through ep_step on an EP_F32 grid.
 * Errors: EP_ERR_ARG (bad description / id), EP_ERR_UNSUPPORTED (model,
 * precision, scheme or stimulus windows outside this mode), EP_ERR_OOM (a
 * request larger than the whole budget), EP_ERR_HIP. */
typedef struct ep_batch_s* ep_batch;

typedef struct {
  int64_t hbm_budget;         /* device bytes for admitted requests (arena) */
  int32_t max_slots;          /* requests resident at once */
  int32_t steps_per_launch;   /* K, steps per graph launch (>= 1) */
  void* stream;               /* hipStream_t or NULL for the batch's own */
} ep_batch_desc;

typedef struct {
  int64_t submitted, admitted, finished, released;
  int32_t resident;           /* requests holding device memory */
  int32_t queued;
  int64_t arena_used, arena_peak;   /* bytes */
  int64_t graph_launches;
  double voxel_steps;         /* tissue voxel-steps advanced so far */
} ep_batch_stats;

EP_API ep_status ep_batch_create(const ep_batch_desc* d, ep_batch* out);
EP_API ep_status ep_batch_submit(ep_batch b, const ep_grid_desc* d, const double* fibre,
                                 const double* scale, double sig_l, double sig_t,
                                 int64_t n_steps, int64_t* id);
EP_API ep_status ep_batch_advance(ep_batch b, int32_t* n_finished);
EP_API ep_status ep_batch_finished(ep_batch b, int64_t* ids, int32_t cap, int32_t* n);
EP_API ep_status ep_batch_read(ep_batch b, int64_t id, ep_field f, double* host_out, size_t n);
EP_API ep_status ep_batch_release(ep_batch b, int64_t id);
EP_API ep_status ep_batch_get_stats(ep_batch b, ep_batch_stats* s);
EP_API ep_status ep_batch_destroy(ep_batch b);
EP_API const char* ep_batch_last_error(ep_batch b);

#ifdef __cplusplus
}
#endif
#endif /* EP_H_ */
