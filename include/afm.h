/*
 * afm.h -- C ABI of the MI355X tip-sample force inversion library (libafm.so).
 *
 * The library solves the two problems posed in Busch, Zou, Ganapathysubramanian, "A near
 * real-time framework for extracting tip-sample forces in dynamic atomic force microscopy"
 * (arXiv 1109.0334):
 *   FP (Sec. 2.2): given the cantilever, the base motion and a parameterised tip-sample force,
 *       compute the tip deflection -- here reduced to the steady-state lock-in amplitude and
 *       phase and to the misfit against a measured trace;
 *   IP (Sec. 2.3): given the measured deflection, find the force parameters, posed as the
 *       unconstrained minimisation of a misfit J (Eq. 5) and solved with particle swarm
 *       optimisation (Sec. 3.4, Eq. 8).
 *
 * Model (Eq. 1-2 reduced to tip-normalised modes):
 *   u = sum_i q_i,  d = z_c + u (tip-sample gap, u positive away from the sample),
 *   q_i'' + (w_i/Q_i) q_i' + w_i^2 q_i = F(d, d'; theta) / M + gamma_i a wd^2 sin(wd t),
 * M = k / w_0^2, base motion y_b = a sin(wd t) (Eq. 9) with a set so that the free tip amplitude
 * is A0.  Classical RK4 with N steps per drive period (Sec. 3.2), n_cycles periods.  Lock-in over
 * the last lockin_cycles periods: X = 2/W sum u cos(2 pi p/N), Y = 2/W sum u sin(2 pi p/N),
 * A = sqrt(X^2 + Y^2), phi = atan2(-X, Y) (u ~ A sin(wd t - phi)).  Misfit over the same window:
 * J = sum (U - u)^2 / sum U^2 (Eq. 5 on the steady-state window, normalised so that sqrt(J) is
 * the relative L2 error of Sec. 3.3).
 *
 * Conventions for every entry point:
 *   - SI units (m, s, N, Pa, J); phases in radians; J dimensionless.
 *   - Array arguments are device pointers owned by the caller (e.g. torch tensor storage),
 *     structure-of-arrays: a [D][n] array holds row j at offset j*n.
 *   - Calls are asynchronous on `stream` (a hipStream_t; NULL = the legacy default stream).
 *     Arguments are validated before anything is enqueued; an invalid call returns
 *     AFM_ERR_INVALID and launches nothing.  A HIP failure returns AFM_ERR_HIP.  The text of the
 *     last error of the calling thread is returned by afm_last_error().
 *   - A trajectory that becomes non-finite or exceeds |u| > div_limit * A0 at the end of a drive
 *     period is not an error: its status word gets AFM_ST_NONFINITE / AFM_ST_DIVERGED, its
 *     amplitude and phase are NaN and its misfit +inf.
 *   - A plan is not thread-safe: use one plan per host thread.  Its workspaces (gradient
 *     checkpoints, polish state, inversion swarms, the lane order of small batches) are reused
 *     by every call, so calls on one plan must be ordered: issue them on one stream, or
 *     synchronise between streams.
 */
#ifndef AFM_H
#define AFM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AFM_MAX_MODES 8
#define AFM_MAX_PARAMS 12

typedef void *afm_stream_t; /* a hipStream_t */

typedef enum {
    AFM_OK = 0,
    AFM_ERR_INVALID = 1,     /* bad argument; nothing was enqueued           */
    AFM_ERR_HIP = 2,         /* HIP runtime failure (launch, copy, capture)  */
    AFM_ERR_NOMEM = 3,       /* device or host allocation failed             */
    AFM_ERR_UNSUPPORTED = 4  /* valid request the library does not implement */
} afm_status;

/* Arithmetic of the forward solve. */
enum {
    AFM_PREC_MIXED = 0, /* FP32 state and RK4 (compensated update), FP64 lock-in and misfit sums */
    AFM_PREC_FP64 = 1   /* plain FP64 throughout: the per-particle baseline                      */
};

/* Tip-sample force laws F(d, d'), F > 0 repulsive.  params[] layouts (z_c always first):
 *   DMT   {z_c, H, E*, a0, R}: -H R/(6 d^2) for d > a0; -H R/(6 a0^2) + 4/3 E* sqrt(R)
 *         (a0 - d)^{3/2} for d <= a0 (Hertz contact with van der Waals adhesion; the paper names
 *         Hertz and van der Waals forces in Sec. 2.2 and adhesion as an extension in Sec. 5).
 *   LJ    {z_c, eps, r0, n, m}: eps n m/(n - m)/d [(r0/d)^n - (r0/d)^m] (Lennard-Jones type, well
 *         depth eps at d = r0); d <= 0 yields a non-finite trajectory.
 *   KV    {z_c, H, E*, a0, R, eta}: DMT plus -eta sqrt(R (a0 - d)) d' in contact (Kelvin-Voigt
 *         dissipation, the spring-damper of Eq. 4 / Eq. 12 applied to a Hertzian contact).
 *   HOOKE {z_c, k_s}: -k_s d for d < 0 (Eq. 3 / Eq. 11).
 *   SD    {z_c, k_s, zeta_s}: -k_s d - zeta_s d' for d < 0 (Eq. 4 / Eq. 12).
 *   NONE  {z_c}: no tip force (the linear driven cantilever).  z_c only offsets the gap: use 0
 *         (the mixed kernel carries mode 1 as the FP32 gap z_c + u, so a z_c far above the
 *         deflection costs its precision).                                                     */
enum { AFM_LAW_DMT = 0, AFM_LAW_LJ = 1, AFM_LAW_KV = 2, AFM_LAW_HOOKE = 3, AFM_LAW_SD = 4,
       AFM_LAW_NONE = 5 };

/* Base motion.  TABLE: the sinusoid of Eq. 9 at drive_freq with the amplitude a fixed by the
 * free amplitude A0 (the force inversions).  PARAMS: the chirp of Eq. 10 (Sec. 4.1),
 * y_b = a sin(2 pi (f + g t) t), with a (m), f (Hz) and g (Hz/s) in params[8], params[9] and
 * params[10] of each trajectory, so that they can be free parameters (the paper's base-motion
 * inversions; g = 0 is Eq. 9).  The RHS then carries -y_b'' = a (w^2 sin(phi) - 4 pi g cos(phi)),
 * phi = 2 pi (f + g t) t, w = 2 pi (f + 2 g t), evaluated per lane at every RK4 stage time
 * (FP64 phase reduced to one revolution, sine and cosine in the plan's precision); the time step
 * stays 1 / (drive_freq N) and the lock-in projects onto drive_freq.  PARAMS requires
 * ic = AFM_IC_REST (the free steady state of a chirp is not defined).  Launch shapes as for
 * TABLE (afm_set_launch_shape) without two trajectories per lane; with one lane per mode the
 * lanes of a trajectory split its drive evaluations between them.  The adjoint
 * (afm_grad_batch, afm_polish, the invert polish) differentiates a, f, g too, one lane per
 * trajectory. */
enum { AFM_DRIVE_TABLE = 0, AFM_DRIVE_PARAMS = 1 };
enum { AFM_P_BASE_A = 8, AFM_P_BASE_F = 9, AFM_P_BASE_G = 10 };

/* Initial state: FREE_STEADY = linear free steady state at t = 0 (q_i = Im(a H_i),
 * q_i' = wd Re(a H_i), H_i = gamma_i wd^2 / (w_i^2 - wd^2 + i w_i wd / Q_i)); REST = zero. */
enum { AFM_IC_FREE_STEADY = 0, AFM_IC_REST = 1 };

/* Per-trajectory status bits.  BAD_INPUT: the trajectory's target row is outside
 * [0, n_targets) or its period count is below lockin_cycles; it is not integrated. */
enum { AFM_ST_NONFINITE = 1, AFM_ST_DIVERGED = 2, AFM_ST_BAD_INPUT = 4 };

/* Problem description, copied by value into a plan (FP: Sec. 2.2; IP search box: Sec. 3.4). */
typedef struct afm_problem {
    int32_t n_modes;         /* 1 (point mass) .. 8 (the paper's beam), tip-normalised modes  */
    int32_t law;             /* AFM_LAW_*                                                     */
    int32_t steps_per_cycle; /* N, RK4 steps per drive period, 4 .. 4096                      */
    int32_t n_cycles;        /* drive periods integrated (default per trajectory)             */
    int32_t lockin_cycles;   /* periods at the end used for lock-in and misfit, >= 1          */
    int32_t ic;              /* AFM_IC_*                                                      */
    double k;                /* first-mode stiffness, N/m                                     */
    double f0;               /* first-mode natural frequency, Hz                              */
    double drive_freq;       /* base drive frequency, Hz                                      */
    double free_amplitude;   /* A0, m; fixes the base amplitude (TABLE), scales div_limit     */
    double div_limit;        /* divergence threshold in units of A0 (0 => 100)                */
    double q[AFM_MAX_MODES];     /* quality factor per mode                                   */
    double ratio[AFM_MAX_MODES]; /* w_i / w_0 (ratio[0] is normally 1)                        */
    double gain[AFM_MAX_MODES];  /* gamma_i, base-drive participation (1 for a point mass)    */
    double params[AFM_MAX_PARAMS];      /* full parameter vector, SI: the law's (slots 0 ..
                                           its count - 1), with PARAMS the base motion's in
                                           slots 8 .. 10; free entries are overwritten per
                                           trajectory by theta; other slots ignored          */
    int32_t n_free;                     /* D: free parameters, 0 .. law count (+ 3 with PARAMS) */
    int32_t free_index[AFM_MAX_PARAMS]; /* params[] slot of free parameter j (a law slot, or
                                           8 .. 10 with PARAMS)                              */
    double lo[AFM_MAX_PARAMS];          /* search box of free parameter j (SI)                */
    double hi[AFM_MAX_PARAMS];
    int32_t log_scale[AFM_MAX_PARAMS];  /* 1: theta = lo (hi/lo)^z, else lo + z (hi - lo)      */
    double pso_w, pso_c1, pso_c2, pso_vmax; /* Eq. 8 weights; 0 => 0.7298, 1.49618, 1.49618, 1 */
    int32_t polish_precision; /* arithmetic of afm_polish and the invert polish: AFM_POLISH_*   */
    int32_t drive_mode;       /* AFM_DRIVE_* (0 = TABLE)                                       */
    double steady_rtol;       /* > 0: adaptive steady-state exit (below); 0 = off              */
} afm_problem;

/* Adaptive steady-state exit (steady_rtol > 0; TABLE drive only): each trajectory integrates
 * period by period; at the end of every period before its window it takes the stroboscopic point
 * P = (u, u'/wd) -- deflection and rate at the same drive phase each time; |P| is the amplitude
 * of a steady sinusoid -- and ends its transient after the first period with
 * |P_c - P_{c-1}| < steady_rtol |P_c| (P_{-1}: the initial state); its lock-in window is then the
 * following lockin_cycles periods.  The period count (problem or per trajectory) stays the cap:
 * without such a period the window is its last lockin_cycles periods, as without the exit.
 * Applies to every forward solve (afm_forward_batch, afm_misfit, afm_forward_points, afm_invert;
 * one trajectory per lane; work-queue batches of afm_invert refill each lane with the next
 * trajectory as its own ends); afm_forward_steady reports the periods each trajectory
 * integrated.  The adjoint is not built for it (afm_grad_batch, afm_polish and the invert polish
 * return AFM_ERR_UNSUPPORTED). */

/* Polish arithmetic: the plan's own precision, or FP32 (mixed) / FP64 adjoint and misfits. */
enum { AFM_POLISH_PLAN = 0, AFM_POLISH_MIXED = 1, AFM_POLISH_FP64 = 2 };

typedef struct afm_plan afm_plan; /* opaque: constants, drive/lock-in tables, workspace */

/* Swarm state, caller-owned device arrays in normalised coordinates z in [0,1]^D for S swarms
 * of P particles (particle g = s*P + p).  theta receives the SI parameters of the positions. */
typedef struct afm_swarm {
    int32_t n_dim, particles, swarms;
    double *z, *v, *pbest_z; /* [D][S*P] */
    double *pbest_J;         /* [S*P]    */
    double *gbest_z;         /* [D][S]   */
    double *gbest_J;         /* [S]      */
    int32_t *gen_to_cutoff;  /* [S]: first generation with sqrt(gbest_J) <= cutoff, or -1   */
    double *theta;           /* [D][S*P]: SI parameters of z (written by init and step)      */
} afm_swarm;

/* Build a plan (the set-up of the FP, Sec. 2.2 and Sec. 3.2): validates the problem, derives
 * the base amplitude a of Eq. 9 from the free amplitude A0 (the linear, damped steady response
 * of Eq. 2 without tip force, summed over the modes at the tip), the initial state, and the
 * non-dimensional constants of Eq. 2 (time in drive radians, lengths in nm, modes from Eq. 6-7
 * and App. B), and uploads the drive and lock-in tables (the base forcing at each RK4 stage and
 * the sin/cos weights, Sec. 3.2).  precision:
 * AFM_PREC_*.  Allocates device memory owned by the plan.  *out is NULL on failure; the message
 * from afm_last_error names the invalid field. */
afm_status afm_plan_create(const afm_problem *problem, int32_t precision, afm_plan **out);

/* Release a plan and its device memory (synchronises the plan's private stream).  NULL is OK. */
afm_status afm_plan_destroy(afm_plan *plan);

/* Launch shape of the plain forward kernel (afm_forward_batch, afm_misfit, the swarm
 * evaluations of afm_invert without per-swarm period counts -- with them too for a
 * parameter-driven base --, polish line searches).  By default
 * (block = 0) it is autotuned per precision, batch size and period-count mode: the first call
 * with a new combination runs the launch once per candidate -- workgroups of 64, 128 or 256
 * lanes, times one trajectory per lane, two trajectories per lane (point-mass problems with the
 * fixed drive and without per-trajectory period counts) or one lane per mode (problems with
 * several modes: 2 lanes per trajectory for 2 modes, 4 for 3 or 4, 8 for 5 to 8; the paper's mapping
 * of modes to threads, Sec. 3.2) --
 * times each with events and keeps the default shape unless another is at least 2 % faster;
 * that call synchronises the stream.  Under stream
 * capture nothing is timed and the default shape is used (64 lanes below 65536 trajectories,
 * else 256; one lane per mode for several modes and at most 16384 trajectories, else one
 * trajectory per lane).  afm_invert tunes before it captures.  Every shape computes
 * bit-identical results.  DMT and Kelvin-Voigt batches below 65536 trajectories (one lane per
 * trajectory or per mode) run a time loop that leaves the contact force out of four-step blocks
 * no lane of a wave can reach contact in; for point-mass batches of 65 to 16384 trajectories
 * their assignment to lanes follows the contact stiffness E* sqrt(R) (ranked on the device
 * before each launch, in plan-owned buffers), which groups similar trajectories in a wave;
 * neither changes any result.  Batches of 65536 or more skip the
 * contact piece per RK4 stage where no lane of a wave is near contact (FP32 point-mass DMT: the
 * same bits as smaller batches) or branch per lane (FP64, and the KV law), which rounds the
 * frozen attraction at d = a0 once ahead: those agree with a smaller batch's to rounding, not
 * bit for bit.
 * block in {64, 128, 256} and tpl in {1, 2, 0} (0 = one lane per mode) pin the shape for this
 * plan (a tpl that does not apply falls back to 1); block = 0 returns to tuning.  Anything
 * else: AFM_ERR_INVALID. */
afm_status afm_set_launch_shape(afm_plan *plan, int32_t block, int32_t tpl);

/* FP for n parameter points.  theta: [n_free][n] SI values of the free parameters (device).
 * n_cycles: [n] per-trajectory period counts, or NULL for the problem's n_cycles (each must be
 * >= lockin_cycles).  Outputs (device): amp [n] in m, phase [n] in rad, status [n]; trace, if
 * not NULL, [n][W] FP64 window deflection in m, W = lockin_cycles * steps_per_cycle. */
afm_status afm_forward_batch(afm_plan *plan, int64_t n, const double *theta,
                             const int32_t *n_cycles, double *amp, double *phase, double *trace,
                             int32_t *status, afm_stream_t stream);

/* afm_forward_batch that also writes periods [n] (device): the drive periods each trajectory
 * integrated -- transient plus window with the adaptive steady-state exit, the period count
 * without it, the periods up to a failure, 0 for a bad input.  periods is required. */
afm_status afm_forward_steady(afm_plan *plan, int64_t n, const double *theta,
                              const int32_t *n_cycles, double *amp, double *phase, double *trace,
                              int32_t *status, int32_t *periods, afm_stream_t stream);

/* Deflection at points along the beam for n parameter points (the paper's deflection points,
 * n_dp, Sec. 3.2): u(x_k, t) = sum_i w[k][i] q_i(t) over the tip-normalised modal coordinates
 * q_i (App. B, Eq. 13), with weights (host, [n_points][n_modes]) w[k][i] = Phi_i(x_k) / Phi_i(L)
 * (afm_beam_shapes gives them for a uniform cantilever; all ones is the tip).  1 <= n_points
 * <= 16.  theta, n_cycles as in afm_forward_batch.  Outputs (device): amp, phase [n_points][n]
 * -- each point's lock-in amplitude (m) and phase over the window --, trace [n_points][n][W]
 * (m) or NULL, status [n]; failed trajectories give NaN.  The forward solve is afm_forward_batch's
 * (same launch shapes and bits); the window's modal coordinates go through a plan-owned
 * workspace of n_modes x W x 8 bytes per trajectory, at most 1 GiB (larger batches run in
 * chunks), grown on demand. */
afm_status afm_forward_points(afm_plan *plan, int64_t n, const double *theta,
                              const int32_t *n_cycles, int32_t n_points, const double *weights,
                              double *amp, double *phase, double *trace, int32_t *status,
                              afm_stream_t stream);

/* Misfit J (Eq. 5 on the lock-in window, normalised) of n parameter points against measured
 * traces.  targets: [n_targets][W] FP64 deflections in m on the window samples (the states after
 * steps N_tot - W + 1 .. N_tot); target_id: [n] row of targets per point, or NULL for row 0
 * (rows outside [0, n_targets) give status AFM_ST_BAD_INPUT).
 * Outputs (device): J [n] (+inf for failed trajectories), status [n]. */
afm_status afm_misfit(afm_plan *plan, int64_t n, const double *theta, const int32_t *n_cycles,
                      const int32_t *target_id, const double *targets, int32_t n_targets,
                      double *J, int32_t *status, afm_stream_t stream);

/* Misfits of S swarms of P points each (one PSO generation's forward solves of afm_invert,
 * without the swarm update): point g = s * P + p, theta [n_free][S * P] (device, SI), is solved
 * with swarm s's parameter vector (swarm_params [AFM_MAX_PARAMS][S], device, free entries
 * ignored, or NULL for the problem's), swarm s's period count (n_cycles [S], device, or NULL for
 * the problem's) and compared with target row s (targets [S][W], device).  Outputs (device):
 * J [S * P] (Eq. 5 on the lock-in window, normalised; +inf on failure), status [S * P].  With
 * period counts the launch is afm_invert's persistent work queue: 64-point chunks of the swarms,
 * longest period count first, taken by the waves of a grid sized to the device.  The order is
 * built on the first call for an n_cycles buffer (a synchronous read of the counts) and reused
 * while the same buffer, S and P come back (the order only balances the load: the results never
 * depend on it, so a buffer refilled with other counts still gives exact results).  Within each
 * swarm the points go to lanes in the order of the force law's contact stiffness (DMT,
 * Kelvin-Voigt), ranked on the device before every launch; every point's result is the same
 * whichever lane computes it.  The queue order, counter and lane order live in a plan-owned workspace
 * (4 (S ceil(P / 64) + 64) + 12 S P bytes).  Without period counts: afm_misfit's tuned plain
 * launch. */
afm_status afm_misfit_swarms(afm_plan *plan, int32_t n_swarms, int32_t particles,
                             const double *theta, const int32_t *n_cycles,
                             const double *swarm_params, const double *targets, double *J,
                             int32_t *status, afm_stream_t stream);

/* Misfit and its exact gradient with respect to the free parameters for n points: the
 * derivative of the forward kernel's discrete RK4 trajectory (Sec. 3.2) and window misfit
 * (Eq. 5) -- an addition beyond the paper, whose inversion is gradient-free (Sec. 3.4); it
 * serves the local refinement after the swarm (afm_polish).  Same arithmetic precision as the
 * plan, with the state checkpointed every ckpt_stride RK4 steps.  Two forms:
 *   SWEEP     the discrete adjoint: per trajectory, each segment recomputed from its checkpoint
 *             and walked backwards through the transposed stage Jacobians (stages reversed);
 *             the result is independent of the stride bit for bit;
 *   SEGMENTS  every (trajectory, segment) pair on its own lane: the segment recomputed from its
 *             checkpoint with its state and parameter tangents carried forward through the same
 *             stages, then a backward recursion over the segments per trajectory (the adjoint
 *             recursion is linear, so the segments combine exactly); the same derivative up to
 *             rounding, with thousands of times more lanes in flight.  Built for the drive table
 *             and up to 4 modes.
 * Arguments as afm_misfit; per-trajectory n_cycles must not exceed the problem's n_cycles.
 * Outputs (device): J [n], dJ [n_free][n] = dJ/dtheta_j in 1/(SI unit of parameter j), status.
 * ckpt_stride: RK4 steps between checkpoints, or 0 = autotuned (the first call with a new n
 * times the strides 16, 64 and 256 with every allowed form -- for SWEEP with several modes one
 * lane per trajectory and one lane per mode -- and keeps the fastest; that call synchronises the
 * stream).  With an explicit stride the form is the one tuned for this n, else SEGMENTS where
 * built, else SWEEP (afm_set_grad_form pins it).  J is afm_misfit's bit for bit in every form.
 * Workspace (checkpoints, segment buffer or segment records: about
 * n x (n_cycles N / stride) x (2 m + c + 1)(2 m + 1) x 8 bytes for SEGMENTS with m modes and a law
 * of c constants) is owned by the plan and grown on demand. */
afm_status afm_grad_batch(afm_plan *plan, int64_t n, const double *theta, const int32_t *n_cycles,
                          const int32_t *target_id, const double *targets, int32_t n_targets,
                          double *J, double *dJ, int32_t ckpt_stride, int32_t *status,
                          afm_stream_t stream);

/* Form of the gradient launches of a plan (afm_grad_batch, afm_grad_batch_noalloc, afm_polish,
 * the invert polish): AUTO (tuned by afm_grad_batch; SEGMENTS where built otherwise), SWEEP, or
 * SEGMENTS (AFM_ERR_UNSUPPORTED for a parameter-driven base or more than 4 modes).  Clears the
 * plan's tuned gradient settings. */
enum { AFM_GRAD_AUTO = 0, AFM_GRAD_SWEEP = 1, AFM_GRAD_SEGMENTS = 2 };
afm_status afm_set_grad_form(afm_plan *plan, int32_t form);

/* afm_grad_batch for callers that cannot allocate device memory (code captured into a HIP graph,
 * tight serving loops, harnesses that forbid allocation): the same kernels, the same results bit
 * for bit, but the checkpoints and the segment buffer live in a fixed library-owned device array
 * of AFM_NOALLOC_SCRATCH_BYTES per device (held from the first call on a device until the process
 * ends) instead of the plan's workspace.  The call allocates nothing and does not synchronise.
 * ckpt_stride: as afm_grad_batch, except that 0 takes the stride afm_grad_batch tuned for this n
 * on this plan, else 256 (no timing is done here); the form is afm_grad_batch's for the same n
 * and stride.  AFM_ERR_INVALID, with nothing enqueued, when the checkpoints,
 * (n_cycles * steps_per_cycle / stride) x 4 x n_modes x n values (FP32 for a mixed plan, FP64
 * otherwise), plus the segment buffer (SWEEP: stride x (2 n_modes + 1) x n values) or segment
 * records (SEGMENTS, as afm_grad_batch states) need more than AFM_NOALLOC_SCRATCH_BYTES, or when
 * the current device is not the plan's.  Every
 * call on one device shares that device's array: calls that overlap in time on one device (other
 * streams, other threads, other plans) race, so order them.  Other arguments and outputs as
 * afm_grad_batch. */
#define AFM_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
afm_status afm_grad_batch_noalloc(afm_plan *plan, int64_t n, const double *theta,
                                  const int32_t *n_cycles, const int32_t *target_id,
                                  const double *targets, int32_t n_targets, double *J,
                                  double *dJ, int32_t ckpt_stride, int32_t *status,
                                  afm_stream_t stream);

/* Initialise a swarm (Sec. 3.4): z, v drawn uniformly over the search box (z ~ U[0,1),
 * v = U[0,1) - z), pbest_z = z, pbest_J = gbest_J = +inf, gen_to_cutoff = -1, theta = SI of z.
 * Random numbers: Philox4x32-10 with key (low 32 bits of seed, swarm) and counter
 * (0, particle, dim << 8 | purpose, high 32 bits of seed), purpose 1 for z, 2 for v; the
 * uniform is ((x0 >> 5) 2^26 + (x1 >> 6)) 2^-53. */
afm_status afm_swarm_init(afm_plan *plan, afm_swarm *swarm, uint64_t seed, afm_stream_t stream);

/* One PSO generation given J [S*P] of the current positions: personal bests (strict <,
 * non-finite J never becomes a best), swarm best (lowest pbest_J, ties to the lowest index),
 * gen_to_cutoff, and -- unless is_last -- the Eq. 8 move v = w v + c1 r1 (pbest - z)
 * + c2 r2 (gbest - z) with r1, r2 from counter (iter, particle, dim << 8 | 0, seed_hi), v
 * clamped to [-vmax, vmax], z = z + v, a coordinate leaving [0,1] is clamped with v = 0; theta
 * is refreshed.  FP64, evaluated in a fixed order without contraction (bit-reproducible). */
afm_status afm_pso_step(afm_plan *plan, afm_swarm *swarm, const double *J, uint64_t seed,
                        int32_t iter, int32_t is_last, double cutoff, afm_stream_t stream);

/* Polish n parameter points with projected L-BFGS on the discrete-adjoint gradient (an
 * addition beyond the paper's gradient-free inversion of Sec. 3.4: it minimises the same
 * misfit, Eq. 5, from the swarm's best points, in the same search box), in the normalised
 * coordinates of the problem's search box: history 5, H0 = s'y / y'y, trial steps
 * 2^-k (k = 0..20) of the direction evaluated together, the first satisfying Armijo (c = 1e-4)
 * accepted, a pair dropped when s'y <= 1e-12 |s||y|; a point with no acceptable step stops.
 * z: [n_free][n] normalised positions (device, in/out); params: [AFM_MAX_PARAMS][n] full
 * parameter vectors of the points (their free entries are ignored) or NULL for the problem's;
 * n_cycles, target_id, targets, n_targets as in afm_misfit; J: [n] misfit at the returned
 * positions (device).  Workspace is owned by the plan.  Enqueues a fixed sequence of launches
 * (no host synchronisation). */
afm_status afm_polish(afm_plan *plan, int64_t n, double *z, const double *params,
                      const int32_t *n_cycles, const int32_t *target_id, const double *targets,
                      int32_t n_targets, int32_t steps, double *J, afm_stream_t stream);

/* Whole inversions (IP, Sec. 2.3) of S independent targets, one swarm of P particles each, T
 * generations: init, then T x [misfit of every particle -> PSO generation]; then, if
 * lbfgs_steps > 0, the lbfgs_topk best personal bests of every swarm are polished by
 * afm_polish and the best polished point replaces the swarm best when lower.  Captured once as
 * a HIP graph and replayed without host round-trips: a later call with the same S, P, T, seed,
 * cutoff, polish settings and input buffers (targets, n_cycles, swarm_params) replays it, with
 * any output buffers; a new graph first tunes the forward launch shape (afm_set_launch_shape)
 * unless the plan holds one for S*P trajectories.  targets: [S][W] (device); n_cycles: [S]
 * per-target period counts or NULL (uneven counts run through the persistent work-queue
 * kernel, longest first).  Outputs (device): best_theta [n_free][S] SI, best_J [S],
 * gen_to_cutoff [S].  swarm_params: [AFM_MAX_PARAMS][S] full parameter vectors per target
 * (e.g. each pixel's separation from its set-point; free entries ignored) or NULL for the
 * problem's.  lbfgs_topk <= particles.  Workspace is owned by the plan; with n_cycles the
 * first call reads the period counts to order the work queue (a synchronous copy). */
afm_status afm_invert(afm_plan *plan, int32_t n_swarms, const double *targets,
                      const int32_t *n_cycles, const double *swarm_params, int32_t particles,
                      int32_t iters, uint64_t seed,
                      double cutoff, int32_t lbfgs_steps, int32_t lbfgs_topk, double *best_theta,
                      double *best_J, int32_t *gen_to_cutoff, afm_stream_t stream);

/* Separation from an amplitude set-point for n_pixels pixels (the amplitude feedback of Sec. 1,
 * which holds the oscillation amplitude at a set-point by moving the sample): z_c[s] (m) is the
 * separation at which the steady amplitude of pixel s equals setpoint[s] * A0.  The steady
 * amplitude is the plain FP64 forward solve of the plan's problem (its drive, modes, initial
 * state and force law; the plan's precision, period counts and exit settings are not used) over
 * `periods` drive periods with lock-in over the last `lockin_periods`.  The search emulates an
 * approach curve: z steps down from A0 + 2 nm by `step` (m; 0 = 0.25 nm) to the first grid point
 * whose amplitude is below the set-point (a failed solve counts as below); the bracket between it
 * and the grid point above is then narrowed `rounds` times (0 .. 64) by 16 equally spaced trial
 * separations each -- to the first trial at or above the set-point and the one before it -- and
 * z_c is the bracket's midpoint (bracket width step / 17^rounds).  Pixels with no crossing
 * (or crossing at the top grid point) get NaN.
 * params: [AFM_MAX_PARAMS][n_pixels] full parameter vectors per pixel (device; their z_c entry
 * is ignored) or NULL for the plan's; setpoint: [n_pixels] (device, fraction of A0); zc:
 * [n_pixels] (device).  Needs the fixed drive table.  Allocates a temporary plan and workspace
 * (about 4.5 x n_pixels x max((A0 + 2 nm) / step, 16) x 8 bytes) and synchronises the stream before it
 * returns. */
afm_status afm_separations(afm_plan *plan, int32_t n_pixels, const double *params,
                           const double *setpoint, int32_t periods, int32_t lockin_periods,
                           double step, int32_t rounds, double *zc, afm_stream_t stream);

/* Modes of a uniform clamped-free Euler-Bernoulli cantilever (Sec. 3.2, Eq. 6-7; App. B), for
 * building afm_problem's ratio and gain: beta_i L from cos(beta L) cosh(beta L) + 1 = 0 (Newton),
 * mode shapes Phi_i in the overflow-free exponential form of Eq. 6 with Eq. 7's G -- its
 * denominator read as 2 e^{-beta L} cos(beta L) + e^{-2 beta L} + 1, since the printed minus on
 * e^{-2 beta L} violates the free-end conditions -- normalised at the tip (phi_i = Phi_i /
 * Phi_i(L)), integrals by Simpson's rule on n_points points (odd, >= 3; the paper uses 501).
 * Outputs (host arrays of n_modes, 1 <= n_modes <= 8): ratio[i] = w_i / w_1 = (beta_i / beta_1)^2;
 * gain[i] = gamma_i = int phi_i dx / int phi_i^2 dx (the base-drive participation of mode i in
 * Eq. 2).  f1 (optional): the first natural frequency beta_1^2 sqrt(E I / (mu L^4)) / (2 pi) in
 * Hz from the modulus E (Pa), section moment I (m^4), mass per length mu (kg/m) and length L
 * (m); NaN unless all four are positive.  Host computation only (no device, no stream). */
afm_status afm_beam_modes(int32_t n_modes, int32_t n_points, double E, double I, double mu,
                          double L, double *ratio, double *gain, double *f1);

/* Tip-normalised mode shapes of a uniform clamped-free cantilever (the shapes of
 * afm_beam_modes) at n_x points x[k] in units of L (0 = clamped base, 1 = tip):
 * w[k * n_modes + i] = Phi_i(x_k L) / Phi_i(L), the weights afm_forward_points takes.  1 <=
 * n_modes <= 8, 0 <= x[k] <= 1.  Host computation only. */
afm_status afm_beam_shapes(int32_t n_modes, int32_t n_x, const double *x, double *w);

/* Text of the calling thread's last error ("" if none). */
const char *afm_last_error(void);

/* Library version string. */
const char *afm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* AFM_H */
