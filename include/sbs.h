/*
 * sbs.h -- C ABI of the MI355X (gfx950) sample-based stochastic (SBS)
 * predictive controller for quadruped locomotion.
 *
 * Method (Turrisi et al., "On the Benefits of GPU Sample-Based Stochastic
 * Predictive Controllers for Legged Locomotion", IROS 2024): every control
 * step samples N decision vectors theta_k = [gait frequency, per-step GRFs]
 * from N(theta, C) (Alg. 1, Sampling), rolls each out over H steps of the
 * single-rigid-body model of Eq. (1) with explicit Euler (Alg. 2), evaluates
 * the quadratic tracking cost of Sec. V plus the frequency regulariser, and
 * updates the sampling mean: MPPI weights (Sec. III-C, Alg. 4), the top-K_e
 * elite mean and covariance (Alg. 1), or the best sample (Sec. III-B, Alg. 3).
 * The mean is warm-started across steps (Sec. III-A) and its first step is the
 * action handed to the low-level controller (Sec. IV, Fig. 2).
 *
 * Ownership and threading
 *   - The caller lends device memory (an "arena", e.g. a torch uint8 tensor)
 *     and a HIP stream; the arena must outlive the runtime.  Every device
 *     buffer of the library is carved from the arena; nothing else is
 *     allocated on the device.  Pinned host staging is allocated with
 *     hipHostMalloc at runtime creation.
 *   - Structs passed by pointer are read (or written) during the call only.
 *   - All functions are thread-safe for one runtime.  Ticks of one controller
 *     execute in submission order.  No exception crosses the ABI.
 *   - Every function returns an sbs_status; on failure a message is kept per
 *     thread and returned by sbs_last_error().
 *
 * Layouts: states are x = [p(3) world, Phi(3) roll/pitch/yaw, v(3) world,
 * omega(3) body]; GRFs are world-frame, leg-major [FL, FR, RL, RR][x, y, z];
 * means are [H][12] row-major.
 */
#ifndef SBS_H
#define SBS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SBS_ABI_VERSION 4

typedef enum {
  SBS_OK = 0,
  SBS_EINVAL = -1,    /* bad argument, non-finite state, unknown id        */
  SBS_ENOMEM = -2,    /* arena or staging exhausted                        */
  SBS_EAGAIN = -3,    /* result not ready yet (fetch with timeout 0)       */
  SBS_ETIMEDOUT = -4, /* fetch timed out                                   */
  SBS_EDEVICE = -5,   /* a HIP call failed                                 */
  SBS_ECANCELED = -6, /* controller destroyed before the tick ran          */
  SBS_ENOENT = -7     /* unknown or already fetched ticket                 */
} sbs_status;

enum { SBS_MPPI = 0, SBS_ELITE = 1, SBS_NAIVE = 2 };
enum { SBS_FREQ_FIXED = 0, SBS_FREQ_UNIFORM = 1, SBS_FREQ_GAUSSIAN = 2, SBS_FREQ_SET = 3 };
enum { SBS_FP32 = 0, SBS_FP64 = 1 };
enum { SBS_FLAG_NONFINITE = 1 };
enum { SBS_MODE_DIRECT = 0, SBS_MODE_SERVING = 1 };

/* Controller configuration.  N samples per iteration (the paper's K), H
 * horizon steps (the paper's N), `iterations` SBS iterations per control step
 * (Alg. 1 repeated from the same state), method SBS_MPPI / SBS_ELITE /
 * SBS_NAIVE, gait-frequency mode SBS_FREQ_* (Sec. IV-C: fixed, uniform on
 * [f_min, f_max], Gaussian around the frequency mean, or one of a small set
 * drawn uniformly as in Sec. V), precision of the
 * rollouts and costs (SBS_FP32 or SBS_FP64).  The frequency is carried as a
 * phase increment per step q = round-half-even(f dt 2^32).
 *
 * knots selects the GRF parametrisation (Sec. IV-B): 0 gives one GRF vector
 * per step (the mean has H rows of 12); P in [2, H] gives P spline knots
 * at instants spread evenly from the first to the last step, each step's
 * GRFs being the cubic Hermite interpolant with finite-difference slopes
 * (centred inside, one-sided at the ends) of the knots (the mean has P rows).
 * Everything indexed by "rows" below is H or P accordingly. */
typedef struct sbs_controller_cfg {
  int32_t N, H, iterations, method, freq_mode, friction_on, precision, knots;
  double dt;            /* step of the discretised dynamics [s]             */
  double lambda;        /* MPPI temperature                                 */
  double elite_frac;    /* K_e = max(1, floor(elite_frac N))                */
  double mu_fric;       /* friction coefficient of the cone clip            */
  double rho;           /* weight of (f_k - f_nominal)^2                    */
  double f_nominal;     /* nominal stepping frequency [Hz]                  */
  double sigma_grf;     /* GRF noise std [N], reset every control step      */
  double sigma_f;       /* frequency noise std [Hz] (Gaussian mode)         */
  double sigma_min_grf, sigma_min_f; /* elite covariance floors           */
  double f_min, f_max;  /* admissible frequency range [Hz]                  */
  double f_fixed;       /* frequency of the fixed mode [Hz]                 */
  double duty;          /* duty factor D_f: stance time D_f / f_s           */
  double mu_f0;         /* initial frequency mean [Hz]                      */
  double mass, gravity;
  double inertia[3];    /* diagonal body inertia [kg m^2]                   */
  double hip[12];       /* body-frame hip offsets [leg][xyz] [m]            */
  double Q[12];         /* diagonal state weights                           */
  double R[12];         /* diagonal GRF weights                             */
  uint32_t phase_offset[4]; /* leg phase offsets, 2^32 = one gait cycle     */
  uint64_t seed;        /* key of the counter-based noise stream            */
  double f_set[4];      /* SBS_FREQ_SET: the admissible frequencies [Hz],   */
  int32_t n_fset;       /* each drawn with probability 1 / n_fset (1..4)    */
  int32_t reserved1;
} sbs_controller_cfg;

/* One control-step request ("Given x0", Alg. 5). */
typedef struct sbs_tick_input {
  double x0[12];        /* current state estimate                           */
  double foot_pos[12];  /* world footholds [leg][xyz] of the stance legs    */
  double p_ref0[3];     /* reference position at the first step             */
  double v_ref[3];      /* reference (desired) velocity                     */
  double yaw_ref;
  uint32_t phase_robot; /* gait phase of the robot, 2^32 = one cycle        */
  uint32_t reserved0;
} sbs_tick_input;

/* Result of one control step. */
typedef struct sbs_action {
  double grf[12];       /* first-step GRFs of the updated mean, masked by the
                           contact flags and clipped to the friction cone   */
  int32_t contact[4];   /* stance flags at the robot's current phase        */
  double freq_hz;       /* updated gait frequency                           */
  double best_cost;     /* lowest cost of the last iteration                */
  uint32_t q;           /* phase increment per step of freq_hz              */
  int32_t flags;        /* SBS_FLAG_*                                        */
  uint32_t tick;        /* control-step counter of the controller           */
  int32_t controller;
  int64_t t_submit_ns, t_launch_ns, t_done_ns; /* CLOCK_MONOTONIC           */
  uint32_t n_active;    /* samples with non-zero weight in the last iteration */
  uint32_t reserved0;
} sbs_action;

typedef struct sbs_runtime sbs_runtime;

/* Create a runtime on the current HIP device.  arena: device pointer of
 * arena_bytes bytes (256-byte aligned); stream: hipStream_t the library
 * enqueues on; mode SBS_MODE_DIRECT launches each submission immediately on
 * the caller's thread, SBS_MODE_SERVING queues submissions for a scheduler
 * thread that admits them by arena memory and batches them (continuous
 * batching).  stream2 (may be NULL) is a second stream the serving scheduler
 * alternates batches on so that consecutive batches overlap. */
int sbs_runtime_create(void *arena, uint64_t arena_bytes, void *stream, void *stream2,
                       int32_t mode, sbs_runtime **out);
/* Waits for all work, then frees host resources.  Pending tickets are
 * cancelled. */
int sbs_runtime_destroy(sbs_runtime *rt);

/* Validate cfg, reserve the controller's persistent device state (mean
 * [rows][12] in the controller precision, frequency mean, spline tables),
 * set the mean to the hover forces (0, 0, m g / 2) on every leg and row
 * (first warm start,
 * Sec. III-A) and return its id.  SBS_ENOMEM if the arena cannot hold it. */
int sbs_init_controller(sbs_runtime *rt, const sbs_controller_cfg *cfg, int32_t *id);
int sbs_destroy_controller(sbs_runtime *rt, int32_t id);

/* Queue one control step of controller id: "given x0" (Alg. 5), sample,
 * roll out, rank and update as in Alg. 1 (MPPI: Alg. 4; best sample:
 * Alg. 3) from the controller's warm-started mean (Sec. III-A).  Never blocks.  Returns a ticket
 * for sbs_fetch_action.  SBS_EINVAL for a non-finite state; SBS_ENOMEM
 * (direct mode) if the arena cannot hold the step's workspace now. */
int sbs_submit_tick(sbs_runtime *rt, int32_t id, const sbs_tick_input *in, uint64_t *ticket);

/* sbs_submit_tick for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the step workspace (noise, costs, weights, chosen samples, per-iteration
 * scalars) lives in a static device array of 64 MiB that the library holds
 * on each GPU it runs on until the process ends, instead of being carved from
 * the arena; the call takes no arena memory and calls no allocator.  Results
 * are those of sbs_submit_tick (same kernels); fetch with sbs_fetch_action.
 * Direct mode only (SBS_EINVAL otherwise); the noise is always made inside
 * the tick (no prefetch).  SBS_EINVAL if the controller's workspace exceeds
 * 64 MiB (e.g. N = 16384 per-step samples at H = 80).  Every call on a GPU
 * shares that GPU's array: calls of one runtime are ordered on its stream,
 * but calls through runtimes on different streams of one GPU that overlap
 * in time race on it. */
int sbs_submit_tick_noalloc(sbs_runtime *rt, int32_t id, const sbs_tick_input *in,
                            uint64_t *ticket);

/* Queue one control step for each of n distinct controllers as one fused
 * launch sequence (one kernel per stage for all of them). */
int sbs_submit_batch(sbs_runtime *rt, int32_t n, const int32_t *ids, const sbs_tick_input *in,
                     uint64_t *tickets);

/* The action of a control step: the first step of the updated mean, the
 * command handed to the low-level controller (Fig. 2, Sec. IV), with the
 * contact flags at the robot's phase and the updated gait frequency.
 * Wait up to timeout_us (0: poll, <0: forever) for a ticket.  SBS_EAGAIN or
 * SBS_ETIMEDOUT if not done; on SBS_OK the ticket is consumed. */
int sbs_fetch_action(sbs_runtime *rt, uint64_t ticket, sbs_action *out, int64_t timeout_us);

/* Every completed control step at once (serving clients polling many
 * robots): writes up to max completed tickets and their actions into
 * tickets[] and out[] (consuming them) and their number into *count; ticks
 * still pending, and failed ones (which sbs_fetch_action reports), are left.
 * With none ready it waits up to timeout_us (0: return at once, <0: until
 * one is ready), yielding the CPU between polls.  The order is unspecified:
 * each action carries its controller and tick.  SBS_EINVAL on a null
 * pointer or max < 0. */
int sbs_fetch_ready(sbs_runtime *rt, int32_t max, uint64_t *tickets, sbs_action *out,
                    int32_t *count, int64_t timeout_us);

/* sbs_fetch_action for n tickets in order (out[i] for tickets[i]), each
 * waited for up to timeout_us: one call for a batch's or plan's tickets.
 * Returns at the first ticket that fails or is not ready with that status;
 * the tickets before it are consumed and their actions written, the rest
 * are left as they were.  SBS_EINVAL on a null pointer or n < 0. */
int sbs_fetch_actions(sbs_runtime *rt, int32_t n, const uint64_t *tickets, sbs_action *out,
                      int64_t timeout_us);

/* Fixed-membership batch for repeated fused ticks: reserves the workspace of
 * the n controllers once and records the whole tick (all stages and
 * iterations) as a HIP graph that sbs_plan_submit replays with new inputs.
 * sbs_plan_submit returns SBS_EAGAIN while the plan's previous replay is
 * still running (its actions can be fetched before its last kernel ends):
 * submit again. */
int sbs_plan_create(sbs_runtime *rt, int32_t n, const int32_t *ids, int32_t use_graph,
                    int32_t *plan);
int sbs_plan_submit(sbs_runtime *rt, int32_t plan, const sbs_tick_input *in, uint64_t *tickets);
int sbs_plan_destroy(sbs_runtime *rt, int32_t plan);

/* Rollout form of a plan: lanes per sample (1, or 4 = one lane per leg; 0 =
 * automatic), workgroup size (64, 128, 256) and step-loop unroll (1, 2).
 * Supported forms: lanes 4 with (64|128|256, 1); lanes 1 with (64|128|256, 1)
 * or (64|128, 2).  The form never changes which samples are
 * drawn; lanes 1 and 4 differ only in FP32 rounding order. */
typedef struct sbs_tune {
  int32_t lanes, block, unroll, reserved;
  double tick_us;       /* measured device time of one tick (autotune)      */
} sbs_tune;
int sbs_plan_set_tune(sbs_runtime *rt, int32_t plan, const sbs_tune *t);

/* Autotuner: runs the plan's tick `reps` times (after one warm-up) in every
 * supported rollout form with the given inputs, restoring each controller's
 * mean, frequency mean and tick counter after every trial, keeps the form
 * with the lowest device time (re-recording the plan's graph) and returns it.
 * Waits for all outstanding work first. */
int sbs_plan_autotune(sbs_runtime *rt, int32_t plan, const sbs_tick_input *in, int32_t reps,
                      sbs_tune *best);

/* Synchronous state access (waits for the controller's pending work):
 * mean [H][12], frequency mean and next tick number.  Used for checkpoint
 * and resume: export, then import into a fresh controller, reproduces the
 * following ticks bit for bit (the noise is counter-based). */
int sbs_get_state(sbs_runtime *rt, int32_t id, double *mu, double *mu_f, uint32_t *tick);  /* mu [rows][12] */
int sbs_set_state(sbs_runtime *rt, int32_t id, const double *mu, double mu_f, uint32_t tick);
/* The same two calls under their checkpoint names: sbs_export_state is
 * sbs_get_state, sbs_import_state is sbs_set_state (the warm-started mean of
 * Sec. III-A is the whole state a controller carries between steps). */
int sbs_export_state(sbs_runtime *rt, int32_t id, double *mu, double *mu_f, uint32_t *tick);
int sbs_import_state(sbs_runtime *rt, int32_t id, const double *mu, double mu_f, uint32_t tick);

/* Debug taps.  sbs_set_debug(1) makes every later tick of the controller
 * keep its per-iteration costs [iterations][N], sampled phase increments
 * [iterations][N] and the updated mean before the warm-start shift [rows][12];
 * sbs_debug_fetch returns those of the last completed tick.
 * sbs_debug_noise runs the noise stage alone for (tick, iteration r) with the
 * controller's current frequency mean and returns z [N][rows][12] and q [N]. */
int sbs_set_debug(sbs_runtime *rt, int32_t id, int32_t enable);
int sbs_debug_fetch(sbs_runtime *rt, int32_t id, double *costs, uint32_t *q, double *mean);
/* sbs_debug_fetch under the name of the cost tap: the rollout costs of
 * Alg. 2 that the last completed tick ranked or weighted. */
int sbs_debug_costs(sbs_runtime *rt, int32_t id, double *costs, uint32_t *q, double *mean);
int sbs_debug_noise(sbs_runtime *rt, int32_t id, uint32_t tick, uint32_t r, float *z, uint32_t *q);

/* Noise prefetch for a single controller in direct mode (needs stream2):
 * the GRF noise depends only on (seed, tick, iteration, sample, step), never
 * on the state, so every submission also produces the next tick's noise on
 * the second stream into a second buffer, and the next tick skips its noise
 * stage.  Results are unchanged; the arena holds two extra noise buffers of
 * iterations x rows x N x 12 floats. */
int sbs_set_prefetch(sbs_runtime *rt, int32_t id, int32_t enable);

/* Serving statistics: ticks completed, batches launched, admission waits. */
int sbs_stats(sbs_runtime *rt, uint64_t *ticks, uint64_t *batches, uint64_t *admit_waits);

/* Rollout lanes per sample for FP32 controllers: 4 (one lane per leg, for
 * launches with few samples), 1 (one lane per sample, for throughput), or 0
 * (automatic: 4 when a launch holds at most 32768 samples).  Results of the
 * two forms agree within FP32 rounding, not bit for bit. */
int sbs_set_rollout_lanes(sbs_runtime *rt, int32_t lanes);

/* Stance-pair rollouts (default on): for a diagonal trot at duty factor 1/2
 * (legs 0 and 3 in phase, legs 1 and 2 half a cycle later) exactly one leg
 * pair is in stance at every step, and the one-lane rollouts form the forces,
 * footholds, costs and torques of that pair only (the other pair's terms of
 * Eq. (1) and of the cost are zero).  0 turns this off: every leg is formed
 * and masked by its contact flag.  Both give the same sums; the switch is
 * for verification and timing.  Takes effect at the next submission; a plan
 * keeps the setting it was created with. */
int sbs_set_rollout_pairs(sbs_runtime *rt, int32_t enable);

/* Noise made inside the rollout (Alg. 1 Sampling; the same counter-based
 * values in every mode).  mode 0: a separate noise launch writes every row
 * and the rollout reads it back.  1: a one-lane FP32 rollout of per-step
 * GRFs draws each step's row itself and stores it for the update.  2
 * (default): as 1, except that the one-lane rollout of a controller in the
 * stance-pair form (diagonal trot at duty 1/2, N at most 16384) draws only
 * its two stance legs' GRF components -- the only ones it uses -- and stores
 * nothing; the update then draws the rows of the samples it needs: the
 * weighed ones of MPPI (quick for the usual few; with thousands of weighed
 * samples one workgroup draws them all, correct but slow), the K_e chosen
 * ones of an elite or best-sample update.  The choice depends on the
 * configuration alone.  Modes 0 and 1 give bit-identical results; mode 2's
 * rollout is compiled apart and agrees with them within FP32 rounding.
 * Takes effect at the next submission; a plan keeps the setting it was
 * created with.  SBS_EINVAL for a null runtime or a mode outside 0..2. */
int sbs_set_rollout_noise(sbs_runtime *rt, int32_t mode);

/* Serving mode: batches the scheduler keeps in flight per stream (1 to 4,
 * default 1).  With one stream and depth 2 the next batch is formed and
 * enqueued while the current one runs, so batches run back to back and
 * each has the device to itself; with two streams and depth 1 consecutive
 * batches overlap.  Each batch in flight holds its own step workspace in the
 * arena.  SBS_EINVAL for a null runtime or a depth outside 1..4. */
int sbs_set_serving_depth(sbs_runtime *rt, int32_t depth);

/* Kernel timing with HIP events on the runtime stream: mode 0 off; 1 the
 * rollout kernel's own start and end (events carried by its dispatch) on
 * one launch in 16, counted from this call; 2 event commands between every
 * stage of every launch (diagnostic: each adds a few microseconds); 3 as 1
 * on every launch.
 * sbs_timing returns the average device time [ns] of each stage's timed
 * launches since the last call (0 noise, 1 rollout, 2 select, 3 update) and
 * resets it. */
int sbs_set_timing(sbs_runtime *rt, int32_t mode);
int sbs_timing(sbs_runtime *rt, double *avg_ns, uint64_t *launches);
/* Rollout timing by form (modes 1 and 3): form 0 FP32 one lane per sample,
 * 1 FP32 four lanes per sample, 2 FP64, 3 FP32 one lane per sample making
 * its own noise rows, 4 FP32 one lane per sample making its stance legs'
 * noise only (sbs_set_rollout_noise).  Returns the average device time
 * [ns] of that form's timed rollout launches since the last call for the
 * form, their number and the rollout-steps (sum of N H over the launches'
 * controllers) they covered, and resets the form's accumulators.  The
 * algorithmic FLOP rate of the rollout (Alg. 2) is then
 * flop_per_step * steps / (avg_ns * launches).  SBS_EINVAL for a null
 * runtime or a form outside 0..4. */
int sbs_timing_rollout(sbs_runtime *rt, int32_t form, double *avg_ns, uint64_t *launches,
                       double *steps);
/* Fixed overhead of dispatch-carried timing events: the average interval [ns]
 * that an empty one-workgroup kernel launched with start/stop events on the
 * runtime's stream spans, over reps launches (1..4096; each waits for its own
 * events).  Every launch timed in modes 1 and 3 includes it once; subtracting
 * it leaves the kernel's execution time as a kernel trace records it.
 * SBS_EINVAL on a null pointer or reps out of range. */
int sbs_timing_overhead(sbs_runtime *rt, int32_t reps, double *avg_ns);

/* Simulated robot for closed-loop runs (host, FP64, not part of the control
 * step): advances the single-rigid-body plant of Eq. (1) by one step dt
 * under the action's GRFs on the stance legs, an external world-frame force
 * ext_force [N] on the CoM, and world-fixed feet; a leg that touches down is
 * placed by the foothold rule of Eq. (2) with the executed frequency and
 * v_ref.  state (x[12], foot_pos[12], phase) is updated in place; the phase
 * advances by action->q.  Uses cfg for the model constants. */
typedef struct sbs_plant_state {
  double x[12];
  double foot_pos[12];
  int32_t contact[4];   /* stance flags of the previous step                */
  uint32_t phase;
  uint32_t reserved0;
} sbs_plant_state;
int sbs_plant_step(const sbs_controller_cfg *cfg, sbs_plant_state *st, const sbs_action *act,
                   const double ext_force[3], const double v_ref[3]);
/* The same step under an external wrench on the CoM: ext_wrench = world-frame
 * force [N] (0..2) and world-frame torque [N m] (3..5), the disturbances of
 * the simulated robustness tests of Sec. V.  Returns SBS_EINVAL on a
 * null pointer; the state is left unchanged then. */
int sbs_plant_step_wrench(const sbs_controller_cfg *cfg, sbs_plant_state *st,
                          const sbs_action *act, const double ext_wrench[6],
                          const double v_ref[3]);
/* One closed-loop cycle of a simulated robot in native code (for host-side
 * simulation loops, where a round trip through an interpreter per call would
 * dominate the cycle): builds the tick input from the plant state -- x0 =
 * state, world footholds, gait phase, reference position (x, y of the state,
 * z_ref), v_ref, yaw_ref -- then sbs_submit_tick, sbs_fetch_action with no
 * time limit, and sbs_plant_step_wrench under the action and ext_wrench.
 * cfg gives the plant's model constants (normally the controller's).  The
 * action is returned in *out; the status is that of the first failing call
 * (the plant is advanced only when all succeed). */
int sbs_closed_loop_step(sbs_runtime *rt, int32_t id, const sbs_controller_cfg *cfg,
                         sbs_plant_state *st, const double ext_wrench[6], const double v_ref[3],
                         double z_ref, double yaw_ref, sbs_action *out);

const char *sbs_last_error(void);
int32_t sbs_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif
