/*
 * oracle.h -- plain FP64 CPU oracle of the sample-based stochastic (SBS)
 * predictive controller for a quadruped (Turrisi et al., "On the Benefits of
 * GPU Sample-Based Stochastic Predictive Controllers for Legged Locomotion",
 * IROS 2024).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The product path
 * (the HIP library under paper_2403_11383_amd/) never calls it, and the two
 * share no code, header, table or constant.
 *
 * Everything is computed in FP64 except the Gaussian noise transform, which
 * is a fixed sequence of IEEE FP32 operations (the noise contract) so that
 * the GPU side can reproduce it bit for bit.
 *
 * What each function follows:
 *   orc_philox4x32_10   Philox4x32-10 block function (Salmon et al., SC'11),
 *                       the counter-based stream behind "theta_k ~ N(theta,C)"
 *                       of Alg. 1 (Sampling).
 *   orc_gauss_pair      Box-Muller transform of two 24-bit uniforms.
 *   orc_noise_step      The 12 GRF noise draws of one sample at one step.
 *   orc_freq_q          Per-sample gait frequency theta_1 (Sec. IV-C, Sec. V).
 *   orc_contact         computeContactSequence(theta_1): periodic gait with
 *                       stance time D_f/f_s (Sec. IV-C).
 *   orc_friction_clip   Friction-cone constraint on the GRF (Sec. IV-B).
 *   orc_rotation        Body orientation R(Phi), roll-pitch-yaw (Sec. IV-A).
 *   orc_srbd_deriv      Single-rigid-body dynamics, Eq. (1).
 *   orc_foothold        Foothold reference, Eq. (2) (Sec. IV-D), used at
 *                       every touchdown inside a rollout.
 *   orc_knot_time       Knot instants t^knot_p of the GRF spline (Sec. IV-B).
 *   orc_spline_eval     The GRF spline sigma((t^knot, theta_2), t) of Sec. IV-B.
 *   orc_rollout         Rollout(theta_k), Alg. 2, with the quadratic cost of
 *                       Sec. V and the frequency regulariser of Sec. V.
 *   orc_mppi_*          MPPI UpdateMean, Sec. III-C / Alg. 4.
 *   orc_elite_*         Elite UpdateMean/UpdateCov over the top K_e, Alg. 1;
 *                       K_e = 1 without covariance update is the naive
 *                       optimiser of Sec. III-B / Alg. 3.
 *   orc_tick            One control step of Alg. 5 with warm start (Sec. III-A).
 *
 * Parity pins (tests/test_oracle_*.py): Philox against the header-only
 * philox_engine shipped with PyTorch's ATen; the Gaussian transform against
 * FP64 libm Box-Muller and distribution tests; dynamics against closed forms
 * (free fall, ballistic, hover, torque-free spin), scipy rotations and the
 * momentum theorems; MPPI against scipy.special.softmax and its limits;
 * elite against numpy sort/mean/var on brute-forced tiny cases; the GRF
 * spline against scipy's cubic Hermite interpolant with numpy's gradient
 * slopes, knot interpolation and exactness on linear data.
 * Parity unpinned: the closed-loop behaviour over many ticks (no values in
 * the paper to compare against).
 */
#ifndef SBS_ORACLE_H
#define SBS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_MPPI = 0, ORC_ELITE = 1, ORC_NAIVE = 2 };
enum { ORC_FREQ_FIXED = 0, ORC_FREQ_UNIFORM = 1, ORC_FREQ_GAUSSIAN = 2, ORC_FREQ_SET = 3 };
enum { ORC_FLAG_NONFINITE = 1 };

typedef struct {
  int32_t N;            /* samples per iteration (the paper's K)            */
  int32_t H;            /* horizon steps (the paper's N)                    */
  int32_t iterations;   /* SBS iterations per control step                  */
  int32_t method;       /* ORC_MPPI / ORC_ELITE / ORC_NAIVE                 */
  int32_t freq_mode;    /* ORC_FREQ_*                                       */
  int32_t friction_on;  /* apply the friction-cone clip                     */
  int32_t knots;        /* 0: one GRF vector per step (theta is [H][12]);   */
                        /* P >= 2: cubic spline through P knots (theta is   */
                        /* [P][12]), Sec. IV-B                              */
  double dt, lambda, elite_frac, mu_fric, rho, f_nominal;
  double sigma_grf, sigma_f, sigma_min_grf, sigma_min_f;
  double f_min, f_max, f_fixed, duty;
  double mass, gravity;
  double inertia[3];    /* diagonal body inertia                            */
  double hip[12];       /* body-frame hip offset of leg i at hip[3*i+c]     */
  double Q[12];         /* diagonal state weight, order [p, Phi, v, omega]  */
  double R[12];         /* diagonal GRF weight                              */
  uint32_t phase_offset[4]; /* leg phase offsets, 2^32 = one gait cycle     */
  uint64_t seed;
  double f_set[4];      /* ORC_FREQ_SET: the admissible frequencies, drawn  */
  int32_t n_fset;       /* with equal probability (n_fset in [1, 4])        */
} orc_cfg;

typedef struct {
  double x0[12];        /* [p(3) world, Phi(3) roll/pitch/yaw, v(3) world, omega(3) body] */
  double foot_pos[12];  /* world foothold of leg i at foot_pos[3*i+c]; used */
                        /* for the legs in stance at the first step         */
  double p_ref0[3];
  double v_ref[3];
  double yaw_ref;
  uint32_t phase_robot; /* robot gait phase at this tick                    */
} orc_input;

typedef struct {
  double grf[12];       /* world-frame GRF of the first step, masked        */
  int32_t contact[4];
  double freq_hz;       /* gait frequency after the update                  */
  uint32_t q;           /* its phase increment per step                     */
  double best_cost;     /* lowest cost of the last iteration                */
  int32_t flags;
} orc_action;

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void orc_gauss_pair(uint32_t w0, uint32_t w1, float out[2]);
void orc_noise_step(uint64_t seed, uint32_t tick, uint32_t r, uint32_t k, uint32_t j,
                    float z[12]);
uint32_t orc_q_of_freq(double f, double dt);
double orc_freq_of_q(uint32_t q, double dt);
uint32_t orc_freq_q(const orc_cfg *cfg, double mu_f, double sigma_f, uint32_t tick,
                    uint32_t r, uint32_t k);
int orc_contact(const orc_cfg *cfg, uint32_t phase_robot, uint32_t q, int32_t j,
                int32_t delta[4]);
void orc_friction_clip(const double f[3], double mu, double out[3]);
void orc_rotation(const double phi[3], double R[9]);
void orc_euler_rate_matrix(const double phi[3], double E[9]);
void orc_srbd_deriv(const orc_cfg *cfg, const double x[12], const double u[12],
                    const double lever[12], double xdot[12]);
void orc_foothold(const orc_cfg *cfg, const double x[12], uint32_t q,
                  const double v_ref[3], int32_t leg, double out[3]);
double orc_knot_time(const orc_cfg *cfg, int32_t p);
void orc_spline_eval(const orc_cfg *cfg, const double *theta, double t, double out[12]);
double orc_rollout(const orc_cfg *cfg, const orc_input *in, const double *theta,
                   uint32_t q, double *xs, double *feet);
int orc_mppi_weights(int32_t n, const double *J, double lambda, double *omega,
                     double *beta, double *Omega);
void orc_weighted_mean(int32_t n, int32_t d, const double *omega, const double *theta,
                       double *mean);
int32_t orc_elite_count(int32_t n, double elite_frac);
void orc_elite_select(int32_t n, const double *J, int32_t ke, int32_t *idx);
void orc_elite_moments(int32_t ke, int32_t d, const int32_t *idx, const double *theta,
                       double *mean, double *var);
int orc_tick(const orc_cfg *cfg, double *mu, double *mu_f, uint32_t tick,
             const orc_input *in, orc_action *out, double *costs_out,
             const double *costs_override, double *mean_out, uint32_t *q_out,
             int32_t nthreads);

#ifdef __cplusplus
}
#endif
#endif
