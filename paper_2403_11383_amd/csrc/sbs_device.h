// sbs_device.h -- descriptors shared by the host runtime and the gfx950
// kernels.  One TickDesc describes one controller's control step; a LaunchTab
// maps the flattened block index of each stage onto the descriptors active in
// one iteration of a fused batch.
#pragma once

#include <stdint.h>

namespace sbs {

constexpr int kNoiseBlock = 256;   // samples per noise workgroup at one step
constexpr int kUpdBlock = 512;     // threads per update workgroup (elite, best sample)
constexpr int kMppiBlock = 1024;   // threads per fused MPPI update workgroup
constexpr int kSelBlock = 1024;    // threads of the per-controller select block
constexpr int kResultDoubles = 24; // action record
constexpr int kItScalars = 16;     // per-iteration scalars
constexpr int kMaxH = 256;         // longest horizon: the rollout stages the mean, std and
                                   // spline tables in LDS (58 KB at FP64 and H = 256)

// result record layout (doubles)
enum : int {
  RES_GRF = 0,        // 12
  RES_CONTACT = 12,   // 4
  RES_FREQ = 16,
  RES_Q = 17,
  RES_BEST = 18,
  RES_FLAGS = 19,
  RES_NACT = 20,      // samples with non-zero weight in the last iteration
  RES_SEQ = 21,       // uint64 bits: tick + 1, stored last with system-scope
                      // release, so a host that reads it sees a whole record
};

// per-iteration scalars (doubles)
enum : int {
  IT_MUF = 0,      // frequency mean for the next sampling round
  IT_SIGF = 1,     // frequency std for the next sampling round
  IT_BETA = 2,     // lowest cost
  IT_OMEGA = 3,    // normaliser (MPPI), K_e (elite), 1 (naive)
  IT_BEST = 4,     // index of the lowest cost
  IT_FNEW = 5,     // updated frequency
  IT_FLAGS = 6,
  IT_SKIP = 7,     // 1 when no cost was finite: keep the mean
  IT_NACT = 8,     // number of samples with non-zero weight
};

struct TickDesc {
  int32_t N, H, R, method, freq_mode, friction_on, precision, Ke;
  int32_t mu_par0;       // the tick's first iteration reads mu_buf[mu_par0]
  int32_t shift0;        // 1: that mean is the previous tick's, read shifted
  uint32_t tick;         // control-step counter (noise counter word 2)
  uint32_t phase_robot;
  uint32_t q_fixed, q_lo, q_hi;
  uint32_t q_set[4];     // frequency-set mode: phase increments of the members
  int32_t n_fset;
  int32_t pad1;
  uint32_t phase_offset[4];
  uint32_t duty_q;       // stance iff phase < duty_q (duty_full: always)
  int32_t duty_full;
  int32_t slot;          // index of this descriptor in the batch
  int32_t M;             // rows of the mean: H, or the spline knot count P
  int32_t spline;        // 1: GRFs of step j are the spline through the knots
  uint64_t seed;
  double dt, inv_lambda, mu_fric, rho, f_nominal, mass, inv_mass, gravity, inv_g;
  double inertia[3], inv_inertia[3], hip[12], Q[12], Rw[12];
  double sigma0, sigma_f0, sigma_min_grf, sigma_min_f, f_min, f_max, f_fixed;
  double half_duty;      // D_f / 2, so T_st / 2 = half_duty / f
  double inv_q_scale;    // 1 / (dt 2^32): f = q * inv_q_scale
  double x0[12], foot[12], p_ref0[3], v_ref[3], yaw_ref;
  // persistent controller state
  // Two [M][12] mean buffers in the controller precision.  Iteration r
  // reads mu_buf[(mu_par0 + r) & 1] and writes the other one.  The warm-start
  // shift of Sec. III-A is applied when a mean is read (shift0): row j of
  // the shifted mean is row j + 1 of the stored one (per-step GRFs) or the
  // stored spline one step later (knots), the last row hover.
  void *mu_buf[2];
  double *ctl;           // [0] frequency mean
  // spline tables (spline == 1): the GRFs of step j are
  //   sum_i sp_w[4 j + i] * theta[sp_b[j] + i]   (knots beyond M - 1 weigh 0)
  // and the shifted mean's knot p < M - 1 is
  //   sum_i sh_w[4 p + i] * mu[sh_b[p] + i]
  const double *sp_w;    // [H][4]
  const int32_t *sp_b;   // [H], non-decreasing
  const double *sh_w;    // [M][4]
  const int32_t *sh_b;   // [M]
  // step workspace
  float *z;              // [M][N][12] noise; iteration r at z + r * z_iter_stride
  uint64_t z_iter_stride; // 0 (one buffer reused per iteration) or M * N * 12
  uint32_t *q;           // [N]
  void *J;               // [N] costs, controller precision
  void *w;               // [N] weights of the active samples, controller precision
  uint32_t *act;         // [N] active sample indices in increasing order
  double *sigma;         // [M][12] elite std of the current iteration
  double *it;            // [kItScalars]
  double *result;        // [kResultDoubles]
  double *dbg_J;         // optional [R][N]
  uint32_t *dbg_q;       // optional [R][N]
  double *dbg_mean;      // optional [M][12]
};

// Block maps of one (iteration, precision, parametrisation) launch over n
// active descriptors:
// start arrays are exclusive prefix sums of each stage's blocks per item.
struct LaunchTab {
  int32_t n;
  int32_t r;             // iteration index
  int32_t total_noise, total_roll, total_upd;
  int32_t max_h;         // longest horizon among the items
  int32_t lanes;         // rollout lanes per sample: 1 or 4 (FP32 only)
  int32_t roll_block;    // rollout workgroup size: 64, 128 or 256
  int32_t unroll;        // rollout step-loop unroll: 1 or 2
  int32_t r_count;       // iterations covered by a noise launch
  int32_t write_q;       // noise launch also writes the frequency draws
  int32_t skip_noise;    // noise already produced (ahead of the tick)
  int32_t n_select;      // items with an elite or best-sample update
  int32_t max_rows;      // most mean rows among the items
  int32_t spline;        // the items use the spline parametrisation
  int32_t noise_rpt;     // noise rows per thread (single-controller launches; 0 = 1)
  int32_t upd_chunk;     // mean rows per elite / best-sample update workgroup (0 or
                         // 1: one); MPPI items have no blocks in upd_start
  int32_t gen_noise;     // the one-lane FP32 rollout makes the noise itself (no noise
                         // launch; per-step GRFs only): 1 every row, stored for the
                         // update; 2 (stance-pair form) only the stance legs'
                         // Gaussians, nothing stored: the updates make the rows they
                         // read
  int32_t pairs;         // one-lane rollouts in the stance-pair form: every item is a
                         // diagonal trot at duty 1/2 (one of the leg pairs {0, 3},
                         // {1, 2} in stance at every step)
  const TickDesc *desc;  // descriptor array of the batch
  const int32_t *item;   // [n] descriptor index
  const int32_t *noise_start;  // [n+1]
  const int32_t *roll_start;   // [n+1]
  const int32_t *upd_start;    // [n+1]
};

}  // namespace sbs
