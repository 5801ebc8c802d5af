/*
 * oracle.c -- plain FP64 CPU oracle (test infrastructure only; see oracle.h).
 *
 * Build: gcc -std=c11 -O2 -ffp-contract=off -fno-fast-math -fPIC -shared
 *        -pthread oracle.c -o liboracle.so -lm
 * Contraction stays off so that every FP32 step of the noise transform is the
 * exact operation written here; fused multiply-adds appear only where fmaf()
 * is called explicitly.
 */
#include "oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define TWO32 4294967296.0

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplies with a   */
/* Weyl-sequence key schedule.                                              */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u; /* golden ratio */
      k1 += 0xBB67AE85u; /* sqrt(3) - 1  */
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------------------ */
/* Box-Muller on two 24-bit uniforms, u1 in (0,1] and u2 in [0,1):            */
/*   z_a = sqrt(-2 ln u1) cos(2 pi u2),  z_b = sqrt(-2 ln u1) sin(2 pi u2).  */
/* ln u1 = e ln2 + ln m with m in [sqrt2/2, sqrt2]; ln m = ln(1 + f), f =   */
/* m - 1 (exact), as f + f^2 (f P(f) - 1/2) with P a degree-7 polynomial:   */
/* a fit of (ln(1+f) - f + f^2/2) / f^3 on the folded range that weighs the */
/* relative error of ln m (weighted least squares on Chebyshev nodes,       */
/* reweighted toward the largest errors), coefficients rounded to FP32; no  */
/* division.  Over all 2^24 inputs ln u1 stays within 0.9 ulp of the exact  */
/* logarithm.  sin/cos of 2 pi u2 by exact reduction in turns to |a| <= 1/8 */
/* and Taylor polynomials.  Every step is one IEEE FP32 operation.          */
/* ------------------------------------------------------------------------ */
static int floor_log2_u32(uint32_t v) {
  int e = -1;
  while (v) { v >>= 1; ++e; }
  return e;
}

void orc_gauss_pair(uint32_t w0, uint32_t w1, float out[2]) {
  uint32_t i1 = (w0 >> 8) + 1u;      /* u1 = i1 * 2^-24, i1 in [1, 2^24] */
  uint32_t i2 = w1 >> 8;             /* u2 = i2 * 2^-24, i2 in [0, 2^24) */

  /* ln u1 */
  int e = floor_log2_u32(i1);        /* 0..24 */
  float m = ldexpf((float)i1, -e);   /* exact, in [1,2) */
  if (m > 0x1.6a09e6p+0f) { m = m * 0.5f; e = e + 1; }
  float f = m - 1.0f;                               /* exact */
  float h = f * f;
  float p = fmaf(f, -0x1.38b4e6p-4f, 0x1.055b58p-3f); /* P(f), highest terms first */
  p = fmaf(f, p, -0x1.0d8556p-3f);
  p = fmaf(f, p, 0x1.22da20p-3f);
  p = fmaf(f, p, -0x1.547242p-3f);
  p = fmaf(f, p, 0x1.99a008p-3f);                     /* ~ 1/5 */
  p = fmaf(f, p, -0x1.000228p-2f);                    /* ~ -1/4 */
  p = fmaf(f, p, 0x1.555554p-2f);                     /* ~ 1/3 */
  float lnm = fmaf(h, fmaf(f, p, -0.5f), f);
  float ke = (float)(e - 24);
  float lnu = fmaf(ke, 0x1.62e4p-1f, fmaf(ke, 0x1.7f7d1cp-20f, lnm)); /* ln2 hi + lo */
  float rho = sqrtf(-2.0f * lnu);

  /* cos, sin of 2 pi u2 */
  uint32_t n = (i2 + (1u << 21)) >> 22;            /* nearest quarter turn, 0..4 */
  int32_t fi = (int32_t)i2 - (int32_t)(n << 22);   /* |fi| <= 2^21 */
  float a = (float)fi * 0x1p-24f;                  /* turns, |a| <= 1/8 */
  float a2 = a * a;
  float ps = fmaf(a2, 0x1.507834p+5f, -0x1.32d2ccp+6f);   /* (2pi)^9/9!, -(2pi)^7/7! */
  ps = fmaf(a2, ps, 0x1.466bc6p+6f);                      /* (2pi)^5/5! */
  ps = fmaf(a2, ps, -0x1.4abbcep+5f);                     /* -(2pi)^3/3! */
  ps = fmaf(a2, ps, 0x1.921fb6p+2f);                      /* 2pi */
  float sn = a * ps;
  float pc = fmaf(a2, -0x1.a6d1f2p+4f, 0x1.e1f506p+5f);   /* -(2pi)^10/10!, (2pi)^8/8! */
  pc = fmaf(a2, pc, -0x1.55d3c8p+6f);                     /* -(2pi)^6/6! */
  pc = fmaf(a2, pc, 0x1.03c1f0p+6f);                      /* (2pi)^4/4! */
  pc = fmaf(a2, pc, -0x1.3bd3ccp+4f);                     /* -(2pi)^2/2! */
  float cs = fmaf(a2, pc, 1.0f);
  float c, sv;
  switch (n & 3u) {
    case 0: c = cs; sv = sn; break;
    case 1: c = -sn; sv = cs; break;
    case 2: c = -cs; sv = -sn; break;
    default: c = sn; sv = -cs; break;
  }
  out[0] = rho * c;
  out[1] = rho * sv;
}

/* Counter map of the noise stream: key = seed, counter = (k, j, tick,      */
/* (r << 8) | call).  Calls 0..2 give the six Box-Muller pairs of row j:     */
/* pair p uses words 2(p mod 2), 2(p mod 2) + 1 of call p / 2.  Each pair    */
/* serves one force component of the two legs of a diagonal: pairs 0..2 the  */
/* x, y, z components of legs 0 and 3 (dims 0..2 and 9..11), pairs 3..5      */
/* those of legs 1 and 2 (dims 3..5 and 6..8).  Call 3 at j = 0 gives the    */
/* frequency draw of sample k.                                              */
static void philox_call(uint64_t seed, uint32_t k, uint32_t j, uint32_t tick, uint32_t r,
                        uint32_t call, uint32_t w[4]) {
  uint32_t ctr[4] = {k, j, tick, (r << 8) | call};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  orc_philox4x32_10(ctr, key, w);
}

/* GRF dimensions of Box-Muller pair p: (first value, second value). */
static const int kPairDims[6][2] = {{0, 9}, {1, 10}, {2, 11}, {3, 6}, {4, 7}, {5, 8}};

void orc_noise_step(uint64_t seed, uint32_t tick, uint32_t r, uint32_t k, uint32_t j,
                    float z[12]) {
  for (uint32_t c = 0; c < 3; ++c) {
    uint32_t w[4];
    philox_call(seed, k, j, tick, r, c, w);
    for (int h = 0; h < 2; ++h) {
      float g[2];
      orc_gauss_pair(w[2 * h], w[2 * h + 1], g);
      const int p = 2 * (int)c + h;
      z[kPairDims[p][0]] = g[0];
      z[kPairDims[p][1]] = g[1];
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Gait frequency theta_1 (Sec. IV-C): the frequency is carried as a uint32  */
/* phase increment per step, q = round-half-even(f * dt * 2^32), so that the */
/* contact schedule is integer arithmetic on both sides.                    */
/* ------------------------------------------------------------------------ */
uint32_t orc_q_of_freq(double f, double dt) {
  double v = rint((f * dt) * TWO32);
  if (!(v > 0.0)) return 0u;           /* also NaN */
  if (v > 4294967295.0) return 4294967295u;
  return (uint32_t)v;
}

double orc_freq_of_q(uint32_t q, double dt) { return (double)q / (dt * TWO32); }

uint32_t orc_freq_q(const orc_cfg *cfg, double mu_f, double sigma_f, uint32_t tick,
                    uint32_t r, uint32_t k) {
  if (cfg->freq_mode == ORC_FREQ_FIXED) return orc_q_of_freq(cfg->f_fixed, cfg->dt);
  uint32_t w[4];
  philox_call(cfg->seed, k, 0u, tick, r, 3u, w);
  if (cfg->freq_mode == ORC_FREQ_UNIFORM) {
    /* uniform over the integer increments of [f_min, f_max] */
    uint32_t qlo = orc_q_of_freq(cfg->f_min, cfg->dt);
    uint32_t qhi = orc_q_of_freq(cfg->f_max, cfg->dt);
    uint64_t span = (uint64_t)(qhi - qlo) + 1u;
    return qlo + (uint32_t)(((uint64_t)w[0] * span) >> 32);
  }
  if (cfg->freq_mode == ORC_FREQ_SET) {
    /* one of the n admissible frequencies, each with probability 1/n */
    uint32_t i = (uint32_t)(((uint64_t)w[0] * (uint64_t)cfg->n_fset) >> 32);
    return orc_q_of_freq(cfg->f_set[i], cfg->dt);
  }
  /* Gaussian around the current mean, clamped to the admissible range */
  float g[2];
  orc_gauss_pair(w[0], w[1], g);
  double f = mu_f + sigma_f * (double)g[0];
  if (f < cfg->f_min) f = cfg->f_min;
  if (f > cfg->f_max) f = cfg->f_max;
  return orc_q_of_freq(f, cfg->dt);
}

/* computeContactSequence (Sec. IV-C): leg i is in stance at step j iff its  */
/* phase (phase_robot + offset_i + j q) mod 2^32 is below D_f * 2^32, i.e.   */
/* stance lasts D_f / f_s seconds and swing (1 - D_f) / f_s.                */
int orc_contact(const orc_cfg *cfg, uint32_t phase_robot, uint32_t q, int32_t j,
                int32_t delta[4]) {
  uint64_t dq = (uint64_t)rint(cfg->duty * TWO32);
  int n = 0;
  for (int i = 0; i < 4; ++i) {
    uint32_t ph = phase_robot + cfg->phase_offset[i] + (uint32_t)j * q;
    delta[i] = ((uint64_t)ph < dq) ? 1 : 0;
    n += delta[i];
  }
  return n;
}

/* Friction cone (Sec. IV-B): normal force non-negative, tangential force    */
/* scaled radially onto the cone |f_t| <= mu f_z.                            */
void orc_friction_clip(const double f[3], double mu, double out[3]) {
  double fz = f[2] > 0.0 ? f[2] : 0.0;
  double ft = sqrt(f[0] * f[0] + f[1] * f[1]);
  double lim = mu * fz;
  double s = (ft > lim) ? lim / ft : 1.0;
  out[0] = f[0] * s;
  out[1] = f[1] * s;
  out[2] = fz;
}

/* ------------------------------------------------------------------------ */
/* SRBD model, Eq. (1).                                                      */
/* ------------------------------------------------------------------------ */
static void matmul3(const double A[9], const double B[9], double C[9]) {
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += A[3 * r + k] * B[3 * k + c];
      C[3 * r + c] = s;
    }
}

/* R = Rz(yaw) Ry(pitch) Rx(roll): body-to-world rotation, row-major. */
void orc_rotation(const double phi[3], double R[9]) {
  double cr = cos(phi[0]), sr = sin(phi[0]);
  double cp = cos(phi[1]), sp = sin(phi[1]);
  double cy = cos(phi[2]), sy = sin(phi[2]);
  double Rx[9] = {1, 0, 0, 0, cr, -sr, 0, sr, cr};
  double Ry[9] = {cp, 0, sp, 0, 1, 0, -sp, 0, cp};
  double Rz[9] = {cy, -sy, 0, sy, cy, 0, 0, 0, 1};
  double T[9];
  matmul3(Ry, Rx, T);
  matmul3(Rz, T, R);
}

/* Map from body angular velocity to roll/pitch/yaw rates for the           */
/* Rz Ry Rx convention: Phi_dot = E'^-1(Phi) omega.                          */
void orc_euler_rate_matrix(const double phi[3], double E[9]) {
  double cr = cos(phi[0]), sr = sin(phi[0]);
  double cp = cos(phi[1]), tp = tan(phi[1]);
  E[0] = 1.0; E[1] = sr * tp; E[2] = cr * tp;
  E[3] = 0.0; E[4] = cr;      E[5] = -sr;
  E[6] = 0.0; E[7] = sr / cp; E[8] = cr / cp;
}

static void cross3(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

/* State x = [p, Phi, v, omega] (p, v world frame; omega body frame).  u is  */
/* the 4x3 world-frame GRF already multiplied by the contact flags; lever is */
/* the world-frame vector from the CoM to each foot, p_f,i - p_c.  The body- */
/* frame torque of Eq. (1), sum_i C(p_cf,i) x C(Gamma_i), equals             */
/* R^T sum_i (p_f,i - p_c) x Gamma_i because a rotation preserves the cross   */
/* product.                                                                  */
void orc_srbd_deriv(const orc_cfg *cfg, const double x[12], const double u[12],
                    const double lever[12], double xdot[12]) {
  const double *phi = &x[3], *v = &x[6], *w = &x[9];
  double R[9], E[9];
  orc_rotation(phi, R);
  orc_euler_rate_matrix(phi, E);
  /* p_dot = v */
  for (int c = 0; c < 3; ++c) xdot[c] = v[c];
  /* Phi_dot = E'^-1 omega */
  for (int r = 0; r < 3; ++r) {
    double s = 0.0;
    for (int c = 0; c < 3; ++c) s += E[3 * r + c] * w[c];
    xdot[3 + r] = s;
  }
  /* v_dot = (1/m) sum_i Gamma_i + g */
  double F[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < 4; ++i)
    for (int c = 0; c < 3; ++c) F[c] += u[3 * i + c];
  xdot[6] = F[0] / cfg->mass;
  xdot[7] = F[1] / cfg->mass;
  xdot[8] = F[2] / cfg->mass - cfg->gravity;
  /* omega_dot = I^-1 (C(p_cf) x C(Gamma) summed - omega x (I omega)) */
  double tw[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < 4; ++i) {
    double t[3];
    cross3(&lever[3 * i], &u[3 * i], t);
    for (int c = 0; c < 3; ++c) tw[c] += t[c];
  }
  double tau[3];
  for (int r = 0; r < 3; ++r) {
    double s = 0.0;
    for (int c = 0; c < 3; ++c) s += R[3 * c + r] * tw[c]; /* R^T */
    tau[r] = s;
  }
  double Iw[3] = {cfg->inertia[0] * w[0], cfg->inertia[1] * w[1], cfg->inertia[2] * w[2]};
  double gyro[3];
  cross3(w, Iw, gyro);
  for (int c = 0; c < 3; ++c) xdot[9 + c] = (tau[c] - gyro[c]) / cfg->inertia[c];
}

/* Foothold reference, Eq. (2): p_f = p_hip + (T_st/2) v^d +                  */
/* sqrt(p_c,z / g) (v_c - v^d), with p_hip = p_c + R h_i the hip of leg i,    */
/* T_st = D_f / f_s the stance time of the sample's gait, v^d = v_ref, and   */
/* the foot on flat ground at z = 0.                                        */
void orc_foothold(const orc_cfg *cfg, const double x[12], uint32_t q,
                  const double v_ref[3], int32_t leg, double out[3]) {
  double R[9];
  orc_rotation(&x[3], R);
  double f = orc_freq_of_q(q, cfg->dt);
  double half_tst = (q > 0u) ? 0.5 * cfg->duty / f : 0.0;
  double zc = x[2] > 0.0 ? x[2] : 0.0;
  double cap = sqrt(zc / cfg->gravity);
  for (int c = 0; c < 2; ++c) {
    double hip = x[c];
    for (int k = 0; k < 3; ++k) hip += R[3 * c + k] * cfg->hip[3 * leg + k];
    out[c] = hip + half_tst * v_ref[c] + cap * (x[6 + c] - v_ref[c]);
  }
  out[2] = 0.0;
}

/* ------------------------------------------------------------------------ */
/* Rollout(theta_k), Alg. 2: for j = 0..H-1, u_j = pi(theta_k, x_j, t_j),     */
/* J += r(u_j, x_j, x^r_j), x_{j+1} = x_j + dt F(x_j, u_j) (explicit Euler).  */
/* The stage cost is the quadratic form of Sec. V; the gait frequency adds   */
/* rho (f_k - f_n)^2 once (Sec. V).  theta is [H][12] world-frame GRFs, or   */
/* [P][12] spline knots whose interpolant gives the GRFs of each step.       */
/* Feet stay where they touched down: legs in stance at the first step use   */
/* the tick's footholds, a leg that touches down later is placed by Eq. (2)  */
/* from the state at that step.                                             */
/* xs, if not NULL, receives the H+1 states; feet, if not NULL, the H x 12   */
/* footholds in use at each step.                                           */
/* ------------------------------------------------------------------------ */
double orc_rollout(const orc_cfg *cfg, const orc_input *in, const double *theta,
                   uint32_t q, double *xs, double *feet) {
  double x[12], pf[12];
  int32_t prev[4] = {0, 0, 0, 0};
  memcpy(x, in->x0, sizeof x);
  memcpy(pf, in->foot_pos, sizeof pf);
  if (xs) memcpy(xs, x, sizeof x);
  double J = 0.0;
  for (int32_t j = 0; j < cfg->H; ++j) {
    int32_t delta[4];
    int nst = orc_contact(cfg, in->phase_robot, q, j, delta);
    for (int i = 0; i < 4; ++i)
      if (j > 0 && delta[i] && !prev[i]) orc_foothold(cfg, x, q, in->v_ref, i, &pf[3 * i]);
    if (feet) memcpy(&feet[12 * j], pf, sizeof pf);
    double u[12], ur[12], lever[12], grf[12];
    double share = cfg->mass * cfg->gravity / (nst > 1 ? (double)nst : 1.0);
    if (cfg->knots > 0) orc_spline_eval(cfg, theta, (double)j * cfg->dt, grf);
    else memcpy(grf, &theta[12 * j], sizeof grf);
    for (int i = 0; i < 4; ++i) {
      double f[3];
      const double *th = &grf[3 * i];
      if (cfg->friction_on) orc_friction_clip(th, cfg->mu_fric, f);
      else { f[0] = th[0]; f[1] = th[1]; f[2] = th[2]; }
      for (int c = 0; c < 3; ++c) {
        u[3 * i + c] = delta[i] ? f[c] : 0.0;
        lever[3 * i + c] = pf[3 * i + c] - x[c];
      }
      ur[3 * i + 0] = 0.0;
      ur[3 * i + 1] = 0.0;
      ur[3 * i + 2] = delta[i] ? share : 0.0;
    }
    /* reference x^r_j: position moves with v_ref, level attitude, yaw_ref */
    double t = (double)j * cfg->dt;
    double xr[12] = {in->p_ref0[0] + t * in->v_ref[0],
                     in->p_ref0[1] + t * in->v_ref[1],
                     in->p_ref0[2] + t * in->v_ref[2],
                     0.0, 0.0, in->yaw_ref,
                     in->v_ref[0], in->v_ref[1], in->v_ref[2],
                     0.0, 0.0, 0.0};
    double stage = 0.0;
    for (int d = 0; d < 12; ++d) {
      double e = x[d] - xr[d];
      stage += cfg->Q[d] * e * e;
    }
    for (int d = 0; d < 12; ++d) {
      double e = u[d] - ur[d];
      stage += cfg->R[d] * e * e;
    }
    J += stage;
    double xd[12];
    orc_srbd_deriv(cfg, x, u, lever, xd);
    for (int d = 0; d < 12; ++d) x[d] = x[d] + cfg->dt * xd[d];
    for (int i = 0; i < 4; ++i) prev[i] = delta[i];
    if (xs) memcpy(&xs[12 * (j + 1)], x, sizeof x);
  }
  double fk = orc_freq_of_q(q, cfg->dt);
  double df = fk - cfg->f_nominal;
  J += cfg->rho * df * df;
  if (!isfinite(J)) J = INFINITY;
  return J;
}

/* ------------------------------------------------------------------------ */
/* GRF spline, Sec. IV-B: the decision variable holds P knots theta_2 at      */
/* instants t^knot_p spread evenly from the first to the last step of the    */
/* horizon, t_p = p (H - 1) dt / (P - 1).  Between knots the force is the     */
/* cubic Hermite interpolant whose slopes are finite differences of the      */
/* knots: centred inside, one-sided at the two ends.  Outside [t_0, t_{P-1}]  */
/* the argument is clamped to the nearest end.                               */
/* ------------------------------------------------------------------------ */
double orc_knot_time(const orc_cfg *cfg, int32_t p) {
  return (double)p * ((double)(cfg->H - 1) * cfg->dt) / (double)(cfg->knots - 1);
}

static double knot_slope(const orc_cfg *cfg, const double *theta, int32_t p, int d) {
  const int32_t P = cfg->knots;
  int32_t a = p > 0 ? p - 1 : 0, b = p < P - 1 ? p + 1 : P - 1;
  return (theta[12 * b + d] - theta[12 * a + d]) / (orc_knot_time(cfg, b) - orc_knot_time(cfg, a));
}

void orc_spline_eval(const orc_cfg *cfg, const double *theta, double t, double out[12]) {
  const int32_t P = cfg->knots;
  const double T = orc_knot_time(cfg, P - 1);
  if (t < 0.0) t = 0.0;
  if (t > T) t = T;
  int32_t p = 0;
  while (p < P - 2 && t >= orc_knot_time(cfg, p + 1)) ++p;  /* segment [t_p, t_{p+1}] */
  const double t0 = orc_knot_time(cfg, p), t1 = orc_knot_time(cfg, p + 1);
  const double h = t1 - t0, s = (t - t0) / h;
  const double s2 = s * s, s3 = s2 * s;
  const double h00 = 2.0 * s3 - 3.0 * s2 + 1.0, h10 = s3 - 2.0 * s2 + s;
  const double h01 = -2.0 * s3 + 3.0 * s2, h11 = s3 - s2;
  for (int d = 0; d < 12; ++d)
    out[d] = h00 * theta[12 * p + d] + h10 * h * knot_slope(cfg, theta, p, d) +
             h01 * theta[12 * (p + 1) + d] + h11 * h * knot_slope(cfg, theta, p + 1, d);
}

/* ------------------------------------------------------------------------ */
/* MPPI, Alg. 4: beta = lowest cost, w_k = exp(-(J_k - beta)/lambda),        */
/* Omega = sum w_k, omega_k = w_k / Omega.  Returns ORC_FLAG_NONFINITE (and  */
/* all-zero omega) when no cost is finite.                                   */
/* ------------------------------------------------------------------------ */
int orc_mppi_weights(int32_t n, const double *J, double lambda, double *omega,
                     double *beta, double *Omega) {
  double b = INFINITY;
  for (int32_t k = 0; k < n; ++k)
    if (J[k] < b) b = J[k];
  *beta = b;
  if (!isfinite(b)) {
    for (int32_t k = 0; k < n; ++k) omega[k] = 0.0;
    *Omega = 0.0;
    return ORC_FLAG_NONFINITE;
  }
  double W = 0.0;
  for (int32_t k = 0; k < n; ++k) {
    omega[k] = exp(-(J[k] - b) / lambda);
    W += omega[k];
  }
  for (int32_t k = 0; k < n; ++k) omega[k] = omega[k] / W;
  *Omega = W;
  return 0;
}

/* theta_new = sum_k omega_k theta_k, theta is [n][d]. */
void orc_weighted_mean(int32_t n, int32_t d, const double *omega, const double *theta,
                       double *mean) {
  for (int32_t c = 0; c < d; ++c) mean[c] = 0.0;
  for (int32_t k = 0; k < n; ++k)
    for (int32_t c = 0; c < d; ++c) mean[c] += omega[k] * theta[(size_t)k * d + c];
}

/* ------------------------------------------------------------------------ */
/* Elite set, Alg. 1: sort ascending by cost (ties by sample index) and keep */
/* the first K_e.                                                            */
/* ------------------------------------------------------------------------ */
int32_t orc_elite_count(int32_t n, double elite_frac) {
  double v = floor(elite_frac * (double)n);
  int32_t ke = (int32_t)v;
  if (ke < 1) ke = 1;
  if (ke > n) ke = n;
  return ke;
}

typedef struct { double J; int32_t k; } cost_key;

static int cmp_cost_key(const void *a, const void *b) {
  const cost_key *x = (const cost_key *)a, *y = (const cost_key *)b;
  if (x->J < y->J) return -1;
  if (x->J > y->J) return 1;
  return (x->k > y->k) - (x->k < y->k);
}

void orc_elite_select(int32_t n, const double *J, int32_t ke, int32_t *idx) {
  cost_key *keys = (cost_key *)malloc(sizeof(cost_key) * (size_t)n);
  for (int32_t k = 0; k < n; ++k) { keys[k].J = J[k]; keys[k].k = k; }
  qsort(keys, (size_t)n, sizeof(cost_key), cmp_cost_key);
  for (int32_t e = 0; e < ke; ++e) idx[e] = keys[e].k;
  free(keys);
}

/* Maximum-likelihood mean and variance (1/K_e) over the elite samples. */
void orc_elite_moments(int32_t ke, int32_t d, const int32_t *idx, const double *theta,
                       double *mean, double *var) {
  for (int32_t c = 0; c < d; ++c) {
    double s = 0.0;
    for (int32_t e = 0; e < ke; ++e) s += theta[(size_t)idx[e] * d + c];
    mean[c] = s / (double)ke;
    double v = 0.0;
    for (int32_t e = 0; e < ke; ++e) {
      double dv = theta[(size_t)idx[e] * d + c] - mean[c];
      v += dv * dv;
    }
    var[c] = v / (double)ke;
  }
}

/* ------------------------------------------------------------------------ */
/* One control step, Alg. 5 (one or more SBS iterations from the same x0),   */
/* followed by the warm start of Sec. III-A.                                 */
/* ------------------------------------------------------------------------ */
typedef struct {
  const orc_cfg *cfg;
  const orc_input *in;
  const double *mu, *sigma;
  double mu_f, sigma_f;
  uint32_t tick, r;
  int32_t k0, k1;
  double *theta;   /* [N][M*12], M = H or the knot count */
  uint32_t *q;     /* [N] */
  double *J;       /* [N] */
  int rollout;
} worker_args;

static int32_t decision_rows(const orc_cfg *cfg) { return cfg->knots > 0 ? cfg->knots : cfg->H; }

static void *sample_and_rollout(void *arg) {
  worker_args *a = (worker_args *)arg;
  const orc_cfg *cfg = a->cfg;
  const int32_t M = decision_rows(cfg), D = 12 * M;
  for (int32_t k = a->k0; k < a->k1; ++k) {
    double *th = &a->theta[(size_t)k * D];
    for (int32_t j = 0; j < M; ++j) {
      float z[12];
      orc_noise_step(cfg->seed, a->tick, a->r, (uint32_t)k, (uint32_t)j, z);
      for (int d = 0; d < 12; ++d)
        th[12 * j + d] = a->mu[12 * j + d] + a->sigma[12 * j + d] * (double)z[d];
    }
    a->q[k] = orc_freq_q(cfg, a->mu_f, a->sigma_f, a->tick, a->r, (uint32_t)k);
    if (a->rollout) a->J[k] = orc_rollout(cfg, a->in, th, a->q[k], NULL, NULL);
  }
  return NULL;
}

int orc_tick(const orc_cfg *cfg, double *mu, double *mu_f, uint32_t tick,
             const orc_input *in, orc_action *out, double *costs_out,
             const double *costs_override, double *mean_out, uint32_t *q_out,
             int32_t nthreads) {
  const int32_t N = cfg->N, H = cfg->H, R = cfg->iterations;
  const int32_t M = decision_rows(cfg), D = 12 * M;
  if (N < 1 || H < 1 || R < 1) return -1;
  if (cfg->knots < 0 || cfg->knots == 1 || cfg->knots > H) return -1;
  if (cfg->freq_mode == ORC_FREQ_SET && (cfg->n_fset < 1 || cfg->n_fset > 4)) return -1;
  for (int d = 0; d < 12; ++d)
    if (!isfinite(in->x0[d])) return -1;
  if (nthreads < 1) nthreads = 1;
  if (nthreads > N) nthreads = N;

  double *theta = (double *)malloc(sizeof(double) * (size_t)N * D);
  double *J = (double *)malloc(sizeof(double) * (size_t)N);
  double *w = (double *)malloc(sizeof(double) * (size_t)N);
  double *fk = (double *)malloc(sizeof(double) * (size_t)N);
  uint32_t *q = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)N);
  int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
  double *cur = (double *)malloc(sizeof(double) * (size_t)D);
  double *sig = (double *)malloc(sizeof(double) * (size_t)D);
  double *var = (double *)malloc(sizeof(double) * (size_t)D);
  pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
  worker_args *args = (worker_args *)malloc(sizeof(worker_args) * (size_t)nthreads);

  memcpy(cur, mu, sizeof(double) * (size_t)D);
  for (int32_t c = 0; c < D; ++c) sig[c] = cfg->sigma_grf; /* sigma reset every tick */
  double mf = *mu_f, sf = cfg->sigma_f;
  double beta = INFINITY;
  int flags = 0;
  int32_t best = 0;

  for (int32_t r = 0; r < R; ++r) {
    /* Sampling and Evaluation, in parallel over samples */
    for (int t = 0; t < nthreads; ++t) {
      args[t] = (worker_args){cfg, in, cur, sig, mf, sf, tick, (uint32_t)r,
                              (int32_t)((int64_t)N * t / nthreads),
                              (int32_t)((int64_t)N * (t + 1) / nthreads),
                              theta, q, J, costs_override == NULL};
      pthread_create(&th[t], NULL, sample_and_rollout, &args[t]);
    }
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    if (costs_override)
      for (int32_t k = 0; k < N; ++k)
        J[k] = isfinite(costs_override[(size_t)r * N + k]) ? costs_override[(size_t)r * N + k]
                                                            : INFINITY;
    if (costs_out) memcpy(&costs_out[(size_t)r * N], J, sizeof(double) * (size_t)N);
    if (q_out) memcpy(&q_out[(size_t)r * N], q, sizeof(uint32_t) * (size_t)N);
    for (int32_t k = 0; k < N; ++k) fk[k] = orc_freq_of_q(q[k], cfg->dt);

    /* Sorting is only needed as far as each update uses it. */
    beta = INFINITY;
    best = 0;
    for (int32_t k = 0; k < N; ++k)
      if (J[k] < beta) { beta = J[k]; best = k; }
    if (!isfinite(beta)) { flags |= ORC_FLAG_NONFINITE; continue; }

    if (cfg->method == ORC_MPPI) {
      double b, W, fnew;
      orc_mppi_weights(N, J, cfg->lambda, w, &b, &W);
      orc_weighted_mean(N, D, w, theta, cur);
      orc_weighted_mean(N, 1, w, fk, &fnew);
      mf = fnew;
    } else if (cfg->method == ORC_NAIVE) {
      memcpy(cur, &theta[(size_t)best * D], sizeof(double) * (size_t)D);
      mf = fk[best];
    } else {
      int32_t ke = orc_elite_count(N, cfg->elite_frac);
      double fm, fv;
      orc_elite_select(N, J, ke, idx);
      orc_elite_moments(ke, D, idx, theta, cur, var);
      orc_elite_moments(ke, 1, idx, fk, &fm, &fv);
      double smin2 = cfg->sigma_min_grf * cfg->sigma_min_grf;
      for (int32_t c = 0; c < D; ++c) sig[c] = sqrt(var[c] > smin2 ? var[c] : smin2);
      double fmin2 = cfg->sigma_min_f * cfg->sigma_min_f;
      sf = sqrt(fv > fmin2 ? fv : fmin2);
      mf = fm;
    }
  }

  if (mean_out) memcpy(mean_out, cur, sizeof(double) * (size_t)D);

  /* Action: first step of the updated mean, masked and clipped as in the   */
  /* rollout, passed to the low-level controller (Sec. IV, Fig. 2).          */
  uint32_t qf = (cfg->freq_mode == ORC_FREQ_FIXED) ? orc_q_of_freq(cfg->f_fixed, cfg->dt)
                                                    : orc_q_of_freq(mf, cfg->dt);
  int32_t delta[4];
  orc_contact(cfg, in->phase_robot, qf, 0, delta);
  for (int i = 0; i < 4; ++i) {
    double f[3];
    if (cfg->friction_on) orc_friction_clip(&cur[3 * i], cfg->mu_fric, f);
    else { f[0] = cur[3 * i]; f[1] = cur[3 * i + 1]; f[2] = cur[3 * i + 2]; }
    for (int c = 0; c < 3; ++c) out->grf[3 * i + c] = delta[i] ? f[c] : 0.0;
    out->contact[i] = delta[i];
  }
  out->freq_hz = (cfg->freq_mode == ORC_FREQ_FIXED) ? cfg->f_fixed : mf;
  out->q = qf;
  out->best_cost = beta;
  out->flags = flags;

  /* Warm start: shift by one step, hover forces (m g / 2 per leg) at the   */
  /* end; the frequency mean carries over.  A spline mean is shifted by      */
  /* re-sampling it one step later at every knot but the last, which takes   */
  /* the hover forces.                                                       */
  for (int32_t j = 0; j + 1 < M; ++j) {
    if (cfg->knots > 0) orc_spline_eval(cfg, cur, orc_knot_time(cfg, j) + cfg->dt, &mu[12 * j]);
    else memcpy(&mu[12 * j], &cur[12 * (j + 1)], sizeof(double) * 12);
  }
  for (int i = 0; i < 4; ++i) {
    mu[12 * (M - 1) + 3 * i + 0] = 0.0;
    mu[12 * (M - 1) + 3 * i + 1] = 0.0;
    mu[12 * (M - 1) + 3 * i + 2] = 0.5 * cfg->mass * cfg->gravity;
  }
  *mu_f = (cfg->freq_mode == ORC_FREQ_FIXED) ? cfg->f_fixed : mf;

  free(theta); free(J); free(w); free(fk); free(q); free(idx);
  free(cur); free(sig); free(var); free(th); free(args);
  return 0;
}
