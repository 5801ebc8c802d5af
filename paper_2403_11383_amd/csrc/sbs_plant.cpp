// sbs_plant.cpp -- host FP64 single-rigid-body plant used as the simulated
// robot of closed-loop runs (the paper's experiments run MuJoCo; this plant
// stands in for it).  Same model as the controller: Eq. (1) with world-fixed
// footholds placed by Eq. (2) at touchdown, explicit Euler at the control
// step, plus an external wrench (world-frame force and torque) on the CoM.
#include <cmath>
#include <cstring>

#include "../../include/sbs.h"

namespace {

void rotation(const double *phi, double R[9]) {
  const double cr = std::cos(phi[0]), sr = std::sin(phi[0]);
  const double cp = std::cos(phi[1]), sp = std::sin(phi[1]);
  const double cy = std::cos(phi[2]), sy = std::sin(phi[2]);
  R[0] = cy * cp; R[1] = cy * sp * sr - sy * cr; R[2] = cy * sp * cr + sy * sr;
  R[3] = sy * cp; R[4] = sy * sp * sr + cy * cr; R[5] = sy * sp * cr - cy * sr;
  R[6] = -sp;     R[7] = cp * sr;                R[8] = cp * cr;
}

}  // namespace

extern "C" int sbs_plant_step_wrench(const sbs_controller_cfg *cfg, sbs_plant_state *st,
                                     const sbs_action *act, const double ext_wrench[6],
                                     const double v_ref[3]) {
  if (!cfg || !st || !act || !ext_wrench || !v_ref) return SBS_EINVAL;
  double *x = st->x;
  double R[9];
  rotation(&x[3], R);
  const double f = (double)act->q / (cfg->dt * 4294967296.0);
  const double half_tst = act->q ? 0.5 * cfg->duty / f : 0.0;
  const double cap = std::sqrt((x[2] > 0 ? x[2] : 0.0) / cfg->gravity);
  for (int l = 0; l < 4; ++l) {
    const bool stance = act->contact[l] != 0;
    if (stance && !st->contact[l]) {  // touchdown: Eq. (2)
      for (int c = 0; c < 2; ++c) {
        double hip = x[c];
        for (int k = 0; k < 3; ++k) hip += R[3 * c + k] * cfg->hip[3 * l + k];
        st->foot_pos[3 * l + c] = hip + half_tst * v_ref[c] + cap * (x[6 + c] - v_ref[c]);
      }
      st->foot_pos[3 * l + 2] = 0.0;
    }
    st->contact[l] = stance ? 1 : 0;
  }
  double F[3] = {ext_wrench[0], ext_wrench[1], ext_wrench[2]};
  double tw[3] = {ext_wrench[3], ext_wrench[4], ext_wrench[5]};
  for (int l = 0; l < 4; ++l) {
    if (!act->contact[l]) continue;
    const double *u = &act->grf[3 * l];
    const double lx = st->foot_pos[3 * l] - x[0], ly = st->foot_pos[3 * l + 1] - x[1],
                 lz = st->foot_pos[3 * l + 2] - x[2];
    F[0] += u[0]; F[1] += u[1]; F[2] += u[2];
    tw[0] += ly * u[2] - lz * u[1];
    tw[1] += lz * u[0] - lx * u[2];
    tw[2] += lx * u[1] - ly * u[0];
  }
  double tb[3];
  for (int r = 0; r < 3; ++r) tb[r] = R[r] * tw[0] + R[3 + r] * tw[1] + R[6 + r] * tw[2];
  const double *w = &x[9];
  const double I[3] = {cfg->inertia[0], cfg->inertia[1], cfg->inertia[2]};
  const double Iw[3] = {I[0] * w[0], I[1] * w[1], I[2] * w[2]};
  const double gy[3] = {w[1] * Iw[2] - w[2] * Iw[1], w[2] * Iw[0] - w[0] * Iw[2],
                        w[0] * Iw[1] - w[1] * Iw[0]};
  const double cr = std::cos(x[3]), sr = std::sin(x[3]), cp = std::cos(x[4]), tp = std::tan(x[4]);
  double xd[12];
  for (int c = 0; c < 3; ++c) xd[c] = x[6 + c];
  xd[3] = w[0] + (sr * w[1] + cr * w[2]) * tp;
  xd[4] = cr * w[1] - sr * w[2];
  xd[5] = (sr * w[1] + cr * w[2]) / cp;
  xd[6] = F[0] / cfg->mass;
  xd[7] = F[1] / cfg->mass;
  xd[8] = F[2] / cfg->mass - cfg->gravity;
  for (int c = 0; c < 3; ++c) xd[9 + c] = (tb[c] - gy[c]) / I[c];
  for (int c = 0; c < 12; ++c) x[c] += cfg->dt * xd[c];
  st->phase += act->q;
  return SBS_OK;
}

extern "C" int sbs_plant_step(const sbs_controller_cfg *cfg, sbs_plant_state *st,
                              const sbs_action *act, const double ext_force[3],
                              const double v_ref[3]) {
  if (!ext_force) return SBS_EINVAL;
  const double w[6] = {ext_force[0], ext_force[1], ext_force[2], 0.0, 0.0, 0.0};
  return sbs_plant_step_wrench(cfg, st, act, w, v_ref);
}

// One closed-loop cycle of a simulated robot, all in native code: the tick
// input from the plant (state estimate, world footholds, gait phase; the
// reference starts at the robot's horizontal position at height z_ref),
// submit, wait for the action, one plant step under it.
extern "C" int sbs_closed_loop_step(sbs_runtime *rt, int32_t id, const sbs_controller_cfg *cfg,
                                    sbs_plant_state *st, const double ext_wrench[6],
                                    const double v_ref[3], double z_ref, double yaw_ref,
                                    sbs_action *out) {
  if (!rt || !cfg || !st || !ext_wrench || !v_ref || !out) return SBS_EINVAL;
  sbs_tick_input in;
  std::memcpy(in.x0, st->x, sizeof in.x0);
  std::memcpy(in.foot_pos, st->foot_pos, sizeof in.foot_pos);
  in.p_ref0[0] = st->x[0];
  in.p_ref0[1] = st->x[1];
  in.p_ref0[2] = z_ref;
  for (int c = 0; c < 3; ++c) in.v_ref[c] = v_ref[c];
  in.yaw_ref = yaw_ref;
  in.phase_robot = st->phase;
  in.reserved0 = 0;
  uint64_t ticket = 0;
  int rc = sbs_submit_tick(rt, id, &in, &ticket);
  if (rc != SBS_OK) return rc;
  rc = sbs_fetch_action(rt, ticket, out, -1);
  if (rc != SBS_OK) return rc;
  return sbs_plant_step_wrench(cfg, st, out, ext_wrench, v_ref);
}
