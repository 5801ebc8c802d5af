"""Pins of the oracle's rollout: SRBD model Eq. (1), explicit Euler of the
discretised dynamics (Sec. IV-A), contact schedule (Sec. IV-C), friction cone
(Sec. IV-B) and the quadratic tracking cost (Sec. V).

The pins use closed forms (free fall, ballistic flight, hover, torque-free
spin), scipy's rotation conventions, the momentum theorems of a rigid body and
brute force over the gait schedule.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from paper_2403_11383_amd import workloads


def cfg0(**over):
    return workloads.config("c0", **over)


def rot_scipy(phi):
    # intrinsic z-y'-x'' = Rz(yaw) Ry(pitch) Rx(roll)
    return Rotation.from_euler("ZYX", [phi[2], phi[1], phi[0]]).as_matrix()


def test_rotation_matches_scipy(orc):
    rng = np.random.default_rng(0)
    for _ in range(200):
        phi = rng.uniform(-1.4, 1.4, 3)
        R = orc.rotation(phi)
        np.testing.assert_allclose(R, rot_scipy(phi), atol=1e-14)
        np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-14)


def test_euler_rate_matrix_by_finite_differences(orc):
    """Phi_dot = E'^-1 omega must make dR/dt = R [omega]x (omega in body frame)."""
    rng = np.random.default_rng(1)
    h = 1e-5
    for _ in range(100):
        phi = rng.uniform(-1.2, 1.2, 3)
        w = rng.normal(size=3)
        dphi = orc.euler_rate_matrix(phi) @ w
        dR = (rot_scipy(phi + h * dphi) - rot_scipy(phi - h * dphi)) / (2 * h)
        wx = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
        np.testing.assert_allclose(dR, rot_scipy(phi) @ wx, atol=1e-8)


def test_linear_momentum_theorem(orc):
    """m v_dot = sum of GRFs + m g (Eq. (1), second row)."""
    rng = np.random.default_rng(2)
    c = cfg0()
    for _ in range(50):
        x = rng.normal(size=12) * 0.3
        u = rng.normal(size=12) * 50
        xd = orc.srbd_deriv(c, x, u, rng.normal(size=12) * 0.3)
        np.testing.assert_allclose(xd[0:3], x[6:9], rtol=0, atol=0)
        F = u.reshape(4, 3).sum(0)
        np.testing.assert_allclose(c["mass"] * xd[6:9], F + np.array([0, 0, -c["mass"] * c["gravity"]]),
                                   rtol=1e-13, atol=1e-12)


def test_angular_momentum_theorem(orc):
    """d/dt (R I omega) = sum_i (p_f,i - p_c) x Gamma_i: the world-frame torque
    of the GRFs about the CoM (Eq. (1), fourth row)."""
    rng = np.random.default_rng(3)
    c = cfg0()
    I = np.diag(c["inertia"])
    for _ in range(100):
        x = rng.normal(size=12) * 0.4
        u = rng.normal(size=12) * 60
        lever = rng.normal(size=(4, 3)) * 0.3
        xd = orc.srbd_deriv(c, x, u, lever)
        R = rot_scipy(x[3:6])
        w, wd = x[9:12], xd[9:12]
        lhs = R @ (np.cross(w, I @ w) + I @ wd)
        rhs = sum(np.cross(lever[i], u[3 * i:3 * i + 3]) for i in range(4))
        np.testing.assert_allclose(lhs, rhs, rtol=1e-12, atol=1e-10)


def test_torque_free_energy_conserved_by_derivative(orc):
    rng = np.random.default_rng(4)
    c = cfg0()
    I = np.diag(c["inertia"])
    for _ in range(50):
        x = rng.normal(size=12)
        xd = orc.srbd_deriv(c, x, np.zeros(12), rng.normal(size=12))
        assert abs(x[9:12] @ I @ xd[9:12]) < 1e-12


def _zero_theta(H, value=(0.0, 0.0, 0.0)):
    return np.tile(np.array(value * 4, dtype=np.float64), (H, 1))


def test_free_fall_closed_form(orc):
    """No foot in contact (duty 0): explicit Euler gives
    v_j = v0 + j dt g and p_j = p0 + j dt v0 + j(j-1)/2 dt^2 g exactly."""
    c = cfg0(duty=0.0, H=40)
    rng = np.random.default_rng(5)
    x0 = [0.1, -0.2, 0.35, 0, 0, 0, *rng.uniform(-0.3, 0.3, 3), 0, 0, 0]
    theta = rng.normal(size=(40, 12)) * 80  # ignored: no stance leg
    J, xs, _ = orc.rollout(c, workloads.tick_input(x0), theta, 120259084, return_states=True)
    g = np.array([0, 0, -c["gravity"]])
    dt = c["dt"]
    for j in range(41):
        v = np.array(x0[6:9]) + j * dt * g
        p = np.array(x0[0:3]) + j * dt * np.array(x0[6:9]) + 0.5 * j * (j - 1) * dt * dt * g
        np.testing.assert_allclose(xs[j, 6:9], v, atol=1e-12)
        np.testing.assert_allclose(xs[j, 0:3], p, atol=1e-12)
        np.testing.assert_array_equal(xs[j, 3:6], 0.0)
        np.testing.assert_array_equal(xs[j, 9:12], 0.0)
    # and it approaches the continuous parabola as O(dt)
    t = 40 * dt
    cont = np.array(x0[0:3]) + t * np.array(x0[6:9]) + 0.5 * t * t * g
    assert np.abs(xs[40, 0:3] - cont).max() <= 0.5 * t * dt * c["gravity"] + 1e-12


def test_ballistic_constant_force(orc):
    """All feet in contact (duty 1) with constant world forces: the CoM moves
    with a = sum F / m + g whatever the attitude does."""
    c = cfg0(duty=1.0, H=30)
    rng = np.random.default_rng(6)
    f = rng.normal(size=12) * 40
    theta = np.tile(f, (30, 1))
    x0 = [0, 0, 0.35, 0.1, -0.05, 0.2, *rng.uniform(-0.3, 0.3, 3), *rng.uniform(-0.3, 0.3, 3)]
    J, xs, _ = orc.rollout(c, workloads.tick_input(x0), theta, 120259084, return_states=True)
    a = f.reshape(4, 3).sum(0) / c["mass"] + np.array([0, 0, -c["gravity"]])
    dt = c["dt"]
    for j in range(31):
        np.testing.assert_allclose(xs[j, 6:9], np.array(x0[6:9]) + j * dt * a, atol=1e-11)
        np.testing.assert_allclose(
            xs[j, 0:3], np.array(x0[0:3]) + j * dt * np.array(x0[6:9]) + 0.5 * j * (j - 1) * dt * dt * a,
            atol=1e-11)


def test_hover_cost_closed_form(orc):
    """Level stand on four feet below the hips, each carrying m g / 4: no net
    force or torque, so the state never moves, the GRF cost vanishes and the
    cost is sum_j (0.3 j dt)^2 + 0.3^2 = 2.4264 at H = 25, dt = 0.02."""
    c = cfg0(duty=1.0)
    theta = _zero_theta(25, (0.0, 0.0, 0.25 * c["mass"] * c["gravity"]))
    x0 = [0, 0, 0.35, 0, 0, 0, 0, 0, 0, 0, 0, 0]
    for phase in (0, 12345, 1 << 31, 0xFFFFFFFF):
        J, xs, _ = orc.rollout(c, workloads.tick_input(x0, phase_robot=phase), theta, 120259084,
                               return_states=True)
        assert abs(J - 2.4264) < 1e-12
        np.testing.assert_allclose(xs, np.tile(x0, (26, 1)), atol=1e-13)


def test_trot_hover_without_reference_motion(orc):
    """Under a trot with v_ref = 0 every touchdown lands straight below its
    hip (Eq. (2) with v = v^d = 0), the stance pair carries m g / 2 each and
    the body stays at rest: J = 0."""
    c = cfg0()
    theta = _zero_theta(25, (0.0, 0.0, 0.5 * c["mass"] * c["gravity"]))
    x0 = [0, 0, 0.35, 0, 0, 0, 0, 0, 0, 0, 0, 0]
    J, xs, feet = orc.rollout(c, workloads.tick_input(x0, v_ref=(0, 0, 0)), theta, 120259084,
                              return_states=True)
    assert abs(J) < 1e-20
    np.testing.assert_allclose(xs, np.tile(x0, (26, 1)), atol=1e-14)
    np.testing.assert_allclose(feet, np.tile(np.array(workloads.feet_under_hips(x0)), (25, 1, 1)),
                               atol=1e-15)


def test_footholds_follow_eq2(orc):
    """Feet stay put during stance; a touchdown at step j lands at
    p_hip + (T_st/2) v^d + sqrt(z/g)(v - v^d) on the ground (Eq. (2)), where
    T_st = D_f / f_s; legs in stance at the first step keep the tick's feet."""
    c = cfg0(H=40)
    rng = np.random.default_rng(12)
    x0 = workloads.initial_state(rng)
    x0[3:6] = rng.uniform(-0.1, 0.1, 3)
    feet0 = np.array(workloads.feet_under_hips(x0)) + rng.normal(size=(4, 3)) * 0.01
    inp = workloads.tick_input(x0, v_ref=(0.3, 0.1, 0.0), foot_pos=feet0, phase_robot=77777)
    theta = np.tile([0.0, 0.0, 105.0] * 4, (40, 1)) + rng.normal(size=(40, 12)) * 5
    q = orc.q_of_freq(1.8, 0.02)
    J, xs, feet = orc.rollout(c, inp, theta, q, return_states=True)
    hips = np.array(c["hip"])
    f = q / (0.02 * 2**32)
    vd = np.array([0.3, 0.1, 0.0])
    touchdowns = 0
    for i in range(4):
        prev = None
        for j in range(40):
            d, _ = orc.contact(c, inp["phase_robot"], q, j)
            if j == 0 and d[i]:
                np.testing.assert_array_equal(feet[0, i], feet0[i])
            if j > 0 and d[i] and not prev:
                x = xs[j]
                R = rot_scipy(x[3:6])
                hip = x[0:3] + R @ hips[i]
                ref = hip + 0.5 * (0.5 / f) * vd + math.sqrt(x[2] / 9.81) * (x[6:9] - vd)
                np.testing.assert_allclose(feet[j, i, :2], ref[:2], atol=1e-13)
                assert feet[j, i, 2] == 0.0
                touchdowns += 1
            elif j > 0 and d[i]:
                np.testing.assert_array_equal(feet[j, i], feet[j - 1, i])
            prev = d[i]
    assert touchdowns >= 4


def test_torque_free_spin(orc):
    c = cfg0(duty=0.0, H=20)
    w = 0.7
    x0 = [0, 0, 0.35, 0, 0, 0, 0, 0, 0, 0, 0, w]
    J, xs, _ = orc.rollout(c, workloads.tick_input(x0), _zero_theta(20), 0, return_states=True)
    for j in range(21):
        assert xs[j, 11] == w and xs[j, 9] == 0 and xs[j, 10] == 0
        assert abs(xs[j, 5] - j * c["dt"] * w) < 1e-14
        assert xs[j, 3] == 0 and xs[j, 4] == 0


def test_stage_cost_counts_states_before_the_step(orc):
    """Alg. 2 accumulates r(u_i, x_i, x^r_i) for i = 0..H-1: the cost of an
    H = 1 rollout depends only on x_0 and u_0."""
    c = cfg0(H=1, duty=1.0)
    rng = np.random.default_rng(8)
    x0 = rng.normal(size=12) * 0.2
    th = rng.normal(size=(1, 12)) * 30
    inp = workloads.tick_input(x0, v_ref=(0.2, -0.1, 0.0), p_ref0=(0.05, 0.02, 0.33), yaw_ref=0.1)
    J = orc.rollout(c, inp, th, 0)
    xr = np.array([0.05, 0.02, 0.33, 0, 0, 0.1, 0.2, -0.1, 0, 0, 0, 0])
    share = c["mass"] * c["gravity"] / 4
    ur = np.tile([0, 0, share], 4)
    ref = np.sum((x0 - xr) ** 2) + 1e-4 * np.sum((th[0] - ur) ** 2)
    assert abs(J - ref) < 1e-12 * max(1.0, ref)


def test_friction_cone_invariants(orc):
    rng = np.random.default_rng(9)
    mu = 0.5
    for _ in range(500):
        f = rng.normal(size=3) * 50
        g = orc.friction_clip(f, mu)
        assert g[2] >= 0
        assert math.hypot(g[0], g[1]) <= mu * g[2] * (1 + 1e-12) + 1e-12
        np.testing.assert_allclose(orc.friction_clip(g, mu), g, rtol=1e-12, atol=1e-12)
        if f[2] < 0:
            np.testing.assert_array_equal(g, 0.0)
        elif math.hypot(f[0], f[1]) <= mu * f[2]:
            np.testing.assert_array_equal(g, f)
        else:  # radial projection keeps the tangential direction
            assert abs(math.atan2(g[1], g[0]) - math.atan2(f[1], f[0])) < 1e-12
            assert abs(math.hypot(g[0], g[1]) - mu * f[2]) < 1e-9


def test_contact_schedule_brute_force(orc):
    """Stance iff the leg phase lies in the first D_f of the cycle, so stance
    lasts D_f / f_s and swing (1 - D_f) / f_s (Sec. IV-C)."""
    c = cfg0()
    rng = np.random.default_rng(10)
    for _ in range(20):
        phase = int(rng.integers(0, 2**32))
        f = float(rng.uniform(1.0, 2.5))
        q = orc.q_of_freq(f, 0.02)
        steps = 2000
        stance = np.zeros((steps, 4), np.int32)
        for j in range(steps):
            d, n = orc.contact(c, phase, q, j)
            assert n == 2  # trot with duty 0.5: two diagonal legs at a time
            stance[j] = d
        np.testing.assert_array_equal(stance[:, 0], stance[:, 3])
        np.testing.assert_array_equal(stance[:, 1], 1 - stance[:, 0])
        assert abs(stance[:, 0].mean() - 0.5) < 2.0 / (steps * 0.02 * f) + 0.01
        # stance runs last D_f / f seconds (to one step)
        runs, cur = [], 0
        for v in stance[:, 0]:
            if v:
                cur += 1
            elif cur:
                runs.append(cur)
                cur = 0
        runs = runs[1:]  # the first run may be cut by the window
        for r in runs:
            assert abs(r * 0.02 - 0.5 / f) <= 0.02 + 1e-12
    # duty 0: never in stance; duty 1: always in stance
    for duty, n_exp in ((0.0, 0), (1.0, 4)):
        for j in range(10):
            d, n = orc.contact(cfg0(duty=duty), 123, 120259084, j)
            assert n == n_exp


def test_phase_boundary_counts_as_swing(orc):
    c = cfg0(phase_offset=[0, 0, 0, 0])
    d, _ = orc.contact(c, 1 << 31, 0, 0)
    assert list(d) == [0, 0, 0, 0]
    d, _ = orc.contact(c, (1 << 31) - 1, 0, 0)
    assert list(d) == [1, 1, 1, 1]


def test_frequency_regulariser(orc):
    """J gains rho (f_k - f_n)^2 once per rollout (Sec. V)."""
    c = cfg0(rho=2.0, H=5)
    theta = _zero_theta(5, (0.0, 0.0, 0.5 * c["mass"] * c["gravity"]))
    x0 = [0, 0, 0.35] + [0] * 9
    inp = workloads.tick_input(x0, v_ref=(0, 0, 0))
    q = orc.q_of_freq(2.2, 0.02)
    J = orc.rollout(c, inp, theta, q)
    f = orc.freq_of_q(q, 0.02)
    assert abs(J - 2.0 * (f - 1.4) ** 2) < 1e-12


def test_nonfinite_rollout_cost_is_inf(orc):
    c = cfg0(H=3)
    x0 = [0, 0, 0.35, 0, 0, 0, 1e200, 0, 0, 0, 0, 0]  # the squared error overflows
    th = _zero_theta(3)
    J = orc.rollout(c, workloads.tick_input(x0), th, 0)
    assert J == math.inf
    x0 = [0, 0, 0.35, 0, 0, 0, math.nan, 0, 0, 0, 0, 0]
    assert orc.rollout(c, workloads.tick_input(x0), th, 0) == math.inf


# ---------------------------------------------------------------------------
# Eq. (2) by hand: exact numbers chosen so that every term is a short decimal
# ---------------------------------------------------------------------------
def _foothold_cfg(**over):
    # dt = 1/64 s and f = 2 Hz make the phase increment q = 2^27 exact, so the
    # executed frequency is exactly 2 Hz and the stance time D_f / f = 0.25 s
    c = cfg0(dt=1.0 / 64.0, duty=0.5)
    c.update(over)
    return c


Q_2HZ = 1 << 27


def test_foothold_steady_gait_is_hip_plus_half_stance_times_vd(orc):
    """Eq. (2) with v = v^d: the capture term vanishes and the foot lands
    (T_st / 2) v^d ahead of the hip: 0.125 s x (0.4, -0.2) m/s = (0.05,
    -0.025) m."""
    c = _foothold_cfg()
    x = [1.0, 2.0, 0.35, 0.0, 0.0, 0.0, 0.4, -0.2, 0.0, 0.0, 0.0, 0.0]
    vd = (0.4, -0.2, 0.0)
    want = {0: (1.29, 2.105), 1: (1.29, 1.845), 2: (0.81, 2.105), 3: (0.81, 1.845)}
    for leg, (wx, wy) in want.items():
        f = orc.foothold(c, x, Q_2HZ, vd, leg)
        np.testing.assert_allclose(f, [wx, wy, 0.0], rtol=0, atol=1e-15)


def test_foothold_capture_term_at_zero_command(orc):
    """Eq. (2) with v^d = 0: the foot lands sqrt(z / g) v from the hip; with
    z = 0.4 m and g = 10 m/s^2 the factor is 0.2 s, so v = (0.3, -0.1) m/s
    moves it by (0.06, -0.02) m."""
    c = _foothold_cfg(gravity=10.0)
    x = [0.0, 0.0, 0.4, 0.0, 0.0, 0.0, 0.3, -0.1, 0.7, 0.0, 0.0, 0.0]
    f = orc.foothold(c, x, Q_2HZ, (0.0, 0.0, 0.0), 0)
    np.testing.assert_allclose(f, [0.30, 0.11, 0.0], rtol=0, atol=1e-15)
    # the vertical velocity and the stance time play no part at v^d = 0
    f2 = orc.foothold(c, x, Q_2HZ >> 1, (0.0, 0.0, 0.0), 0)
    np.testing.assert_allclose(f2, f, rtol=0, atol=1e-15)


def test_foothold_both_terms_and_yawed_hip(orc):
    """Both terms of Eq. (2) together on a body yawed by 90 degrees: the
    front-left hip (0.24, 0.13) then sits at (-0.13, 0.24) from the CoM; with
    v^d = (0.4, 0), v = (0.2, 0.1), z = 0.4, g = 10 and T_st = 0.25 s the
    foot lands at hip + 0.125 (0.4, 0) + 0.2 (-0.2, 0.1) = hip + (0.01, 0.02)."""
    c = _foothold_cfg(gravity=10.0)
    x = [0.0, 0.0, 0.4, 0.0, 0.0, math.pi / 2, 0.2, 0.1, 0.0, 0.0, 0.0, 0.0]
    f = orc.foothold(c, x, Q_2HZ, (0.4, 0.0, 0.0), 0)
    np.testing.assert_allclose(f, [-0.12, 0.26, 0.0], rtol=0, atol=1e-15)
    # a CoM below the ground keeps the foot under the hip term alone
    x[2] = -0.1
    f = orc.foothold(c, x, Q_2HZ, (0.4, 0.0, 0.0), 0)
    np.testing.assert_allclose(f, [-0.13 + 0.05, 0.24, 0.0], rtol=0, atol=1e-15)
