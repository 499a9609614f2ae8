"""Pins of the CPU oracle's external force and equations of motion (Sec. 2.2
Newton and Euler equations; gravity and buoyancy of Sec. 5.1) against closed
forms: constant acceleration under semi-implicit Euler, free rotation about a
fixed axis, Euler's torque-free equations to first order, and fixed particles."""
import math

import numpy as np
import pytest

from paper_2312_14172_amd import workloads as W


def _rot(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _qmul(a, b):
    return np.array([a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3],
                     a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2],
                     a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1],
                     a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0]])


def test_constant_force_closed_form(oracle_mod):
    """With dt = 1: U_t = U_0 + t a and X_t = X_0 + t U_0 + a t (t + 1) / 2,
    a = (F + (m - rho_f V) g) / m (weight minus buoyancy, Sec. 5.1)."""
    g = (0.0, 0.0, -1e-5)
    orc = oracle_mod.Oracle((200, 200, 200), gravity=g, rho_f=1.0)
    rec = W.make_particle(W.SPHERE, (4.0,), (50.0, 60.0, 70.0), vel=(1e-3, -2e-3, 0.0),
                          density_ratio=2.0)
    P = orc.to_parts(np.array([rec]))
    F = np.array([[2e-3, 1e-3, -3e-3]])
    T = np.zeros((1, 3))
    m, V = rec["mass"], rec["volume"]
    acc = (F[0] + (m - V) * np.array(g)) / m
    for t in range(1, 31):
        orc.apply_eom(P, F, T)
        np.testing.assert_allclose(P["U"][0], rec["vel"] + t * acc, rtol=1e-13, atol=1e-18)
        np.testing.assert_allclose(P["X"][0], rec["pos"] + t * rec["vel"] + acc * t * (t + 1) / 2,
                                   rtol=1e-14)
    # buoyancy: a neutrally buoyant particle feels no gravity
    neutral = W.make_particle(W.SPHERE, (4.0,), (50.0, 60.0, 70.0), density_ratio=1.0)
    Pn = orc.to_parts(np.array([neutral]))
    orc.apply_eom(Pn, np.zeros((1, 3)), T)
    assert np.all(Pn["U"][0] == 0)


def test_periodic_wrap_of_position(oracle_mod):
    orc = oracle_mod.Oracle((20, 20, 20))
    rec = W.make_particle(W.SPHERE, (3.0,), (19.9, 0.05, 10.0), vel=(0.3, -0.2, 0.0))
    P = orc.to_parts(np.array([rec]))
    orc.apply_eom(P, np.zeros((1, 3)), np.zeros((1, 3)))
    np.testing.assert_allclose(P["X"][0], [0.2, 19.85, 10.0], atol=1e-12)


@pytest.mark.parametrize("seed", range(3))
def test_free_rotation_about_fixed_axis_is_exact(oracle_mod, seed):
    """A torque-free sphere keeps omega; the exponential map then gives
    q_t = q_0 (x) (cos(t|w_b|/2), sin(t|w_b|/2) w_b/|w_b|) exactly."""
    rng = np.random.default_rng(seed)
    orc = oracle_mod.Oracle((64, 64, 64))
    q0 = np.array(W.shoemake_quaternion(rng))
    om = 0.05 * rng.standard_normal(3)
    rec = W.make_particle(W.SPHERE, (4.0,), (30.0, 30.0, 30.0), quat=tuple(q0), omega=tuple(om))
    P = orc.to_parts(np.array([rec]))
    wb = _rot(q0).T @ om
    ang = np.linalg.norm(wb)
    for t in range(1, 41):
        orc.apply_eom(P, np.zeros((1, 3)), np.zeros((1, 3)))
        ref = _qmul(q0, np.concatenate([[math.cos(t * ang / 2)], math.sin(t * ang / 2) * wb / ang]))
        np.testing.assert_allclose(P["q"][0], ref, atol=2e-14)
        np.testing.assert_allclose(P["W"][0], om, atol=1e-15)
        assert abs(np.linalg.norm(P["q"][0]) - 1) < 1e-15


def test_torque_free_euler_equations_first_order(oracle_mod):
    """One step of size 1 with a small body angular velocity changes it by the
    textbook Euler equations: I1 dw1 = (I2 - I3) w2 w3 and cyclic."""
    orc = oracle_mod.Oracle((64, 64, 64))
    I = np.array([3.0, 5.0, 7.0])
    wb = np.array([2e-3, -1.5e-3, 1e-3])
    rec = W.make_particle(W.SPHEROID, (6.0, 3.0), (30, 30, 30), omega=tuple(wb))
    rec["inertia"] = I
    P = orc.to_parts(np.array([rec]))
    orc.apply_eom(P, np.zeros((1, 3)), np.zeros((1, 3)))
    wb_new = _rot(P["q"][0]).T @ P["W"][0]
    expect = wb + np.array([(I[1] - I[2]) * wb[1] * wb[2] / I[0],
                            (I[2] - I[0]) * wb[2] * wb[0] / I[1],
                            (I[0] - I[1]) * wb[0] * wb[1] / I[2]])
    np.testing.assert_allclose(wb_new, expect, rtol=0, atol=1e-17)
    # applied torque in the world frame enters through the body frame
    rng = np.random.default_rng(4)
    q0 = np.array(W.shoemake_quaternion(rng))
    rec2 = W.make_particle(W.SPHEROID, (6.0, 3.0), (30, 30, 30), quat=tuple(q0))
    rec2["inertia"] = I
    P2 = orc.to_parts(np.array([rec2]))
    Tw = np.array([[1e-4, -2e-4, 3e-4]])
    orc.apply_eom(P2, np.zeros((1, 3)), Tw)
    wb2 = _rot(P2["q"][0]).T @ P2["W"][0]
    np.testing.assert_allclose(wb2, (_rot(q0).T @ Tw[0]) / I, rtol=1e-12)


def test_fixed_particle_does_not_move(oracle_mod):
    orc = oracle_mod.Oracle((32, 32, 32), gravity=(0, 0, -1e-3))
    rec = W.make_particle(W.SPHERE, (4.0,), (16.0, 16.0, 16.0), vel=(0.01, 0, 0), fixed=True)
    P = orc.to_parts(np.array([rec]))
    before = P.copy()
    orc.apply_eom(P, np.ones((1, 3)), np.ones((1, 3)))
    assert P.tobytes() == before.tobytes()
