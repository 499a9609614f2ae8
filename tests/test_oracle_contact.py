"""Pins of the oracle's sphere contact (the Glowinski et al. 2001 short-range
repulsion the equations of motion add when contact is set; the paper itself
runs without a contact model).

Each check is a property of the force law rather than the law retyped:
special values (touching spheres give k, half the range gives k/4, zero at
the range), the force as minus the gradient of its potential
k zeta / 3 ((R_p + R_q + zeta - d) / zeta)^3 by central differences,
Newton's third law, superposition, translation invariance across a periodic
boundary, the wall as the mirror-image sphere, and the first step of the
equations of motion from rest (U = F_contact / m)."""
import numpy as np
import pytest

from paper_2312_14172_amd import workloads as W


@pytest.fixture(scope="module")
def O(oracle_mod):
    return oracle_mod


def _parts(O, orc, specs):
    recs = np.array([W.make_particle(sh, prm, pos) for sh, prm, pos in specs])
    return orc.to_parts(recs)


def _pair(O, R1, R2, d, direction=(0.3, -0.5, 0.8), k=0.7, zeta=1.3, n=(64, 64, 64)):
    orc = O.Oracle(n, (0, 0, 0))
    e = np.asarray(direction, float)
    e /= np.linalg.norm(e)
    X1 = np.array([20.0, 31.0, 26.0])
    P = _parts(O, orc, [(W.SPHERE, (R1,), X1), (W.SPHERE, (R2,), X1 - d * e)])
    return orc.contact_forces(P, (zeta, k, 0.0)), e


def test_special_values_and_direction(O):
    k, zeta = 0.7, 1.3
    F, e = _pair(O, 3.0, 2.0, 5.0, k=k, zeta=zeta)       # touching
    np.testing.assert_allclose(F[0], k * e, rtol=1e-14)
    F, e = _pair(O, 3.0, 2.0, 5.0 + zeta / 2, k=k, zeta=zeta)
    np.testing.assert_allclose(F[0], k / 4 * e, rtol=1e-13)
    F, _ = _pair(O, 3.0, 2.0, 5.0 + zeta, k=k, zeta=zeta)  # continuous at the range (up to rounding of d)
    assert np.abs(F).max() <= 1e-20
    for d in (5.0 + zeta + 0.1, 9.0):
        F, _ = _pair(O, 3.0, 2.0, d, k=k, zeta=zeta)
        assert np.all(F == 0.0)
    F, e = _pair(O, 3.0, 2.0, 4.2, k=k, zeta=zeta)        # overlapping: still repulsive, larger than k
    assert np.dot(F[0], e) > k and np.allclose(np.cross(F[0], e), 0.0, atol=1e-14)


def test_force_is_minus_gradient_of_potential(O):
    k, zeta, R1, R2 = 0.7, 1.3, 3.0, 2.0

    def U(d):
        s = (R1 + R2 + zeta - d) / zeta
        return k * zeta / 3.0 * s ** 3 if s > 0 else 0.0

    for d in (4.6, 5.2, 5.9, 6.25):
        F, e = _pair(O, R1, R2, d, k=k, zeta=zeta)
        h = 1e-6
        dU = (U(d + h) - U(d - h)) / (2 * h)
        np.testing.assert_allclose(np.dot(F[0], e), -dU, rtol=1e-8)


def test_third_law_and_superposition(O):
    orc = O.Oracle((48, 48, 48), (0, 0, 0))
    specs = [(W.SPHERE, (3.0,), (20.0, 20.0, 20.0)), (W.SPHERE, (2.5,), (25.6, 21.0, 19.5)),
             (W.SPHERE, (2.0,), (17.0, 15.6, 21.2)), (W.ROUNDED_CUBE, (3.0, 0.6), (36.0, 36.0, 36.0))]
    P = _parts(O, orc, specs)
    c = (1.1, 0.9, 0.0)
    F = orc.contact_forces(P, c)
    assert np.any(F[0] != 0) and np.all(F[3] == 0.0)      # the rounded cube is out of range
    np.testing.assert_allclose(F.sum(axis=0), 0.0, atol=1e-15)
    F01 = orc.contact_forces(P[[0, 1]], c)
    F02 = orc.contact_forces(P[[0, 2]], c)
    np.testing.assert_allclose(F[0], F01[0] + F02[0], rtol=1e-14)


def test_periodic_minimum_image(O):
    orc = O.Oracle((40, 40, 40), (0, 0, 0))
    c = (1.0, 0.5, 0.0)
    across = _parts(O, orc, [(W.SPHERE, (3.0,), (1.5, 20.0, 20.0)), (W.SPHERE, (3.0,), (34.8, 21.0, 19.0))])
    inside = _parts(O, orc, [(W.SPHERE, (3.0,), (21.5, 20.0, 20.0)), (W.SPHERE, (3.0,), (14.8, 21.0, 19.0))])
    Fa, Fi = orc.contact_forces(across, c), orc.contact_forces(inside, c)
    assert np.any(Fa != 0)
    np.testing.assert_allclose(Fa, Fi, rtol=1e-12)


def test_wall_acts_as_mirror_image(O):
    zeta, kw, R = 1.2, 0.4, 2.5
    for h in (2.0, 2.6, 3.0):
        walled = O.Oracle((32, 32, 32), (0, 0, 1))
        P = _parts(O, walled, [(W.SPHERE, (R,), (10.0, 12.0, h))])
        Fw = walled.contact_forces(P, (zeta, 0.0, kw))
        free = O.Oracle((32, 32, 64), (0, 0, 0))
        Q = _parts(O, free, [(W.SPHERE, (R,), (10.0, 12.0, 30.0 + h)), (W.SPHERE, (R,), (10.0, 12.0, 30.0 - h))])
        Fm = free.contact_forces(Q, (zeta, kw, 0.0))
        np.testing.assert_allclose(Fw[0], Fm[0], rtol=1e-14, atol=1e-300)
        top = O.Oracle((32, 32, 32), (0, 0, 1))
        Pt = _parts(O, top, [(W.SPHERE, (R,), (10.0, 12.0, 32.0 - h))])
        np.testing.assert_allclose(top.contact_forces(Pt, (zeta, 0.0, kw))[0], -Fw[0], rtol=1e-14)


def test_first_step_from_rest_moves_by_contact_force(O):
    """Resting spheres in a resting fluid: the momentum exchange gives zero, so
    after one step U = F_contact / m and X moved by U; without contact nothing
    moves."""
    n = (24, 24, 24)
    c = (1.0, 2e-3, 0.0)
    recs = np.array([W.make_particle(W.SPHERE, (3.0,), (10.2, 11.7, 12.1)),
                     W.make_particle(W.SPHERE, (2.5,), (15.4, 12.3, 11.6))])
    orc = O.Oracle(n, (0, 0, 0), contact=c)
    P = orc.to_parts(recs)
    Fc = orc.contact_forces(P)
    assert np.linalg.norm(Fc[0]) > 1e-4
    X0 = P["X"].copy()
    F, _ = orc.run(P, orc.equilibrium(), 1)
    assert np.all(F == 0.0)
    np.testing.assert_allclose(P["U"], Fc / recs["mass"][:, None], rtol=1e-13)
    np.testing.assert_allclose(P["X"] - X0, P["U"], rtol=0, atol=1e-14)
    plain = O.Oracle(n, (0, 0, 0))
    P2 = plain.to_parts(recs)
    plain.run(P2, plain.equilibrium(), 1)
    assert np.all(P2["U"] == 0.0)
