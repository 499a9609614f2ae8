"""Pins of the oracle's contact for non-spherical particles: the sphere
repulsion written as a volume law and evaluated on surface nodes against the
partner's signed distance (the oracle's header states the model).

The node sums are pinned against closed forms of the same integrals for
bodies of spherical shape taken through the non-spherical path (a spheroid
with equal semi-axes, a rounded cube whose corner radius equals its
half-size), where the integrals can be done by hand:
  * two equal spheres of radius R, centre distance D, range zeta: with
    A = zeta + R and L = D - R, the axial force is
        K (pi R / D^2) [ (D^2 - R^2) (A - L)^2 / 2 + A^4 / 12 - A L^3 / 3 + L^4 / 4 ],
    K = k / (pi (R / 2) zeta^2) (the surface integral of the depth times the
    axial component of the partner's normal, over both caps, halved);
  * a sphere at height H above a wall: exactly the mirror-image sphere law
    k_w ((2 R + zeta - 2 H) / zeta)^2.
Both are met to the quadrature error of the Fibonacci nodes (at 4096 nodes
0.2 % on the smallest contact patch, where the depth has a kink at the
patch edge; a wrong weight, a lost factor 1/2 or an unprojected normal each
move the force by 5 % or more).  Beyond those: Newton's third law and the balance of angular
momentum for rotated rounded cubes and spheroids, zero force beyond the
range, and the limit of the sphere law for R >> zeta."""
import numpy as np
import pytest

from paper_2312_14172_amd import workloads as W


@pytest.fixture(scope="module")
def O(oracle_mod):
    yield oracle_mod
    oracle_mod.Oracle.set_contact_nodes(1024)


def _closed_pair(R, D, zeta, k):
    A, L = zeta + R, D - R
    if L >= A:
        return 0.0
    c = D * D - R * R
    I = c * (A - L) ** 2 / 2 + A ** 4 / 12 - A * L ** 3 / 3 + L ** 4 / 4
    return k / (np.pi * (R / 2) * zeta ** 2) * (np.pi * R / D ** 2) * I


def _sphere_shaped(shape, R):
    return (R, R, 0.0)


@pytest.mark.parametrize("shape", [W.SPHEROID, W.ROUNDED_CUBE])
@pytest.mark.parametrize("gap", [1.5, 0.4, -0.5])
def test_pair_of_sphere_shaped_bodies_matches_closed_form(O, shape, gap):
    R, zeta, k = 6.0, 2.0, 0.8
    O.Oracle.set_contact_nodes(4096)
    orc = O.Oracle((64, 48, 48), (0, 0, 0))
    e = np.array([0.36, -0.48, 0.8])
    rng = np.random.default_rng(5)
    X1 = np.array([2.0, 20.0, 24.0])          # the pair straddles the periodic x face
    D = 2 * R + gap
    recs = [W.make_particle(shape, _sphere_shaped(shape, R), X1, quat=W.shoemake_quaternion(rng)),
            W.make_particle(shape, _sphere_shaped(shape, R), (X1 - D * e) % [64, 48, 48],
                            quat=W.shoemake_quaternion(rng))]
    F, T = orc.contact_forces(orc.to_parts(np.array(recs)), (zeta, k, 0.0), torque=True)
    ref = _closed_pair(R, D, zeta, k)
    np.testing.assert_allclose(F[0], ref * e, rtol=0, atol=3e-3 * ref)
    np.testing.assert_allclose(F[1], -ref * e, rtol=0, atol=3e-3 * ref)
    # central forces of a sphere: no torque beyond the quadrature noise
    assert np.abs(T).max() <= 3e-3 * ref * R


@pytest.mark.parametrize("side", [0, 1])
def test_sphere_shaped_body_at_a_wall_is_the_mirror_law(O, side):
    R, zeta, kw, nz = 5.0, 2.0, 0.6, 40
    O.Oracle.set_contact_nodes(4096)
    orc = O.Oracle((32, 32, nz), (0, 0, 1))
    for H in (5.4, 5.0, 4.6):
        z = H if side == 0 else nz - H
        recs = [W.make_particle(W.SPHEROID, (R, R, 0.0), (16.0, 15.0, z),
                                quat=W.shoemake_quaternion(np.random.default_rng(int(10 * H))))]
        F = orc.contact_forces(orc.to_parts(np.array(recs)), (zeta, 0.0, kw))
        ref = kw * ((2 * R + zeta - 2 * H) / zeta) ** 2
        np.testing.assert_allclose(F[0], [0.0, 0.0, ref if side == 0 else -ref], rtol=0, atol=3e-3 * ref)


def test_third_law_and_angular_momentum(O):
    O.Oracle.set_contact_nodes(1024)
    orc = O.Oracle((64, 64, 64), (1, 1, 1))
    rng = np.random.default_rng(9)
    cube = W.equal_volume_params(W.ROUNDED_CUBE, 5.0)
    sph = W.equal_volume_params(W.SPHEROID, 5.0)
    recs = [W.make_particle(W.ROUNDED_CUBE, cube, (30.0, 31.0, 29.0), quat=W.shoemake_quaternion(rng)),
            W.make_particle(W.SPHEROID, sph, (38.5, 33.0, 30.0), quat=W.shoemake_quaternion(rng)),
            W.make_particle(W.SPHERE, (4.0,), (31.0, 40.0, 30.5))]
    P = orc.to_parts(np.array(recs))
    F, T = orc.contact_forces(P, (2.0, 1.0, 0.0), torque=True)
    assert np.abs(F).max() > 1e-3                        # the bodies do touch
    scale = np.abs(F).max()
    np.testing.assert_allclose(F.sum(0), 0.0, atol=1e-13 * scale)
    X = np.array([r["pos"] for r in recs])
    L = T.sum(0) + np.cross(X, F).sum(0)
    np.testing.assert_allclose(L, 0.0, atol=1e-12 * scale * 40)
    # pairwise superposition: the three-body force is the sum of the pairs
    F01 = orc.contact_forces(P[[0, 1]], (2.0, 1.0, 0.0))
    F02 = orc.contact_forces(P[[0, 2]], (2.0, 1.0, 0.0))
    np.testing.assert_allclose(F[0], F01[0] + F02[0], rtol=1e-13, atol=1e-15)


def test_zero_beyond_the_range_and_the_large_sphere_limit(O):
    O.Oracle.set_contact_nodes(1024)
    orc = O.Oracle((96, 96, 96), (0, 0, 0))
    prm = W.equal_volume_params(W.SPHEROID, 5.0)
    a = prm[0]
    recs = [W.make_particle(W.SPHEROID, prm, (30.0, 40.0, 40.0)),
            W.make_particle(W.SPHEROID, prm, (30.0 + 2 * a + 2.01, 40.0, 40.0))]
    F = orc.contact_forces(orc.to_parts(np.array(recs)), (2.0, 1.0, 1.0))
    assert np.all(F == 0.0)
    # R >> zeta: the node law tends to the sphere law k ((2R + zeta - D) / zeta)^2
    O.Oracle.set_contact_nodes(16384)
    R, zeta, k = 40.0, 1.0, 1.0
    orc = O.Oracle((256, 128, 128), (0, 0, 0))
    D = 2 * R + 0.5
    recs = [W.make_particle(W.SPHEROID, (R, R, 0.0), (60.0, 64.0, 64.0)),
            W.make_particle(W.SPHEROID, (R, R, 0.0), (60.0 + D, 64.0, 64.0))]
    F = orc.contact_forces(orc.to_parts(np.array(recs)), (zeta, k, 0.0))
    law = k * ((2 * R + zeta - D) / zeta) ** 2
    assert abs(-F[0, 0] / law - 1) < 0.02
