"""Input generators (CPU): the particle counts the paper prints for its
hindered-settling cube, the shape volumes and inertia, and the placement
guarantees (no overlap, wall clearance) of both sequential-addition
generators."""
import math
import os

import numpy as np
import pytest

from paper_2312_14172_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_paper_particle_counts():
    """Sec. 5.1 / 5.4: a periodic cube of edge 12 D holds 166 spheres at
    phi = 0.05 and 991 at phi = 0.3, i.e. the smallest N reaching phi."""
    rows = [ln.split() for ln in open(os.path.join(GOLD, "hindered_settling_counts.txt"))
            if ln.strip() and not ln.startswith("#")]
    for phi, count in rows:
        n = math.ceil(float(phi) * 12.0 ** 3 / (math.pi / 6.0))
        assert n == int(count)


@pytest.mark.parametrize("shape", [W.SPHERE, W.ROUNDED_CUBE, W.SPHEROID])
def test_equal_volume_shapes(shape):
    prm = W.equal_volume_params(shape, 6.0)
    assert abs(W.shape_volume(shape, prm) - 4.0 / 3.0 * math.pi * 216.0) < 1e-9 * 905
    p = W.make_particle(shape, prm, (10, 10, 10), density_ratio=2.5)
    assert abs(p["mass"] - 2.5 * p["volume"]) < 1e-12 * p["mass"]
    assert np.all(p["inertia"] > 0)


def test_rounded_cube_volume_steiner():
    """Minkowski sum of a cube of side 2b and a ball of radius r:
    V = 8 b^3 + 6 (2b)^2 r ... = 8b^3 + 24 b^2 r + 6 pi b r^2 + 4/3 pi r^3."""
    h, r = 5.0, 1.0
    b = h - r
    steiner = 8 * b ** 3 + 24 * b ** 2 * r + 6 * math.pi * b * r ** 2 + 4.0 / 3.0 * math.pi * r ** 3
    assert abs(W.rounded_cube_moments(h, r)[0] - steiner) < 1e-9 * steiner


def test_voxel_rsa_disjoint_footprints():
    rng = np.random.default_rng(0)
    n, bc = (48, 40, 36), (0, 0, 1)
    count = 40
    shapes = np.array([W.SPHERE, W.ROUNDED_CUBE, W.SPHEROID] * 14)[:count]
    prms = [W.equal_volume_params(int(s), float(r)) for s, r in zip(shapes, rng.uniform(2.0, 3.5, count))]
    quats = [W.shoemake_quaternion(rng) for _ in range(count)]
    pos = W.voxel_rsa_positions(rng, shapes, prms, quats, n, bc, gap=1.0)
    occ = np.zeros(n[::-1], dtype=np.int32)
    for s, p, q, x in zip(shapes, prms, quats, pos):
        base = np.floor(x).astype(int)
        cells = W._footprint(int(s), p, q, x - base, 0.5) + base
        cells[:, 0] %= n[0]
        cells[:, 1] %= n[1]
        assert cells[:, 2].min() >= 1 and cells[:, 2].max() <= n[2] - 2
        occ[cells[:, 2], cells[:, 1], cells[:, 0]] += 1
    assert occ.max() == 1


def test_circumsphere_rsa_gap():
    rng = np.random.default_rng(1)
    n = (40, 40, 40)
    radii = rng.uniform(2.0, 4.0, 30)
    pos = W.rsa_positions(rng, radii, n, (0, 0, 1), gap=1.0)
    for i in range(len(radii)):
        d = pos - pos[i]
        d[:, :2] -= 40 * np.round(d[:, :2] / 40)
        dist = np.sqrt((d ** 2).sum(1))
        dist[i] = np.inf
        assert np.all(dist >= radii + radii[i] + 1.0 - 1e-12)
        assert radii[i] + 1.0 <= pos[i, 2] <= 40 - radii[i] - 1.0


def test_named_workloads_solid_fractions():
    assert abs(W.get("spheres128").solid_fraction - 0.089) < 2e-3
    assert abs(W.get("mixed256").solid_fraction - 0.108) < 2e-3


@pytest.mark.slow
def test_hindered_settling_solid_fraction():
    wl = W.get("hindered384")
    assert len(wl.particles) == 11265
    assert abs(wl.solid_fraction - 0.2) < 2e-3


@pytest.mark.slow
def test_hindered_settling_20000_variant_solid_fraction():
    """20 000 particles with r_eq ~ U[3.30, 6.61]: the radius range scaled by
    0.826 so that the stated count and solid fraction 0.2 hold together."""
    wl = W.get("hindered384b")
    assert len(wl.particles) == 20000
    assert abs(wl.solid_fraction - 0.2) < 2e-3
