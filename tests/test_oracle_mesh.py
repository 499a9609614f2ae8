"""Oracle pins for triangle-mesh particles (shape 3): the distance and
inside/outside sign of a closed mesh against shapes with closed forms (a
cube, a finely tessellated sphere), and the solid's volume from the sign
(Monte Carlo) against the divergence-theorem volume of the mesh."""
import math

import numpy as np
import pytest

from paper_2312_14172_amd import workloads as W

CUBE_V = np.array([[x, y, z] for z in (-0.5, 0.5) for y in (-0.5, 0.5) for x in (-0.5, 0.5)])
# two triangles per face, counter-clockwise seen from outside
CUBE_T = np.array([[0, 2, 1], [1, 2, 3], [4, 5, 6], [5, 7, 6], [0, 1, 4], [1, 5, 4],
                   [2, 6, 3], [3, 6, 7], [0, 4, 2], [2, 4, 6], [1, 3, 5], [3, 7, 5]])


def _box_sdf(p, h):
    q = np.abs(p) - h
    return float(np.linalg.norm(np.maximum(q, 0.0)) + min(q.max(), 0.0))


def test_cube_mesh_is_the_box_sdf(oracle_mod):
    O = oracle_mod.Oracle
    vol, inertia = W.mesh_mass_properties(CUBE_V, CUBE_T)
    assert abs(vol - 1.0) < 1e-14                      # outward orientation, unit cube
    assert np.allclose(inertia, np.eye(3) / 6.0, atol=1e-14)
    O.set_mesh(CUBE_V, CUBE_T)
    rng = np.random.default_rng(0)
    s = 2.0  # scale: half-extent 1
    for p in rng.uniform(-2.5, 2.5, (400, 3)):
        assert abs(O.sdf(3, [s, 0, 0], p) - _box_sdf(p, 1.0)) < 1e-12


def test_fine_icosphere_approaches_the_sphere(oracle_mod):
    O = oracle_mod.Oracle
    v, t = W.icosphere(3)
    O.set_mesh(v, t)
    # the faces lie between the sphere and the sphere of the least face-plane distance
    a, b, c = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    n = np.cross(b - a, c - a)
    inner = float(np.min(np.einsum("ij,ij->i", a, n) / np.linalg.norm(n, axis=1)))
    gap = 1.0 - inner
    assert 0 < gap < 5e-3
    rng = np.random.default_rng(1)
    for _ in range(300):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        r = rng.uniform(0.3, 1.7)
        assert abs(O.sdf(3, [1.0, 0, 0], r * d) - (r - 1.0)) <= gap + 1e-12
    # icosahedron volume: (5/12)(3 + sqrt 5) a^3 for edge a = 4 / sqrt(10 + 2 sqrt 5)
    v0, t0 = W.icosphere(0)
    edge = 4.0 / math.sqrt(10 + 2 * math.sqrt(5))
    assert abs(W.mesh_mass_properties(v0, t0)[0] - 5.0 / 12.0 * (3 + math.sqrt(5)) * edge ** 3) < 1e-12


def test_bumpy_mesh_sign_gives_its_volume(oracle_mod):
    O = oracle_mod.Oracle
    v, t = W.MESH_UNIT
    O.set_mesh(v, t)
    vol = W.mesh_mass_properties(v, t)[0]
    rng = np.random.default_rng(2)
    pts = rng.uniform(-1.25, 1.25, (20000, 3))
    inside = np.mean([O.sdf(3, [1.0, 0, 0], p) <= 0.0 for p in pts])
    est = inside * 2.5 ** 3
    sigma = 2.5 ** 3 * math.sqrt(inside * (1 - inside) / len(pts))
    assert abs(est - vol) < 4 * sigma
    # scale: distances scale linearly, the sign is scale-invariant
    for p in pts[:50]:
        assert abs(O.sdf(3, [3.0, 0, 0], 3.0 * p) - 3.0 * O.sdf(3, [1.0, 0, 0], p)) < 1e-12
    # the circumradius of a mesh particle is scale x the largest vertex radius
    P = np.zeros(1, dtype=[("pos", "<f8", 3), ("quat", "<f8", 4), ("vel", "<f8", 3), ("omega", "<f8", 3),
                           ("mass", "<f8"), ("volume", "<f8"), ("inertia", "<f8", 3), ("param", "<f8", 3),
                           ("shape", "<i4")])
    P["param"] = [[2.0, 0, 0]]
    P["shape"] = 3
    P["quat"] = [[1, 0, 0, 0]]
    P["inertia"] = 1.0
    P["pos"] = 16.0
    orc = oracle_mod.Oracle((32, 32, 32), (0, 0, 0), 0.8)
    parts = orc.to_parts(P)
    assert abs(orc.circumradius(3, parts[0]["prm"]) - 2.0 * W.MESH_RC) < 1e-12
