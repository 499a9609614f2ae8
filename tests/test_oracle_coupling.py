"""Pins of the CPU oracle's particle coupling (Sec. 3.2): the trigonometric
indicator's printed pieces, the signed distance functions against brute force,
the momentum-exchange force against a brute-force momentum balance across one
streaming step, the force-free uniform fluid, and the mirror symmetry of the
single-sphere workload."""
import itertools
import math
import os

import numpy as np
import pytest

from paper_2312_14172_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_indicator_matches_printed_pieces(oracle_mod):
    rows = [ln.split() for ln in open(os.path.join(GOLD, "indicator_paper.txt"))
            if ln.strip() and not ln.startswith("#")]
    eps = float(rows[0][1])
    orc = oracle_mod.Oracle((4, 4, 4), eps=eps)
    for d, b in rows[1:]:
        assert abs(orc.indicator(float(d)) - float(b)) < 1e-15, d
    # monotone, continuous, flat at both band edges
    ds = np.linspace(-0.4, 0.4, 2001)
    B = np.array([orc.indicator(d) for d in ds])
    assert np.all(np.diff(B) <= 0)
    h = 1e-6
    for edge in (-eps / 2, eps / 2):
        assert abs(orc.indicator(edge + h) - orc.indicator(edge - h)) < 1e-9


def test_sphere_sdf_exact(oracle_mod):
    rng = np.random.default_rng(0)
    for _ in range(50):
        p = rng.uniform(-6, 6, 3)
        r = rng.uniform(1, 5)
        assert abs(oracle_mod.Oracle.sdf(W.SPHERE, (r, 0, 0), p) - (np.linalg.norm(p) - r)) < 1e-14


def _rounded_cube_brute(h, rc, p, n=81, levels=6):
    """Distance to the Minkowski sum of the core cube and a ball, by brute
    force: the nearest point of the core cube's surface is searched over a
    dense sampling of each face, zooming in around the best sample."""
    b = h - rc
    if np.all(np.abs(p) <= b):
        return -np.min(b - np.abs(p)) - rc   # inside the core: nearest face plane
    best = np.inf
    for ax in range(3):
        for s in (-b, b):
            o = [k for k in range(3) if k != ax]
            lo = np.array([-b, -b])
            hi = np.array([b, b])
            for _ in range(levels):
                t0 = np.linspace(lo[0], hi[0], n)
                t1 = np.linspace(lo[1], hi[1], n)
                A, Bg = np.meshgrid(t0, t1, indexing="ij")
                pts = np.zeros((n * n, 3))
                pts[:, ax] = s
                pts[:, o[0]] = A.ravel()
                pts[:, o[1]] = Bg.ravel()
                dd = np.linalg.norm(pts - p[None, :], axis=1)
                k = int(np.argmin(dd))
                ctr = pts[k, o]
                half = np.array([t0[1] - t0[0], t1[1] - t1[0]])
                lo = np.maximum(ctr - half, -b)
                hi = np.minimum(ctr + half, b)
            best = min(best, float(dd[k]))
    return best - rc


@pytest.mark.parametrize("seed", range(3))
def test_rounded_cube_sdf_brute_force(oracle_mod, seed):
    rng = np.random.default_rng(10 + seed)
    h, rc = 4.876, 0.975
    for _ in range(40):
        p = rng.uniform(-7, 7, 3)
        d = oracle_mod.Oracle.sdf(W.ROUNDED_CUBE, (h, rc, 0), p)
        ref = _rounded_cube_brute(h, rc, p)
        assert abs(d - ref) < 1e-9, (p, d, ref)


def _spheroid_brute(a, b, p, n=2400):
    """Distance to the spheroid surface by brute force: the body is symmetric
    about x, so the nearest point lies in the plane through x and p; sample that
    ellipse densely and refine around the best sample."""
    r = math.hypot(p[1], p[2])
    th = np.linspace(0, math.pi, n)
    best = None
    for _ in range(4):
        ex, ey = a * np.cos(th), b * np.sin(th)
        dd = np.hypot(ex - p[0], ey - r)
        k = int(np.argmin(dd))
        best = dd[k]
        lo, hi = th[max(k - 1, 0)], th[min(k + 1, len(th) - 1)]
        th = np.linspace(lo, hi, n)
    inside = (p[0] / a) ** 2 + (r / b) ** 2 <= 1
    return -best if inside else best


@pytest.mark.parametrize("ab", [(9.524, 4.762), (3.0, 6.0)])
def test_spheroid_sdf_brute_force(oracle_mod, ab):
    a, b = ab
    rng = np.random.default_rng(7)
    pts = list(rng.uniform(-1.3 * max(a, b), 1.3 * max(a, b), (40, 3)))
    pts += [np.array([0.3, 0, 0]), np.array([0, 0, 0]), np.array([0, 0.2, 0.1]),
            np.array([a + 1, 0, 0]), np.array([0, 0, b + 2])]
    for p in pts:
        d = oracle_mod.Oracle.sdf(W.SPHEROID, (a, b, 0), p)
        assert abs(d - _spheroid_brute(a, b, p)) < 1e-9, (p, d)


@pytest.mark.parametrize("shape", [W.ROUNDED_CUBE, W.SPHEROID])
def test_sdf_gradient_has_unit_norm(oracle_mod, shape):
    prm = W.equal_volume_params(shape, 6.0)
    rng = np.random.default_rng(3)
    h = 1e-5
    checked = 0
    for p in rng.uniform(-10, 10, (200, 3)):
        g = np.array([(oracle_mod.Oracle.sdf(shape, prm, p + h * e) -
                       oracle_mod.Oracle.sdf(shape, prm, p - h * e)) / (2 * h) for e in np.eye(3)])
        if shape == W.ROUNDED_CUBE and np.all(np.abs(p) < prm[0] - prm[1]):
            continue   # medial-axis region of the core: gradient defined, but skip kinks
        n = np.linalg.norm(g)
        if abs(n - 1) > 1e-4:
            # allow the medial axis (kinks) only
            assert oracle_mod.Oracle.sdf(shape, prm, p) < 0
            continue
        checked += 1
    assert checked > 120


@pytest.mark.parametrize("shape", [W.SPHERE, W.ROUNDED_CUBE, W.SPHEROID])
def test_inside_cell_count_converges_to_volume(oracle_mod, shape):
    """Cells whose centre has d_s <= 0 approximate the analytic volume; the
    error, averaged over random placements and orientations, falls as the
    shape is scaled up."""
    rng = np.random.default_rng(5)
    mean_err = []
    for r_eq in (3.0, 10.0):
        prm = W.equal_volume_params(shape, r_eq)
        vol = W.shape_volume(shape, prm)
        R = W.circumradius(shape, prm) + 1
        errs = []
        for _ in range(3):
            w_, x_, y_, z_ = W.shoemake_quaternion(rng)
            Rm = np.array([[1 - 2 * (y_ * y_ + z_ * z_), 2 * (x_ * y_ - w_ * z_), 2 * (x_ * z_ + w_ * y_)],
                           [2 * (x_ * y_ + w_ * z_), 1 - 2 * (x_ * x_ + z_ * z_), 2 * (y_ * z_ - w_ * x_)],
                           [2 * (x_ * z_ - w_ * y_), 2 * (y_ * z_ + w_ * x_), 1 - 2 * (x_ * x_ + y_ * y_)]])
            off = rng.random(3)
            ax = [np.arange(-math.ceil(R), math.ceil(R) + 1) + 0.5 - off[k] for k in range(3)]
            pts = np.stack(np.meshgrid(*ax, indexing="ij"), -1).reshape(-1, 3)
            pts = pts[np.linalg.norm(pts, axis=1) <= R]
            body = pts @ Rm
            cnt = sum(1 for pb in body if oracle_mod.Oracle.sdf(shape, prm, pb) <= 0)
            errs.append(abs(cnt - vol) / vol)
        mean_err.append(np.mean(errs))
    assert mean_err[-1] < 0.01 and mean_err[-1] < mean_err[0], mean_err


# ---------------------------------------------------------------------------
# Momentum exchange
# ---------------------------------------------------------------------------
def _numpy_stream_periodic(fs, c, n):
    """Independent push streaming on a periodic box for f[cell, i]."""
    nx, ny, nz = n
    g = fs.reshape(nz, ny, nx, 19)
    out = np.empty_like(g)
    for i in range(19):
        out[..., i] = np.roll(g[..., i], shift=(c[i][2], c[i][1], c[i][0]), axis=(0, 1, 2))
    return out.reshape(-1, 19)


def _cell_centres(n):
    nx, ny, nz = n
    z, y, x = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5,
                          indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)


@pytest.mark.parametrize("seed,shape", [(0, W.SPHERE), (1, W.ROUNDED_CUBE), (2, W.SPHEROID),
                                        (3, W.SPHERE)])
def test_mea_equals_momentum_balance_across_streaming(oracle_mod, seed, shape):
    """For every cell x, F_h(x) as printed equals P*(x) - P(x) - u_p(x)(M*(x) - M(x)),
    where starred sums are the post-collision populations before streaming and
    unstarred the streamed ones (both follow from f_i(x + c_i, t) = f*_i(x, t-1)).
    So the force on the particle, -sum F_h over the inside cells, must equal the
    brute-force change of momentum minus u_p times the change of mass of those
    cells across one streaming step; the torque likewise with the lever arm."""
    n = (17, 16, 15)
    rng = np.random.default_rng(seed)
    orc = oracle_mod.Oracle(n)
    c, w, _ = orc.tables()
    prm = W.equal_volume_params(shape, 3.2)
    rec = W.make_particle(shape, prm, rng.uniform(3, 12, 3), quat=W.shoemake_quaternion(rng),
                          vel=tuple(0.02 * rng.standard_normal(3)),
                          omega=tuple(0.01 * rng.standard_normal(3)))
    P = orc.to_parts(np.array([rec]))
    fs = w[None, :] * (1 + 0.1 * rng.standard_normal((orc.N, 19)))
    f = _numpy_stream_periodic(fs, c, n)
    F, T = orc.mea(P, f)
    # brute force over all cells
    X = rec["pos"]
    d = _cell_centres(n) - X
    d -= np.array(n) * np.round(d / np.array(n))
    q = rec["quat"]
    w_, x_, y_, z_ = q
    Rm = np.array([[1 - 2 * (y_ * y_ + z_ * z_), 2 * (x_ * y_ - w_ * z_), 2 * (x_ * z_ + w_ * y_)],
                   [2 * (x_ * y_ + w_ * z_), 1 - 2 * (x_ * x_ + z_ * z_), 2 * (y_ * z_ - w_ * x_)],
                   [2 * (x_ * z_ - w_ * y_), 2 * (y_ * z_ + w_ * x_), 1 - 2 * (x_ * x_ + y_ * y_)]])
    body = d @ Rm
    inside = np.array([oracle_mod.Oracle.sdf(shape, prm, p) <= 0 for p in body])
    assert inside.sum() > 50
    up = rec["vel"][None, :] + np.cross(rec["omega"][None, :], d)
    dP = f @ c - fs @ c
    dM = f.sum(1) - fs.sum(1)
    per_cell = dP - up * dM[:, None]          # = -F_h(x)
    F_ref = per_cell[inside].sum(0)
    T_ref = np.cross(d[inside], per_cell[inside]).sum(0)
    scale = np.abs(per_cell[inside]).sum()
    np.testing.assert_allclose(F[0], F_ref, atol=1e-13 * scale)
    np.testing.assert_allclose(T[0], T_ref, atol=1e-12 * scale * 5)
    assert np.linalg.norm(F[0]) > 1e-6 * scale


@pytest.mark.parametrize("seed", range(3))
def test_uniform_fluid_exerts_no_force(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    n = (20, 19, 18)
    orc = oracle_mod.Oracle(n)
    rho = 1 + 0.1 * rng.random()
    u = 0.05 * rng.standard_normal(3)
    f = orc.equilibrium(np.full(orc.N, rho), np.repeat(u[:, None], orc.N, axis=1))
    recs = W.random_particles_small(n, 2, seed, bc=(0, 0, 0))
    F, T = orc.mea(orc.to_parts(recs), f)
    np.testing.assert_allclose(F, 0, atol=1e-14)
    np.testing.assert_allclose(T, 0, atol=1e-13)


def test_single_sphere_symmetry(oracle_mod):
    """The sphere sits on the corner shared by eight cells at the box centre,
    so the lattice is mirror-symmetric in x and y about it and gravity acts
    along z: F_x = F_y = 0 and T = 0 up to round-off, while F_z is finite."""
    wl = W.single_sphere()
    orc = oracle_mod.Oracle(wl.n, wl.bc, wl.tau, gravity=wl.gravity)
    P = orc.to_parts(wl.particles)
    f = orc.equilibrium()
    F, T = orc.run(P, f, 12)
    Fz = abs(F[0, 2])
    assert Fz > 1e-5
    assert abs(F[0, 0]) < 1e-11 * Fz and abs(F[0, 1]) < 1e-11 * Fz
    assert np.all(np.abs(T[0]) < 1e-11 * Fz)
    assert P["U"][0, 2] < 0   # the heavy sphere starts to fall along -z
    B, us = orc.coupling(P)
    assert (B == 1.0).sum() == 208 and ((B > 0) & (B < 1)).sum() == 96


def test_overlapping_indicators_combine(oracle_mod):
    """Reading for overlapping smooth regions: B = min(1, sum B_p) and u_s is the
    B-weighted mean of the particle velocities."""
    n = (16, 16, 16)
    orc = oracle_mod.Oracle(n)
    a = W.make_particle(W.SPHERE, (3.0,), (7.3, 8.1, 8.2), vel=(0.01, 0, 0))
    b = W.make_particle(W.SPHERE, (3.0,), (9.4, 8.0, 7.9), vel=(-0.02, 0.01, 0))
    P2 = orc.to_parts(np.array([a, b]))
    B2, u2 = orc.coupling(P2)
    Ba, ua = orc.coupling(orc.to_parts(np.array([a])))
    Bb, ub = orc.coupling(orc.to_parts(np.array([b])))
    S0 = Ba + Bb
    np.testing.assert_allclose(B2, np.minimum(1, S0), atol=1e-15)
    m = S0 > 0
    np.testing.assert_allclose(u2[:, m], (Ba * ua + Bb * ub)[:, m] / S0[m], atol=1e-15)
    assert np.any(S0 > 1)


def _brute_coupling(orc, P, n, bc):
    """B = min(1, sum_p B(d_p)) and u_s = sum_p B_p u_p / sum_p B_p over EVERY
    cell of the lattice, with d_p from the oracle's signed distance (pinned
    above against brute-force surface search) at the body-frame offset of the
    cell centre.  The rotation of each particle comes from scipy's quaternion
    routine, the offset is the minimum image on periodic axes, and the
    particle velocity is U + w x (x - X) (Sec. 3.2)."""
    from scipy.spatial.transform import Rotation
    nx, ny, nz = n
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    cen = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1) + 0.5
    S0 = np.zeros(len(cen))
    S1 = np.zeros((3, len(cen)))
    for p in P:
        dl = cen - p["X"]
        for k in range(3):
            if bc[k] == 0:
                dl[:, k] -= n[k] * np.round(dl[:, k] / n[k])
        w, qx, qy, qz = p["q"]
        Rm = Rotation.from_quat([qx, qy, qz, w]).as_matrix()   # body -> world
        body = dl @ Rm                                          # R^T (x - X) per row
        d = np.array([orc.sdf(int(p["shape"]), p["prm"], b) for b in body])
        Bp = np.array([orc.indicator(v) for v in d])
        up = p["U"][:, None] + np.cross(p["W"], dl).T
        S0 += Bp
        S1 += Bp * up
    B = np.minimum(1.0, S0)
    us = np.where(S0 > 0, S1 / np.where(S0 > 0, S0, 1.0), 0.0)
    return B, us, S0


def test_nonspherical_coupling_against_all_cells(oracle_mod):
    """The oracle's coupling visits, per particle, the cells whose centre is
    within the circumradius + eps/2 (wrapped, clipped at walls); here its B and
    u_s are compared with a brute-force evaluation over every cell for a
    rotating rounded cube across the periodic x face, a spinning spheroid at a
    z wall, a mesh particle overlapping the cube's smooth region, and a
    sphere.  The tips and corners of the non-spherical bodies reach within one
    cell of their circumradius, so a visiting box short by a cell would drop
    cells that have B > 0 here."""
    n, bc = (26, 24, 22), (0, 0, 1)
    orc = oracle_mod.Oracle(n, bc, 0.8)
    oracle_mod.Oracle.set_mesh(*W.MESH_UNIT)
    rng = np.random.default_rng(5)
    cube = W.equal_volume_params(W.ROUNDED_CUBE, 4.0)
    sph = W.equal_volume_params(W.SPHEROID, 3.5)
    mesh = (4.0 / W.MESH_RC * 1.3, 0.0, 0.0)
    recs = np.array([
        W.make_particle(W.ROUNDED_CUBE, cube, (1.3, 8.2, 9.7), quat=W.shoemake_quaternion(rng),
                        vel=(0.01, -0.004, 0.002), omega=(0.002, -0.003, 0.004)),
        W.make_particle(W.SPHEROID, sph, (14.6, 15.1, 3.4), quat=W.shoemake_quaternion(rng),
                        vel=(-0.003, 0.002, 0.006), omega=(-0.004, 0.001, 0.003)),
        W.make_particle(W.MESH, mesh, (8.9, 9.3, 11.2), quat=W.shoemake_quaternion(rng),
                        vel=(0.002, 0.001, -0.003), omega=(0.001, 0.005, -0.002)),
        W.make_particle(W.SPHERE, (3.2,), (19.5, 3.1, 16.0), vel=(0.0, 0.005, 0.0), omega=(0.0, 0.0, 0.01)),
    ])
    P = orc.to_parts(recs)
    B, us = orc.coupling(P)
    Bb, usb, S0 = _brute_coupling(orc, P, n, bc)
    # the two rotations and offsets round differently (~1e-15 in d); B moves
    # at most pi / eps per unit of d
    np.testing.assert_allclose(B, Bb, rtol=0, atol=1e-12)
    np.testing.assert_allclose(us, usb, rtol=0, atol=1e-13)
    assert np.sum(B > 0) > 1000
    assert np.any(S0 > 1.0)            # an overlap of smooth regions is covered
    # cells with B_p > 0 within one cell of each body's circumradius exist
    from scipy.spatial.transform import Rotation
    z, y, x = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    cen = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1) + 0.5
    for p in P[:3]:
        dl = cen - p["X"]
        for k in range(3):
            if bc[k] == 0:
                dl[:, k] -= n[k] * np.round(dl[:, k] / n[k])
        r = np.linalg.norm(dl, axis=1)
        rc = orc.circumradius(int(p["shape"]), p["prm"])
        near = np.where(r > rc - 1.0)[0]
        w, qx, qy, qz = p["q"]
        body = dl[near] @ Rotation.from_quat([qx, qy, qz, w]).as_matrix()
        d = np.array([orc.sdf(int(p["shape"]), p["prm"], b) for b in body])
        assert np.any(d < 0.5 * orc.eps), int(p["shape"])
