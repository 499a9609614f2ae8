"""Seeded synthetic inputs for the HLBM step: lattice configurations, particle
lists and initial fields.

This module generates inputs only.  It holds none of the method's arithmetic
(no populations, indicator, momentum exchange or equations of motion) and is
the single piece of code shared by the HIP path's tests/benchmarks and the
CPU oracle's tests.  Shapes, sizes and distributions follow the paper's
hindered-settling workload (Sec. 5.1: resolved spheres of 12-27 cells per
diameter, solid fractions 0.05-0.3, tau = 0.55) scaled to the five workloads
below; every random draw comes from ``numpy.random.default_rng(seed)``.

Particle records use ``PARTICLE_DTYPE`` (field names, not byte layout, are the
contract: each binding copies them into its own record).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SPHERE, ROUNDED_CUBE, SPHEROID, MESH = 0, 1, 2, 3
SHAPE_NAMES = {SPHERE: "sphere", ROUNDED_CUBE: "rounded_cube", SPHEROID: "spheroid", MESH: "mesh"}


# ---------------------------------------------------------------------------
# Triangle-mesh particles: a closed mesh at unit scale (param[0] = scale)
# ---------------------------------------------------------------------------
def icosphere(level: int):
    """Unit icosphere: the icosahedron with every triangle split into four
    `level` times, new vertices pushed onto the sphere.  Triangles are
    counter-clockwise seen from outside."""
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    v = [np.array(p, dtype=np.float64) / math.sqrt(1 + t * t) for p in v]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
         (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11),
         (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(level):
        mid = {}

        def m(a, b):
            key = (min(a, b), max(a, b))
            if key not in mid:
                c = v[a] + v[b]
                v.append(c / np.linalg.norm(c))
                mid[key] = len(v) - 1
            return mid[key]

        f = [t2 for a, b, c in f for t2 in ((a, m(a, b), m(c, a)), (b, m(b, c), m(a, b)), (c, m(c, a), m(b, c)),
                                            (m(a, b), m(b, c), m(c, a)))]
    return np.array(v), np.array(f, dtype=np.int32)


def bumpy_mesh(level: int = 2, amp: float = 0.5):
    """A star-shaped closed mesh with cubic symmetry: the icosphere's vertices
    moved to radius 1 + amp (x^4 + y^4 + z^4 - 3/5) along their direction
    (bulges along the axes, dents along the diagonals).  Vertices rounded to
    FP32, the precision the library stores them in."""
    d, tri = icosphere(level)
    r = 1.0 + amp * ((d ** 4).sum(axis=1) - 0.6)
    v = (d * r[:, None]).astype(np.float32).astype(np.float64)
    return v, tri


def mesh_mass_properties(v, tri):
    """Volume and inertia tensor (unit density) of the solid bounded by a
    closed, outward-oriented triangle mesh, summed over the tetrahedra
    (origin, a, b, c): signed volume det[a b c] / 6 and second moments
    int x x^T = V / 20 (a a^T + b b^T + c c^T + s s^T), s = a + b + c."""
    a, b, c = v[tri[:, 0]], v[tri[:, 1]], v[tri[:, 2]]
    vol_t = np.einsum("ij,ij->i", a, np.cross(b, c)) / 6.0
    ssum = a + b + c
    second = sum(np.einsum("i,ij,ik->jk", vol_t, x, x) for x in (a, b, c, ssum)) / 20.0
    vol = float(vol_t.sum())
    inertia = np.trace(second) * np.eye(3) - second
    return vol, inertia


MESH_UNIT = bumpy_mesh()
_MESH_VOL, _MESH_INERTIA = mesh_mass_properties(*MESH_UNIT)
MESH_RC = float(np.sqrt((MESH_UNIT[0] ** 2).sum(axis=1)).max())

PARTICLE_DTYPE = np.dtype([
    ("pos", "<f8", 3), ("quat", "<f8", 4), ("vel", "<f8", 3), ("omega", "<f8", 3),
    ("mass", "<f8"), ("volume", "<f8"), ("inertia", "<f8", 3), ("param", "<f8", 3),
    ("shape", "<i4"), ("flags", "<i4")])


# ---------------------------------------------------------------------------
# Shape geometry of the inputs: volume, mass, principal inertia, circumradius
# ---------------------------------------------------------------------------
def _gauss_legendre(n, a, b):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (b - a) * x + 0.5 * (b + a), 0.5 * (b - a) * w


def rounded_cube_moments(h: float, rc: float):
    """Volume and I_zz/mass-density of the Minkowski sum of a cube of
    half-extent b = h - rc with a ball of radius rc (unit density).

    Integrated slice by slice: at height z the cross-section is a square of
    half-side b with corners rounded to radius rho(z) (rho = rc in the core,
    sqrt(rc^2 - s^2) at distance s above it)."""
    b = h - rc

    def area(rho):
        return 4 * b * b + 8 * b * rho + math.pi * rho * rho

    def polar(rho):  # integral of x^2 + y^2 over the rounded square
        core = 8 * b ** 4 / 3
        sides = 4 * (2 * b * ((b + rho) ** 3 - b ** 3) / 3 + 2 * b ** 3 * rho / 3)
        corners = 4 * (math.pi * b * b * rho * rho / 2 + 4 * b * rho ** 3 / 3
                       + math.pi * rho ** 4 / 8)
        return core + sides + corners

    phi, w = _gauss_legendre(64, 0.0, 0.5 * math.pi)
    rho = rc * np.cos(phi)
    jac = rc * np.cos(phi)
    vol = 2 * b * area(rc) + 2 * float(np.sum(w * jac * area(rho)))
    izz = 2 * b * polar(rc) + 2 * float(np.sum(w * jac * polar(rho)))
    return vol, izz


def shape_volume(shape: int, prm) -> float:
    if shape == SPHERE:
        return 4.0 / 3.0 * math.pi * prm[0] ** 3
    if shape == ROUNDED_CUBE:
        return rounded_cube_moments(prm[0], prm[1])[0]
    if shape == SPHEROID:
        return 4.0 / 3.0 * math.pi * prm[0] * prm[1] * prm[1]
    if shape == MESH:
        return _MESH_VOL * prm[0] ** 3
    raise ValueError(shape)


def shape_inertia(shape: int, prm, mass: float):
    if shape == SPHERE:
        v = 0.4 * mass * prm[0] ** 2
        return (v, v, v)
    if shape == ROUNDED_CUBE:
        vol, izz = rounded_cube_moments(prm[0], prm[1])
        v = mass / vol * izz
        return (v, v, v)
    if shape == SPHEROID:  # symmetry axis = body x
        a, b = prm[0], prm[1]
        return (0.4 * mass * b * b, 0.2 * mass * (a * a + b * b), 0.2 * mass * (a * a + b * b))
    if shape == MESH:  # cubic symmetry: the body axes are principal
        return tuple(mass / _MESH_VOL * prm[0] ** 2 * np.diag(_MESH_INERTIA))
    raise ValueError(shape)


def circumradius(shape: int, prm) -> float:
    if shape == SPHERE:
        return float(prm[0])
    if shape == ROUNDED_CUBE:
        return math.sqrt(3.0) * (prm[0] - prm[1]) + prm[1]
    if shape == SPHEROID:
        return float(max(prm[0], prm[1]))
    if shape == MESH:
        return MESH_RC * prm[0]
    raise ValueError(shape)


def equal_volume_params(shape: int, r_eq: float):
    """Shape parameters with the volume of a sphere of radius r_eq:
    rounded cube with corner radius 0.2 h, prolate 2:1 spheroid."""
    if shape == SPHERE:
        return (r_eq, 0.0, 0.0)
    if shape == ROUNDED_CUBE:
        v_target = 4.0 / 3.0 * math.pi * r_eq ** 3
        unit = rounded_cube_moments(1.0, 0.2)[0]
        h = (v_target / unit) ** (1.0 / 3.0)
        return (h, 0.2 * h, 0.0)
    if shape == SPHEROID:
        b = r_eq / 2 ** (1.0 / 3.0)
        return (2 * b, b, 0.0)
    if shape == MESH:
        return ((4.0 / 3.0 * math.pi / _MESH_VOL) ** (1.0 / 3.0) * r_eq, 0.0, 0.0)
    raise ValueError(shape)


def make_particle(shape: int, prm, pos, quat=(1.0, 0.0, 0.0, 0.0), density_ratio=2.0,
                  rho_f=1.0, vel=(0.0, 0.0, 0.0), omega=(0.0, 0.0, 0.0), fixed=False):
    rec = np.zeros((), dtype=PARTICLE_DTYPE)
    prm = tuple(float(v) for v in prm) + (0.0,) * (3 - len(prm))
    vol = shape_volume(shape, prm)
    mass = density_ratio * rho_f * vol
    rec["pos"] = pos
    rec["quat"] = quat
    rec["vel"] = vel
    rec["omega"] = omega
    rec["volume"] = vol
    rec["inertia"] = shape_inertia(shape, prm, mass)
    rec["mass"] = -1.0 if fixed else mass
    rec["param"] = prm
    rec["shape"] = shape
    return rec


def shoemake_quaternion(rng: np.random.Generator):
    """Uniformly random unit quaternion (Shoemake, Graphics Gems III, 1992)."""
    u1, u2, u3 = rng.random(3)
    a, b = math.sqrt(1 - u1), math.sqrt(u1)
    return (b * math.cos(2 * math.pi * u3), a * math.sin(2 * math.pi * u2),
            a * math.cos(2 * math.pi * u2), b * math.sin(2 * math.pi * u3))


# ---------------------------------------------------------------------------
# Random sequential addition on circumspheres
# ---------------------------------------------------------------------------
def rsa_positions(rng, radii, n, bc, gap=1.0, wall_margin=1.0, batch=64, max_attempts=5_000_000):
    """Place spheres of the given radii (in the given order) uniformly at
    random without overlap: centre distance >= r_i + r_j + gap, minimum image
    on periodic axes, and at least r + wall_margin from a wall.  Candidates are
    checked against the already placed spheres of the neighbouring buckets of
    a uniform grid."""
    n = np.asarray(n, dtype=np.float64)
    bc = np.asarray(bc)
    radii = np.asarray(radii, dtype=np.float64)
    rmax = float(radii.max()) if len(radii) else 1.0
    h = 2 * rmax + gap
    nb = np.maximum(1, np.floor(n / h)).astype(int)
    hs = n / nb
    buckets = {}
    pos = np.zeros((len(radii), 3))
    per = bc == 0
    attempts = 0
    for i, r in enumerate(radii):
        lo = np.where(bc == 1, r + wall_margin, 0.0)
        hi = np.where(bc == 1, n - r - wall_margin, n)
        placed = False
        while not placed:
            cand = lo + (hi - lo) * rng.random((batch, 3))
            for c in cand:
                attempts += 1
                if attempts > max_attempts:
                    raise RuntimeError(f"RSA stalled after placing {i} of {len(radii)}")
                cell = np.minimum((c // hs).astype(int), nb - 1)
                near = []
                for dz in (-1, 0, 1):
                    for dy in (-1, 0, 1):
                        for dx in (-1, 0, 1):
                            k = cell + (dx, dy, dz)
                            if np.any((k < 0) | (k >= nb)):
                                if np.any(((k < 0) | (k >= nb)) & ~per):
                                    continue
                                k = k % nb
                            near.extend(buckets.get(tuple(k), ()))
                if near:
                    idx = np.array(near)
                    d = pos[idx] - c
                    d[:, per] -= n[per] * np.round(d[:, per] / n[per])
                    if np.any(np.sqrt(np.sum(d * d, axis=1)) < radii[idx] + r + gap):
                        continue
                pos[i] = c
                buckets.setdefault(tuple(cell), []).append(i)
                placed = True
                break
    return pos


# ---------------------------------------------------------------------------
# Random sequential addition on a voxel-occupancy grid (true shapes)
# ---------------------------------------------------------------------------
def _rotation(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _footprint(shape, prm, q, frac, grow):
    """Offsets (relative to floor(X)) of the cells whose centre lies in the
    shape grown by `grow` (a superset of its grow-neighbourhood for the
    spheroid), for a centre at floor(X) + frac.  Placement geometry only."""
    reach = circumradius(shape, prm) + grow
    k = int(math.ceil(reach)) + 1
    ax = np.arange(-k, k + 1)
    gz, gy, gx = np.meshgrid(ax, ax, ax, indexing="ij")
    off = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)
    d = off + 0.5 - np.asarray(frac)
    b = d @ _rotation(q)  # body-frame coordinates R^T d, row-wise
    if shape == SPHERE:
        inside = np.sum(b * b, axis=1) <= (prm[0] + grow) ** 2
    elif shape == ROUNDED_CUBE:
        core = prm[0] - prm[1]
        o = np.maximum(np.abs(b) - core, 0.0)
        inside = np.sum(o * o, axis=1) <= (prm[1] + grow) ** 2
    else:
        a, c = prm[0] + grow, prm[1] + grow
        inside = (b[:, 0] / a) ** 2 + (b[:, 1] ** 2 + b[:, 2] ** 2) / c ** 2 <= 1.0
    return off[inside]


def voxel_rsa_positions(rng, shapes, prms, quats, n, bc, gap=1.0, wall_margin=1.0, max_attempts=20_000_000):
    """Place the given oriented shapes (in the given order) uniformly at random
    so that their footprints grown by gap/2 occupy disjoint cells of the
    lattice (surface gap >= gap at lattice resolution), wrapping on periodic
    axes and keeping every footprint cell at least wall_margin cells from a
    wall."""
    n = tuple(int(v) for v in n)
    occ = np.zeros(n[::-1], dtype=bool)  # [z, y, x]
    pos = np.zeros((len(shapes), 3))
    attempts = 0
    nn = np.array(n)
    for i in range(len(shapes)):
        shape, prm, q = int(shapes[i]), prms[i], quats[i]
        reach = circumradius(shape, prm) + 0.5 * gap
        lo = np.array([0.0 if bc[k] == 0 else reach + wall_margin for k in range(3)])
        hi = np.array([float(n[k]) if bc[k] == 0 else n[k] - reach - wall_margin for k in range(3)])
        # a core of cells inside the footprint for every centre in the base
        # cell: the ball of the inscribed radius of the grown shape (an early
        # rejection that never rejects an attempt the full test would accept)
        r_in = (prm[0] if shape != SPHEROID else min(prm[0], prm[1])) + 0.5 * gap
        k = int(math.ceil(r_in)) + 1
        ax = np.arange(-k, k + 1)
        gz, gy, gx = np.meshgrid(ax, ax, ax, indexing="ij")
        off = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)
        far = np.sqrt(np.sum((np.abs(off) + 0.5) ** 2, axis=1))  # farthest centre over the base cell
        core = off[far <= r_in]
        while True:
            attempts += 1
            if attempts > max_attempts:
                raise RuntimeError(f"voxel RSA stalled after placing {i} of {len(shapes)}")
            X = lo + (hi - lo) * rng.random(3)
            base = np.floor(X).astype(int)
            if occ[base[2] % n[2], base[1] % n[1], base[0] % n[0]]:
                continue
            if len(core):
                cc = core + base
                inside = True
                for a in range(3):
                    if bc[a] == 0:
                        cc[:, a] %= nn[a]
                    elif cc[:, a].min() < wall_margin or cc[:, a].max() > n[a] - 1 - wall_margin:
                        inside = False
                if not inside or occ[cc[:, 2], cc[:, 1], cc[:, 0]].any():
                    continue
            cells = _footprint(shape, prm, q, X - base, 0.5 * gap) + base
            ok = True
            for k in range(3):
                if bc[k] == 0:
                    cells[:, k] %= n[k]
                elif cells[:, k].min() < wall_margin or cells[:, k].max() > n[k] - 1 - wall_margin:
                    ok = False
            if not ok or occ[cells[:, 2], cells[:, 1], cells[:, 0]].any():
                continue
            occ[cells[:, 2], cells[:, 1], cells[:, 0]] = True
            pos[i] = X
            break
    return pos


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    n: tuple
    bc: tuple
    tau: float
    steps: int
    precision: str
    gravity: tuple = (0.0, 0.0, -1e-5)
    density_ratio: float = 2.0
    eps: float = 0.5
    rho_f: float = 1.0
    fluid_accel: tuple = (0.0, 0.0, 0.0)
    seed: int = 0
    description: str = ""
    learned: bool = False
    particles: np.ndarray = field(default=None, repr=False)

    @property
    def ncells(self):
        return self.n[0] * self.n[1] * self.n[2]

    @property
    def solid_fraction(self):
        return float(np.sum(self.particles["volume"]) / self.ncells) if len(self.particles) else 0.0


def single_sphere(n=32, r=4.0, tau=0.8, steps=100, precision="fp64"):
    """One sphere of radius 4 centred on the corner shared by eight cells at the
    box centre, periodic 32^3, tau = 0.8, density ratio 2, g = 1e-5."""
    w = Workload("sphere32", (n, n, n), (0, 0, 0), tau, steps, precision, seed=1,
                 description="32^3 periodic, one sphere r=4 at the box centre, tau=0.8")
    w.particles = np.array([make_particle(SPHERE, (r,), (n / 2, n / 2, n / 2), density_ratio=2.0)])
    return w


def settling_spheres(n=128, count=200, seed=2, tau=0.6, steps=1000, precision="fp32"):
    """Spheres with radius U[5,7] placed by RSA (gap >= 1) in a box periodic in
    x, y with half-way walls at z = 0 and z = n; tau = 0.6; density ratio 2."""
    rng = np.random.default_rng(seed)
    radii = rng.uniform(5.0, 7.0, count)
    order = np.argsort(-radii, kind="stable")
    pos = rsa_positions(rng, radii[order], (n, n, n), (0, 0, 1))
    recs = []
    for k, i in enumerate(order):
        recs.append(make_particle(SPHERE, (radii[i],), pos[k], density_ratio=2.0))
    w = Workload(f"spheres{n}", (n, n, n), (0, 0, 1), tau, steps, precision, seed=seed,
                 description=f"{n}^3, z walls, {count} spheres r~U[5,7], tau={tau}")
    w.particles = np.array(recs)
    return w


def mixed_shapes(n=256, count=2000, r_eq=6.0, seed=3, tau=0.6, steps=1000, precision="fp16s",
                 learned=False, density_ratio=2.0, r_eq_range=None, gap=1.0):
    """Spheres, rounded cubes (corner radius 0.2 h) and prolate 2:1 spheroids in
    equal thirds, equal volume r_eq (or r_eq ~ U[r_eq_range]), uniformly random
    orientations, RSA on circumspheres, z walls."""
    rng = np.random.default_rng(seed)
    shapes = np.array([SPHERE, ROUNDED_CUBE, SPHEROID] * (count // 3 + 1))[:count]
    if r_eq_range is None:
        req = np.full(count, float(r_eq))
    else:
        req = rng.uniform(r_eq_range[0], r_eq_range[1], count)
    prms = [equal_volume_params(int(s), float(r)) for s, r in zip(shapes, req)]
    rcirc = np.array([circumradius(int(s), p) for s, p in zip(shapes, prms)])
    quats = [shoemake_quaternion(rng) for _ in range(count)]
    order = np.argsort(-rcirc, kind="stable")
    pos = rsa_positions(rng, rcirc[order], (n, n, n), (0, 0, 1), gap=gap)
    recs = []
    for k, i in enumerate(order):
        recs.append(make_particle(int(shapes[i]), prms[i], pos[k], quat=quats[i],
                                  density_ratio=density_ratio))
    w = Workload(f"mixed{n}" + ("_learned" if learned else ""), (n, n, n), (0, 0, 1), tau, steps,
                 precision, seed=seed,
                 density_ratio=density_ratio, learned=learned,
                 description=f"{n}^3, z walls, {count} mixed shapes r_eq={r_eq}, tau={tau}")
    w.particles = np.array(recs)
    return w


def hindered_settling(n=384, count=11265, r_eq_range=(4.0, 8.0), seed=5, tau=0.55, steps=5000,
                      precision="fp32", density_ratio=2.5, gap=1.0, name=None):
    """Hindered settling: spheres, rounded cubes and prolate 2:1 spheroids in
    equal thirds with equivalent radius r_eq ~ U[4, 8] (solid fraction ~0.2 at
    11 265 particles in 384^3), uniformly random orientations, voxel-occupancy
    RSA with surface gap >= 1, z walls, tau = 0.55, density ratio 2.5."""
    rng = np.random.default_rng(seed)
    shapes = np.array([SPHERE, ROUNDED_CUBE, SPHEROID] * (count // 3 + 1))[:count]
    req = rng.uniform(r_eq_range[0], r_eq_range[1], count)
    prms = [equal_volume_params(int(s), float(r)) for s, r in zip(shapes, req)]
    rcirc = np.array([circumradius(int(s), p) for s, p in zip(shapes, prms)])
    quats = [shoemake_quaternion(rng) for _ in range(count)]
    order = np.argsort(-rcirc, kind="stable")
    pos = voxel_rsa_positions(rng, shapes[order], [prms[i] for i in order], [quats[i] for i in order],
                              (n, n, n), (0, 0, 1), gap=gap)
    recs = [make_particle(int(shapes[i]), prms[i], pos[k], quat=quats[i], density_ratio=density_ratio)
            for k, i in enumerate(order)]
    w = Workload(name or f"hindered{n}", (n, n, n), (0, 0, 1), tau, steps, precision, seed=seed,
                 density_ratio=density_ratio,
                 description=f"{n}^3, z walls, {count} mixed shapes r_eq~U{r_eq_range}, tau={tau}")
    w.particles = np.array(recs)
    return w


def smooth_fields(n, seed, rho_amp=1e-3, u_amp=1e-2, modes=3):
    """Smooth periodic random density and velocity fields (sums of a few
    Fourier modes with seeded amplitudes and phases).  Returns rho[N], u[3,N]
    in cell order x + nx*(y + ny*z)."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = n
    z, y, x = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5,
                          indexing="ij")

    def field1():
        acc = np.zeros_like(x)
        for _ in range(modes):
            k = rng.integers(0, 3, 3)
            ph = rng.random() * 2 * math.pi
            a = rng.normal()
            acc += a * np.sin(2 * math.pi * (k[0] * x / nx + k[1] * y / ny + k[2] * z / nz) + ph)
        return acc / modes

    rho = 1.0 + rho_amp * field1()
    u = np.stack([u_amp * field1() for _ in range(3)])
    return rho.reshape(-1).copy(), u.reshape(3, -1).copy()


def random_particles_small(n, count, seed, shapes=(SPHERE, ROUNDED_CUBE, SPHEROID), r_eq=(2.5, 4.0),
                           bc=(0, 0, 1), moving=True, density_ratio=2.0, gap=0.5):
    """A few mixed particles for small parity lattices: random shapes, sizes,
    orientations and (optionally) velocities and angular velocities."""
    rng = np.random.default_rng(seed)
    sh = [shapes[i % len(shapes)] for i in range(count)]
    req = rng.uniform(r_eq[0], r_eq[1], count)
    prms = [equal_volume_params(int(s), float(r)) for s, r in zip(sh, req)]
    rcirc = np.array([circumradius(int(s), p) for s, p in zip(sh, prms)])
    pos = rsa_positions(rng, rcirc, n, bc, gap=gap, wall_margin=1.5)
    recs = []
    for i in range(count):
        vel = tuple(rng.uniform(-0.01, 0.01, 3)) if moving else (0.0, 0.0, 0.0)
        om = tuple(rng.uniform(-0.004, 0.004, 3)) if moving else (0.0, 0.0, 0.0)
        recs.append(make_particle(int(sh[i]), prms[i], pos[i], quat=shoemake_quaternion(rng),
                                  vel=vel, omega=om, density_ratio=density_ratio))
    return np.array(recs)


def small_spheres(n=128, count=4200, seed=11, tau=0.6, steps=100, precision="fp32"):
    """Many small spheres, radius U[1.5, 2.5], RSA (gap >= 1), z walls, tau 0.6,
    density ratio 2: a parity case with enough particles for the
    momentum exchange's dispatch for large particle counts."""
    rng = np.random.default_rng(seed)
    radii = np.sort(rng.uniform(1.5, 2.5, count))[::-1]
    pos = rsa_positions(rng, radii, (n, n, n), (0, 0, 1))
    w = Workload(f"small{count}", (n, n, n), (0, 0, 1), tau, steps, precision, seed=seed,
                 description=f"{n}^3, z walls, {count} spheres r~U[1.5,2.5], tau={tau}")
    w.particles = np.array([make_particle(SPHERE, (r,), x, density_ratio=2.0) for r, x in zip(radii, pos)])
    return w


def mesh_particles(n=128, count=100, r_eq=6.0, seed=13, tau=0.8, steps=1000, precision="fp32", learned=False):
    """Triangle-mesh particles (the bumpy 320-triangle mesh MESH_UNIT) with
    the volume of a sphere of radius r_eq, random orientations, RSA on
    circumspheres (gap 2), z walls."""
    rng = np.random.default_rng(seed)
    s = equal_volume_params(MESH, r_eq)
    rc = circumradius(MESH, s)
    pos = rsa_positions(rng, np.full(count, rc), (n, n, n), (0, 0, 1), gap=2.0, wall_margin=2.0)
    w = Workload(f"meshes{n}" + ("_learned" if learned else ""), (n, n, n), (0, 0, 1), tau, steps, precision,
                 seed=seed, learned=learned,
                 description=f"{n}^3, z walls, {count} meshes of {len(MESH_UNIT[1])} triangles, r_eq {r_eq}")
    w.particles = np.array([make_particle(MESH, s, x, quat=shoemake_quaternion(rng)) for x in pos])
    return w


def get(name: str, **kw) -> Workload:
    """Named workloads:
    sphere32   -- 32^3 periodic, one sphere (parity case);
    spheres128 -- 128^3, z walls, 200 spheres r~U[5,7], tau 0.6;
    mixed256   -- 256^3, z walls, 2000 mixed shapes r_eq 6, tau 0.6;
    mixed256_learned -- as mixed256 with the learned indicator for non-spheres;
    hindered384 -- 384^3, z walls, 11 265 mixed shapes r_eq~U[4,8], tau 0.55;
    hindered384b -- as hindered384 with 20 000 particles, r_eq~U[3.30,6.61]
                  (the same solid fraction 0.2);
    small4200  -- 128^3, z walls, 4200 spheres r~U[1.5,2.5] (parity case);
    meshes128 / meshes128_learned -- 128^3, z walls, 100 triangle meshes
                  (r_eq 6), exact distance / learned indicator.
    """
    if name == "sphere32":
        return single_sphere(**kw)
    if name == "spheres128":
        return settling_spheres(**kw)
    if name == "mixed256":
        return mixed_shapes(**kw)
    if name == "mixed256_learned":
        return mixed_shapes(learned=True, **kw)
    if name == "hindered384":
        return hindered_settling(**kw)
    if name == "hindered384b":
        return hindered_settling(count=20000, r_eq_range=(3.30, 6.61), name="hindered384b", **kw)
    if name == "meshes128":
        return mesh_particles(**kw)
    if name == "meshes128_learned":
        return mesh_particles(learned=True, **kw)
    if name == "small4200":
        return small_spheres(**kw)
    raise KeyError(name)


# ---------------------------------------------------------------------------
# Signed-distance surrogate network: initial parameters and sample points
# ---------------------------------------------------------------------------
MLP_HIDDEN = 64
MLP_NPARAM = 64 * 3 + 64 + 64 * 64 + 64 + 64 * 64 + 64 + 64 + 1


def mlp_init_params(seed):
    """Initial network parameters (uniform, He-style limits sqrt(6 / fan_in),
    zero biases) as one flat float32 vector in the order W1 (64x3), b1,
    W2 (64x64), b2, W3 (64x64), b3, W4 (64), b4."""
    rng = np.random.default_rng(seed)
    parts = [rng.uniform(-math.sqrt(6 / 3), math.sqrt(6 / 3), 64 * 3), np.zeros(64),
             rng.uniform(-math.sqrt(6 / 64), math.sqrt(6 / 64), 64 * 64), np.zeros(64),
             rng.uniform(-math.sqrt(6 / 64), math.sqrt(6 / 64), 64 * 64), np.zeros(64),
             rng.uniform(-math.sqrt(6 / 64), math.sqrt(6 / 64), 64), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)


def mlp_points(seed, n, half=1.1):
    """n points uniform in the cube [-half, half]^3 (normalised body frame)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-half, half, (n, 3))
