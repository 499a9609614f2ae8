"""Pins of the CPU oracle's lattice Boltzmann part against facts fixed by the
paper (Sec. 3.1) and by mathematics: the printed velocity set and weights,
closed-form moments of the equilibrium, conservation in collision, streaming
of an impulse, reduction to textbook BGK when no particle is present, and the
analytic discrete Poiseuille profile."""
import itertools
import os

import numpy as np
import pytest

from paper_2312_14172_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _no_particles():
    return np.zeros(0, dtype=W.PARTICLE_DTYPE)


def test_velocity_set_and_weights_match_paper(oracle_mod):
    c, w, opp = oracle_mod.Oracle.tables()
    rows = [ln.split() for ln in open(os.path.join(GOLD, "d3q19_paper.txt"))
            if ln.strip() and not ln.startswith("#")]
    groups = {r[0]: r for r in rows if r[0] != "cs2"}
    norms = np.sum(c * c, axis=1)
    assert len(c) == 19 and np.all(np.abs(c) <= 1)
    assert len({tuple(v) for v in c}) == 19
    assert tuple(c[0]) == (0, 0, 0)
    for name, r in groups.items():
        sel = norms == int(r[1])
        assert sel.sum() == int(r[2])
        np.testing.assert_allclose(w[sel], int(r[3]) / int(r[4]), rtol=0, atol=0)
    # opposite table
    for i in range(19):
        assert np.all(c[opp[i]] == -c[i])
    # isotropy of the quadrature: sum w c_a c_b = cs^2 delta_ab; 4th order = cs^4 (3 delta delta)
    cs2 = 1.0 / 3.0
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", w, c, c), cs2 * np.eye(3), atol=1e-16)
    np.testing.assert_allclose(np.einsum("i,ia->a", w, c), 0.0, atol=1e-17)
    d = np.eye(3)
    t4 = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    iso = cs2 ** 2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
                      + np.einsum("ad,bc->abcd", d, d))
    np.testing.assert_allclose(t4, iso, atol=1e-16)


@pytest.mark.parametrize("seed", range(5))
def test_equilibrium_moments_closed_form(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    c, w, _ = oracle_mod.Oracle.tables()
    rho = 1 + 0.2 * rng.standard_normal()
    u = 0.1 * rng.standard_normal(3)
    feq = oracle_mod.Oracle.feq(rho, u)
    assert abs(feq.sum() - rho) < 1e-15
    np.testing.assert_allclose(c.T @ feq, rho * u, atol=1e-16)
    # second moment of the second-order equilibrium: rho (cs^2 I + u u)
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", feq, c, c),
                               rho * (np.eye(3) / 3 + np.outer(u, u)), atol=1e-15)
    # rest state equals the weights
    np.testing.assert_array_equal(oracle_mod.Oracle.feq(1.0, np.zeros(3)), w)


@pytest.mark.parametrize("seed", range(6))
def test_collision_conserves_mass_and_adds_rho_du(oracle_mod, seed):
    rng = np.random.default_rng(100 + seed)
    tau = 0.55 + rng.random()
    af = 1e-4 * rng.standard_normal(3)
    orc = oracle_mod.Oracle((4, 4, 4), tau=tau, fluid_accel=tuple(af))
    c, w, _ = orc.tables()
    f = orc.feq(1 + 0.05 * rng.standard_normal(), 0.05 * rng.standard_normal(3))
    f = f + 1e-3 * w * rng.standard_normal(19)      # non-equilibrium part
    B = [0.0, 1.0, rng.random()][seed % 3]
    us = 0.02 * rng.standard_normal(3)
    fs = orc.collide_cell(f, B, us)
    rho = f.sum()
    u = c.T @ f / rho
    du = B * (us - u) + (1 - B) * af
    assert abs(fs.sum() - rho) < 2e-16 * 19
    np.testing.assert_allclose(c.T @ fs, rho * (u + du), atol=1e-16)
    if B == 1.0:   # solid cell: post-collision momentum is exactly rho * u_s
        np.testing.assert_allclose(c.T @ fs / rho, us, atol=1e-16)
    # EDM identity: BGK with source equals plain BGK applied to f + S
    S = orc.feq(rho, u + du) - orc.feq(rho, u)
    g = f + S
    plain = g - (g - orc.feq(g.sum(), c.T @ g / g.sum())) / tau
    np.testing.assert_allclose(fs, plain, atol=1e-16)
    # the non-equilibrium second moment relaxes by (1 - 1/tau)
    if B == 0.0 and not af.any():
        neq = f - orc.feq(rho, u)
        neq_s = fs - orc.feq(rho, u)
        np.testing.assert_allclose(np.einsum("i,ia,ib->ab", neq_s, c, c),
                                   (1 - 1 / tau) * np.einsum("i,ia,ib->ab", neq, c, c), atol=1e-17)


@pytest.mark.parametrize("bc", [(0, 0, 0), (0, 1, 1), (1, 1, 1)])
def test_stream_moves_an_impulse_along_c(oracle_mod, bc):
    n = (5, 4, 3)
    orc = oracle_mod.Oracle(n, bc=bc)
    c, w, opp = orc.tables()
    N = orc.N
    for cell in [(0, 0, 0), (4, 3, 2), (2, 1, 1)]:
        x = cell[0] + n[0] * (cell[1] + n[1] * cell[2])
        for i in range(19):
            fs = np.zeros((N, 19))
            fs[x, i] = 1.0
            fn = orc.stream(fs)
            assert fn.sum() == 1.0
            tgt = np.array(cell) + c[i]
            past_wall = any(bc[k] == 1 and not (0 <= tgt[k] < n[k]) for k in range(3))
            if past_wall:   # half-way bounce-back: back into the same cell, reversed
                assert fn[x, opp[i]] == 1.0
            else:
                tgt = tgt % np.array(n)
                y = tgt[0] + n[0] * (tgt[1] + n[1] * tgt[2])
                assert fn[y, i] == 1.0


def test_rest_state_is_a_fixed_point(oracle_mod):
    # the momentum sum of the rest weights cancels only to round-off in the
    # oracle's summation order, so rest is a fixed point to ~1 ulp
    orc = oracle_mod.Oracle((6, 5, 4), bc=(0, 0, 1), tau=0.7)
    f = orc.equilibrium()
    f0 = f.copy()
    orc.run(orc.to_parts(_no_particles()), f, 5)
    np.testing.assert_allclose(f, f0, rtol=0, atol=2e-16)


def _textbook_bgk(f_xyz, tau, steps):
    """Independent plain D3Q19 BGK on a periodic box: f[i, z, y, x], np.roll streaming."""
    vel = [v for v in itertools.product((-1, 0, 1), repeat=3) if sum(a * a for a in v) <= 2]
    ws = {0: 1 / 3, 1: 1 / 18, 2: 1 / 36}
    wt = np.array([ws[sum(a * a for a in v)] for v in vel])
    cv = np.array(vel, dtype=np.float64)
    f = f_xyz.copy()
    for _ in range(steps):
        rho = f.sum(axis=0)
        j = np.einsum("ia,izyx->azyx", cv, f)
        u = j / rho
        cu = np.einsum("ia,azyx->izyx", cv, u)
        uu = np.sum(u * u, axis=0)
        feq = wt[:, None, None, None] * rho * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * uu)
        f = f - (f - feq) / tau
        for i, v in enumerate(vel):
            f[i] = np.roll(f[i], shift=(v[2], v[1], v[0]), axis=(0, 1, 2))
    return f, vel


@pytest.mark.parametrize("seed", [0, 1])
def test_no_particles_reduces_to_textbook_bgk(oracle_mod, seed):
    n = (7, 6, 5)
    tau = 0.6 + 0.3 * seed
    orc = oracle_mod.Oracle(n, tau=tau)
    c, w, _ = orc.tables()
    rho, u = W.smooth_fields(n, seed, rho_amp=0.02, u_amp=0.05)
    f = orc.equilibrium(rho, u)
    rng = np.random.default_rng(seed)
    f += 1e-3 * w[None, :] * rng.standard_normal(f.shape)
    # the same state as f[i, z, y, x] in the textbook ordering
    ref0, vel = None, None
    grid = f.reshape(n[2], n[1], n[0], 19)
    _, vel = _textbook_bgk(np.zeros((19, 1, 1, 1)) + 1, tau, 0)
    perm = [next(i for i in range(19) if tuple(c[i]) == v) for v in vel]
    ref0 = np.stack([grid[..., perm[k]] for k in range(19)])
    steps = 7
    ref, _ = _textbook_bgk(ref0, tau, steps)
    orc.run(orc.to_parts(_no_particles()), f, steps)
    out = np.stack([f.reshape(n[2], n[1], n[0], 19)[..., perm[k]] for k in range(19)])
    np.testing.assert_allclose(out, ref, rtol=0, atol=5e-16)


@pytest.mark.parametrize("H,tau", [(16, 0.8), (8, 1.2), (12, 0.7)])
def test_poiseuille_discrete_closed_form(oracle_mod, H, tau):
    """Body-force channel flow between half-way walls at z = 0 and z = H.
    For BGK with exact-difference forcing the steady discrete solution is
    u_phys(z) = a z (H - z) / (2 nu) + a (6 nu - 1/(8 nu)) at cell centres
    z = k + 1/2, nu = (tau - 1/2)/3.  The parabola's curvature -a/nu holds for
    every tau; the constant is the tau-dependent wall slip."""
    a = 1e-6
    orc = oracle_mod.Oracle((1, 1, H), bc=(0, 0, 1), tau=tau, fluid_accel=(a, 0, 0))
    P = orc.to_parts(_no_particles())
    f = orc.equilibrium()
    nu = (tau - 0.5) / 3
    orc.run(P, f, int(40 * H * H / (nu * np.pi ** 2)))
    rho, u, up, B = orc.fields(P, f)
    z = np.arange(H) + 0.5
    exact = a * z * (H - z) / (2 * nu) + a * (6 * nu - 1 / (8 * nu))
    np.testing.assert_allclose(up[0], exact, rtol=2e-10, atol=0)
    np.testing.assert_allclose(np.diff(up[0], 2), -a / nu, rtol=1e-9)
    assert np.all(np.abs(up[1:]) < 1e-10 * np.max(exact))  # round-off only
    np.testing.assert_allclose(rho, 1.0, atol=1e-13)
