"""Pins of the oracle's partially saturated collision (the PSM family that
Sec. 3.2 names as a possible host of the scheme; operator of Noble and
Torczynski 1998): the solid weight's limits, mass conservation, the momentum
change rho [B_n (u_s - u) + (1 - B_n) a_f] that follows from the operator's
moments, the fluid limit (identical to the exact-difference collision), the
solid limit (momentum rho u_s, non-equilibrium reversed)."""
import numpy as np
import pytest


def _random_f(orc, rng):
    rho = 1 + 0.05 * rng.standard_normal()
    u = 0.05 * rng.standard_normal(3)
    return orc.feq(rho, u) * (1 + 0.02 * rng.standard_normal(19))


def _moments(c, f):
    return f.sum(), c.T @ f


@pytest.mark.parametrize("tau", [0.55, 0.8, 1.3])
def test_solid_weight_limits(oracle_mod, tau):
    orc = oracle_mod.Oracle((4, 4, 4), tau=tau, coupling="psm")
    assert orc.psm_weight(0.0) == 0.0
    assert abs(orc.psm_weight(1.0) - 1.0) < 1e-15
    B = np.linspace(0, 1, 101)
    w = np.array([orc.psm_weight(b) for b in B])
    assert np.all(np.diff(w) > 0)
    # below the solid fraction for any finite relaxation time
    assert np.all(w[1:-1] < B[1:-1])
    # and tends to it for a very long relaxation time
    big = oracle_mod.Oracle((4, 4, 4), tau=1e9, coupling="psm")
    assert max(abs(big.psm_weight(b) - b) for b in B) < 1e-8


@pytest.mark.parametrize("seed", range(4))
def test_mass_and_momentum_change(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    af = 1e-4 * rng.standard_normal(3)
    orc = oracle_mod.Oracle((4, 4, 4), tau=0.6 + rng.random(), fluid_accel=af, coupling="psm")
    c, _, _ = orc.tables()
    for B in (0.0, 0.3, 0.77, 1.0):
        f = _random_f(orc, rng)
        us = 0.03 * rng.standard_normal(3)
        fs = orc.collide_cell(f, B, us)
        rho, j = _moments(c, f)
        rho_s, j_s = _moments(c, fs)
        Bn = orc.psm_weight(B)
        u = j / rho
        assert abs(rho_s - rho) < 1e-15
        np.testing.assert_allclose(j_s - j, rho * (Bn * (us - u) + (1 - Bn) * af), rtol=0, atol=2e-16)


def test_fluid_limit_equals_exact_difference_collision(oracle_mod):
    rng = np.random.default_rng(7)
    af = (2e-5, -1e-5, 3e-5)
    psm = oracle_mod.Oracle((4, 4, 4), tau=0.7, fluid_accel=af, coupling="psm")
    edm = oracle_mod.Oracle((4, 4, 4), tau=0.7, fluid_accel=af)
    for _ in range(5):
        f = _random_f(psm, rng)
        np.testing.assert_allclose(psm.collide_cell(f, 0.0, (0.01, 0, 0)), edm.collide_cell(f, 0.0, (0.01, 0, 0)),
                                   rtol=0, atol=1e-17)


def test_solid_limit_reverses_nonequilibrium(oracle_mod):
    """B = 1: f*_i - feq_i(rho, u_s) = f_opp(i) - feq_opp(i)(rho, u), so the
    post-collision momentum is rho u_s whatever the fluid did."""
    rng = np.random.default_rng(8)
    orc = oracle_mod.Oracle((4, 4, 4), tau=0.9, fluid_accel=(1e-4, 0, 0), coupling="psm")
    c, _, opp = orc.tables()
    f = _random_f(orc, rng)
    us = np.array([0.02, -0.01, 0.005])
    fs = orc.collide_cell(f, 1.0, us)
    rho, j = _moments(c, f)
    feq = orc.feq(rho, j / rho)
    np.testing.assert_allclose(fs - orc.feq(rho, us), (f - feq)[opp], rtol=0, atol=6e-17)
    np.testing.assert_allclose(c.T @ fs, rho * us, rtol=0, atol=1e-16)


def test_whole_step_without_particles_is_plain_bgk(oracle_mod):
    """No particles: every cell is fluid and the PSM run equals the HLBM run."""
    from paper_2312_14172_amd import workloads as W
    n = (12, 10, 8)
    rho, u = W.smooth_fields(n, 3, rho_amp=1e-2, u_amp=2e-2)
    runs = []
    for coupling in ("hlbm", "psm"):
        orc = oracle_mod.Oracle(n, (0, 1, 0), 0.7, fluid_accel=(1e-5, 0, 0), coupling=coupling)
        f = orc.equilibrium(rho, u)
        orc.run(orc.to_parts(np.zeros(0, dtype=W.PARTICLE_DTYPE)), f, 5)
        runs.append(f)
    np.testing.assert_array_equal(runs[0], runs[1])


@pytest.mark.parametrize("B", [0.25, 0.6])
def test_stress_relaxes_at_the_reduced_rate(oracle_mod, B):
    """With u_s = u and no body force the solid collision reverses the
    non-equilibrium part, which leaves its second moment unchanged, so the
    non-equilibrium stress relaxes by 1 - (1 - B_n)/tau per step."""
    rng = np.random.default_rng(11)
    orc = oracle_mod.Oracle((4, 4, 4), tau=0.8, coupling="psm")
    c, _, _ = orc.tables()
    f = _random_f(orc, rng)
    rho, j = _moments(c, f)
    u = j / rho
    fs = orc.collide_cell(f, B, u)
    feq = orc.feq(rho, u)
    cc = np.einsum("ia,ib->iab", c, c)
    Pi = np.einsum("iab,i->ab", cc, f - feq)
    Pis = np.einsum("iab,i->ab", cc, fs - feq)
    Bn = orc.psm_weight(B)
    np.testing.assert_allclose(Pis, (1 - (1 - Bn) / 0.8) * Pi, rtol=0, atol=1e-15)
