"""Hindered-settling reference values (CPU): the Schiller-Naumann terminal
Reynolds number, the expansion indices and correlations of Sec. 5, and the
set-up in lattice units.  Pinned against their limits and closed forms."""
import math

import pytest

from paper_2312_14172_amd import settling as S


def test_schiller_naumann_balance_and_stokes_limit():
    # the returned Re satisfies (3/4) C_d Re^2 = Ar with C_d = 24/Re (1 + 0.15 Re^0.687)
    for Ar in (1.0, 100.0, 1500.0, 5e4):
        Re = S.reynolds_schiller_naumann(Ar)
        cd = 24.0 / Re * (1.0 + 0.15 * Re ** 0.687)
        assert abs(0.75 * cd * Re * Re - Ar) <= 1e-9 * Ar
    # creeping flow: C_d -> 24/Re, so Re -> Ar / 18 (Stokes settling); the
    # relative gap is the Schiller-Naumann correction 0.15 Re^0.687
    for Ar in (1e-6, 1e-3):
        Re = S.reynolds_schiller_naumann(Ar)
        gap = (Ar / 18.0 - Re) / Re
        assert 0.0 < gap <= 0.151 * Re ** 0.687


def test_expansion_indices():
    assert S.n_richardson_zaki(0.1) == 4.65
    assert S.n_richardson_zaki(600.0) == 2.39
    assert abs(S.n_richardson_zaki(0.5) - 4.35 * 0.5 ** -0.03) < 1e-15
    assert abs(S.n_richardson_zaki(31.84) - 4.45 * 31.84 ** -0.1) < 1e-15
    # Garside-Al-Dibouni: 5.1 in creeping flow, 2.7 at high Re
    assert abs(S.n_garside_al_dibouni(1e-12) - 5.1) < 1e-9
    assert abs(S.n_garside_al_dibouni(1e12) - 2.7) < 1e-6


def test_barnea_mizrahi_and_power_law_limits():
    assert S.barnea_mizrahi(0.0) == 1.0
    # monotone decrease in phi
    vals = [S.barnea_mizrahi(p) for p in (0.05, 0.1, 0.2, 0.3)]
    assert all(a > b for a, b in zip(vals, vals[1:]))
    assert S.power_law(0.0, 4.0) == 1.0
    assert abs(S.power_law(0.2, 2.0) - 0.64) < 1e-15


def test_particle_counts_and_lattice_setup():
    # Sec. 5.1 / 5.4: 166 spheres at phi = 0.05 and 991 at phi = 0.3 in a 12 D cube
    assert S.particle_count(0.05) == 166
    assert S.particle_count(0.3) == 991
    s = S.setup(Ar=1500.0, ratio=1.3, tau=0.55, N=12)
    nu = 0.05 / 3.0
    assert abs(s["nu"] - nu) < 1e-15
    # Ar recovered from g, D, the density ratio and nu
    assert abs(s["g"] * 12 ** 3 * 0.3 / nu ** 2 - 1500.0) < 1e-9
    # u* from Re, and the Stokes velocity g D^2 (ratio - 1) / (18 nu)
    assert abs(s["u_star"] * 12 / nu - s["Re"]) < 1e-9
    assert abs(s["u_st"] - s["g"] * 144 * 0.3 / (18 * nu)) < 1e-15
    assert abs(s["t_star"] - 12 / s["u_st"]) < 1e-12


@pytest.mark.parametrize("N", [5, 12, 27])
def test_setup_scales_with_resolution(N):
    # at fixed Ar and tau: g ~ N^-3, u* ~ N^-1, t* ~ N^2
    a, b = S.setup(N=12), S.setup(N=N)
    r = N / 12.0
    assert abs(b["g"] * r ** 3 - a["g"]) < 1e-12 * a["g"]
    assert abs(b["u_star"] * r - a["u_star"]) < 1e-12 * a["u_star"]
    assert abs(b["t_star"] / r ** 2 - a["t_star"]) < 1e-9 * a["t_star"]
    assert math.isclose(b["Re"], a["Re"])
