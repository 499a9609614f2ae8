"""Edge cases of the GPU path through the C ABI: the largest particles the
binning and the momentum-exchange layout accept (circumradius 27.4, a box of
56 z-layers and 16 tiles per axis), overlapping smooth regions (S0 > 1,
Sec. 3 indicator sum), and the capacity and divergence errors the kernels
report through the status word.

Tolerances of the FP64 parity case as in test_gpu_parity.py."""
import numpy as np
import pytest

from paper_2312_14172_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2312_14172_amd import hlbm
    hlbm.lib()
    return hlbm


def _log(msg):
    print(msg, flush=True)


def _l2rel(a, b, floor):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), floor * np.sqrt(b.size)))


def test_largest_particles_overlapping_fp64(H, oracle_mod):
    """A sphere of radius 27.4 and a spheroid of semi-axes 27.2 / 8 that
    overlap it, both moving and spinning, on a 64^3 periodic lattice: the
    largest boxes the library accepts (56 momentum-exchange layers, 16 tiles
    per axis), cells covered by both smooth regions, 3 steps against the
    oracle."""
    n, bc, tau, g = (64, 64, 64), (0, 0, 0), 0.8, (0.0, 0.0, -1e-5)
    q = np.array([0.9, 0.2, -0.3, 0.25])
    q /= np.linalg.norm(q)
    parts = np.array([
        W.make_particle(W.SPHERE, (27.4,), (31.3, 32.6, 30.9), vel=(0.004, -0.003, 0.002), omega=(0.0, 2e-4, -1e-4)),
        W.make_particle(W.SPHEROID, (27.2, 8.0), (36.2, 28.7, 35.4), quat=tuple(q), vel=(-0.003, 0.002, 0.001),
                        omega=(3e-4, 0.0, 2e-4)),
    ])
    rho, u = W.smooth_fields(n, 21, rho_amp=1e-3, u_amp=5e-3)
    _log("gpu: largest particles, overlapping, 64^3 FP64")
    sim = H.Simulation(n, bc, tau, "fp64", max_particles=2, gravity=g)
    sim.set_fields(rho, u)
    sim.set_particles(parts)
    sim.step(1)
    sim.step(2)
    F, T, st = sim.get_forces()
    fl = sim.get_fields()
    sim.close()
    orc = oracle_mod.Oracle(n, bc, tau, gravity=g)
    P = orc.to_parts(parts)
    f = orc.equilibrium(rho, u)
    Fo, To = orc.run(P, f, 3)
    rho_o, u_o, up_o, B_o = orc.fields(P, f)
    both = np.sum(B_o > 0.999)
    _log(f"  L2rel(u)={_l2rel(fl['u'], u_o, 1e-4):.3e}  |F| {np.abs(Fo).max():.3e}  solid cells {both}")
    assert _l2rel(fl["u"], u_o, 1e-4) <= 1e-12
    assert _l2rel(fl["u_phys"], up_o, 1e-4) <= 1e-12
    assert np.max(np.abs(fl["rho"] - rho_o)) <= 1e-14
    np.testing.assert_allclose(fl["B"], B_o, rtol=0, atol=1e-13)
    np.testing.assert_allclose(F, Fo, rtol=0, atol=1e-10 * np.max(np.abs(Fo)))
    np.testing.assert_allclose(T, To, rtol=0, atol=1e-9 * np.max(np.abs(To)))
    np.testing.assert_allclose(st["pos"], P["X"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(st["quat"], P["q"], rtol=0, atol=1e-12)


def test_tile_overflow_is_reported(H):
    """49 or more particles whose coupling boxes touch one 64 x 4 x 4 tile
    exceed the tile lists: set_particles reports HLBM_EUNSUPPORTED; with 48
    the same layout binds and steps."""
    n = (64, 8, 8)
    recs = [W.make_particle(W.SPHERE, (0.6,), (0.7 + 1.25 * i, 2.0, 2.0)) for i in range(50)]
    sim = H.Simulation(n, (0, 0, 0), 0.8, "fp32", max_particles=50)
    with pytest.raises(H.HLBMError) as e:
        sim.set_particles(np.array(recs))
    assert e.value.code == -6
    sim.set_particles(np.array(recs[:48]))
    sim.step(3)
    F, _, _ = sim.get_forces()
    assert F.shape == (48, 3) and np.all(np.isfinite(F))
    sim.close()


def test_particle_leaving_through_wall_is_reported(H):
    """A heavy sphere driven through a wall: once its centre is outside the
    walls the next get_* call reports HLBM_EUNSTABLE, and the context is
    usable again after new particles are set."""
    n, bc = (16, 16, 32), (0, 0, 1)
    rec = W.make_particle(W.SPHERE, (2.0,), (8.0, 8.0, 4.0), density_ratio=200.0, vel=(0.0, 0.0, -0.1))
    sim = H.Simulation(n, bc, 0.8, "fp32", max_particles=1, gravity=(0.0, 0.0, 0.0))
    sim.set_particles(np.array([rec]))
    sim.step(80)
    with pytest.raises(H.HLBMError) as e:
        sim.get_forces()
    assert e.value.code == -5
    _log(f"  reported: {e.value}")
    sim.set_fields(None, None)
    rec["pos"] = (8.0, 8.0, 16.0)
    rec["vel"] = (0.0, 0.0, 0.0)
    sim.set_particles(np.array([rec]))
    sim.step(2)
    F, _, st = sim.get_forces()
    assert np.all(np.isfinite(F)) and abs(st["pos"][0][2] - 16.0) < 1e-3
    sim.close()
