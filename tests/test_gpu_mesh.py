"""Triangle-mesh particles (HLBM_MESH) through the library against the FP64
oracle, and the learned indicator's gain over the exact mesh distance.

The library reads the distance of mesh particles from a per-particle table
over the coupling box (the layout the learned indicator uses), filled each
step with the exact distance (FP64, stored in FP32).  The FP32 storage bounds
the parity of the FP64 path: the indicator depends on d only in the band
|d| < eps/2, where it moves by at most its slope pi / eps times the FP32
rounding of d (eps/2 2^-24), i.e. 1e-7 (measured 1.4e-8); velocity, force
and torque follow at that level (measured 5e-11, 3e-10, 3e-9 relative)."""
import time

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


def _l2rel(a, b, floor=0.0):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), floor * np.sqrt(b.size), 1e-300))


def _mesh_case(seed=5):
    rng = np.random.default_rng(seed)
    s = W.equal_volume_params(W.MESH, 4.0)
    recs = []
    for x in ((16.0, 24.0, 14.0), (40.0, 20.0, 25.0), (30.0, 36.0, 20.0)):
        recs.append(W.make_particle(W.MESH, s, np.array(x) + rng.uniform(-0.5, 0.5, 3),
                                    quat=W.shoemake_quaternion(rng), vel=tuple(rng.normal(0, 2e-3, 3)),
                                    omega=tuple(rng.normal(0, 2e-4, 3)), density_ratio=2.0))
    recs.append(W.make_particle(W.SPHERE, (3.0,), (50.3, 40.6, 12.2), density_ratio=2.0))
    return np.array(recs)


def test_mesh_particles_match_oracle(H, oracle_mod):
    n, bc, tau, g = (64, 48, 40), (0, 0, 1), 0.8, (0.0, 0.0, -1e-5)
    v, t = W.MESH_UNIT
    parts = _mesh_case()
    rho, u = W.smooth_fields(n, 21, rho_amp=1e-3, u_amp=1e-2)
    steps = (1, 9, 10)
    _log(f"gpu: {len(t)}-triangle mesh particles, fp64, steps {steps}")
    sim = H.Simulation(n, bc, tau, "fp64", max_particles=len(parts), gravity=g, max_mesh_triangles=len(t),
                       learned_max_circumradius=6.0)
    sim.set_mesh(v, t)
    sim.set_fields(rho, u)
    sim.set_particles(parts)
    for k in steps:
        sim.step(k)
    F, T, st = sim.get_forces()
    fl = sim.get_fields()
    sim.close()
    _log("oracle")
    oracle_mod.Oracle.set_mesh(v, t)
    orc = oracle_mod.Oracle(n, bc, tau, gravity=g)
    P = orc.to_parts(parts)
    f = orc.equilibrium(rho, u)
    Fo, To = orc.run(P, f, sum(steps))
    rho_o, u_o, up_o, B_o = orc.fields(P, f)
    eB = float(np.max(np.abs(fl["B"] - B_o)))
    eu = _l2rel(fl["u"], u_o, 1e-4)
    eF = float(np.max(np.abs(F - Fo)) / np.max(np.abs(Fo)))
    eT = float(np.max(np.abs(T - To)) / np.max(np.abs(To)))
    ex = float(np.max(np.abs(st["pos"] - P["X"])))
    _log(f"  max|dB| {eB:.2e}  L2rel(u) {eu:.2e}  F {eF:.2e}  T {eT:.2e}  max|dX| {ex:.2e}")
    assert eB <= 1e-7
    assert eu <= 1e-9
    assert float(np.max(np.abs(fl["rho"] - rho_o))) <= 1e-12
    assert eF <= 1e-8 and eT <= 1e-7
    assert ex <= 1e-10
