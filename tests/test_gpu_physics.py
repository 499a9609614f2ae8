"""Physics checks of the GPU path through the C ABI (the path itself is held
to the oracle by tests/test_gpu_parity.py): the discrete Poiseuille closed
form, and first-order convergence of the sphere-array drag towards Hasimoto's
correlation (Sec. 5.2 reports EOC ~ 1 for the method)."""
import math

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


@pytest.mark.parametrize("precision,tol", [("fp64", 2e-10), ("fp32", 2e-4)])
def test_poiseuille_closed_form(H, precision, tol):
    H_, tau, a = 16, 0.8, 1e-6
    nu = (tau - 0.5) / 3
    sim = H.Simulation((8, 4, H_), (0, 0, 1), tau, precision, fluid_accel=(a, 0, 0))
    sim.step(int(40 * H_ * H_ / (nu * math.pi ** 2)))
    up = sim.get_fields(H.FIELD_U_PHYS)["u_phys"][0].reshape(H_, 4, 8)
    z = np.arange(H_) + 0.5
    exact = a * z * (H_ - z) / (2 * nu) + a * (6 * nu - 1 / (8 * nu))
    np.testing.assert_allclose(up, np.broadcast_to(exact[:, None, None], up.shape), rtol=tol)
    sim.close()


def _drag(H, a, tau=0.8):
    L = 8 * a
    nu = (tau - 0.5) / 3
    af = 4e-7 * (4.0 / a) ** 3
    vol = 4 / 3 * math.pi * a ** 3
    phi = vol / L ** 3
    Kh = 1 / (1 - 1.7601 * phi ** (1 / 3) + phi - 1.5593 * phi ** 2)
    t_relax = L ** 3 / (6 * math.pi * nu * a * Kh)
    sim = H.Simulation((L, L, L), (0, 0, 0), tau, "fp32", max_particles=1, fluid_accel=(af, 0, 0))
    u0 = np.zeros((3, L ** 3))
    u0[0] = af * (L ** 3 - vol) / (6 * math.pi * nu * a * Kh)
    sim.set_fields(None, u0)
    sim.set_particles(np.array([W.make_particle(W.SPHERE, (float(a),), (L / 2,) * 3, fixed=True)]))
    sim.step(int(8 * t_relax))
    fl = sim.get_fields(H.FIELD_RHO | H.FIELD_U_PHYS | H.FIELD_SOLID)
    F, _, _ = sim.get_forces()
    drive = af * np.sum(fl["rho"] * (1 - fl["B"]))
    K = drive / (6 * math.pi * nu * a * fl["u_phys"][0].mean())
    sim.close()
    return K / Kh - 1, F[0, 0] / drive


def test_sphere_array_drag_converges_first_order(H):
    radii = [4, 6, 8, 12]
    res = [_drag(H, a) for a in radii]
    errs = [e for e, _ in res]
    print("drag errors vs Hasimoto:", dict(zip(radii, [f"{e:+.4f}" for e in errs])), flush=True)
    assert all(e < 0 for e in errs)
    assert all(abs(errs[k + 1]) < abs(errs[k]) for k in range(len(errs) - 1))
    assert errs[-1] > -0.04
    eoc = math.log(errs[0] / errs[-1]) / math.log(radii[-1] / radii[0])
    assert 0.5 < eoc < 1.5, eoc
    assert all(0.85 < fb <= 1.0 for _, fb in res)
