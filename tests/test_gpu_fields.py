"""Observables through the C ABI: FP32 field output (the same values as the
FP64 output, rounded to nearest) and the library's volume-flux reduction
(mean u_phys over all cells and over the pure-fluid cells, B = 0) against the
oracle's fields on the same state."""
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


def _state(H, precision="fp64"):
    n, bc = (70, 26, 30), (0, 0, 1)
    parts = W.random_particles_small(n, 4, 5, r_eq=(2.5, 3.5), bc=bc)
    rho, u = W.smooth_fields(n, 17, rho_amp=1e-3, u_amp=1e-2)
    a = (1e-6, -2e-6, 3e-6)
    sim = H.Simulation(n, bc, 0.8, precision, max_particles=len(parts), gravity=(0, 0, -1e-5), fluid_accel=a)
    sim.set_fields(rho, u)
    sim.set_particles(parts)
    sim.step(7)
    return sim, n, bc, parts, rho, u, a


def test_fp32_fields_are_fp64_fields_rounded(H):
    sim, *_ = _state(H)
    f64 = sim.get_fields()
    f32 = sim.get_fields(dtype="fp32")
    dev32 = sim.get_fields(H.FIELD_U_PHYS | H.FIELD_SOLID, on_device=True, dtype="fp32").cpu().numpy()
    sim.close()
    for k in ("rho", "u", "u_phys", "B"):
        assert f32[k].dtype == np.float32
        np.testing.assert_array_equal(f32[k], f64[k].astype(np.float32))
    np.testing.assert_array_equal(dev32[:3], f64["u_phys"].astype(np.float32))
    np.testing.assert_array_equal(dev32[3], f64["B"].astype(np.float32))


def test_bad_dtype_rejected(H):
    import ctypes
    sim = H.Simulation((16, 8, 8), (0, 0, 0), 0.8, "fp32")
    out = np.zeros(16 * 8 * 8)
    rc = H.lib().hlbm_get_fields(sim._ctx, H.FIELD_RHO, 2, out.ctypes.data, 0)
    assert rc == -1
    sim.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_mean_velocity_matches_oracle_fields(H, oracle_mod, precision):
    sim, n, bc, parts, rho, u, a = _state(H, precision)
    mean_all, mean_fluid, nfluid = sim.get_mean_velocity()
    fl = sim.get_fields(H.FIELD_U_PHYS | H.FIELD_SOLID)
    sim.close()
    # the same reduction of the library's own FP64 fields
    fluid = fl["B"] == 0.0
    np.testing.assert_allclose(mean_all, fl["u_phys"].mean(axis=1), rtol=1e-12, atol=1e-18)
    np.testing.assert_allclose(mean_fluid, fl["u_phys"][:, fluid].mean(axis=1), rtol=1e-12, atol=1e-18)
    assert nfluid == int(fluid.sum())
    # against the oracle's state after the same steps
    orc = oracle_mod.Oracle(n, bc, 0.8, gravity=(0, 0, -1e-5), fluid_accel=a)
    P = orc.to_parts(parts)
    f = orc.equilibrium(rho, u)
    orc.run(P, f, 7)
    _, _, up_o, B_o = orc.fields(P, f)
    fo = B_o == 0.0
    assert nfluid == int(fo.sum())
    scale = float(np.max(np.abs(up_o)))
    tol = 1e-13 if precision == "fp64" else 1e-5
    np.testing.assert_allclose(mean_all, up_o.mean(axis=1), rtol=0, atol=tol * scale)
    np.testing.assert_allclose(mean_fluid, up_o[:, fo].mean(axis=1), rtol=0, atol=tol * scale)


def test_mean_velocity_is_reproducible(H):
    sim, *_ = _state(H, "fp32")
    a = sim.get_mean_velocity()
    b = sim.get_mean_velocity()
    sim.close()
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
