"""Training kernels of the learned indicator against the oracle, through the
C ABI: the Adam update of the FP32 master parameters (two consecutive steps,
fed the GPU's own gradients) against the FP64 Adam of oracle/mlp_oracle.py,
the packed operands the step updates in place against a full repack,
the bitwise reproducibility of a training,
and the exact-distance training samples the GPU generator draws against the
oracle's signed distance at the returned points.

Tolerances: Adam, |theta_gpu - theta_ref| <= 4 ulp(theta) + 1e-5 lr per
parameter (FP32 moments and update; the oracle repeats them in FP64 on the
GPU's gradient); samples, |t - clip(d_ref)| <= 1e-6 (the points are rounded
to FP32 after the GPU evaluated d at the unrounded point, |grad d| = 1)."""
import numpy as np
import pytest

from oracle import mlp_oracle as M
from oracle import oracle as O
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


def _sim(H, **kw):
    return H.Simulation((32, 32, 32), (0, 0, 0), 0.8, "fp64", max_particles=4, learned_max_circumradius=10.0,
                        learned_samples=200_000, **kw)


@pytest.mark.parametrize("shape,n", [(W.ROUNDED_CUBE, 4096), (W.SPHEROID, 777)])
def test_adam_steps_match_oracle(H, shape, n):
    _log(f"gpu: adam steps shape {shape} n {n}")
    sim = _sim(H)
    theta0 = W.mlp_init_params(40 + shape)
    sim.mlp_set_params(shape, theta0)
    prm = W.equal_volume_params(shape, 1.0)
    rc = W.circumradius(shape, prm)
    pts = W.mlp_points(50 + shape, n)
    t = np.array([O.Oracle.sdf(shape, np.array(prm) / rc, p) for p in pts])
    ref = theta0.astype(np.float64)
    m = np.zeros_like(ref)
    v = np.zeros_like(ref)
    for step, lr in ((1, 1e-3), (2, 5e-4)):
        g, _ = sim.mlp_train_step(shape, pts, t, lr, step)
        theta = sim.mlp_get_params(shape).astype(np.float64)
        ref, m, v = M.adam_step(ref, m, v, g, step, lr)
        ulp = np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
        err = np.abs(theta - ref)
        bound = 4 * ulp + 1e-5 * lr
        _log(f"  step {step}: max|dtheta - ref| {err.max():.3e}, moved {np.abs(theta - theta0).max():.3e}")
        assert np.all(err <= bound), int(np.argmax(err - bound))
        # the step moved every parameter with a nonzero gradient by about lr
        assert np.all(np.abs(theta - theta0)[np.abs(g) > 1e-3] > 0)
        # continue from the GPU's rounded parameters, as the GPU does
        ref = theta
    # the step rewrites the packed BF16 operands in place: the network must
    # evaluate bit for bit as after a full repack of the new parameters
    y_step = sim.mlp_eval(shape, pts[:512])
    sim.mlp_set_params(shape, sim.mlp_get_params(shape))
    np.testing.assert_array_equal(sim.mlp_eval(shape, pts[:512]), y_step)
    sim.close()


def test_train_step_rejects_bad_arguments(H):
    sim = _sim(H)
    sim.mlp_set_params(W.SPHEROID, W.mlp_init_params(1))
    pts = W.mlp_points(3, 64)
    with pytest.raises(H.HLBMError):
        sim.mlp_train_step(W.SPHEROID, pts, np.zeros(64), 0.0, 1)
    with pytest.raises(H.HLBMError):
        sim.mlp_train_step(W.SPHEROID, pts, np.zeros(64), 1e-3, 0)
    sim.close()


@pytest.mark.parametrize("shape", [W.ROUNDED_CUBE, W.SPHEROID, W.MESH])
def test_samples_match_oracle_sdf(H, shape):
    _log(f"gpu: sdf samples shape {shape}")
    if shape == W.MESH:
        sim = _sim(H, max_mesh_triangles=len(W.MESH_UNIT[1]))
        sim.set_mesh(*W.MESH_UNIT)
        O.Oracle.set_mesh(*W.MESH_UNIT)
        prm = (6.0 / W.MESH_RC, 0.0, 0.0)
        n = 3000
    else:
        sim = _sim(H)
        prm = W.equal_volume_params(shape, 6.0)
        n = 20000
    box, band, clip, share = 1.1, 0.1, 0.25, 0.8
    s = sim.mlp_samples(shape, prm[:2], n, seed=9, box=box, band=band, clip=clip, band_share=share)
    sim.close()
    rc = W.circumradius(shape, prm) if shape != W.MESH else prm[0] * W.MESH_RC
    nprm = np.array([prm[0] / rc, prm[1] / rc, 0.0])
    if shape == W.MESH:
        nprm = np.array([prm[0] / rc, 1.0, 0.0])
    d = np.array([O.Oracle.sdf(shape, nprm, p) for p in s[:, :3]])
    err = np.abs(s[:, 3] - np.clip(d, -clip, clip))
    inband = np.mean(np.abs(d) <= band)
    _log(f"  max|t - clip(d)| {err.max():.3e}; share within the band {inband:.3f}")
    assert err.max() <= 1e-6
    assert np.all(np.abs(s[:, :3]) <= box * (1 + 1e-7))
    # a band_share of the samples is redrawn into the band; the rest is uniform
    assert inband >= share - 0.02
    # the counter-based generator gives every sample its own draw
    assert len(np.unique(s[:, 0])) > 0.99 * n


def test_training_is_bitwise_reproducible(H):
    """The training path has no floating-point atomics (fixed-order partial
    sums, one workgroup per 64 parameters for the Adam step), so two
    trainings from the same parameters and seed end at the same network bit
    for bit, in two separate contexts."""
    _log("gpu: training reproducibility, 2 x 300 Adam steps")
    prm = W.equal_volume_params(W.SPHEROID, 6.0)
    res = []
    for _ in range(2):
        sim = _sim(H)
        sim.mlp_set_params(W.SPHEROID, W.mlp_init_params(5))
        rep = sim.train_indicator(W.SPHEROID, prm[:2], samples=100_000, holdout=10_000, iterations=300,
                                  batch=8192, gate_rms=1.0, gate_max=10.0)
        res.append((sim.mlp_get_params(W.SPHEROID), rep))
        sim.close()
    (t0, r0), (t1, r1) = res
    assert r0["loss_last"] < r0["loss_first"]
    np.testing.assert_array_equal(t0, t1)
    assert r0["loss_last"] == r1["loss_last"] and r0["rms_err"] == r1["rms_err"]
