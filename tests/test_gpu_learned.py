"""Learned indicator on the GPU, through the C ABI: the BF16 matrix-core
forward pass and gradient against the FP64 oracle network fed the same
BF16-rounded operands, training on exact signed distances, the acceptance
gate and its exact fallback, and the learned coupling against the exact one.

Tolerances: forward |y - y_ref| <= 2e-3 max|y_ref| (FP32 accumulation and the
rare BF16 rounding flip of an activation computed in FP32 instead of FP64);
gradient L2-relative <= 1e-3 overall and <= 1e-2 per parameter block."""
import numpy as np
import pytest

from oracle import mlp_oracle as M
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


def _sim(H, n=(32, 32, 32), bc=(0, 0, 0), precision="fp64", max_particles=4, rmax=10.0,
         samples=300_000, **kw):
    return H.Simulation(n, bc, 0.8, precision, max_particles=max_particles,
                        learned_max_circumradius=rmax, learned_samples=samples, **kw)


BLOCKS = [("W1", 0, 192), ("b1", 192, 256), ("W2", 256, 4352), ("b2", 4352, 4416),
          ("W3", 4416, 8512), ("b3", 8512, 8576), ("W4", 8576, 8640), ("b4", 8640, 8641)]


@pytest.mark.parametrize("seed", [0, 1])
def test_forward_matches_oracle(H, seed):
    _log(f"gpu: mlp forward seed {seed}")
    sim = _sim(H)
    theta = W.mlp_init_params(seed)
    sim.mlp_set_params(W.ROUNDED_CUBE, theta)
    pts = W.mlp_points(seed + 20, 3000)
    y = sim.mlp_eval(W.ROUNDED_CUBE, pts)
    yref, _ = M.forward(theta.astype(np.float64), pts, bf16=True)
    err = np.abs(y - yref)
    _log(f"  max err {err.max():.3e} median {np.median(err):.3e} scale {np.abs(yref).max():.3e}")
    assert err.max() <= 2e-3 * np.abs(yref).max()
    assert np.median(err) <= 1e-5 * np.abs(yref).max()
    np.testing.assert_array_equal(sim.mlp_get_params(W.ROUNDED_CUBE), theta)
    sim.close()


@pytest.mark.parametrize("seed,n", [(0, 4096), (1, 1000), (2, 77), (3, 20000)])
def test_gradient_matches_oracle(H, seed, n):
    """Batch sizes that fill, and do not fill, the 32-sample pairs and the
    gradient workgroups; 20 000 samples give each workgroup two pairs (the
    two wavefronts' per-lane sums then span several tiles) and a last
    workgroup with one."""
    _log(f"gpu: mlp gradient seed {seed} n {n}")
    sim = _sim(H)
    theta = W.mlp_init_params(seed + 3)
    sim.mlp_set_params(W.SPHEROID, theta)
    pts = W.mlp_points(seed + 30, n)
    prm = W.equal_volume_params(W.SPHEROID, 1.0)
    rc = W.circumradius(W.SPHEROID, prm)
    from oracle import oracle as O
    t = np.array([O.Oracle.sdf(W.SPHEROID, np.array(prm) / rc, p) for p in pts])
    g, L = sim.mlp_gradient(W.SPHEROID, pts, t)
    gref, Lref = M.gradient(theta.astype(np.float64), pts, t, bf16=True)
    rel = np.linalg.norm(g - gref) / np.linalg.norm(gref)
    _log(f"  loss {L:.6e} ref {Lref:.6e}  grad rel {rel:.3e}")
    assert abs(L - Lref) <= 1e-3 * Lref
    assert rel <= 1e-3
    for name, a, b in BLOCKS:
        rb = np.linalg.norm(g[a:b] - gref[a:b]) / max(np.linalg.norm(gref[a:b]), 1e-30)
        assert rb <= 1e-2, (name, rb)
    sim.close()


def _train(sim, shape, r_eq, iterations, **kw):
    prm = W.equal_volume_params(shape, r_eq)
    sim.mlp_set_params(shape, W.mlp_init_params(7 + shape))
    rep = sim.train_indicator(shape, prm[:2], iterations=iterations, **kw)
    return prm, rep


def test_training_reduces_loss_and_falls_back_to_exact(H):
    """A gate no network can pass keeps the exact indicator: the coupled run is
    bitwise the run of a context that never trained."""
    n, bc = (40, 40, 40), (0, 0, 1)
    parts = np.array([W.make_particle(W.ROUNDED_CUBE, W.equal_volume_params(W.ROUNDED_CUBE, 5.0),
                                      (20.3, 19.6, 21.1), quat=W.shoemake_quaternion(
                                          np.random.default_rng(2)))])
    sim = _sim(H, n, bc, samples=240_000)
    _log("gpu: short training, impossible gate")
    prm, rep = _train(sim, W.ROUNDED_CUBE, 5.0, 400, samples=200_000, holdout=20_000, batch=4096,
                      gate_rms=1e-9, gate_max=1e-9)
    _log(f"  {rep}")
    assert rep["loss_last"] < 0.2 * rep["loss_first"]
    assert rep["accepted"] == 0
    sim.set_particles(parts)
    sim.step(20)
    F, T, _ = sim.get_forces()
    ref = _sim(H, n, bc, samples=1000)
    ref.set_particles(parts)
    ref.step(20)
    Fr, Tr, _ = ref.get_forces()
    np.testing.assert_array_equal(F, Fr)
    np.testing.assert_array_equal(T, Tr)
    sim.close()
    ref.close()


TRAIN = dict(samples=1_000_000, holdout=100_000, iterations=30000, batch=8192, lr=1e-2, lr_final=1e-5,
             band=0.1, clip=0.25, band_share=0.8, gate_rms=0.05, gate_max=0.5)


def test_learned_coupling_against_exact(H):
    """Rounded cubes and spheroids (volume of a sphere of radius 6) with
    trained networks against the exact indicator on the same workload:
    porosity on smoothed-boundary cells, solid volume, time-averaged forces
    (<= 1 % RMS over particles) and the step time with each."""
    import time
    import torch
    n, bc = (96, 96, 96), (0, 0, 1)
    rng = np.random.default_rng(11)
    shapes = [W.ROUNDED_CUBE, W.SPHEROID] * 3
    prms = [W.equal_volume_params(s, 6.0) for s in shapes]
    rcs = np.array([W.circumradius(s, p) for s, p in zip(shapes, prms)])
    pos = W.rsa_positions(rng, rcs, n, bc, gap=2.0, wall_margin=2.0)
    parts = np.array([W.make_particle(s, p, x, quat=W.shoemake_quaternion(rng))
                      for s, p, x in zip(shapes, prms, pos)])
    out = {}
    for mode in ("exact", "learned"):
        _log(f"gpu: coupled run, {mode} indicator")
        sim = _sim(H, n, bc, "fp32", max_particles=8, samples=1_100_000, gravity=(0, 0, -1e-5))
        if mode == "learned":
            for s in (W.ROUNDED_CUBE, W.SPHEROID):
                p = W.equal_volume_params(s, 6.0)
                sim.mlp_set_params(s, W.mlp_init_params(7 + s))
                rep = sim.train_indicator(s, p[:2], ref_circumradius=W.circumradius(s, p), **TRAIN)
                _log(f"  family {s}: {rep}")
                assert rep["accepted"] == 1
        sim.set_particles(parts)
        B0 = sim.get_fields(H.FIELD_SOLID)["B"]
        acc = np.zeros((len(parts), 3))
        for _ in range(30):
            sim.step(10)
            acc += sim.get_forces()[0]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(200)
        torch.cuda.synchronize()
        out[mode] = dict(B0=B0, F=acc / 30, ms=(time.perf_counter() - t0) / 200 * 1e3)
        sim.close()
    ex, le = out["exact"], out["learned"]
    band = ((ex["B0"] > 0) & (ex["B0"] < 1)) | ((le["B0"] > 0) & (le["B0"] < 1))
    dB = np.abs(le["B0"] - ex["B0"])[band]
    ferr = np.sqrt(np.mean(np.sum((le["F"] - ex["F"]) ** 2, 1)) / np.mean(np.sum(ex["F"] ** 2, 1)))
    _log(f"  porosity L1 {dB.mean():.4f} Linf {dB.max():.4f}  volume {le['B0'].sum():.1f} vs "
         f"{ex['B0'].sum():.1f}  force RMS rel {ferr:.4f}  step ms learned {le['ms']:.4f} "
         f"exact {ex['ms']:.4f} (learned/exact {le['ms'] / ex['ms']:.2f})")
    assert ferr <= 0.01
    assert dB.mean() <= 0.05
    assert abs(le["B0"].sum() / ex["B0"].sum() - 1) <= 5e-3
    assert le["ms"] > 0 and ex["ms"] > 0


@pytest.mark.parametrize("shape,r_eq,eps", [(W.ROUNDED_CUBE, 6.0, 0.5), (W.SPHEROID, 6.0, 0.5), (W.MESH, 6.0, 0.5),
                                            (W.SPHEROID, 2.0, 2.0)])
def test_band_grid_settles_only_far_cells(H, oracle_mod, shape, r_eq, eps):
    """The band grid of a trained shape settles the table cells whose distance
    is certainly beyond +-eps/2 and leaves the others to the network.  With a
    network that answers d = 0 everywhere, every cell the network decides has
    B = 1/2 exactly, so the settled cells can be told apart: each must carry
    the exact indicator of the FP64 oracle (0 or 1), every cell of the exact
    band 0 < B < 1 must have been left to the network, and the cells left to
    it may number at most four times the band (without the grid the whole
    shell between r_in - eps/2 and R_c + eps/2 is queried).  The small
    spheroid with eps = 2 reaches past the grid (|b| up to 1.31 of R_c
    against its half-width 1.25): those cells are always queried."""
    n, bc = (48, 36, 32), (0, 0, 1)
    rng = np.random.default_rng(3 + shape)
    prm = W.equal_volume_params(shape, r_eq)
    # the particle straddles the periodic x face
    parts = np.array([W.make_particle(shape, prm, (1.3, 17.6, 15.2), quat=W.shoemake_quaternion(rng))])
    kw = {}
    if shape == W.MESH:
        v, t = W.MESH_UNIT
        kw["max_mesh_triangles"] = len(t)
    sim = _sim(H, n, bc, "fp64", max_particles=1, samples=8192, eps=eps, **kw)
    if shape == W.MESH:
        sim.set_mesh(v, t)
    _log(f"gpu: band grid of shape {shape}, r_eq {r_eq}, eps {eps}, network d = 0")
    sim.mlp_set_params(shape, W.mlp_init_params(7 + shape))
    sim.train_indicator(shape, prm[:2], samples=4096, holdout=64, iterations=1, batch=1024,
                        gate_rms=1e-9, gate_max=1e-9)
    sim.mlp_set_params(shape, np.zeros(H.MLP_NPARAM, dtype=np.float32))
    sim.set_indicator(shape, H.INDICATOR_LEARNED)
    sim.set_particles(parts)
    B = sim.get_fields(H.FIELD_SOLID)["B"]
    sim.close()
    if shape == W.MESH:
        oracle_mod.Oracle.set_mesh(v, t)
    orc = oracle_mod.Oracle(n, bc, 0.8, eps=eps)
    Bo, _ = orc.coupling(orc.to_parts(parts))
    queried = np.abs(B - 0.5) <= 1e-12
    band = (Bo > 0) & (Bo < 1)
    _log(f"  queried {int(queried.sum())}  exact band {int(band.sum())}  "
         f"settled {int((~queried).sum())} (B = 1: {int((B == 1).sum())})")
    np.testing.assert_array_equal(B[~queried], Bo[~queried])
    assert queried[band].all()
    assert band.sum() > 100 and queried.sum() <= 4 * band.sum()
    if eps > 1.0:  # cells beyond the grid are queried even where far from the surface
        assert queried.sum() > band.sum()
