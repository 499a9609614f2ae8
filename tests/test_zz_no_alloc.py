"""The allocation-free gradient entry point against hlbm_mlp_gradient, through
the C ABI: two calls in a row on the same GPU (the second with fewer samples,
so the fixed scratch holds the first call's partials when it starts), each
equal bitwise to the context entry point's gradient and loss (same kernels,
same partition); sizes beyond the fixed scratch are refused."""
import numpy as np
import pytest

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


def test_noalloc_gradient_matches_context_gradient(H):
    import torch
    theta = W.mlp_init_params(5)
    sim = H.Simulation((32, 32, 32), (0, 0, 0), 0.8, "fp64", max_particles=1, learned_max_circumradius=10.0,
                       learned_samples=10000)
    sim.mlp_set_params(W.SPHEROID, theta)
    prm = W.equal_volume_params(W.SPHEROID, 1.0)
    rc = W.circumradius(W.SPHEROID, prm)
    d_theta = torch.tensor(theta, dtype=torch.float32, device="cuda")
    d_grad = torch.empty(H.MLP_NPARAM + 1, dtype=torch.float32, device="cuda")
    for n, seed in ((2048, 61), (700, 62)):
        pts = W.mlp_points(seed, n)
        t = np.array([O.Oracle.sdf(W.SPHEROID, np.array(prm) / rc, p) for p in pts])
        g_ctx, loss_ctx = sim.mlp_gradient(W.SPHEROID, pts, t)
        smp = np.concatenate([pts, t[:, None]], axis=1).astype(np.float32)
        d_smp = torch.tensor(smp, device="cuda")
        H.mlp_gradient_noalloc(d_theta, d_smp, d_grad)
        torch.cuda.synchronize()
        g = d_grad.cpu().numpy()
        print(f"n {n}: max|g - g_ctx| {np.abs(g[:-1] - g_ctx).max():.3e}", flush=True)
        np.testing.assert_array_equal(g[:-1], g_ctx.astype(np.float32))
        # the context entry point reports the loss as the FP32 quotient sse / n
        assert np.float32(g[-1]) / np.float32(n) == np.float32(loss_ctx)
    sim.close()


def test_noalloc_rejects_sizes_beyond_scratch(H):
    import torch
    d_theta = torch.zeros(H.MLP_NPARAM, dtype=torch.float32, device="cuda")
    d_grad = torch.empty(H.MLP_NPARAM + 1, dtype=torch.float32, device="cuda")
    d_smp = torch.zeros((2049, 4), dtype=torch.float32, device="cuda")
    with pytest.raises(H.HLBMError) as e:
        H.mlp_gradient_noalloc(d_theta, d_smp, d_grad)
    assert e.value.code == -6
