"""The allocation-free gradient pass (mc_mlp_grad_noalloc) against the
allocating one (mc_mlp_grad), through the C ABI: the same kernels on the
same inputs, so loss and gradient agree to the last bit; two calls in a row,
the second with a smaller batch (the workspace keeps the first call's
contents), and the size limit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_noalloc_gradient_matches_the_allocating_pass(oracle):
    from paper_1602_05716_amd import mc
    rng = np.random.default_rng(77)
    p = oracle.bf16(rng.normal(0.0, 0.08, oracle.da_nparam()))
    for batch in (256, 64):
        print("[gpu-case] noalloc batch %d" % batch, flush=True)
        f = rng.integers(0, 5, (batch, 256)).astype(np.uint8)
        y = rng.normal(0.0, 1.0, batch)
        loss, g = mc.mlp_grad_noalloc(f, y, p)
        ref_loss, ref_g = mc.mlp_grad(f, y, p)
        assert loss == ref_loss
        assert np.array_equal(g, ref_g)
        # and both against the oracle's double backpropagation
        o_loss, o_g = oracle.mlp_loss_grad(p, f[:, :128].astype(float), f[:, 128:].astype(float), y)
        assert loss == pytest.approx(o_loss, rel=2e-3)
        assert np.linalg.norm(g[:-1] - o_g[:-1]) <= 1e-2 * np.linalg.norm(o_g[:-1])
    with pytest.raises(mc.MCError) as ei:
        mc.mlp_grad_noalloc(np.zeros((288, 256), np.uint8), np.zeros(288), p)
    assert ei.value.code == -1 and "exceeds" in str(ei.value)
