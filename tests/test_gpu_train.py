"""Training of the delayed-acceptance surrogate on the GPU (C ABI).

The forward and backward passes (bfloat16 matrix-core products with float
sums) are checked against the oracle's double-precision backpropagation on
the same bfloat16 weights and inputs -- norm-wise relative error <= 1e-2 per
parameter block.  Training on moves logged from a plain run must lower the
loss, predict held-out dE, and -- what the network buys the two-stage test --
cut the stage-2 rejection rate of stage-1 passes below that of the test
without a network (dEh = 0: stage 1 passes everything and stage 2 is the
plain Metropolis test).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)


BLOCKS = [("W1", 0, 128 * 128), ("b1", 128 * 128, 128), ("W2", 128 * 128 + 128, 128 * 128),
          ("b2", 2 * 128 * 128 + 128, 128), ("w3", 2 * 128 * 128 + 256, 128)]


@pytest.mark.parametrize("batch,scale", [(64, 0.1), (256, 0.05)])
def test_gradients_match_double_backprop(oracle, batch, scale):
    from paper_1602_05716_amd import mc
    rng = np.random.default_rng(batch)
    p = oracle.bf16(rng.normal(0.0, scale, oracle.da_nparam()))
    f = rng.integers(0, 4, (batch, 256)).astype(np.uint8)
    y = rng.normal(0.0, 1.0, batch)
    _say("mlp grad batch=%d" % batch)
    loss, g = mc.mlp_grad(f, y, p)
    ref_loss, ref_g = oracle.mlp_loss_grad(p, f[:, :128].astype(float), f[:, 128:].astype(float), y)
    assert loss == pytest.approx(ref_loss, rel=2e-3)
    for name, o, n in BLOCKS:
        a, b = g[o:o + n], ref_g[o:o + n]
        err = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        assert err <= 1e-2, (name, err)
    assert abs(g[-1]) < 1e-5  # b3 cancels in the difference


def test_training_learns_dE_and_helps_the_two_stage_test(oracle):
    from paper_1602_05716_amd import inputs, mc
    sy = inputs.electrolyte(2048, 2048, 1.0, -1.0, 1.0, 1.0, 0.05, 0.7)
    sy.xyz = inputs.random_start(sy, 51)
    sweeps = 12
    n_log = sweeps * sy.n
    _say("log %d moves, N=%d" % (n_log, sy.n))
    with mc.Chain(sy.xyz, sy.q, sy.sigma, sy.R, sy.lB, precision="fp32", max_disp=1.5, log_moves=n_log,
                  resum_every=0, waves=4) as ch:
        ch.sweep(sweeps, 77)
        lg = ch.get_log(n_log)
        tr = ch.train_surrogate(n_log, epochs=12, batch=512, lr=2e-3, seed=5)
        zero = np.zeros(oracle.da_nparam())
        z = ch.train_surrogate(n_log, epochs=1, batch=512, lr=1e-12, seed=5, params_in=zero)
        _say("losses", np.round(tr["loss"], 4), "val", tr["val_loss"], "ref", tr["ref_stage2_reject"],
             "zero-network ref", z["ref_stage2_reject"])
        # the loss falls and held-out dE is predicted
        ok = ((lg["flags"] & 0x87) == 0x80)
        y = lg["dE"][ok] / sy.lB
        assert tr["loss"][-1] < 0.6 * tr["loss"][0]
        assert tr["val_loss"] < 0.5 * np.var(y), (tr["val_loss"], np.var(y))
        # the gain: stage 2 rejects far fewer of the stage-1 passes
        assert tr["ref_stage2_reject"] < 0.7 * z["ref_stage2_reject"]
        # and the trained network drives the chain: the two-stage test runs
        ch.set_surrogate(tr["params"], tr["ref_stage2_reject"], True)
        st0 = ch.stats()
        ch.sweep(4, 78)
        st1 = ch.stats()
        passed = st1["da_stage1_passed"] - st0["da_stage1_passed"]
        rej2 = st1["da_stage2_rejected"] - st0["da_stage2_rejected"]
        assert passed > 1000 and st1["da_active"] == 1
        _say("stage-2 rejection rate in the run %.4f (reference %.4f)" % (rej2 / passed, tr["ref_stage2_reject"]))
        assert abs(rej2 / passed - tr["ref_stage2_reject"]) < 0.1
