"""The non-learned first stage (truncated Coulomb sum over the histogram
range) as network weights, evaluated by the oracle's network: its output
difference is l_B times Eq. (Delta E_ij) of a 1:1 electrolyte restricted to
the neighbours within rc, each placed at its bin centre, up to the bfloat16
rounding of the two hidden activations that carry it."""
import numpy as np


def test_truncated_coulomb_surrogate(oracle):
    from paper_1602_05716_amd import inputs, surrogate
    rc, lB = 4.0, 0.7
    p = surrogate.truncated_coulomb_params(rc)
    assert p.size == oracle.da_nparam() and np.array_equal(p, oracle.bf16(p))
    s = inputs.electrolyte(300, 300, 1.0, -1.0, 1.0, 1.0, 0.05, lB)
    s.xyz = inputs.random_start(s, 3)
    rng = np.random.default_rng(8)
    dr = rc / 64
    for i in rng.choice(s.n, 25, replace=False):
        xt = s.xyz[i] + rng.uniform(-1.0, 1.0, 3)
        want, scale = 0.0, 0.0
        for sign, pos in ((1.0, xt), (-1.0, s.xyz[i])):
            d = np.linalg.norm(s.xyz - pos, axis=1)
            near = (d < rc) & (np.arange(s.n) != i)
            terms = s.q[i] * s.q[near] / ((np.floor(d[near] / dr) + 0.5) * dr)
            want += sign * lB * float(np.sum(terms))
            scale += lB * float(np.sum(np.abs(terms)))
        f0 = oracle.da_features(s.xyz, s.q, i, s.xyz[i], rc)
        f1 = oracle.da_features(s.xyz, s.q, i, xt, rc)
        got = lB * (oracle.mlp_eps(p, f1) - oracle.mlp_eps(p, f0))
        # each 1/r_k held at bfloat16 (2^-9 of every term) and the
        # activation rounded (2^-9 of the net sum)
        assert abs(got - want) <= 2.0 ** -7 * scale + 1e-12, (i, got, want)
