"""CPU checks of the batch planner (mc_plan_schedule, host only): the plan
that decides how many workgroups each chain of a batch gets and which chains
share a workgroup.  The sharing rule and the cost model are the library's
own design (the paper runs one chain per device); these tests pin the plan's
invariants and that sharing never makes the predicted sweep time worse."""
import numpy as np
import pytest

A, B = 1.2, 1.3


def _plan(nb, scale=None, measured=None, budget=512, a=A, b=B):
    from paper_1602_05716_amd import mc
    return mc.plan_schedule(nb, scale, measured, a, b, budget)


def _cost(nb, scale, w, a=A, b=B):
    return scale * (a * nb + b * nb * nb / max(1, w))


def _check_valid(nb, scale, measured, budget, wg, items, n_launch):
    nb = np.asarray(nb)
    n = len(nb)
    assert n_launch <= budget
    assert (wg >= 1).all() and (wg <= nb).all()
    # every chain's workgroups 0..w-1 appear exactly once
    for k in range(n):
        idx = sorted(items[items[:, 0] == k, 1].tolist())
        assert idx == list(range(wg[k])), (k, idx, wg[k])
    # launch workgroups 0..n_launch-1 each run at least one item
    assert sorted(set(items[:, 2].tolist())) == list(range(n_launch))
    # a shared launch workgroup holds only measured single-workgroup chains
    for w in range(n_launch):
        ks = items[items[:, 2] == w, 0]
        if len(ks) > 1:
            for k in ks:
                assert measured is not None and measured[k] and wg[k] == 1, (w, ks)


def _predicted_ms(nb, scale, wg, items, n_launch):
    t = np.zeros(n_launch)
    for k, j, w in items:
        t[w] += _cost(nb[k], scale[k], wg[k])
    return t.max()


def test_single_chain_takes_the_budget_up_to_its_groups():
    wg, items, nl = _plan([512], budget=512)
    assert wg.tolist() == [512] and nl == 512
    wg, items, nl = _plan([100], budget=512)
    assert wg.tolist() == [100] and nl == 100
    wg, items, nl = _plan([1], budget=7)
    assert wg.tolist() == [1] and nl == 1


def test_equal_chains_split_the_budget_evenly():
    wg, items, nl = _plan([64] * 8, budget=512)
    assert wg.tolist() == [64] * 8 and nl == 512


def test_unmeasured_chains_never_share():
    rng = np.random.default_rng(3)
    nb = rng.integers(1, 80, size=40)
    wg, items, nl = _plan(nb, budget=256)
    _check_valid(nb, np.ones(40), None, 256, wg, items, nl)
    assert nl == wg.sum()


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4])
def test_measured_small_chains_share_and_time_does_not_grow(seed):
    rng = np.random.default_rng(seed)
    n = 48
    nb = np.concatenate([rng.integers(1, 8, size=n - 4), rng.integers(40, 64, size=4)]).astype(np.int32)
    scale = rng.uniform(0.7, 1.4, size=n)
    measured = np.ones(n, np.uint8)
    budget = 96
    wg, items, nl = _plan(nb, scale, measured, budget)
    _check_valid(nb, scale, measured, budget, wg, items, nl)
    assert nl < wg.sum(), "small measured chains should share workgroups"
    t_pack = _predicted_ms(nb, scale, wg, items, nl)
    wg0, items0, nl0 = _plan(nb, scale, None, budget)
    _check_valid(nb, scale, None, budget, wg0, items0, nl0)
    t_plain = _predicted_ms(nb, scale, wg0, items0, nl0)
    assert t_pack <= t_plain * (1 + 1e-9), (t_pack, t_plain)


def test_only_measured_chains_are_packed():
    nb = np.array([2, 2, 2, 2, 2, 2, 50], np.int32)
    measured = np.array([1, 1, 1, 0, 0, 0, 1], np.uint8)
    wg, items, nl = _plan(nb, None, measured, budget=20)
    _check_valid(nb, np.ones(7), measured, 20, wg, items, nl)
    shared = [w for w in range(nl) if (items[:, 2] == w).sum() > 1]
    assert shared, "the three measured small chains should share"
    for w in shared:
        assert set(items[items[:, 2] == w, 0].tolist()) <= {0, 1, 2}


def test_large_measured_chains_do_not_share():
    # every chain needs more than one workgroup to stay within the sweep time
    nb = np.full(8, 64, np.int32)
    wg, items, nl = _plan(nb, None, np.ones(8, np.uint8), budget=512)
    assert wg.tolist() == [64] * 8 and nl == 512


def test_grid_orders_heavy_with_light():
    # launch workgroup i and i + W/2 pair heavy work with light work
    nb = np.array([200, 10], np.int32)
    wg, items, nl = _plan(nb, budget=40)
    work = np.zeros(nl)
    for k, j, w in items:
        work[w] += nb[k] ** 2 / wg[k]
    half = (nl + 1) // 2
    assert work[:half].min() >= work[half:].max()


def test_rejects_bad_arguments():
    from paper_1602_05716_amd import mc
    with pytest.raises(mc.MCError):
        _plan([4, 4, 4], budget=2)
    with pytest.raises(mc.MCError):
        _plan([0], budget=4)
    with pytest.raises(mc.MCError):
        _plan([4], scale=[-1.0], budget=4)
    with pytest.raises(mc.MCError):
        _plan([4], budget=4, a=0.0)
