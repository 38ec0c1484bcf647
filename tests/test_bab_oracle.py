"""Pins of the oracle's branch and bound (App. B.1, Alg. 1) against the exact
minimum of tiny networks, found by enumerating every activation pattern of the
root-unstable neurons (each pattern makes the network affine; its minimum over
the box and the pattern's half-planes is found by vertex enumeration).  No GPU."""
import itertools

import numpy as np
import pytest

from oracle import bab as ob
from oracle import beta_crown as bc
from tests import pinlib


def tiny_net(seed, widths=(2, 5, 4, 1), eps=0.6):
    rng = np.random.default_rng(seed)
    net = pinlib.random_net(rng, list(widths))
    x0 = rng.uniform(-0.5, 0.5, size=widths[0])
    x_lo, x_hi = x0 - eps, x0 + eps
    lo, up = bc.root_bounds(net, x_lo, x_hi)
    return net, x_lo, x_hi, lo, up


def exact_min(net, C, x_lo, x_hi, lo, up):
    uns = [(i, j) for i in range(len(lo)) for j in range(lo[i].shape[0]) if lo[i][j] < 0 < up[i][j]]
    best = np.inf
    for signs in itertools.product((1, -1), repeat=len(uns)):
        split = [np.zeros(l.shape[0], np.int8) for l in lo]
        for (i, j), s in zip(uns, signs):
            split[i][j] = s
        best = min(best, pinlib.vertex_min_2d(net, C, x_lo, x_hi, lo, up, split)[0])
    return best, len(uns)


def shifted(net, t):
    """The same network with t subtracted from its single output."""
    W, b = net[-1]
    return net[:-1] + [(W, b - t)]


@pytest.mark.parametrize("seed", range(6))
def test_bab_decides_like_the_exact_minimum(seed):
    net, x_lo, x_hi, lo, up = tiny_net(seed + 500)
    C = np.ones((1, 1))
    fstar, n_uns = exact_min(net, C, x_lo, x_hi, lo, up)
    if n_uns > 9 or n_uns < 2:
        pytest.skip("enumeration size")
    cfg = bc.AdamConfig(iters=60, lr_alpha=0.1, lr_beta=0.2)
    for t in (fstar - 0.05 * max(1.0, abs(fstar)), fstar + 0.05 * max(1.0, abs(fstar))):
        r = ob.bab(shifted(net, t), x_lo, x_hi, C, lo, up, batch=4, max_rounds=400, cfg=cfg)
        target = fstar - t
        # sound both ways, and complete on the proving side (every neuron split makes the bound exact,
        # Theorem 3.1 / Cor. 3.2.1); a counter-example needs the box minimiser x* of some leaf to be one,
        # which Alg. 1 does not promise, so a false property may end undecided
        assert r["lb"] <= target + 1e-9 and r["ub"] >= target - 1e-9, (r, target)
        if target > 0:
            assert r["verdict"] == "verified", (r, target)
        else:
            assert r["verdict"] in ("falsified", "unknown"), (r, target)


def test_branch_order_is_by_chord_intercept():
    lo = [np.array([-1.0, -3.0, 0.5, -2.0]), np.array([-1.0, 2.0])]
    up = [np.array([1.0, 1.0, 2.0, 2.0]), np.array([4.0, 3.0])]
    # intercepts -l u / (u - l): 0.5, 0.75, stable, 1.0 | 0.8, stable
    assert ob.branch_order(lo, up) == [(0, 3), (1, 0), (0, 1), (0, 0)]


def test_root_already_verified_or_falsified():
    net, x_lo, x_hi, lo, up = tiny_net(3)
    C = np.ones((1, 1))
    fstar, _ = exact_min(net, C, x_lo, x_hi, lo, up)
    r = ob.bab(shifted(net, fstar - 100.0), x_lo, x_hi, C, lo, up)
    assert r["verdict"] == "verified" and r["rounds"] == 0 and r["domains"] == 1
    r = ob.bab(shifted(net, fstar + 100.0), x_lo, x_hi, C, lo, up)
    assert r["verdict"] == "falsified" and r["rounds"] == 0


def test_library_branch_order_matches_oracle():
    """The library driver's host-side branching order (layers 1-based) is the oracle's."""
    from oracle import bab as ob
    from paper_2103_06624_amd import bab as gb
    rng = np.random.default_rng(1)
    lo = [rng.uniform(-2, 1, size=7), rng.uniform(-2, 1, size=5)]
    up = [l + rng.uniform(0.1, 3, size=l.shape) for l in lo]
    o = ob.branch_order(lo, up)
    g = gb.branch_order(np.concatenate(lo), np.concatenate(up), [7, 5])
    assert g == [(i + 1, j) for i, j in o]


@pytest.mark.parametrize("seed", range(6))
def test_warm_started_bab_keeps_the_guarantees(seed):
    """Children started from their parent's final alpha, beta: still sound
    both ways and complete on the proving side (any start gives a sound bound,
    and a fully split subdomain's bound is exact)."""
    net, x_lo, x_hi, lo, up = tiny_net(seed + 500)
    C = np.ones((1, 1))
    fstar, n_uns = exact_min(net, C, x_lo, x_hi, lo, up)
    if n_uns > 9 or n_uns < 2:
        pytest.skip("enumeration size")
    cfg = bc.AdamConfig(iters=60, lr_alpha=0.1, lr_beta=0.2)
    for t in (fstar - 0.05 * max(1.0, abs(fstar)), fstar + 0.05 * max(1.0, abs(fstar))):
        r = ob.bab(shifted(net, t), x_lo, x_hi, C, lo, up, batch=4, max_rounds=400, cfg=cfg, warm=True)
        target = fstar - t
        assert r["lb"] <= target + 1e-9 and r["ub"] >= target - 1e-9, (r, target)
        if target > 0:
            assert r["verdict"] == "verified", (r, target)
        else:
            assert r["verdict"] in ("falsified", "unknown"), (r, target)


def test_delta_exit_stops_once_the_bounds_meet():
    """Alg. 1's f-bar - f-underbar <= delta exit: a delta wider than the
    root's gap stops before any round; a moderate one stops as soon as the
    gap closes to it (the search without delta runs on), and the reported
    bounds still bracket the exact minimum."""
    for seed in range(500, 520):
        net, x_lo, x_hi, lo, up = tiny_net(seed)
        C = np.ones((1, 1))
        fstar, n_uns = exact_min(net, C, x_lo, x_hi, lo, up)
        if 3 <= n_uns <= 9:
            break
    cfg = bc.AdamConfig(iters=60, lr_alpha=0.1, lr_beta=0.2)
    t = fstar - 0.05 * max(1.0, abs(fstar))  # a true property: the search proves it
    net_t = shifted(net, t)
    full = ob.bab(net_t, x_lo, x_hi, C, lo, up, batch=1, max_rounds=400, cfg=cfg)
    wide = ob.bab(net_t, x_lo, x_hi, C, lo, up, batch=1, max_rounds=400, cfg=cfg, delta=1e6)
    assert wide["rounds"] == 0 and wide["verdict"] == "unknown"
    assert wide["lb"] <= fstar - t <= wide["ub"] + 1e-9
    gap0 = wide["ub"] - wide["lb"]
    mid = ob.bab(net_t, x_lo, x_hi, C, lo, up, batch=1, max_rounds=400, cfg=cfg, delta=0.5 * gap0)
    assert mid["lb"] <= fstar - t + 1e-9
    assert mid["rounds"] <= full["rounds"]
    if mid["verdict"] == "unknown":
        assert mid["ub"] - mid["lb"] <= 0.5 * gap0 + 1e-12
