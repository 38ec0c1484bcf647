"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

No GPU.  Every test below would fail on a plausible slip in the oracle: a
dropped constant term, a wrong sign of S, a swapped relaxation branch, a
transposed weight or a wrong box minimiser.
"""
import json
import os

import numpy as np
import pytest

from oracle import beta_crown as bc
from tests import pinlib

HERE = os.path.dirname(os.path.abspath(__file__))


def tiny_case(seed, widths=(2, 6, 5, 2), eps=0.6, m=2):
    rng = np.random.default_rng(seed)
    net = pinlib.random_net(rng, list(widths))
    x0 = rng.uniform(-0.5, 0.5, size=widths[0])
    x_lo, x_hi = x0 - eps, x0 + eps
    lo, up = bc.root_bounds(net, x_lo, x_hi)
    C = rng.standard_normal((m, widths[-1]))
    return rng, net, x0, eps, x_lo, x_hi, lo, up, C


def unstable_list(lo, up):
    return [(i, j) for i in range(len(lo)) for j in range(lo[i].shape[0]) if lo[i][j] < 0 < up[i][j]]


def random_vars(rng, lo, m, split=None, beta_scale=1.0):
    alpha = [rng.uniform(0, 1, size=(m, l.shape[0])) for l in lo]
    beta = [rng.uniform(0, beta_scale, size=(m, l.shape[0])) * (0 if split is None else (split[i] != 0))
            for i, l in enumerate(lo)]
    return alpha, beta


def random_split(rng, lo, up, k):
    split = [np.zeros(l.shape[0], np.int8) for l in lo]
    uns = unstable_list(lo, up)
    if not uns:
        return split
    for t in rng.choice(len(uns), size=min(k, len(uns)), replace=False):
        i, j = uns[t]
        split[i][j] = rng.choice([-1, 1])
    return split


# ---------------------------------------------------------------------------
# network plumbing


@pytest.mark.parametrize("cfg", [((3, 8, 8), 5, 4, 2, 1), ((8, 16, 16), 7, 4, 2, 1), ((8, 16, 16), 8, 3, 1, 1),
                                 ((3, 9, 9), 4, 4, 2, 0), ((2, 5, 7), 3, 3, 2, 1)])
def test_conv_matrix_matches_library_conv(cfg):
    torch = pytest.importorskip("torch")
    (ci, h, w), co, k, s, p = cfg
    rng = np.random.default_rng(0)
    wt = rng.standard_normal((co, ci, k, k))
    ho, wo = (h + 2 * p - k) // s + 1, (w + 2 * p - k) // s + 1
    M = bc.conv_as_matrix(wt, (ci, h, w), (co, ho, wo), s, p)
    x = rng.standard_normal((ci, h, w))
    ref = torch.nn.functional.conv2d(torch.from_numpy(x)[None], torch.from_numpy(wt), stride=s, padding=p)[0]
    assert np.allclose(M @ x.ravel(), ref.numpy().ravel(), atol=1e-12)


def test_first_layer_bounds_are_exact_interval_bounds():
    _, net, _, _, x_lo, x_hi, lo, up, _ = tiny_case(1, widths=(3, 7, 4, 2))
    W, b = net[0]
    ctr, rad = (x_lo + x_hi) / 2, (x_hi - x_lo) / 2
    assert np.allclose(lo[0], W @ ctr - np.abs(W) @ rad + b, atol=1e-12)
    assert np.allclose(up[0], W @ ctr + np.abs(W) @ rad + b, atol=1e-12)


@pytest.mark.parametrize("seed", range(4))
def test_root_bounds_enclose_grid(seed):
    _, net, _, _, x_lo, x_hi, lo, up, _ = tiny_case(seed, widths=(2, 7, 6, 5, 2))
    zs, _ = pinlib.forward_all(net, pinlib.grid(x_lo, x_hi, 401))
    for i, z in enumerate(zs):
        assert np.all(z.min(0) >= lo[i] - 1e-9) and np.all(z.max(0) <= up[i] + 1e-9)
    # the relaxations actually bite (otherwise the other pins are vacuous)
    assert len(unstable_list(lo, up)) >= 3


# ---------------------------------------------------------------------------
# T1: soundness against brute force, any alpha in [0,1], beta >= 0


@pytest.mark.parametrize("seed", range(6))
def test_sound_against_grid(seed):
    rng, net, _, _, x_lo, x_hi, lo, up, C = tiny_case(seed, widths=(2, 6, 6, 2), m=2)
    for trial in range(4):
        split = random_split(rng, lo, up, k=trial)
        alpha, beta = random_vars(rng, lo, C.shape[0], split, beta_scale=2.0)
        g = bc.bound(net, x_lo, x_hi, C, lo, up, split, alpha, beta)
        gm = pinlib.grid_min(net, C, x_lo, x_hi, split, n=601)
        assert np.all(g <= gm + 1e-9), (g, gm)


def test_sound_against_dense_grid_2001():
    rng, net, _, _, x_lo, x_hi, lo, up, C = tiny_case(7, widths=(2, 8, 6, 2), m=2)
    split = random_split(rng, lo, up, k=2)
    cfg = bc.AdamConfig(iters=60, lr_alpha=0.1, lr_beta=0.1)
    best, *_ = bc.optimize(net, x_lo, x_hi, C, lo, up, split, [bc.default_alpha(l, u) * np.ones((2, 1)) for l, u in
                                                                 zip(lo, up)], [np.zeros((2, l.shape[0])) for l in lo], cfg)
    gm = pinlib.grid_min(net, C, x_lo, x_hi, split, n=2001)
    assert np.all(best <= gm + 1e-9)


# ---------------------------------------------------------------------------
# T4 / Cor. 3.2.1: weak duality against the LP, and the LP duals attain it


@pytest.mark.parametrize("seed", range(5))
def test_weak_duality_and_dual_attainment(seed):
    rng, net, _, _, x_lo, x_hi, lo, up, C = tiny_case(seed + 20, widths=(2, 6, 5, 2), m=1)
    split = random_split(rng, lo, up, k=2)
    p_lp, res, tags = pinlib.lp_verify_split(net, x_lo, x_hi, C[0], lo, up, split)
    assert res.status == 0
    for _ in range(5):
        alpha, beta = random_vars(rng, lo, 1, split, beta_scale=3.0)
        g = bc.bound(net, x_lo, x_hi, C, lo, up, split, alpha, beta)[0]
        assert g <= p_lp + 1e-8
    a_star, b_star = pinlib.duals_to_alpha_beta(res, tags, [l.shape[0] for l in lo])
    g_star = bc.bound(net, x_lo, x_hi, C, lo, up, split, [a[None] for a in a_star], [b[None] for b in b_star])[0]
    assert abs(g_star - p_lp) <= 1e-7 * max(1.0, abs(p_lp)), (g_star, p_lp)


# ---------------------------------------------------------------------------
# T6: exactness when every unstable neuron is split


@pytest.mark.parametrize("seed", range(8))
def test_exact_when_fully_split(seed):
    rng, net, _, _, x_lo, x_hi, lo, up, C = tiny_case(seed + 40, widths=(2, 5, 4, 2), m=1)
    uns = unstable_list(lo, up)
    if len(uns) > 9:
        pytest.skip("too many unstable neurons for the enumeration")
    split = [np.zeros(l.shape[0], np.int8) for l in lo]
    for (i, j) in uns:
        split[i][j] = rng.choice([-1, 1])
    exact = pinlib.vertex_min_2d(net, C, x_lo, x_hi, lo, up, split)[0]
    p_lp, res, _ = pinlib.lp_verify_split(net, x_lo, x_hi, C[0], lo, up, split)
    alpha0 = [np.zeros((1, l.shape[0])) for l in lo]
    slots = [(i, j) for i in range(len(lo)) for j in np.nonzero(split[i])[0]]

    def affine(bvec):
        beta = [np.zeros((1, l.shape[0])) for l in lo]
        for v, (i, j) in zip(bvec, slots):
            beta[i][0, j] = v
        g, A0, _ = bc.bound(net, x_lo, x_hi, C, lo, up, split, alpha0, beta, keep=True)
        return A0[0], g[0] - np.minimum(A0[0] * x_lo, A0[0] * x_hi).sum()

    g_max = pinlib.max_over_beta_lp(affine, len(slots), x_lo, x_hi)
    if np.isinf(exact):
        # T7: an infeasible split pattern has an unbounded dual
        assert res.status == 2 and np.isinf(g_max)
    else:
        assert abs(exact - p_lp) <= 1e-7 * max(1, abs(exact))
        assert abs(g_max - exact) <= 1e-7 * max(1, abs(exact)), (g_max, exact)
        # and the concave beta problem is reachable by the projected ascent
        cfg = bc.AdamConfig(iters=400, lr_alpha=0.0, lr_beta=0.05, decay=0.995)
        best, *_ = bc.optimize(net, x_lo, x_hi, C, lo, up, split, alpha0, [np.zeros((1, l.shape[0])) for l in lo], cfg)
        assert best[0] <= exact + 1e-9 and best[0] >= exact - 2e-2 * max(1, abs(exact))


# ---------------------------------------------------------------------------
# T2: three formulas for g agree


@pytest.mark.parametrize("seed", range(6))
def test_dual_nu_form_matches(seed):
    rng, net, x0, eps, x_lo, x_hi, lo, up, C = tiny_case(seed + 60, widths=(3, 6, 5, 4, 2), m=2)
    split = random_split(rng, lo, up, k=3)
    alpha, beta = random_vars(rng, lo, 2, split, beta_scale=2.0)
    g = bc.bound(net, x_lo, x_hi, C, lo, up, split, alpha, beta)
    for r in range(2):
        gd, _ = pinlib.dual_nu_bound(net, x0, eps, C[r], lo, up, split, [a[r] for a in alpha], [b[r] for b in beta])
        assert abs(gd - g[r]) <= 1e-10 * max(1, abs(g[r]))


@pytest.mark.parametrize("seed", range(6))
def test_explicit_theorem_form_matches(seed):
    rng, net, x0, eps, x_lo, x_hi, lo, up, C = tiny_case(seed + 80, widths=(3, 6, 5, 4, 2), m=2)
    split = random_split(rng, lo, up, k=3)
    alpha, beta = random_vars(rng, lo, 2, split, beta_scale=2.0)
    g = bc.bound(net, x_lo, x_hi, C, lo, up, split, alpha, beta)
    for r in range(2):
        _, nuhats = pinlib.dual_nu_bound(net, x0, eps, C[r], lo, up, split, [a[r] for a in alpha],
                                         [b[r] for b in beta])
        Ds, lbs = [], []
        for i, nh in enumerate(nuhats):  # A(i) = -nu-hat(i); D, lowerb by Eq. definition_D/lowerb
            A = -nh
            l, u, s = lo[i], up[i], split[i]
            D = np.zeros_like(A)
            lb = np.zeros_like(A)
            for j in range(A.shape[0]):
                if s[j] > 0 or (s[j] == 0 and l[j] >= 0):
                    D[j] = 1.0
                elif s[j] < 0 or u[j] <= 0:
                    D[j] = 0.0
                elif A[j] >= 0:
                    D[j] = alpha[i][r, j]
                else:
                    D[j] = u[j] / (u[j] - l[j])
                    lb[j] = -u[j] * l[j] / (u[j] - l[j])
            Ds.append(D)
            lbs.append(lb)
        ge = pinlib.explicit_bound(net, x_lo, x_hi, C[r], Ds, lbs, split, [b[r] for b in beta])
        assert abs(ge - g[r]) <= 1e-10 * max(1, abs(g[r]))


# ---------------------------------------------------------------------------
# T3: beta = 0 reproduces alpha-CROWN with splits as modified bounds


@pytest.mark.parametrize("seed", range(6))
def test_beta_zero_is_alpha_crown(seed):
    rng, net, _, _, x_lo, x_hi, lo, up, C = tiny_case(seed + 100, widths=(4, 8, 7, 6, 3), m=3)
    split = random_split(rng, lo, up, k=4)
    alpha, _ = random_vars(rng, lo, 3)
    beta0 = [np.zeros((3, l.shape[0])) for l in lo]
    g = bc.bound(net, x_lo, x_hi, C, lo, up, split, alpha, beta0)
    for r in range(3):
        ref = pinlib.alpha_crown_modified_bounds(net, x_lo, x_hi, C[r], lo, up, split, [a[r] for a in alpha])
        assert abs(ref - g[r]) <= 1e-11 * max(1, abs(g[r]))


# ---------------------------------------------------------------------------
# T8: gradient against central finite differences


@pytest.mark.parametrize("seed", range(4))
def test_gradient_matches_central_differences(seed):
    rng, net, _, _, x_lo, x_hi, lo, up, C = tiny_case(seed + 120, widths=(5, 8, 7, 6, 3), m=2)
    split = random_split(rng, lo, up, k=3)
    alpha, beta = random_vars(rng, lo, 2, split, beta_scale=0.5)
    alpha = [np.clip(a, 0.05, 0.95) for a in alpha]
    beta = [np.where(s != 0, b + 0.1, 0.0) for b, s in zip(beta, split)]
    g, ga, gb = bc.bound_and_grad(net, x_lo, x_hi, C, lo, up, split, alpha, beta)
    h = 1e-3

    def pattern(a, b):
        _, A0, tr = bc.bound(net, x_lo, x_hi, C, lo, up, split, a, b, keep=True)
        return [np.sign(A0)] + [np.sign(t[0]) for t in tr]

    base = pattern(alpha, beta)
    checked = 0
    for which, vars_, grads in (("a", alpha, ga), ("b", beta, gb)):
        for i in range(len(vars_)):
            for r in range(2):
                for j in range(vars_[i].shape[1]):
                    uns = lo[i][j] < 0 < up[i][j] and split[i][j] == 0
                    if (which == "a" and not uns) or (which == "b" and split[i][j] == 0):
                        assert grads[i][r, j] == 0.0
                        continue
                    p, q = [v.copy() for v in vars_], [v.copy() for v in vars_]
                    p[i][r, j] += h
                    q[i][r, j] -= h
                    args_p = (p, beta) if which == "a" else (alpha, p)
                    args_q = (q, beta) if which == "a" else (alpha, q)
                    if any((np.any(x != y) or np.any(x != z)) for x, y, z in
                           zip(base, pattern(*args_p), pattern(*args_q))):
                        continue
                    fd = (bc.bound(net, x_lo, x_hi, C, lo, up, split, *args_p)[r] -
                          bc.bound(net, x_lo, x_hi, C, lo, up, split, *args_q)[r]) / (2 * h)
                    assert abs(fd - grads[i][r, j]) <= 1e-7 + 1e-6 * abs(fd), (which, i, r, j, fd, grads[i][r, j])
                    checked += 1
    assert checked >= 10


# ---------------------------------------------------------------------------
# hand-derived values (tests/golden/hand_example.json holds the derivations)


def test_hand_derived_example():
    with open(os.path.join(HERE, "golden", "hand_example.json")) as f:
        fx = json.load(f)
    for case in fx["cases"]:
        net = [(np.array(W, float), np.array(b, float)) for W, b in case["net"]]
        lo = [np.array(v, float) for v in case["l"]]
        up = [np.array(v, float) for v in case["u"]]
        split = [np.array(v, np.int8) for v in case["split"]]
        C = np.array(case["C"], float)
        alpha = [np.array(v, float)[None] for v in case["alpha"]]
        beta = [np.array(v, float)[None] for v in case["beta"]]
        x_lo, x_hi = np.array(case["x_lo"], float), np.array(case["x_hi"], float)
        g, ga, gb = bc.bound_and_grad(net, x_lo, x_hi, C, lo, up, split, alpha, beta)
        assert abs(g[0] - case["g"]) <= 1e-12, (case["name"], g[0], case["g"])
        if "dg_dalpha" in case:
            assert np.allclose(ga[0][0], case["dg_dalpha"], atol=1e-12), case["name"]
            assert np.allclose(gb[0][0], case["dg_dbeta"], atol=1e-12), case["name"]


# ---------------------------------------------------------------------------
# optimiser


def test_adam_first_step_is_normalised_sign():
    cfg = bc.AdamConfig()
    th, m, v = bc.adam_ascent_step(np.array([0.5, 0.5, 0.5]), np.array([3.0, -0.02, 0.0]), np.zeros(3), np.zeros(3), 1,
                                   0.01, cfg)
    assert np.allclose(th, [0.51, 0.49, 0.5], atol=1e-7)


def test_adam_schedule_constant_gradient_trajectories():
    """The 20-step schedule itself: decay exponent, both learning rates and
    both projections (tests/golden/adam_schedule.json derives every value)."""
    with open(os.path.join(HERE, "golden", "adam_schedule.json")) as f:
        fx = json.load(f)
    net = [(np.array(W, float), np.array(b, float)) for W, b in fx["net"]]
    x_lo, x_hi = np.array(fx["x_lo"], float), np.array(fx["x_hi"], float)
    lo = [np.array(v, float) for v in fx["l"]]
    up = [np.array(v, float) for v in fx["u"]]
    C = np.array(fx["C"], float)
    for case in fx["cases"]:
        split = [np.array(case["split"], np.int8)]
        a0 = [np.array([[case["alpha0"]]])]
        b0 = [np.array([[case["beta0"]]])]
        cfg = bc.AdamConfig(iters=fx["iters"], lr_alpha=case["lr_alpha"], lr_beta=case["lr_beta"], decay=fx["decay"])
        best, a, b, _ = bc.optimize(net, x_lo, x_hi, C, lo, up, split, a0, b0, cfg)
        assert abs(a[0][0, 0] - case["alpha_final"]) <= 1e-12, (case["name"], a[0][0, 0])
        assert abs(b[0][0, 0] - case["beta_final"]) <= 1e-12, (case["name"], b[0][0, 0])
        assert abs(best[0] - case["best"]) <= 1e-11, (case["name"], best[0])


def test_default_alpha_rule():
    assert list(bc.default_alpha(np.array([-1.0, -2.0, -1.0]), np.array([2.0, 1.0, 1.0]))) == [1.0, 0.0, 1.0]


@pytest.mark.parametrize("seed", range(3))
def test_optimise_monotone_and_below_lp(seed):
    rng, net, _, _, x_lo, x_hi, lo, up, C = tiny_case(seed + 140, widths=(2, 6, 5, 2), m=1)
    split = random_split(rng, lo, up, k=2)
    a0 = [bc.default_alpha(l, u)[None] for l, u in zip(lo, up)]
    b0 = [np.zeros((1, l.shape[0])) for l in lo]
    g0 = bc.bound(net, x_lo, x_hi, C, lo, up, split, a0, b0)
    best, a, b, gf = bc.optimize(net, x_lo, x_hi, C, lo, up, split, a0, b0, bc.AdamConfig(lr_alpha=0.1))
    p_lp, res, _ = pinlib.lp_verify_split(net, x_lo, x_hi, C[0], lo, up, split)
    assert best[0] >= g0[0] - 1e-12 and best[0] >= gf[0]
    assert best[0] <= p_lp + 1e-8
    assert all(np.all((x >= 0) & (x <= 1)) for x in a) and all(np.all(x >= 0) for x in b)


# ---------------------------------------------------------------------------
# The primal side: ub = C f(x*) at the box minimiser (Alg. 1 and its footnote)


@pytest.mark.parametrize("seed", range(6))
def test_upper_bound_is_the_network_at_the_dual_minimiser(seed):
    """x* rebuilt from the Theorem 3.2 dual form (coefficient of x = -nu-hat(0),
    minimised over the l-inf ball coordinate by coordinate); the network run
    forward at that point by an independent evaluator gives ub, its split
    pre-activations give sat and margin."""
    rng, net, x0, eps, x_lo, x_hi, lo, up, C = tiny_case(seed + 200, widths=(3, 6, 5, 4, 2), m=2)
    split = random_split(rng, lo, up, k=3)
    alpha, beta = random_vars(rng, lo, 2, split, beta_scale=2.0)
    g, ub, sat, margin = bc.upper_bound(net, x_lo, x_hi, C, lo, up, split, alpha, beta)
    for r in range(2):
        gd, _, nh0 = pinlib.dual_nu_bound(net, x0, eps, C[r], lo, up, split, [a[r] for a in alpha],
                                          [b[r] for b in beta], with_input=True)
        assert abs(gd - g[r]) <= 1e-10 * max(1, abs(g[r]))
        coef = -nh0
        xs = np.where(coef > 0, x_lo, np.where(coef < 0, x_hi, x0))
        zs, logits = pinlib.forward_all(net, xs[None, :])
        assert abs(ub[r] - C[r] @ logits[0]) <= 1e-10 * max(1, abs(ub[r]))
        ok = all(np.all(z[0][s > 0] >= 0) and np.all(z[0][s < 0] <= 0) for z, s in zip(zs, split))
        mg = min([np.abs(z[0][s != 0]).min() for z, s in zip(zs, split) if (s != 0).any()] + [np.inf])
        assert bool(sat[r]) == ok
        assert mg == margin[r] or abs(mg - margin[r]) <= 1e-12 * max(1.0, mg)


@pytest.mark.parametrize("seed", range(4))
def test_upper_bound_meets_lower_bound_where_the_network_is_affine(seed):
    """Biases large enough that every hidden neuron is active on the box: the
    network is affine there, the relaxation is exact, and x* is the true
    minimiser, so g = ub."""
    rng = np.random.default_rng(seed + 300)
    net = pinlib.random_net(rng, [3, 5, 4, 2])
    # hidden layers after the first take |W| so that positive inputs stay positive
    net = [(W if i == 0 or i == len(net) - 1 else np.abs(W), b + (25.0 if i < len(net) - 1 else 0.0))
           for i, (W, b) in enumerate(net)]
    x_lo = rng.uniform(-0.5, 0.0, size=3)
    x_hi = x_lo + 0.8
    lo, up = bc.root_bounds(net, x_lo, x_hi)
    assert all((l > 0).all() for l in lo)
    C = rng.standard_normal((3, 2))
    alpha = [rng.uniform(0, 1, size=(3, l.shape[0])) for l in lo]
    beta = [np.zeros((3, l.shape[0])) for l in lo]
    split = [np.zeros(l.shape[0], np.int8) for l in lo]
    g, ub, sat, margin = bc.upper_bound(net, x_lo, x_hi, C, lo, up, split, alpha, beta)
    assert np.allclose(g, ub, rtol=0, atol=1e-9 * max(1.0, np.abs(g).max()))
    assert sat.all() and np.isinf(margin).all()


@pytest.mark.parametrize("seed", range(6))
def test_upper_bound_brackets_the_minimum(seed):
    """x* is a point of the box, so ub is at least the unsplit problem's
    minimum, hence at least any sound lower bound of it (here the brute-force
    grid minimum minus the grid's reach is not needed: the unsplit bound at any
    alpha is below the minimum); where x* meets the splits, the subdomain's
    own lower bound is below ub too."""
    rng, net, _, _, x_lo, x_hi, lo, up, C = tiny_case(seed + 400, widths=(2, 6, 6, 2), m=2)
    none = [np.zeros(l.shape[0], np.int8) for l in lo]
    for trial in range(4):
        split = random_split(rng, lo, up, k=trial)
        alpha, beta = random_vars(rng, lo, 2, split, beta_scale=2.0)
        g, ub, sat, _ = bc.upper_bound(net, x_lo, x_hi, C, lo, up, split, alpha, beta)
        g_free = bc.bound(net, x_lo, x_hi, C, lo, up, none, alpha, [np.zeros_like(b) for b in beta])
        gm = pinlib.grid_min(net, C, x_lo, x_hi, none, n=401)
        assert np.all(ub >= g_free - 1e-12)
        # the grid holds points no better than the true minimum, which ub cannot beat by more than the
        # grid's resolution; here checked one-sided: ub is never below a sound lower bound of the minimum
        assert np.all(g_free <= gm + 1e-9)
        assert np.all(g[sat] <= ub[sat] + 1e-12)


# ---------------------------------------------------------------------------
# Optimised intermediate bounds (Sec. 3.3, each bound with its own alpha')


@pytest.mark.parametrize("seed", range(4))
def test_optimised_root_bounds_tighter_sound_and_below_the_lp(seed):
    """At least as tight as CROWN's (the ascent keeps its best iterate, which
    starts at CROWN's default), enclosing the pre-activations on a dense grid
    of the box, equal to the exact interval bound on the first layer, and
    never beyond the LP relaxation of the same neuron (weak duality)."""
    rng, net, _, _, x_lo, x_hi, lo, up, C = tiny_case(seed + 600, widths=(2, 6, 5, 4, 2))
    lo_o, up_o = bc.root_bounds_opt(net, x_lo, x_hi, bc.AdamConfig(iters=40, lr_alpha=0.1))
    assert np.array_equal(lo_o[0], lo[0]) and np.array_equal(up_o[0], up[0])
    for l, u, lc, uc in zip(lo_o, up_o, lo, up):
        assert (l >= lc - 1e-12).all() and (u <= uc + 1e-12).all()
    assert any((l > lc + 1e-6).any() or (u < uc - 1e-6).any() for l, u, lc, uc in zip(lo_o, up_o, lo, up))
    zs, _ = pinlib.forward_all(net, pinlib.grid(x_lo, x_hi, 301))
    for z, l, u in zip(zs, lo_o, up_o):
        assert (z >= l - 1e-9).all() and (z <= u + 1e-9).all()
    # layer 2 neurons against the LP with the optimised layer-1 bounds
    sub = net[:2]
    none = [np.zeros(lo_o[0].shape[0], np.int8)]
    for j in range(lo_o[1].shape[0]):
        for sgn, val in ((1.0, lo_o[1][j]), (-1.0, -up_o[1][j])):
            c = np.zeros(lo_o[1].shape[0])
            c[j] = sgn
            p_lp, res, _ = pinlib.lp_verify_split(sub, x_lo, x_hi, c, lo_o[:1], up_o[:1], none)
            assert res.status == 0 and val <= p_lp + 1e-8


# ---------------------------------------------------------------------------
# l2-ball input sets (the q-norm form of Eq. beta_crown_lp, q = p = 2)


@pytest.mark.parametrize("seed", range(6))
def test_l2_ball_matches_dual_form_and_minimiser(seed):
    """The bound over the l2 ball equals Theorem 3.2's dual form with the
    2-norm of nu-hat(0); x* lies on the sphere and attains the linear part's
    minimum; ub is the network at that x* (independent forward)."""
    rng, net, x0, eps, x_lo, x_hi, lo, up, C = tiny_case(seed + 700, widths=(3, 6, 5, 4, 2), m=2)
    split = random_split(rng, lo, up, k=3)
    alpha, beta = random_vars(rng, lo, 2, split, beta_scale=2.0)
    ball = (x0, eps)
    g, A0, _ = bc.bound(net, x_lo, x_hi, C, lo, up, split, alpha, beta, keep=True, ball=ball)
    _, ub, sat, _ = bc.upper_bound(net, x_lo, x_hi, C, lo, up, split, alpha, beta, ball)
    xs = bc.minimiser(A0, x_lo, x_hi, ball)
    for r in range(2):
        gd, _, nh0 = pinlib.dual_nu_bound(net, x0, eps, C[r], lo, up, split, [a[r] for a in alpha],
                                          [b[r] for b in beta], with_input=True, q=2)
        assert abs(gd - g[r]) <= 1e-10 * max(1, abs(g[r]))
        coef = -nh0
        assert abs(np.linalg.norm(xs[r] - x0) - eps) <= 1e-12
        assert abs(coef @ xs[r] - (coef @ x0 - eps * np.linalg.norm(coef))) <= 1e-10 * max(1.0, abs(coef @ x0))
        _, logits = pinlib.forward_all(net, xs[r][None, :])
        assert abs(ub[r] - C[r] @ logits[0]) <= 1e-10 * max(1, abs(ub[r]))


@pytest.mark.parametrize("seed", range(4))
def test_l2_ball_bound_sound_on_the_disk(seed):
    """Below the network's minimum over a dense sampling of the disk (2-D
    input) restricted to the split half-spaces, and at least the bound over
    the enclosing box at the same variables (the ball lies inside the box:
    A x0 - eps ||A||_2 >= A x0 - eps ||A||_1)."""
    rng, net, x0, eps, x_lo, x_hi, lo, up, C = tiny_case(seed + 800, widths=(2, 6, 6, 2), m=2)
    th = np.linspace(0, 2 * np.pi, 721)[:-1]
    rad = np.sqrt(np.linspace(0, 1, 301))
    X = (x0[None, None, :] + eps * rad[:, None, None] * np.stack([np.cos(th), np.sin(th)], 1)[None]).reshape(-1, 2)
    for trial in range(3):
        split = random_split(rng, lo, up, k=trial)
        alpha, beta = random_vars(rng, lo, 2, split, beta_scale=2.0)
        g = bc.bound(net, x_lo, x_hi, C, lo, up, split, alpha, beta, ball=(x0, eps))
        g_box = bc.bound(net, x_lo, x_hi, C, lo, up, split, alpha, beta)
        assert np.all(g >= g_box - 1e-12)
        zs, logits = pinlib.forward_all(net, X)
        ok = np.ones(X.shape[0], bool)
        for z, s in zip(zs, split):
            ok &= np.all((z[:, s > 0] >= 0), axis=1) & np.all((z[:, s < 0] <= 0), axis=1)
        if ok.any():
            fmin = (logits[ok] @ C.T).min(axis=0)
            assert np.all(g <= fmin + 1e-9), (g, fmin)


@pytest.mark.parametrize("seed", range(3))
def test_l2_ball_gradient_matches_central_differences(seed):
    rng, net, x0, eps, x_lo, x_hi, lo, up, C = tiny_case(seed + 900, widths=(5, 8, 7, 3), m=2)
    split = random_split(rng, lo, up, k=2)
    alpha, beta = random_vars(rng, lo, 2, split, beta_scale=0.5)
    alpha = [np.clip(a, 0.05, 0.95) for a in alpha]
    beta = [np.where(s != 0, b + 0.1, 0.0) for b, s in zip(beta, split)]
    ball = (x0, eps)
    g, ga, gb = bc.bound_and_grad(net, x_lo, x_hi, C, lo, up, split, alpha, beta, ball)
    h = 1e-4

    def pattern(a, b):
        _, A0, tr = bc.bound(net, x_lo, x_hi, C, lo, up, split, a, b, keep=True, ball=ball)
        return [np.sign(t[0]) for t in tr]

    base = pattern(alpha, beta)
    checked = 0
    for which, vars_, grads in (("a", alpha, ga), ("b", beta, gb)):
        for i in range(len(vars_)):
            for r in range(2):
                for j in range(vars_[i].shape[1]):
                    uns = lo[i][j] < 0 < up[i][j] and split[i][j] == 0
                    if (which == "a" and not uns) or (which == "b" and split[i][j] == 0):
                        continue
                    p, q = [v.copy() for v in vars_], [v.copy() for v in vars_]
                    p[i][r, j] += h
                    q[i][r, j] -= h
                    args_p = (p, beta) if which == "a" else (alpha, p)
                    args_q = (q, beta) if which == "a" else (alpha, q)
                    if any(np.any(x != y) or np.any(x != z) for x, y, z in
                           zip(base, pattern(*args_p), pattern(*args_q))):
                        continue
                    fd = (bc.bound(net, x_lo, x_hi, C, lo, up, split, *args_p, ball=ball)[r] -
                          bc.bound(net, x_lo, x_hi, C, lo, up, split, *args_q, ball=ball)[r]) / (2 * h)
                    assert abs(fd - grads[i][r, j]) <= 1e-6 + 1e-5 * abs(fd), (which, i, r, j, fd, grads[i][r, j])
                    checked += 1
    assert checked >= 10


# ---------------------------------------------------------------------------
# general l_p-ball input sets (Eq. beta_crown_lp with the dual exponent q)

LP_PS = (1.5, 3.0, 6.0)


@pytest.mark.parametrize("p", LP_PS)
@pytest.mark.parametrize("seed", range(3))
def test_lp_ball_matches_dual_form_and_hoelder_equality(seed, p):
    """The bound over the l_p ball equals Theorem 3.2's dual form with the
    q-norm of nu-hat(0) (1/p + 1/q = 1); x* lies on the ball's surface
    (||x* - x0||_p = eps) and attains Hoelder's equality for the linear part;
    ub is the network at that x* (independent forward)."""
    rng, net, x0, eps, x_lo, x_hi, lo, up, C = tiny_case(seed + 1700, widths=(4, 6, 5, 4, 2), m=2)
    split = random_split(rng, lo, up, k=2)
    alpha, beta = random_vars(rng, lo, 2, split, beta_scale=2.0)
    q = p / (p - 1.0)
    ball = (x0, eps, p)
    g, A0, _ = bc.bound(net, x_lo, x_hi, C, lo, up, split, alpha, beta, keep=True, ball=ball)
    _, ub, _, _ = bc.upper_bound(net, x_lo, x_hi, C, lo, up, split, alpha, beta, ball)
    xs = bc.minimiser(A0, x_lo, x_hi, ball)
    for r in range(2):
        gd, _, nh0 = pinlib.dual_nu_bound(net, x0, eps, C[r], lo, up, split, [a[r] for a in alpha],
                                          [b[r] for b in beta], with_input=True, q=q)
        assert abs(gd - g[r]) <= 1e-10 * max(1, abs(g[r]))
        coef = -nh0
        assert abs(np.sum(np.abs(xs[r] - x0) ** p) ** (1 / p) - eps) <= 1e-12
        assert abs(coef @ xs[r] - (coef @ x0 - eps * np.sum(np.abs(coef) ** q) ** (1 / q))) \
            <= 1e-10 * max(1.0, abs(coef @ x0))
        _, logits = pinlib.forward_all(net, xs[r][None, :])
        assert abs(ub[r] - C[r] @ logits[0]) <= 1e-10 * max(1, abs(ub[r]))


@pytest.mark.parametrize("seed", range(3))
def test_lp_ball_bound_orders_with_the_ball_and_reduces_to_l2_and_box(seed):
    """At fixed variables the l_p balls of one radius are nested (p < r gives
    the smaller ball), so the bound falls as p grows: l_1.5 >= l_2 >= l_3 >=
    l_6 >= box (the box is the l_inf ball).  p = 2 reproduces the l2 form
    exactly, and p = 1000 is within d^(1/p) - 1 of the box's eps-term."""
    rng, net, x0, eps, x_lo, x_hi, lo, up, C = tiny_case(seed + 1800, widths=(5, 7, 6, 3), m=3)
    split = random_split(rng, lo, up, k=2)
    alpha, beta = random_vars(rng, lo, 3, split, beta_scale=1.0)
    gs = [bc.bound(net, x_lo, x_hi, C, lo, up, split, alpha, beta, ball=(x0, eps, p)) for p in (1.5, 2.0, 3.0, 6.0)]
    g_box, A0, _ = bc.bound(net, x_lo, x_hi, C, lo, up, split, alpha, beta, keep=True)
    for a, b in zip(gs, gs[1:] + [g_box]):
        assert np.all(a >= b - 1e-12)
    g_l2 = bc.bound(net, x_lo, x_hi, C, lo, up, split, alpha, beta, ball=(x0, eps))
    assert np.array_equal(gs[1], g_l2)
    g_big = bc.bound(net, x_lo, x_hi, C, lo, up, split, alpha, beta, ball=(x0, eps, 1000.0))
    gap = eps * np.abs(A0).sum(axis=1) * (x0.shape[0] ** (1 / 1000.0) - 1)
    assert np.all(g_big >= g_box - 1e-12) and np.all(g_big - g_box <= gap + 1e-12)


@pytest.mark.parametrize("p", (1.5, 3.0))
@pytest.mark.parametrize("seed", range(3))
def test_lp_ball_bound_sound_on_the_ball(seed, p):
    """Below the network's minimum over a dense sampling of the 2-D l_p ball
    (direction times radius, each direction scaled to unit p-norm) restricted
    to the split half-spaces."""
    rng, net, x0, eps, x_lo, x_hi, lo, up, C = tiny_case(seed + 1900, widths=(2, 6, 6, 2), m=2)
    th = np.linspace(0, 2 * np.pi, 721)[:-1]
    d = np.stack([np.cos(th), np.sin(th)], 1)
    d /= (np.abs(d) ** p).sum(axis=1, keepdims=True) ** (1 / p)
    rad = np.linspace(0, 1, 301) ** 0.5
    X = (x0[None, None, :] + eps * rad[:, None, None] * d[None]).reshape(-1, 2)
    for trial in range(3):
        split = random_split(rng, lo, up, k=trial)
        alpha, beta = random_vars(rng, lo, 2, split, beta_scale=2.0)
        g = bc.bound(net, x_lo, x_hi, C, lo, up, split, alpha, beta, ball=(x0, eps, p))
        zs, logits = pinlib.forward_all(net, X)
        ok = np.ones(X.shape[0], bool)
        for z, s in zip(zs, split):
            ok &= np.all((z[:, s > 0] >= 0), axis=1) & np.all((z[:, s < 0] <= 0), axis=1)
        if ok.any():
            fmin = (logits[ok] @ C.T).min(axis=0)
            assert np.all(g <= fmin + 1e-9), (g, fmin)


@pytest.mark.parametrize("p", (1.5, 3.0))
def test_lp_ball_gradient_matches_central_differences(p):
    rng, net, x0, eps, x_lo, x_hi, lo, up, C = tiny_case(2000 + int(p * 10), widths=(5, 8, 7, 3), m=2)
    split = random_split(rng, lo, up, k=2)
    alpha, beta = random_vars(rng, lo, 2, split, beta_scale=0.5)
    alpha = [np.clip(a, 0.05, 0.95) for a in alpha]
    beta = [np.where(s != 0, b + 0.1, 0.0) for b, s in zip(beta, split)]
    ball = (x0, eps, p)
    g, ga, gb = bc.bound_and_grad(net, x_lo, x_hi, C, lo, up, split, alpha, beta, ball)
    h = 1e-5

    def pattern(a, b):
        _, A0, tr = bc.bound(net, x_lo, x_hi, C, lo, up, split, a, b, keep=True, ball=ball)
        return [np.sign(t[0]) for t in tr]

    base = pattern(alpha, beta)
    checked = 0
    for which, vars_, grads in (("a", alpha, ga), ("b", beta, gb)):
        for i in range(len(vars_)):
            for r in range(2):
                for j in range(vars_[i].shape[1]):
                    uns = lo[i][j] < 0 < up[i][j] and split[i][j] == 0
                    if (which == "a" and not uns) or (which == "b" and split[i][j] == 0):
                        continue
                    pp, qq = [v.copy() for v in vars_], [v.copy() for v in vars_]
                    pp[i][r, j] += h
                    qq[i][r, j] -= h
                    args_p = (pp, beta) if which == "a" else (alpha, pp)
                    args_q = (qq, beta) if which == "a" else (alpha, qq)
                    if any(np.any(x != y) or np.any(x != z) for x, y, z in
                           zip(base, pattern(*args_p), pattern(*args_q))):
                        continue
                    fd = (bc.bound(net, x_lo, x_hi, C, lo, up, split, *args_p, ball=ball)[r] -
                          bc.bound(net, x_lo, x_hi, C, lo, up, split, *args_q, ball=ball)[r]) / (2 * h)
                    assert abs(fd - grads[i][r, j]) <= 1e-6 + 1e-5 * abs(fd), (which, i, r, j, fd, grads[i][r, j])
                    checked += 1
    assert checked >= 10
