"""Pins of the joint optimisation of intermediate bounds (oracle.joint; Sec. 3.3,
Eq. opt_non_convex) against what the paper and the mathematics fix: the torch
recursion equals the pinned NumPy bound and its hand adjoint; at the starting
point the intermediate bounds are per-layer CROWN's (an independent function);
each computed intermediate bound is Theorem 3.1's bound of the sub-network with
the layer's shared variables broadcast to its rows; every bound is sound on a
dense grid and at most the LP with the same splits and the same earlier
bounds; one ReLU layer leaves nothing to optimise jointly; run long, the joint
bound is at least the fixed-bounds optimum."""
import numpy as np
import pytest

from oracle import beta_crown as bc
from tests import pinlib

torch = pytest.importorskip("torch")
jt = pytest.importorskip("oracle.joint")


def case(seed, widths=(2, 8, 8, 6, 2), eps=0.6, m=2):
    rng = np.random.default_rng(seed)
    net = pinlib.random_net(rng, list(widths))
    x0 = rng.uniform(-0.5, 0.5, size=widths[0])
    x_lo, x_hi = x0 - eps, x0 + eps
    lo, up = bc.root_bounds(net, x_lo, x_hi)
    C = rng.standard_normal((m, widths[-1]))
    return rng, net, x_lo, x_hi, lo, up, C


def random_split(rng, lo, up, k):
    split = [np.zeros(l.shape[0], np.int8) for l in lo]
    uns = [(i, j) for i in range(len(lo)) for j in range(lo[i].shape[0]) if lo[i][j] < 0 < up[i][j]]
    for t in rng.choice(len(uns), size=min(k, len(uns)), replace=False):
        i, j = uns[t]
        split[i][j] = rng.choice([-1, 1])
    return split


def default_vars(lo, up, m):
    alpha = [np.tile(bc.default_alpha(l, u), (m, 1)) for l, u in zip(lo, up)]
    beta = [np.zeros((m, l.shape[0])) for l in lo]
    return alpha, beta


def random_jv(rng, net, lo, up, split):
    jv = jt.init_vars(net, lo, up)
    for i in jv.ap:
        for side in (0, 1):
            jv.ap[i][side] = [torch.tensor(rng.uniform(0, 1, a.shape[0])) for a in jv.ap[i][side]]
            jv.bp[i][side] = [torch.tensor(rng.uniform(0, 1, b.shape[0]) * (split[k] != 0))
                              for k, b in enumerate(jv.bp[i][side])]
    return jv


def T(xs):
    return [torch.tensor(np.asarray(x, np.float64)) for x in xs]


@pytest.mark.parametrize("seed", range(5))
def test_torch_bound_equals_numpy_bound_and_its_adjoint(seed):
    """bound_t at random variables, bounds and splits is the NumPy oracle's
    bound (1e-12), and autograd's gradient is the hand adjoint's (the Danskin
    z-bar A rule), away from the sign decisions where both are exact."""
    rng, net, x_lo, x_hi, lo, up, C = case(seed + 10, widths=(4, 7, 6, 5, 3), m=3)
    split = random_split(rng, lo, up, 3)
    alpha = [rng.uniform(0, 1, (3, l.shape[0])) for l in lo]
    beta = [rng.uniform(0, 1, (3, l.shape[0])) * (s != 0) for l, s in zip(lo, split)]
    g_np, ga, gb = bc.bound_and_grad(net, x_lo, x_hi, C, lo, up, split, alpha, beta)
    a_t = [x.requires_grad_(True) for x in T(alpha)]
    b_t = [x.requires_grad_(True) for x in T(beta)]
    g_t = jt.bound_t([(torch.tensor(W), torch.tensor(b)) for W, b in net], torch.tensor(x_lo), torch.tensor(x_hi),
                     torch.tensor(C), T(lo), T(up), [torch.tensor(s.astype(np.int64)) for s in split], a_t, b_t)
    assert np.abs(g_t.detach().numpy() - g_np).max() <= 1e-12 * max(1.0, np.abs(g_np).max())
    grads = torch.autograd.grad(g_t.sum(), a_t + b_t)
    for x, y in zip(grads, ga + gb):
        assert np.abs(x.numpy() - y).max() <= 1e-10


@pytest.mark.parametrize("seed", range(4))
def test_starting_point_gives_per_layer_crown_bounds(seed):
    """No splits, alpha' at CROWN's slopes, beta' = 0: every intermediate
    bound is per-layer CROWN's (bc.root_bounds, an independent NumPy path)
    and the final bound is the plain bound at those bounds."""
    rng, net, x_lo, x_hi, lo, up, C = case(seed + 20, widths=(3, 9, 8, 7, 6, 2))
    split = [np.zeros(l.shape[0], np.int8) for l in lo]
    alpha, beta = default_vars(lo, up, 2)
    g, lj, uj = jt.joint_bound(net, x_lo, x_hi, C, lo, up, split, T(alpha), T(beta), jt.init_vars(net, lo, up))
    for k in range(len(lo)):
        assert np.abs(lj[k].numpy() - lo[k]).max() <= 1e-12
        assert np.abs(uj[k].numpy() - up[k]).max() <= 1e-12
    assert np.abs(g.numpy() - bc.bound(net, x_lo, x_hi, C, lo, up, split, alpha, beta)).max() <= 1e-12


@pytest.mark.parametrize("seed", range(4))
def test_each_intermediate_bound_is_the_subnetwork_bound_with_shared_variables(seed):
    """At random alpha', beta' and splits, layer i's bounds are the NumPy
    bound of the sub-network 1..i with specification [I] (lower) or [-I]
    (upper), every row given the side's shared alpha', beta', earlier layers
    at the joint bounds, then clipped by the root bounds; the final bound is
    the NumPy bound at the joint bounds."""
    rng, net, x_lo, x_hi, lo, up, C = case(seed + 30, widths=(3, 8, 7, 6, 2))
    split = random_split(rng, lo, up, 3)
    jv = random_jv(rng, net, lo, up, split)
    alpha = [rng.uniform(0, 1, (2, l.shape[0])) for l in lo]
    beta = [rng.uniform(0, 1, (2, l.shape[0])) * (s != 0) for l, s in zip(lo, split)]
    g, lj, uj = jt.joint_bound(net, x_lo, x_hi, C, lo, up, split, T(alpha), T(beta), jv)
    lj = [x.detach().numpy() for x in lj]
    uj = [x.detach().numpy() for x in uj]
    for i in range(2, len(net)):
        d = net[i - 1][0].shape[0]
        for side, sgn in ((0, 1.0), (1, -1.0)):
            a_rows = [np.tile(a.numpy(), (d, 1)) for a in jv.ap[i][side]]
            b_rows = [np.tile(b.numpy(), (d, 1)) for b in jv.bp[i][side]]
            r = bc.bound(net[:i], x_lo, x_hi, sgn * np.eye(d), lj[:i - 1], uj[:i - 1], split[:i - 1], a_rows, b_rows)
            want = np.maximum(r, lo[i - 1]) if side == 0 else np.minimum(-r, up[i - 1])
            got = lj[i - 1] if side == 0 else uj[i - 1]
            assert np.abs(got - want).max() <= 1e-12
    assert np.abs(g.detach().numpy() - bc.bound(net, x_lo, x_hi, C, lj, uj, split, alpha, beta)).max() <= 1e-12


@pytest.mark.parametrize("seed", range(4))
def test_joint_bounds_are_sound_on_a_dense_grid_and_below_the_lp(seed):
    """After 20 joint iterations (lr 0.1 / 0.05): the best bound lies below the
    network's minimum over a 1001^2 grid of the subdomain; every intermediate
    bound of the final iterate encloses its pre-activation on the grid's
    subdomain points and is at most the LP minimum of z(i)_j (maximum for u)
    with the same splits and the same earlier bounds; the final iterate's
    bound is at most the LP of the objective at the final intermediate
    bounds."""
    rng, net, x_lo, x_hi, lo, up, C = case(seed + 40, widths=(2, 7, 7, 6, 2))
    cfg = bc.AdamConfig(iters=20, lr_alpha=0.1, lr_beta=0.05)
    X = pinlib.grid(x_lo, x_hi, 1001)
    zs, out = pinlib.forward_all(net, X)
    for trial in range(2):
        split = random_split(rng, lo, up, trial + 1)
        alpha, beta = default_vars(lo, up, 2)
        best, a, b, gf, lj, uj = jt.joint_optimize(net, x_lo, x_hi, C, lo, up, split, alpha, beta, cfg)
        ok = np.ones(X.shape[0], bool)
        for z, s in zip(zs, split):
            for j in np.nonzero(s)[0]:
                ok &= (z[:, j] >= 0) if s[j] > 0 else (z[:, j] <= 0)
        if ok.any():
            assert np.all(best <= (out[ok] @ C.T).min(axis=0) + 1e-9)
            for k in range(len(lj)):
                assert np.all(lj[k] <= zs[k][ok].min(axis=0) + 1e-9)
                assert np.all(uj[k] >= zs[k][ok].max(axis=0) - 1e-9)
        for i in range(2, len(net)):
            for j in range(lj[i - 1].shape[0]):
                if lj[i - 1][j] > lo[i - 1][j]:  # computed, not the root's
                    e = np.zeros(lj[i - 1].shape[0])
                    e[j] = 1.0
                    p_lp, res, _ = pinlib.lp_verify_split(net[:i], x_lo, x_hi, e, lj[:i - 1], uj[:i - 1],
                                                          split[:i - 1])
                    assert res.status in (0, 2) and lj[i - 1][j] <= p_lp + 1e-7
        for r in range(C.shape[0]):
            p_lp, res, _ = pinlib.lp_verify_split(net, x_lo, x_hi, C[r], lj, uj, split)
            assert res.status in (0, 2) and gf[r] <= p_lp + 1e-7


@pytest.mark.parametrize("seed", range(3))
def test_one_relu_layer_leaves_only_the_final_variables(seed):
    """L = 2: no intermediate layer has variables, so the joint optimiser is
    the plain one (bc.optimize), iterate for iterate."""
    rng, net, x_lo, x_hi, lo, up, C = case(seed + 50, widths=(3, 9, 3), m=3)
    split = random_split(rng, lo, up, 2)
    alpha, beta = default_vars(lo, up, 3)
    cfg = bc.AdamConfig(iters=15, lr_alpha=0.1, lr_beta=0.05)
    best, a, b, gf, _, _ = jt.joint_optimize(net, x_lo, x_hi, C, lo, up, split, alpha, beta, cfg)
    best2, a2, b2, g2 = bc.optimize(net, x_lo, x_hi, C, lo, up, split, alpha, beta, cfg)
    assert np.abs(best - best2).max() <= 1e-12 and np.abs(gf - g2).max() <= 1e-12
    for x, y in zip(a + b, a2 + b2):
        assert np.abs(x - y).max() <= 1e-12


@pytest.mark.parametrize("seed", range(4))
def test_long_joint_run_reaches_at_least_the_fixed_bounds_optimum(seed):
    """Run long (400 iterations, decay 0.99), the plain optimiser approaches
    the LP with the root bounds (the concave problem of Theorem 3.3; it stays
    below it) and the joint one its own bounds' optimum, which is at least
    that: the joint bounds are never looser than the root's, and the LP over
    a smaller relaxation is no lower."""
    rng, net, x_lo, x_hi, lo, up, C = case(seed + 60, widths=(3, 8, 8, 2))
    split = random_split(rng, lo, up, 1)
    alpha, beta = default_vars(lo, up, 2)
    cfg = bc.AdamConfig(iters=400, lr_alpha=0.05, lr_beta=0.05, decay=0.99)
    best, *_ = jt.joint_optimize(net, x_lo, x_hi, C, lo, up, split, alpha, beta, cfg)
    best_p, *_ = bc.optimize(net, x_lo, x_hi, C, lo, up, split, alpha, beta, cfg)
    lp = np.array([pinlib.lp_verify_split(net, x_lo, x_hi, C[r], lo, up, split)[0] for r in range(2)])
    assert np.all(best_p <= lp + 1e-7)
    assert np.all(best >= best_p - 1e-6 * np.maximum(1, np.abs(best_p)))


def test_gradient_reaches_the_shared_variables_through_the_bounds():
    """The autograd gradient of sum g with respect to alpha' and beta' matches
    central differences of the whole pipeline (intermediate bounds
    recomputed), at points whose sign decisions are stable under +-h, and is
    non-zero for some entry (the bounds do feed the final relaxation)."""
    rng, net, x_lo, x_hi, lo, up, C = case(71, widths=(3, 8, 7, 6, 2))
    split = random_split(rng, lo, up, 2)
    jv = random_jv(rng, net, lo, up, split)
    alpha, beta = default_vars(lo, up, 2)
    leaves = jv.leaves()
    for x in leaves:
        x.requires_grad_(True)
    g, _, _ = jt.joint_bound(net, x_lo, x_hi, C, lo, up, split, T(alpha), T(beta), jv)
    grads = torch.autograd.grad(g.sum(), leaves, allow_unused=True)
    h = 1e-6
    checked, nonzero = 0, 0
    for x, gr in zip(leaves, grads):
        gr = torch.zeros_like(x) if gr is None else gr
        for j in range(x.shape[0]):
            vals = []
            with torch.no_grad():
                for dlt in (h, -h):
                    x[j] += dlt
                    vals.append(jt.joint_bound(net, x_lo, x_hi, C, lo, up, split, T(alpha), T(beta), jv)[0].sum())
                    x[j] -= dlt
            fd = float(vals[0] - vals[1]) / (2 * h)
            if abs(fd - float(gr[j])) > 1e-5 * max(1.0, abs(fd)):
                # a sign decision or a root clip switched within +-h: skip the coordinate
                continue
            checked += 1
            nonzero += abs(fd) > 1e-8
    assert checked >= 0.9 * sum(x.shape[0] for x in leaves)
    assert nonzero >= 3


def test_a_split_decides_its_neuron_even_against_its_bounds():
    """Hand case: x in [-1, 1], z = x + 2 (bounds [1, 3]), split z < 0 -- an
    empty subdomain, which only jointly tightened bounds can produce.  The
    split decides the relaxation (z-hat = 0 with its beta term), so for
    y = relu(z): Lambda = beta, c = 2 beta, A(0) = beta and g = beta;
    letting the bounds decide (z-hat = z) would give 1 + beta."""
    net = [(torch.tensor([[1.0]], dtype=torch.float64), torch.tensor([2.0], dtype=torch.float64)),
           (torch.tensor([[1.0]], dtype=torch.float64), torch.tensor([0.0], dtype=torch.float64))]
    for b in (0.0, 0.5, 2.0):
        g = jt.bound_t(net, torch.tensor([-1.0], dtype=torch.float64), torch.tensor([1.0], dtype=torch.float64),
                       torch.tensor([[1.0]], dtype=torch.float64), [torch.tensor([1.0], dtype=torch.float64)],
                       [torch.tensor([3.0], dtype=torch.float64)], [torch.tensor([-1])],
                       [torch.tensor([[0.5]], dtype=torch.float64)], [torch.tensor([[b]], dtype=torch.float64)])
        assert abs(float(g[0]) - b) <= 1e-15


def test_shared_layouts_round_trip():
    """The batch driver's mapping of the library's shared alpha' / beta'
    layouts: writing each subdomain's starting variables into the flat
    arrays and reading them back gives the same bound, bounds and gradient
    as the starting variables themselves (mlp_deep, splits on several
    layers)."""
    from tests import cases
    wl, lo, up, lo64, up64, orc = cases.small_case("mlp_deep")
    a0 = orc.default_alpha_flat()
    z = np.zeros(orc.nnz * orc.m)
    L = len(orc.net64)
    flat = {}
    for i in range(2, L):
        oa, ob = orc.joint_offsets(i)
        ash, bsh = np.zeros(oa[-1]), np.zeros(ob[-1])
        for b in range(orc.B):
            us, ts = orc.joint_layout(b, i)
            p = int(orc.dom_prop[b])
            dflt = bc.default_alpha(orc.lo[p][us], orc.up[p][us])
            ash[oa[b]:oa[b + 1]] = np.concatenate([dflt, dflt])
        flat[i] = (ash, bsh)
    for b in (0, 7, 31):
        g1, l1, u1, gr1 = orc.joint_eval(b, a0, z, orc.joint_vars(b, flat), grad=True)
        g2, l2, u2, gr2 = orc.joint_eval(b, a0, z, orc.joint_start(b), grad=True)
        assert np.array_equal(g1, g2) and np.array_equal(l1, l2) and np.array_equal(u1, u2)
        for i in gr1:
            assert np.array_equal(gr1[i][0], gr2[i][0]) and np.array_equal(gr1[i][1], gr2[i][1])
            assert gr1[i][0].shape[0] == 2 * orc.joint_layout(b, i)[0].shape[0]
        assert any(np.abs(gr1[i][0]).max(initial=0) > 0 for i in gr1)
