"""GPU parity over general l_p-ball input sets (cv_bound_set_input_lp) against
the FP64 oracle on the same balls: bound, gradients, optimiser and upper
bound at p = 1.5 (dual q = 3) and p = 3 (q = 1.5), the 1e-4 guarded relative
bar of the box tests.  Over an l_p ball the last step of Theorem 3.1's bound
is A(0) x0 - eps ||A(0)||_q, with the minimiser
x* = x0 - eps sign(A(0)) |A(0)|^(q-1) / ||A(0)||_q^(q-1).
"""
import sys

import numpy as np
import pytest

from tests import cases
from tests.cases import guarded_rel

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

TOL = 1e-4
PS = (1.5, 3.0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2103_06624_amd import binding
    binding.lib()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda()


def problem(name, p):
    from paper_2103_06624_amd.api import BoundProblem
    wl, lo, up, x0, eps, orc = cases.small_lp_case(name, p)
    pb = BoundProblem.from_workload(wl, lo, up)
    pb.set_input_lp(x0, eps, p)
    return wl, orc, pb, x0, eps


@pytest.mark.parametrize("p", PS)
@pytest.mark.parametrize("name", ["mlp_small", "mlp_deep", "cnn_base", "cnn_wide", "cnn_odd"])
def test_lp_eval_parity(name, p):
    say("lp eval parity", name, p)
    wl, orc, pb, _, _ = problem(name, p)
    alpha, beta = cases.random_vars(orc, seed=31)
    lb = pb.eval(dev(alpha), dev(beta)).cpu().numpy()
    ref = np.stack([orc.eval(b, alpha, beta) for b in range(orc.B)])
    err = guarded_rel(lb, ref)
    say(name, p, "max rel err", err.max())
    assert err.max() <= TOL


@pytest.mark.parametrize("p", PS)
@pytest.mark.parametrize("name", ["mlp_small", "cnn_base", "cnn_odd"])
def test_lp_grad_parity(name, p):
    """Bound and gradients at random (alpha, beta), on the rows clear of a
    float32 sign decision (the box test's criterion)."""
    from tests.test_gpu_parity import kink_free_rows
    say("lp grad parity", name, p)
    wl, orc, pb, _, _ = problem(name, p)
    alpha, beta = cases.random_vars(orc, seed=32)
    lb, ga, gb = pb.grad(dev(alpha), dev(beta))
    lb, ga, gb = lb.cpu().numpy(), ga.cpu().numpy(), gb.cpu().numpy().reshape(-1, orc.m)
    checked, worst = 0, 0.0
    for b in range(orc.B):
        g, ra, rb = orc.grad(b, alpha, beta)
        assert guarded_rel(lb[b], g).max() <= TOL
        ok = kink_free_rows(orc, b, alpha, beta)
        U = ra.shape[0] // orc.m
        a_gpu = ga[orc.alpha_off[b]:orc.alpha_off[b + 1]].reshape(orc.m, U)
        a_ref = ra.reshape(orc.m, U)
        b_gpu = gb[orc.ptr[b]:orc.ptr[b + 1]]
        for k in np.nonzero(ok)[0]:
            scale = max(1.0, np.abs(a_ref[k]).max(initial=0), np.abs(rb[:, k]).max(initial=0))
            worst = max(worst, np.abs(a_gpu[k] - a_ref[k]).max(initial=0) / scale,
                        np.abs(b_gpu[:, k] - rb[:, k]).max(initial=0) / scale)
            checked += 1
    say(name, p, "grad rows checked", checked, "of", orc.B * orc.m, "worst", worst)
    assert checked >= 0.75 * orc.B * orc.m
    assert worst <= TOL


@pytest.mark.parametrize("name,p,nparts", [("mlp_small", 3.0, 1), ("cnn_base", 1.5, 1), ("mlp_deep", 1.5, 2)])
def test_lp_optimize_parity(name, p, nparts):
    """20 projected-Adam steps from CROWN's alpha and beta = 0 (two concurrent
    sub-batches for mlp_deep: the balls and their exponent reach the new
    sub-batch handles)."""
    say("lp optimize parity", name, p, nparts)
    wl, orc, pb, _, _ = problem(name, p)
    pb.set_parts(nparts)
    a = pb.alpha_init()
    b = pb.zeros_beta()
    best, last = pb.optimize(a, b, iters=20, lr_alpha=0.01, lr_beta=0.05, decay=0.98)
    best, last = best.cpu().numpy(), last.cpu().numpy()
    a_gpu, b_gpu = a.cpu().numpy(), b.cpu().numpy()
    a0 = orc.default_alpha_flat()
    z = np.zeros(orc.nnz * orc.m)
    doms = range(orc.B) if orc.B <= 24 else np.random.default_rng(5).choice(orc.B, 12, replace=False)
    errs, ex = [], []
    for d in doms:
        rbest, _, _, _ = orc.optimize(d, a0, z)
        errs.append(guarded_rel(best[d], rbest).max())
        g64 = orc.eval(d, a_gpu, b_gpu)
        ex.append(((last[d] - g64) / np.maximum(np.abs(g64), 1.0)).max())
    say(name, p, "opt max rel err", max(errs), "max rel excess at own vars", max(ex))
    assert np.all(a_gpu >= 0) and np.all(a_gpu <= 1) and np.all(b_gpu >= 0)
    assert max(errs) <= TOL
    assert max(ex) <= TOL


@pytest.mark.parametrize("p", PS)
@pytest.mark.parametrize("name", ["mlp_small", "cnn_base"])
def test_lp_upper_bound_parity(name, p):
    """ub = C f(x*) at the l_p minimiser on every row, the split check where
    the smallest split pre-activation at x* is clear of zero, lb <= ub where
    sat."""
    say("lp upper bound", name, p)
    wl, orc, pb, _, _ = problem(name, p)
    alpha, beta = cases.random_vars(orc, seed=33)
    lb, ub, sat = [t.cpu().numpy() for t in pb.upper(dev(alpha), dev(beta))]
    n_sat = 0
    for b in range(orc.B):
        g, u, st, mg = orc.upper(b, alpha, beta)
        assert guarded_rel(lb[b], g).max() <= TOL
        assert guarded_rel(ub[b], u).max() <= TOL, (b, ub[b], u)
        for k in np.nonzero(mg > 1e-3)[0]:
            assert bool(sat[b, k]) == bool(st[k]), (b, k, mg[k])
            n_sat += 1
    s1 = sat.astype(bool)
    assert (lb[s1] <= ub[s1] + TOL * np.maximum(1.0, np.abs(ub[s1]))).all()
    say(name, p, "sat checked", n_sat, "sat=1", int(s1.sum()), "of", sat.size)


@pytest.mark.parametrize("p", PS)
def test_lp_bound_below_sampled_network_values(p):
    """Soundness over the ball: with no splits, every optimised lower bound
    (20 steps) lies below C f(x) at points on and inside the property's l_p
    ball (Gaussian directions scaled to unit p-norm), the network in FP64."""
    from paper_2103_06624_amd.api import BoundProblem
    wl, lo, up, x0, eps, orc = cases.small_lp_case("mlp_small", p)
    P = x0.shape[0]
    pb = BoundProblem(wl.net.layers, wl.x_lo, wl.x_hi, wl.C, lo, up, np.arange(P, dtype=np.int32),
                      np.zeros(P + 1, np.int64), [], [], [])
    pb.set_input_lp(x0, eps, p)

    def forward(x):
        h = x.T
        for i, (W, bias) in enumerate(orc.net64):
            h = W @ h + bias[:, None]
            if i < len(orc.net64) - 1:
                h = np.maximum(h, 0.0)
        return h.T

    best, _ = pb.optimize(pb.alpha_init(), pb.zeros_beta(), iters=20)
    best = best.cpu().numpy()
    rng = np.random.default_rng(8)
    d0 = x0.shape[1]
    for k in range(P):
        d = rng.standard_normal((512, d0))
        d /= (np.abs(d) ** p).sum(axis=1, keepdims=True) ** (1 / p)
        r = np.concatenate([np.ones(256), rng.uniform(0, 1, 256) ** (1.0 / d0)])
        xs = x0[k].astype(np.float64)[None] + eps[k] * r[:, None] * d
        vmin = (forward(xs) @ orc.C[k].T).min(axis=0)
        assert (best[k] <= vmin + 1e-5 * np.maximum(1.0, np.abs(vmin))).all(), (k, best[k], vmin)


@pytest.mark.parametrize("name", ["mlp_small", "cnn_base"])
def test_lp_two_is_the_l2_ball_and_the_balls_order(name):
    """p = 2 through cv_bound_set_input_lp gives the l2 entry point's bounds
    bit for bit; at the same variables the bounds fall as p grows
    (l_1.5 >= l_2 >= l_3 >= box), the nesting of the balls."""
    wl, orc, pb, x0, eps = problem(name, 2.0)
    alpha, beta = cases.random_vars(orc, seed=34)
    a, b = dev(alpha), dev(beta)
    g2 = pb.eval(a, b).cpu().numpy()
    pb.set_input_l2(x0, eps)
    assert np.array_equal(pb.eval(a, b).cpu().numpy(), g2)
    pb.set_input_lp(x0, eps, 1.5)
    g15 = pb.eval(a, b).cpu().numpy()
    pb.set_input_lp(x0, eps, 3.0)
    g3 = pb.eval(a, b).cpu().numpy()
    pb.set_input_lp(None, None, 2.0)
    gbox = pb.eval(a, b).cpu().numpy()
    slack = 1e-5 * np.maximum(1.0, np.abs(g2))
    assert (g15 >= g2 - slack).all() and (g2 >= g3 - slack).all() and (g3 >= gbox - slack).all()


def test_lp_rejects_bad_exponents_and_sound_mode():
    from paper_2103_06624_amd.binding import CvError
    wl, orc, pb, x0, eps = problem("mlp_small", 3.0)
    for bad_p in (1.0, 1.2, np.inf, np.nan, -2.0):
        with pytest.raises(CvError):
            pb.set_input_lp(x0, eps, bad_p)
    with pytest.raises(CvError):  # sound mode is for boxes and l2 balls
        pb.set_sound(1)
    pb.set_input_lp(x0, eps, 2.0)
    pb.set_sound(1)
    with pytest.raises(CvError):
        pb.set_input_lp(x0, eps, 3.0)
