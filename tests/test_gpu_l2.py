"""GPU parity over l2-ball input sets (cv_bound_set_input_l2) against the FP64
oracle on the same balls: bound, gradients, optimiser and upper bound, same
1e-4 guarded relative bar as the box tests.  Over a ball the last step of
Theorem 3.1's bound is A(0) x0 - eps ||A(0)||_2, smooth in A(0) away from
A(0) = 0, so the minimiser x* and the upper bound are compared on every row.
"""
import sys

import numpy as np
import pytest

from tests import cases
from tests.cases import guarded_rel

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

TOL = 1e-4


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


def problem(name):
    from paper_2103_06624_amd.api import BoundProblem
    wl, lo, up, x0, eps, orc = cases.small_l2_case(name)
    pb = BoundProblem.from_workload(wl, lo, up)
    pb.set_input_l2(x0, eps)
    return wl, orc, pb, x0, eps


@pytest.mark.parametrize("name", ["mlp_small", "mlp_deep", "cnn_base", "cnn_wide", "cnn_deep", "cnn_odd"])
def test_l2_eval_parity(name):
    say("l2 eval parity", name)
    wl, orc, pb, _, _ = problem(name)
    alpha, beta = cases.random_vars(orc, seed=21)
    lb = pb.eval(dev(alpha), dev(beta)).cpu().numpy()
    ref = np.stack([orc.eval(b, alpha, beta) for b in range(orc.B)])
    err = guarded_rel(lb, ref)
    say(name, "max rel err", err.max())
    assert err.max() <= TOL


@pytest.mark.parametrize("name", ["mlp_small", "cnn_base", "cnn_wide", "cnn_odd"])
def test_l2_grad_parity(name):
    """Bound and gradients at random (alpha, beta).  Rows are compared where
    no hidden-layer sign decision is within float32 reach of a kink (the
    box test's criterion, which also skips near-zero A(0) entries: harmless
    over a ball, only fewer rows)."""
    from tests.test_gpu_parity import kink_free_rows
    say("l2 grad parity", name)
    wl, orc, pb, _, _ = problem(name)
    alpha, beta = cases.random_vars(orc, seed=22)
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
    say(name, "grad rows checked", checked, "of", orc.B * orc.m, "worst", worst)
    assert checked >= 0.75 * orc.B * orc.m
    assert worst <= TOL


@pytest.mark.parametrize("name,nparts", [("mlp_small", 1), ("cnn_base", 1), ("mlp_deep", 2)])
def test_l2_optimize_parity(name, nparts):
    """20 projected-Adam steps from CROWN's alpha and beta = 0 (over two
    concurrent sub-batches for mlp_deep: the ball set before the split must
    reach the new sub-batch handles)."""
    say("l2 optimize parity", name, nparts)
    wl, orc, pb, _, _ = problem(name)
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
    say(name, "opt max rel err", max(errs), "max rel excess at own vars", max(ex))
    assert np.all(a_gpu >= 0) and np.all(a_gpu <= 1) and np.all(b_gpu >= 0)
    assert max(errs) <= TOL
    assert max(ex) <= TOL


@pytest.mark.parametrize("name", ["mlp_small", "cnn_base", "mlp_deep"])
def test_l2_upper_bound_parity(name):
    """ub = C f(x*) at x* = x0 - eps A(0)/||A(0)||_2 on every row, the split
    check where the smallest split pre-activation at x* is clear of zero, and
    lb <= ub where sat."""
    say("l2 upper bound", name)
    wl, orc, pb, _, _ = problem(name)
    alpha, beta = cases.random_vars(orc, seed=23)
    lb, ub, sat = [t.cpu().numpy() for t in pb.upper(dev(alpha), dev(beta))]
    n_sat = 0
    for b in range(orc.B):
        g, u, st, mg = orc.upper(b, alpha, beta)
        assert guarded_rel(lb[b], g).max() <= TOL
        assert guarded_rel(ub[b], u).max() <= TOL, (b, ub[b], u)
        for k in np.nonzero(mg > 1e-3)[0]:
            assert bool(sat[b, k]) == bool(st[k]), (b, k, mg[k])
            n_sat += 1
        if orc.ptr[b + 1] == orc.ptr[b]:
            assert (sat[b] == 1).all()
    s1 = sat.astype(bool)
    assert (lb[s1] <= ub[s1] + TOL * np.maximum(1.0, np.abs(ub[s1]))).all()
    say(name, "sat checked", n_sat, "sat=1", int(s1.sum()), "of", sat.size)


def test_l2_bound_below_sampled_network_values():
    """Soundness over the ball: with no splits (one subdomain per property),
    every optimised lower bound (20 steps) lies below C f(x) at points drawn
    on and inside the property's ball, the network evaluated in FP64."""
    from paper_2103_06624_amd.api import BoundProblem
    wl, lo, up, x0, eps, orc = cases.small_l2_case("mlp_small")
    P = x0.shape[0]
    pb = BoundProblem(wl.net.layers, wl.x_lo, wl.x_hi, wl.C, lo, up, np.arange(P, dtype=np.int32),
                      np.zeros(P + 1, np.int64), [], [], [])
    pb.set_input_l2(x0, eps)

    def forward(x):
        h = x.T
        for i, (W, bias) in enumerate(orc.net64):
            h = W @ h + bias[:, None]
            if i < len(orc.net64) - 1:
                h = np.maximum(h, 0.0)
        return h.T

    best, _ = pb.optimize(pb.alpha_init(), pb.zeros_beta(), iters=20)
    best = best.cpu().numpy()
    rng = np.random.default_rng(7)
    d0 = x0.shape[1]
    for p in range(P):
        d = rng.standard_normal((512, d0))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        r = np.concatenate([np.ones(256), rng.uniform(0, 1, 256) ** (1.0 / d0)])
        xs = x0[p].astype(np.float64)[None] + eps[p] * r[:, None] * d
        vmin = (forward(xs) @ orc.C[p].T).min(axis=0)
        assert (best[p] <= vmin + 1e-5 * np.maximum(1.0, np.abs(vmin))).all(), (p, best[p], vmin)


def test_l2_off_returns_to_box():
    """Switching the balls off gives back the box bounds bit for bit."""
    from paper_2103_06624_amd.api import BoundProblem
    wl, lo, up, x0, eps, orc = cases.small_l2_case("mlp_small")
    pb = BoundProblem.from_workload(wl, lo, up)
    alpha, beta = cases.random_vars(orc, seed=24)
    box = pb.eval(dev(alpha), dev(beta)).cpu().numpy()
    pb.set_input_l2(x0, eps)
    ball = pb.eval(dev(alpha), dev(beta)).cpu().numpy()
    pb.set_input_l2(None, None)
    again = pb.eval(dev(alpha), dev(beta)).cpu().numpy()
    assert np.array_equal(box, again)
    assert not np.array_equal(box, ball)


def test_l2_rejects_bad_values():
    from paper_2103_06624_amd.binding import CvError
    wl, orc, pb, x0, eps = problem("mlp_small")
    for bad_eps in (-1.0, np.inf, np.nan):
        with pytest.raises(CvError):
            pb.set_input_l2(x0, np.full_like(eps, bad_eps))
    bad_x = x0.copy()
    bad_x[0, 0] = np.nan
    with pytest.raises(CvError):
        pb.set_input_l2(bad_x, eps)


SOUND_TOL = 1e-6  # the float64 evaluation's margin plus one float ulp, relative to max(|bound|, 1)


@pytest.mark.parametrize("name", ["mlp_small", "cnn_base", "mlp_deep"])
def test_l2_sound_mode_is_below_the_exact_bound(name):
    """Sound mode over l2 balls: every bound lies below the FP64 oracle's
    bound on the same balls at the same variables (every row, no tolerance)
    and within SOUND_TOL of it; the optimiser's final iterate too.  Switching
    sound mode off restores the plain bounds bit for bit, and setting the
    balls before or after switching sound mode on gives the same bounds."""
    from paper_2103_06624_amd.api import BoundProblem
    wl, orc, pb, x0, eps = problem(name)
    alpha, beta = cases.random_vars(orc, seed=25)
    lb_plain = pb.eval(dev(alpha), dev(beta)).cpu().numpy()
    pb.set_sound(1)
    lb = pb.eval(dev(alpha), dev(beta)).cpu().numpy()
    ref = np.stack([orc.eval(b, alpha, beta) for b in range(orc.B)])
    assert (lb <= ref).all()
    assert guarded_rel(lb, ref).max() <= SOUND_TOL
    say(name, "sound excess", float(np.maximum(lb - ref, 0).max()), "gap max", float(guarded_rel(lb, ref).max()))
    a = pb.alpha_init()
    b = pb.zeros_beta()
    best, last = pb.optimize(a, b, iters=5)
    a_h, b_h = a.cpu().numpy(), b.cpu().numpy()
    ref_last = np.stack([orc.eval(d, a_h, b_h) for d in range(orc.B)])
    assert (last.cpu().numpy() <= ref_last).all()
    # the other order: sound mode first, then the balls
    wl2, lo, up, _, _, _ = cases.small_l2_case(name)
    pb2 = BoundProblem.from_workload(wl2, lo, up)
    pb2.set_sound(1)
    pb2.set_input_l2(x0, eps)
    assert np.array_equal(pb2.eval(dev(alpha), dev(beta)).cpu().numpy(), lb)
    pb.set_sound(0)
    assert np.array_equal(pb.eval(dev(alpha), dev(beta)).cpu().numpy(), lb_plain)


def test_l2_zero_radius_is_the_point():
    """Degenerate balls (eps = 0): the bound matches the oracle, and the upper
    bound is the network at x0 itself on every row (x* = x0), checked against
    an FP64 forward pass."""
    wl, orc, pb, x0, eps = problem("mlp_small")
    z = np.zeros_like(eps)
    pb.set_input_l2(x0, z)
    orc_z = cases.small_l2_case("mlp_small")[5]
    alpha, beta = cases.random_vars(orc, seed=26)
    saved = orc_z.l2
    try:
        orc_z.set_l2(x0, z)
        lb, ub, sat = [t.cpu().numpy() for t in pb.upper(dev(alpha), dev(beta))]
        ref = np.stack([orc_z.eval(b, alpha, beta) for b in range(orc_z.B)])
        assert guarded_rel(lb, ref).max() <= TOL
    finally:
        orc_z.l2 = saved
    for b in range(orc.B):
        p = int(orc.dom_prop[b])
        h = x0[p].astype(np.float64)
        for i, (W, bias) in enumerate(orc.net64):
            h = W @ h + bias
            if i < len(orc.net64) - 1:
                h = np.maximum(h, 0.0)
        assert guarded_rel(ub[b], orc.C[p] @ h).max() <= TOL
    s1 = sat.astype(bool)  # where x0 meets the subdomain's splits
    assert (lb[s1] <= ub[s1] + TOL * np.maximum(1.0, np.abs(ub[s1]))).all()
