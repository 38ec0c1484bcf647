"""GPU parity of the joint optimisation of intermediate bounds
(cv_bound_optimize_joint; Sec. 3.3, Eq. opt_non_convex) against the FP64 oracle
(oracle.joint) on the same subdomains: the bound and every intermediate bound
at the GPU's own final variables, the gradient in the shared variables at the
start, the bound at the start, and the 20-iteration trajectory's best bound.
Bar: 1e-4 guarded relative."""
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


def problem(name):
    from paper_2103_06624_amd.api import BoundProblem
    wl, lo, up, lo64, up64, orc = cases.small_case(name)
    return wl, orc, BoundProblem.from_workload(wl, lo, up)


def gpu_joint_vars(pb, orc):
    """{layer i: (alpha', beta', g alpha', g beta')} of every intermediate layer, host arrays."""
    return {i: tuple(t.cpu().numpy() for t in pb.joint_vars(i)) for i in range(2, len(orc.net64))}


CASES = [("mlp_small", 16), ("cnn_odd", 12), ("mlp_deep", 6)]


@pytest.mark.parametrize("name,n_check", CASES)
def test_joint_bounds_at_the_gpus_own_variables(name, n_check):
    """After 20 joint iterations: the final bound and every intermediate bound
    of the final iterate against the FP64 oracle's joint bound evaluated at
    the GPU's own final alpha, beta, alpha' and beta' (the trajectory itself
    is rounding-dependent; the bound at given variables is unique)."""
    say("joint at own variables", name)
    wl, orc, pb = problem(name)
    a = pb.alpha_init()
    b = pb.zeros_beta()
    best, last, lo_g, up_g = pb.optimize_joint(a, b, iters=20, bounds=True)
    last, lo_g, up_g = last.cpu().numpy(), lo_g.cpu().numpy(), up_g.cpu().numpy()
    a_g, b_g = a.cpu().numpy(), b.cpu().numpy()
    jflat = {i: (v[0], v[1]) for i, v in gpu_joint_vars(pb, orc).items()}
    for i, (ash, bsh) in jflat.items():
        assert np.all(ash >= 0) and np.all(ash <= 1) and np.all(bsh >= 0)
    assert np.all(a_g >= 0) and np.all(a_g <= 1) and np.all(b_g >= 0)
    doms = range(orc.B) if orc.B <= n_check else np.random.default_rng(9).choice(orc.B, n_check, replace=False)
    worst = 0.0
    for d in doms:
        g, l_j, u_j = orc.joint_eval(d, a_g, b_g, orc.joint_vars(d, jflat))
        e = max(guarded_rel(last[d], g).max(), guarded_rel(lo_g[d], l_j).max(), guarded_rel(up_g[d], u_j).max())
        worst = max(worst, e)
    say(name, "max rel err at own variables", worst)
    assert worst <= TOL


@pytest.mark.parametrize("name,n_check", CASES)
def test_joint_gradient_at_the_start(name, n_check):
    """One joint iteration: the gradient of sum g with respect to every
    layer's shared alpha', beta' at the start (alpha' at CROWN's slopes,
    beta' = 0), against the oracle's autograd gradient, per subdomain and
    layer relative to the largest entry of the two blocks."""
    say("joint gradient", name)
    wl, orc, pb = problem(name)
    a = pb.alpha_init()
    b = pb.zeros_beta()
    pb.optimize_joint(a, b, iters=1)
    gv = gpu_joint_vars(pb, orc)
    a0 = orc.default_alpha_flat()
    z = np.zeros(orc.nnz * orc.m)
    doms = range(orc.B) if orc.B <= n_check else np.random.default_rng(10).choice(orc.B, n_check, replace=False)
    worst, nz = 0.0, 0
    for d in doms:
        *_, gref = orc.joint_eval(d, a0, z, orc.joint_start(d), grad=True)
        for i, (ga_ref, gb_ref) in gref.items():
            oa, ob = orc.joint_offsets(i)
            ga = gv[i][2][oa[d]:oa[d + 1]]
            gb = gv[i][3][ob[d]:ob[d + 1]]
            scale = max(1.0, np.abs(ga_ref).max(initial=0), np.abs(gb_ref).max(initial=0))
            worst = max(worst, np.abs(ga - ga_ref).max(initial=0) / scale, np.abs(gb - gb_ref).max(initial=0) / scale)
            nz += int((np.abs(ga_ref) > 1e-6).sum())
    say(name, "gradient max rel err", worst, "non-zero entries", nz)
    assert nz > 0
    assert worst <= TOL


@pytest.mark.parametrize("name,n_check", CASES)
def test_joint_trajectory_against_the_oracle(name, n_check):
    """20 joint iterations from the same start on both sides (lr 0.01 / 0.05,
    decay 0.98): the best bound of each checked subdomain against the
    oracle's."""
    say("joint trajectory", name)
    wl, orc, pb = problem(name)
    a = pb.alpha_init()
    b = pb.zeros_beta()
    best, _ = pb.optimize_joint(a, b, iters=20)
    best = best.cpu().numpy()
    a0 = orc.default_alpha_flat()
    z = np.zeros(orc.nnz * orc.m)
    doms = range(orc.B) if orc.B <= n_check else np.random.default_rng(9).choice(orc.B, n_check, replace=False)
    errs = []
    for d in doms:
        rbest = orc.joint_optimize(d, a0, z)[0]
        errs.append(guarded_rel(best[d], rbest).max())
        say(f"  dom {d} best {errs[-1]:.2e}")
    say(name, "best max rel err", max(errs))
    assert max(errs) <= TOL


@pytest.mark.parametrize("name", ["mlp_small", "cnn_odd", "mlp_deep"])
def test_zero_iterations_is_the_bound_at_the_start(name):
    """iters = 0: one evaluation with alpha' at CROWN's slopes and beta' = 0;
    the intermediate bounds are the computed ones where tighter than the root
    (splits make them so), and the bound is the oracle's joint bound at the
    start, on every subdomain."""
    from oracle import joint as jt
    say("joint zero iterations", name)
    wl, orc, pb = problem(name)
    a = pb.alpha_init()
    b = pb.zeros_beta()
    best, last, lo_g, up_g = pb.optimize_joint(a, b, iters=0, bounds=True)
    best, lo_g, up_g = best.cpu().numpy(), lo_g.cpu().numpy(), up_g.cpu().numpy()
    a0 = orc.default_alpha_flat()
    z = np.zeros(orc.nnz * orc.m)
    errs = []
    for d in range(min(orc.B, 24)):
        p, lo, up, split = orc.domain(d)
        g, l_j, u_j = jt.joint_bound(orc.net64, orc.x_lo[p], orc.x_hi[p], orc.C[p], lo, up, split,
                                     [torch.tensor(x) for x in orc.alpha_to_layers(d, a0)],
                                     [torch.tensor(x) for x in orc.beta_to_layers(d, z)],
                                     jt.init_vars(orc.net64, lo, up))
        errs.append(guarded_rel(best[d], g.numpy()).max())
        errs.append(guarded_rel(lo_g[d], np.concatenate([x.numpy() for x in l_j])).max())
        errs.append(guarded_rel(up_g[d], np.concatenate([x.numpy() for x in u_j])).max())
    say(name, "max rel err", max(errs))
    assert max(errs) <= TOL


def test_joint_rejects_sound_mode_and_balls():
    from paper_2103_06624_amd.binding import CvError
    wl, orc, pb = problem("mlp_small")
    a, b = pb.alpha_init(), pb.zeros_beta()
    pb.set_sound(1)
    with pytest.raises(CvError):
        pb.optimize_joint(a, b, iters=2)
    pb.set_sound(0)
    x0 = np.asarray(wl.x0, np.float32)
    pb.set_input_l2(x0, np.full(x0.shape[0], 0.01, np.float32))
    with pytest.raises(CvError):
        pb.optimize_joint(a, b, iters=2)
    pb.set_input_l2(None, None)
    with pytest.raises(CvError):
        pb.optimize_joint(a, b, iters=-1)
    best, _ = pb.optimize_joint(a, b, iters=1)
    assert torch.isfinite(best).all()
