"""GPU parity of libcvbound against the FP64 oracle, through the C ABI.

Bar: bounds and gradients within 1e-4 guarded relative error
(|x - x64| / max(|x64|, 1)) at identical (alpha, beta); optimised bounds
within the same bar after the 20-step projected-Adam trajectory.  The
soundness excess max(0, g_gpu - g64(alpha_gpu, beta_gpu)) is reported: in
plain float32 it is bounded by the same rounding tolerance, in sound mode it
is zero on every row.
"""
import sys

import numpy as np
import pytest

from tests import cases
from tests.cases import guarded_rel

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

TOL = 1e-4
SOUND_TOL = 1e-6  # sound mode: the float64 evaluation's margin plus one float ulp, relative to max(|bound|, 1)
NAMES = list(cases.SMALL)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2103_06624_amd import binding
    binding.lib()


def problem(name, full=False):
    from paper_2103_06624_amd.api import BoundProblem
    wl, lo, up, _, _, orc = cases.case(name) if full else cases.small_case(name)
    return wl, orc, BoundProblem.from_workload(wl, lo, up)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda()


def sample_doms(orc, k, seed=0):
    rng = np.random.default_rng(seed)
    return sorted(rng.choice(orc.B, size=min(k, orc.B), replace=False).tolist())


@pytest.mark.parametrize("name", NAMES)
def test_eval_parity(name):
    say("eval parity", name)
    wl, orc, pb = problem(name)
    alpha, beta = cases.random_vars(orc, seed=1)
    lb = pb.eval(dev(alpha), dev(beta)).cpu().numpy()
    ref = np.stack([orc.eval(b, alpha, beta) for b in range(orc.B)])
    err = guarded_rel(lb, ref)
    say(name, "max rel err", err.max(), "excess", np.maximum(lb - ref, 0).max())
    assert err.max() <= TOL
    assert np.all(lb - ref <= TOL * np.maximum(np.abs(ref), 1.0))


def test_config1_default_alpha_zero_beta():
    """mlp_small as stated: CROWN default alpha, beta = 0, 16 x 9 bounds."""
    wl, orc, pb = problem("mlp_small")
    a = pb.alpha_init()
    lb = pb.eval(a, pb.zeros_beta()).cpu().numpy()
    assert lb.shape == (16, 9)
    a_ref = orc.default_alpha_flat()
    assert np.array_equal(a.cpu().numpy(), a_ref.astype(np.float32))
    ref = np.stack([orc.eval(b, a_ref, np.zeros(orc.nnz * orc.m)) for b in range(orc.B)])
    assert guarded_rel(lb, ref).max() <= TOL


def kink_free_rows(orc, b, alpha, beta, ulps=100.0):
    """Rows whose FP64 sign decisions are out of float32 reach of a kink: every
    A(i)_j at an unstable neuron and every A(0)_j is either exactly 0
    (structural, identical in float32) or larger than `ulps` float32 ulps of
    its own accumulation magnitude (|Lambda(i+1)| |W(i+1)|)_j."""
    from oracle import beta_crown as bc
    p, lo, up, split = orc.domain(b)
    beta_l = orc.beta_to_layers(b, beta)
    g, A0, tr = bc.bound(orc.net64, orc.x_lo[p], orc.x_hi[p], orc.C[p], lo, up, split,
                         orc.alpha_to_layers(b, alpha), beta_l, keep=True)
    eps = ulps * np.finfo(np.float32).eps

    def near(A, mag):
        ax = np.abs(A)
        return ((ax > 0) & (ax <= eps * mag)).any(axis=1)

    L = len(orc.net64)
    ok = np.ones(A0.shape[0], bool)
    for i in range(1, L):  # A(i-1) = Lambda(i) W(i)
        A, D, _ = tr[i - 1]
        lam = A * D + beta_l[i - 1] * bc.split_sign(split[i - 1])
        mag = np.abs(lam) @ np.abs(orc.net64[i - 1][0])
        if i == 1:
            ok &= ~near(A0, mag)
        else:
            _, _, uns = bc.neuron_kind(lo[i - 2], up[i - 2], split[i - 2])
            Aprev = tr[i - 2][0]
            ok &= ~near(Aprev[:, uns], mag[:, uns])
    return ok


def oracle_grads(orc, alpha, beta):
    """Per subdomain: the oracle's bound and gradients, and which spec rows
    are clear of kinks."""
    return [(*orc.grad(b, alpha, beta), kink_free_rows(orc, b, alpha, beta)) for b in range(orc.B)]


def check_grad(name, orc, pb, alpha, beta, ref=None):
    """Bound and gradient of every subdomain against the oracle; gradient rows
    are compared where no sign decision is within float32 reach of a kink."""
    ref = ref or oracle_grads(orc, alpha, beta)
    lb, ga, gb = pb.grad(dev(alpha), dev(beta))
    lb, ga, gb = lb.cpu().numpy(), ga.cpu().numpy(), gb.cpu().numpy().reshape(-1, orc.m)
    checked = 0
    worst = 0.0
    for b in range(orc.B):
        g, ra, rb, ok = ref[b]
        assert guarded_rel(lb[b], g).max() <= TOL
        U = ra.shape[0] // orc.m
        a_gpu = ga[orc.alpha_off[b]:orc.alpha_off[b + 1]].reshape(orc.m, U)
        a_ref = ra.reshape(orc.m, U)
        b_gpu = gb[orc.ptr[b]:orc.ptr[b + 1]]
        for k in np.nonzero(ok)[0]:
            scale = max(1.0, np.abs(a_ref[k]).max(initial=0), np.abs(rb[:, k]).max(initial=0))
            e1 = np.abs(a_gpu[k] - a_ref[k]).max(initial=0) / scale
            e2 = np.abs(b_gpu[:, k] - rb[:, k]).max(initial=0) / scale
            worst = max(worst, e1, e2)
            checked += 1
    say(name, "grad rows checked", checked, "of", orc.B * orc.m, "worst", worst)
    assert checked >= 0.75 * orc.B * orc.m
    assert worst <= TOL


@pytest.mark.parametrize("name", NAMES)
def test_grad_parity(name):
    say("grad parity", name)
    wl, orc, pb = problem(name)
    alpha, beta = cases.random_vars(orc, seed=2)
    check_grad(name, orc, pb, alpha, beta)


@pytest.mark.parametrize("name,plan", [("mlp_deep", (0, 0)), ("mlp_deep", (1, 1)), ("mlp_deep", (1, 0)),
                                       ("mlp_deep", (0, 1)), ("cnn_deep", (0, 0)), ("cnn_deep", (1, 0))])
def test_plan_parity(name, plan):
    """Fused dense chains and per-layer kernels, each direction on its own
    (cnn_deep's dense tail is one layer deep: a back-substitution chain only)."""
    say("plan parity", name, plan)
    wl, orc, pb = problem(name)
    pb.set_plan(*plan)
    alpha, beta = cases.random_vars(orc, seed=6)
    lb = pb.eval(dev(alpha), dev(beta)).cpu().numpy()
    ref = np.stack([orc.eval(b, alpha, beta) for b in range(orc.B)])
    assert guarded_rel(lb, ref).max() <= TOL
    check_grad(name, orc, pb, alpha, beta)


@pytest.mark.parametrize("name,plan", [(n, None) for n in NAMES] + [("mlp_deep", (1, 0))])
def test_upper_bound_parity(name, plan):
    """ub = C f(x*) at each row's box minimiser and the split check, against
    the oracle.  ub is compared on rows whose A(0) signs are out of float32
    reach of a tie (x* is then the same point); sat where the smallest split
    pre-activation at x* is clear of zero.  Rows without splits must have
    sat = 1, and sat = 1 rows must have lb <= ub."""
    say("upper bound", name, plan)
    wl, orc, pb = problem(name)
    if plan:
        pb.set_plan(*plan)
    alpha, beta = cases.random_vars(orc, seed=11)
    lb, ub, sat = [t.cpu().numpy() for t in pb.upper(dev(alpha), dev(beta))]
    lb_eval = pb.eval(dev(alpha), dev(beta)).cpu().numpy()
    assert np.array_equal(lb, lb_eval)
    n_ub = n_sat = 0
    for b in range(orc.B):
        g, u, st, mg = orc.upper(b, alpha, beta)
        assert guarded_rel(lb[b], g).max() <= TOL
        ok = kink_free_rows(orc, b, alpha, beta)
        for k in np.nonzero(ok)[0]:
            assert guarded_rel(ub[b, k], u[k]) <= TOL, (b, k, ub[b, k], u[k])
            n_ub += 1
            if mg[k] > 1e-3:
                assert bool(sat[b, k]) == bool(st[k]), (b, k, mg[k])
                n_sat += 1
        if orc.ptr[b + 1] == orc.ptr[b]:
            assert (sat[b] == 1).all()
    assert n_ub >= 0.75 * orc.B * orc.m
    s1 = sat.astype(bool)
    assert (lb[s1] <= ub[s1] + TOL * np.maximum(1.0, np.abs(ub[s1]))).all()
    say(name, "ub rows checked", n_ub, "sat checked", n_sat, "sat=1", int(s1.sum()), "of", sat.size)


@pytest.mark.parametrize("name", NAMES)
def test_sound_mode_is_below_the_exact_bound(name):
    """Sound mode: the bound is evaluated in float64 with a rigorous bound on
    its float64 rounding and rounded down to float, so every bound lies below
    the FP64 oracle's bound at the same variables -- every row, no tolerance --
    and within SOUND_TOL of it.  The optimiser's final iterate is reported the
    same way (below the oracle at the returned variables); its best bound is
    at least that.  Switching sound mode off restores the plain bounds."""
    wl, orc, pb = problem(name)
    alpha, beta = cases.random_vars(orc, seed=12)
    lb_plain = pb.eval(dev(alpha), dev(beta)).cpu().numpy()
    pb.set_sound(1)
    lb = pb.eval(dev(alpha), dev(beta)).cpu().numpy()
    ref = np.stack([orc.eval(b, alpha, beta) for b in range(orc.B)])
    gap = guarded_rel(lb, ref)
    say(name, "plain excess", float(np.maximum(lb_plain - ref, 0).max()), "sound excess",
        float(np.maximum(lb - ref, 0).max()), "sound gap max", float(gap.max()))
    assert (lb <= ref).all()
    assert gap.max() <= SOUND_TOL
    # the bound of cv_bound_grad and cv_bound_upper in sound mode is the same
    lb_g, _, _ = pb.grad(dev(alpha), dev(beta))
    assert np.array_equal(lb_g.cpu().numpy(), lb)
    a = pb.alpha_init()
    b = pb.zeros_beta()
    best, last = pb.optimize(a, b, iters=5)
    a_h, b_h = a.cpu().numpy(), b.cpu().numpy()
    ref_last = np.stack([orc.eval(d, a_h, b_h) for d in range(orc.B)])
    last = last.cpu().numpy()
    assert (last <= ref_last).all()
    assert guarded_rel(last, ref_last).max() <= SOUND_TOL
    assert (best.cpu().numpy() >= last).all()
    pb.set_sound(0)
    assert np.array_equal(pb.eval(dev(alpha), dev(beta)).cpu().numpy(), lb_plain)


@pytest.mark.parametrize("name", NAMES)
def test_sound_optimised_bounds_meet_the_parity_bar_with_zero_violations(name):
    """Sound mode end to end: the 20-step optimised bounds are within TOL of the
    FP64 oracle's 20-step optimisation from the same start, and no row is
    unsound -- the final iterate's bound lies below the FP64 bound at the
    GPU's own final variables on every row."""
    from oracle.beta_crown import AdamConfig
    wl, orc, pb = problem(name)
    pb.set_sound(1)
    a, b = pb.alpha_init(), pb.zeros_beta()
    best, last = pb.optimize(a, b, iters=20)
    best, last = best.cpu().numpy(), last.cpu().numpy()
    a_h, b_h = a.cpu().numpy(), b.cpu().numpy()
    a0, z0 = orc.default_alpha_flat(), np.zeros(orc.nnz * orc.m)
    ref_best = np.stack([orc.optimize(d, a0, z0, AdamConfig(iters=20))[0] for d in range(orc.B)])
    ref_last = np.stack([orc.eval(d, a_h, b_h) for d in range(orc.B)])
    err = guarded_rel(best, ref_best)
    viol = int(np.sum(last > ref_last))
    say(name, "sound optimised: max rel err", float(err.max()), "violations", viol, "of", last.size)
    assert viol == 0
    assert err.max() <= TOL


def test_sound_root_bounds_enclose_sampled_preactivations():
    """The library's root bounds are sound: every pre-activation of the
    float64 network at random points of the box lies inside them."""
    from paper_2103_06624_amd import api, synth
    for name in ["mlp_deep", "cnn_base"]:
        wl = synth.make(name)
        lo, up = api.root_bounds(wl.net.layers, wl.x_lo, wl.x_hi, sound=True)
        lo_p, up_p = api.root_bounds(wl.net.layers, wl.x_lo, wl.x_hi)
        # the float64 evaluation: within float rounding of the plain bounds
        assert np.abs(lo - lo_p).max() <= 1e-4 * max(1.0, np.abs(lo_p).max())
        assert np.abs(up - up_p).max() <= 1e-4 * max(1.0, np.abs(up_p).max())
        from oracle import beta_crown as bc
        net64 = bc.dense_net(wl.net.layers)
        rng = np.random.default_rng(5)
        for p in range(min(2, wl.x_lo.shape[0])):
            xl, xh = wl.x_lo[p].astype(np.float64), wl.x_hi[p].astype(np.float64)
            X = xl + (xh - xl) * rng.uniform(size=(256, xl.shape[0]))
            X[:32] = np.where(rng.uniform(size=(32, xl.shape[0])) < 0.5, xl, xh)  # box corners
            h = X
            off = 0
            for W, b in net64[:-1]:
                z = h @ W.T + b
                d = z.shape[1]
                assert (z >= lo[p, off:off + d] - 0.0).all() and (z <= up[p, off:off + d] + 0.0).all(), name
                h = np.maximum(z, 0.0)
                off += d


@pytest.mark.parametrize("name", ["mlp_small", "cnn_base", "cnn_odd", "mlp_deep"])
def test_optimised_root_bounds_parity(name):
    """Intermediate bounds each maximised over its own alpha' (10 Adam steps):
    against the oracle's, at least as tight as the library's CROWN bounds, and
    (in sound mode) enclosing sampled pre-activations."""
    from oracle import beta_crown as bc
    from paper_2103_06624_amd.api import root_bounds
    wl, lo32, up32, lo64, up64, orc = cases.small_case(name)
    lo, up = root_bounds(wl.net.layers, wl.x_lo, wl.x_hi, opt_iters=10, lr_alpha=0.1, decay=0.98)
    lo_c, up_c = root_bounds(wl.net.layers, wl.x_lo, wl.x_hi)
    assert (lo >= lo_c - 1e-6 * np.maximum(1, np.abs(lo_c))).all() and (up <= up_c + 1e-6 * np.maximum(1, np.abs(up_c))).all()
    assert (lo > lo_c + 1e-4).any() or (up < up_c - 1e-4).any()
    cfg = bc.AdamConfig(iters=10, lr_alpha=0.1, decay=0.98)
    for p in range(min(2, wl.x_lo.shape[0])):
        lo_o, up_o = bc.root_bounds_opt(orc.net64, wl.x_lo[p].astype(np.float64), wl.x_hi[p].astype(np.float64), cfg)
        e = max(guarded_rel(lo[p], np.concatenate(lo_o)).max(), guarded_rel(up[p], np.concatenate(up_o)).max())
        say(name, "optimised root bounds rel err", e, "property", p)
        assert e <= TOL
    lo_s, up_s = root_bounds(wl.net.layers, wl.x_lo, wl.x_hi, sound=True, opt_iters=10, lr_alpha=0.1, decay=0.98)
    # sound: evaluated in float64 and rounded outward, within float rounding
    # of the plain optimised bounds, and enclosing the sampled pre-activations
    assert guarded_rel(lo_s, lo).max() <= TOL and guarded_rel(up_s, up).max() <= TOL
    rng = np.random.default_rng(3)
    xl, xh = wl.x_lo[0].astype(np.float64), wl.x_hi[0].astype(np.float64)
    h = xl + (xh - xl) * rng.uniform(size=(128, xl.shape[0]))
    off = 0
    for W, b in orc.net64[:-1]:
        z = h @ W.T + b
        d = z.shape[1]
        assert (z >= lo_s[0, off:off + d]).all() and (z <= up_s[0, off:off + d]).all()
        h = np.maximum(z, 0.0)
        off += d


def test_sound_rejects_bad_values():
    from paper_2103_06624_amd.binding import CvError
    wl, orc, pb = problem("mlp_small")
    for bad in [-1, 2]:
        with pytest.raises(CvError):
            pb.set_sound(bad)


@pytest.mark.parametrize("name", ["mlp_small", "mlp_deep"])
def test_every_tiling(name):
    """Every GEMM tiling (tile shape, K slab, loads in flight) on every dense
    layer: bounds and gradients against the oracle."""
    from paper_2103_06624_amd.api import BoundProblem
    wl, orc, pb = problem(name)
    alpha, beta = cases.random_vars(orc, seed=9)
    ref = oracle_grads(orc, alpha, beta)
    lb_ref = np.stack([r[0] for r in ref])
    n = BoundProblem.num_tilings()
    assert n >= 30
    for t in range(n):
        say("tiling", name, t)
        pb.set_tiling(t)
        lb = pb.eval(dev(alpha), dev(beta)).cpu().numpy()
        assert guarded_rel(lb, lb_ref).max() <= TOL, t
        check_grad(name, orc, pb, alpha, beta, ref)
    pb.set_tiling(-1)
    lb = pb.eval(dev(alpha), dev(beta)).cpu().numpy()
    assert guarded_rel(lb, lb_ref).max() <= TOL


@pytest.mark.parametrize("name", ["cnn_base", "cnn_wide", "cnn_deep", "cnn_odd"])
def test_every_conv_variant(name):
    """Every conv kernel variant (row-major or subdomain-major, weights in LDS
    or global memory) on every conv layer in both directions: bounds,
    gradients and a 5-step optimisation against the oracle, and the tuned
    choice afterwards."""
    from paper_2103_06624_amd.api import BoundProblem
    wl, orc, pb = problem(name)
    alpha, beta = cases.random_vars(orc, seed=19)
    ref = oracle_grads(orc, alpha, beta)
    lb_ref = np.stack([r[0] for r in ref])
    a0 = orc.default_alpha_flat()
    z0 = np.zeros(orc.nnz * orc.m)
    from oracle.beta_crown import AdamConfig
    opt_ref = np.stack([orc.optimize(d, a0, z0, AdamConfig(iters=5))[0] for d in range(orc.B)])
    n = BoundProblem.num_conv_variants()
    assert n == 4
    conv_layers = [i + 1 for i, ly in enumerate(wl.net.layers) if ly.kind == 1]
    for var in range(n):
        pb.set_conv_variant(var)
        ran = [(pb.conv_variant(i, 0), pb.conv_variant(i, 1)) for i in conv_layers]
        say("conv variant", name, var, "layers run", ran)
        lb = pb.eval(dev(alpha), dev(beta)).cpu().numpy()
        assert guarded_rel(lb, lb_ref).max() <= TOL, var
        check_grad(name, orc, pb, alpha, beta, ref)
        best, _ = pb.optimize(dev(a0), dev(z0), iters=5)
        assert guarded_rel(best.cpu().numpy(), opt_ref).max() <= TOL, var
    pb.autotune()
    ran = [(pb.conv_variant(i, 0), pb.conv_variant(i, 1)) for i in conv_layers]
    say("tuned", name, ran)
    assert all(0 <= v < n for pair in ran for v in pair)
    lb = pb.eval(dev(alpha), dev(beta)).cpu().numpy()
    assert guarded_rel(lb, lb_ref).max() <= TOL
    pb.set_conv_variant(-1)
    with pytest.raises(Exception):
        pb.set_conv_variant(n)


def test_tiling_rejects_bad_values():
    from paper_2103_06624_amd.api import BoundProblem
    from paper_2103_06624_amd.binding import CvError
    wl, orc, pb = problem("mlp_small")
    for bad in [-2, BoundProblem.num_tilings()]:
        with pytest.raises(CvError):
            pb.set_tiling(bad)


def test_plan_rejects_bad_values():
    from paper_2103_06624_amd.binding import CvError
    wl, orc, pb = problem("mlp_small")
    for bad in [(2, 0), (0, -1), (16, 16)]:
        with pytest.raises(CvError):
            pb.set_plan(*bad)
    wl, orc, pb = problem("cnn_deep")
    with pytest.raises(CvError):
        pb.set_plan(1, 1)  # no adjoint chain above a single dense layer


@pytest.mark.parametrize("name,plan", [("mlp_small", None), ("mlp_deep", None), ("cnn_base", None),
                                       ("cnn_deep", None), ("cnn_odd", None), ("mlp_deep", (0, 0)),
                                       ("cnn_deep", (0, 0))])
def test_optimize_parity(name, plan):
    say("optimize parity", name, plan)
    wl, orc, pb = problem(name)
    if plan is not None:
        pb.set_plan(*plan)
    a = pb.alpha_init()
    b = pb.zeros_beta()
    best, last = pb.optimize(a, b, iters=20, lr_alpha=0.01, lr_beta=0.05, decay=0.98)
    best, last = best.cpu().numpy(), last.cpu().numpy()
    a_gpu, b_gpu = a.cpu().numpy(), b.cpu().numpy()
    a0 = orc.default_alpha_flat()
    errs, ex = [], []
    for d in range(orc.B):
        rbest, _, _, rlast = orc.optimize(d, a0, np.zeros(orc.nnz * orc.m))
        errs.append(guarded_rel(best[d], rbest).max())
        # soundness at the GPU's own final variables
        g64 = orc.eval(d, a_gpu, b_gpu)
        ex.append(((last[d] - g64) / np.maximum(np.abs(g64), 1.0)).max())
    errs = np.array(errs)
    say(name, "opt max rel err", errs.max(), "mean", errs.mean(), "max rel excess at own vars", max(ex))
    assert np.all(a_gpu >= 0) and np.all(a_gpu <= 1) and np.all(b_gpu >= 0)
    assert errs.max() <= TOL
    assert max(ex) <= TOL


@pytest.mark.parametrize("name", NAMES)
def test_root_bounds_parity(name):
    say("root bounds", name)
    from paper_2103_06624_amd.api import root_bounds
    wl, lo32, up32, lo64, up64, orc = cases.small_case(name)
    lo, up = root_bounds(wl.net.layers, wl.x_lo, wl.x_hi)
    e = max(guarded_rel(lo, lo64).max(), guarded_rel(up, up64).max())
    say(name, "root bounds max rel err", e)
    assert e <= TOL


def test_alpha_layout_matches_documentation():
    wl, orc, pb = problem("cnn_deep")
    for b in [0, orc.B // 2, orc.B - 1]:
        p = int(orc.dom_prop[b])
        for t, flat in enumerate(orc.unstable[p][:50]):
            i = int(np.searchsorted(orc.offs, flat, side="right"))
            j = int(flat - orc.offs[i - 1])
            for k in (0, orc.m - 1):
                assert pb.alpha_offset(b, k, i, j) == orc.alpha_off[b] + k * orc.unstable[p].shape[0] + t
    assert pb.n_alpha == orc.n_alpha and pb.n_beta == orc.nnz * orc.m


@pytest.mark.parametrize("name,nparts", [("mlp_deep", None), ("mlp_deep", 2), ("cnn_odd", 3)])
def test_deterministic_and_graph_replay(name, nparts):
    """The optimiser's first call runs its loop directly, later calls replay
    the captured graph(s) (one per concurrent sub-batch): every replay, with
    eager work and synchronisations in between, equals the first call bit for
    bit."""
    say("graph replay", name, nparts)
    wl, orc, pb = problem(name)
    if nparts is not None:
        pb.set_parts(nparts)
    alpha, beta = cases.random_vars(orc, seed=3)
    x1 = pb.eval(dev(alpha), dev(beta)).cpu().numpy()
    x2 = pb.eval(dev(alpha), dev(beta)).cpu().numpy()
    assert np.array_equal(x1, x2)
    a = pb.alpha_init()
    b = pb.zeros_beta()
    a0, b0 = a.clone(), b.clone()
    best1, _ = pb.optimize(a, b)
    r1 = (best1.cpu().numpy().copy(), a.cpu().numpy().copy())
    for _ in range(3):  # replays of the captured graph, eager work in between
        a.copy_(a0)
        b.copy_(b0)
        _ = pb.eval(a, b)
        torch.cuda.synchronize()
        best2, _ = pb.optimize(a, b)
        assert np.array_equal(best2.cpu().numpy(), r1[0]) and np.array_equal(a.cpu().numpy(), r1[1])


@pytest.mark.parametrize("name", ["mlp_deep", "cnn_base", "cnn_odd"])
def test_autotune_keeps_parity(name):
    """After the autotuner's choice of dense tilings and plans and (on a CNN)
    of the conv kernel variant per layer and direction."""
    wl, orc, pb = problem(name)
    pb.autotune()
    alpha, beta = cases.random_vars(orc, seed=4)
    lb = pb.eval(dev(alpha), dev(beta)).cpu().numpy()
    ref = np.stack([orc.eval(b, alpha, beta) for b in range(orc.B)])
    assert guarded_rel(lb, ref).max() <= TOL


def test_autograd_function_matches_grad():
    from paper_2103_06624_amd.api import BetaCrownBound
    wl, orc, pb = problem("cnn_base")
    alpha, beta = cases.random_vars(orc, seed=5)
    a = dev(alpha).requires_grad_(True)
    b = dev(beta).requires_grad_(True)
    lb = BetaCrownBound.apply(a, b, pb)
    w = torch.linspace(0.5, 1.5, lb.numel(), device="cuda").view_as(lb)
    (lb * w).sum().backward()
    _, ga, gb = pb.grad(dev(alpha), dev(beta))
    ra, rb = pb.row_maps()
    assert torch.allclose(a.grad, ga * w.reshape(-1)[ra])
    assert torch.allclose(b.grad, gb * w.reshape(-1)[rb])


@pytest.mark.parametrize("name", ["mlp_small", "cnn_odd"])
def test_init_without_bounds_runs_gpu_crown(name):
    """cv_bound_init with l = u = NULL computes the root bounds itself (per-layer
    CROWN on the GPU): the handle's bounds equal those of a handle built on
    cv_bound_root_bounds' output, bit for bit."""
    import ctypes

    from paper_2103_06624_amd import api, synth
    from paper_2103_06624_amd import binding as B
    say("init without bounds", name)
    wl = synth.make(name, **cases.SMALL[name])
    lo, up = api.root_bounds(wl.net.layers, wl.x_lo, wl.x_hi)
    sp = synth.attach_splits(wl, lo, up)
    ref = api.BoundProblem.from_workload(wl, lo, up, sp)
    arr, keep = api.make_layers(wl.net.layers)
    c = lambda x, t: np.ascontiguousarray(x, t)
    bufs = [c(wl.x_lo, np.float32), c(wl.x_hi, np.float32), c(wl.C, np.float32), c(sp.dom_prop, np.int32),
            c(sp.split_ptr, np.int64), c(sp.layer, np.int32), c(sp.neuron, np.int32), c(sp.side, np.int8)]
    p = [ctypes.c_void_p(x.ctypes.data) for x in bufs]
    h = ctypes.c_void_p()
    B.check(B.cv_bound_init(ctypes.byref(h), arr, len(arr), wl.n_props, p[0], p[1], wl.m, p[2], None, None,
                            len(sp.dom_prop), p[3], p[4], p[5], p[6], p[7], None))
    na, nb, nr = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    B.check(B.cv_bound_sizes(h, ctypes.byref(na), ctypes.byref(nb), ctypes.byref(nr)))
    assert (na.value, nb.value, nr.value) == (ref.n_alpha, ref.n_beta, ref.n_rows)
    a = torch.empty(max(na.value, 1), device="cuda")
    bb = torch.zeros(max(nb.value, 1), device="cuda")
    lb = torch.empty(nr.value, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    B.check(B.cv_bound_alpha_init(h, ctypes.c_void_p(a.data_ptr()), s))
    B.check(B.cv_bound_eval(h, ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(bb.data_ptr()),
                            ctypes.c_void_p(lb.data_ptr()), s))
    lb_ref = ref.eval(ref.alpha_init(), ref.zeros_beta()).reshape(-1)
    assert torch.equal(lb, lb_ref)
    B.cv_bound_destroy(h)
    ref.close()


def test_edge_cases_depth_and_tiny_batches():
    """Subdomains with no split, every unstable neuron split, one subdomain."""
    from oracle import batch as ob
    from paper_2103_06624_amd import synth
    from paper_2103_06624_amd.api import BoundProblem
    wl, lo, up, _, _, orc0 = cases.small_case("mlp_small")
    unst = np.nonzero((lo[0] < 0) & (up[0] > 0))[0]
    offs = orc0.offs
    rng = np.random.default_rng(7)
    doms = [[], list(unst), list(unst[:3])]
    ptr, lay, neu, side = [0], [], [], []
    for d in doms:
        for flat in d:
            i = int(np.searchsorted(offs, flat, side="right"))
            lay.append(i)
            neu.append(int(flat - offs[i - 1]))
            side.append(int(rng.choice([-1, 1])))
        ptr.append(len(lay))
    for sel in ([0, 1, 2], [1]):
        ptr_s = [0]
        l2, n2, s2 = [], [], []
        for d in sel:
            l2 += lay[ptr[d]:ptr[d + 1]]
            n2 += neu[ptr[d]:ptr[d + 1]]
            s2 += side[ptr[d]:ptr[d + 1]]
            ptr_s.append(len(l2))
        dp = np.zeros(len(sel), np.int32)
        pb = BoundProblem(wl.net.layers, wl.x_lo, wl.x_hi, wl.C, lo, up, dp, ptr_s, l2, n2, s2)
        orc = ob.OracleProblem(wl.net.layers, wl.x_lo, wl.x_hi, wl.C, lo, up, dp, ptr_s, l2, n2, s2,
                               net64=orc0.net64)
        alpha, beta = cases.random_vars(orc, seed=8, beta_hi=1.0)
        lb = pb.eval(dev(alpha), dev(beta)).cpu().numpy()
        ref = np.stack([orc.eval(b, alpha, beta) for b in range(orc.B)])
        assert guarded_rel(lb, ref).max() <= TOL


@pytest.mark.parametrize("name", ["mlp_small", "cnn_odd"])
def test_empty_batch(name):
    """No subdomains: every entry point returns at once with empty outputs."""
    from paper_2103_06624_amd.api import BoundProblem
    say("empty batch", name)
    wl, lo, up, _, _, _ = cases.small_case(name)
    pb = BoundProblem(wl.net.layers, wl.x_lo, wl.x_hi, wl.C, lo, up, np.zeros(0, np.int32), [0], [], [], [])
    assert pb.n_alpha == 0 and pb.n_beta == 0
    a, b = pb.alpha_init(), pb.zeros_beta()
    assert pb.eval(a, b).numel() == 0
    lb, ga, gb = pb.grad(a, b)
    assert lb.numel() == 0 and ga.numel() == 0 and gb.numel() == 0
    best, last = pb.optimize(a, b)
    assert best.numel() == 0
    out = pb.upper(a, b)
    assert all(t.numel() == 0 for t in out)
    torch.cuda.synchronize()


@pytest.mark.parametrize("name", ["mlp_small", "cnn_odd"])
def test_point_box_gives_the_network_value(name):
    """A zero-width box: every neuron is stable, there is no alpha, and the
    bound of each spec row is C f(x0) itself (the relaxation is exact)."""
    from oracle import batch as ob
    from oracle import beta_crown as bc
    from paper_2103_06624_amd import synth
    from paper_2103_06624_amd.api import BoundProblem
    say("point box", name)
    wl = synth.make(name, **cases.SMALL[name])
    x0 = np.asarray(wl.x0, np.float32)
    net64 = bc.dense_net(wl.net.layers)
    lo64, up64 = ob.root_bounds_all(net64, x0.astype(np.float64), x0.astype(np.float64))
    lo, up = bc.outward_f32(lo64, up64)
    P, B = x0.shape[0], 3 * x0.shape[0]
    dp = np.repeat(np.arange(P, dtype=np.int32), 3)
    pb = BoundProblem(wl.net.layers, x0, x0, wl.C, lo, up, dp, np.zeros(B + 1, np.int64), [], [], [])
    a, b = pb.alpha_init(), pb.zeros_beta()
    lb = pb.eval(a, b).cpu().numpy()
    best, _ = pb.optimize(a, b)
    best = best.cpu().numpy()
    for d in range(B):
        z = x0[dp[d]].astype(np.float64)
        for W, bias in net64[:-1]:
            z = np.maximum(W @ z + bias, 0.0)
        W, bias = net64[-1]
        ref = np.asarray(wl.C[dp[d]], np.float64) @ (W @ z + bias)
        assert guarded_rel(lb[d], ref).max() <= TOL
        assert guarded_rel(best[d], ref).max() <= TOL


def test_no_relu_layer_upper_bound_in_sound_mode():
    """A network with no ReLU layer: the bound is the exact box minimum of
    C (W x + b), attained at x*.  In sound mode only lb is lowered by the
    rounding margin; ub stays the network's value at x* (an upper bound of
    the minimum), identical to plain mode's."""
    from oracle import beta_crown as bc
    from paper_2103_06624_amd import synth
    from paper_2103_06624_amd.api import BoundProblem
    say("no ReLU layer, sound mode upper bound")
    rng = np.random.default_rng(5)
    d0, d1, P, m = 37, 6, 2, 5
    W = rng.standard_normal((d1, d0)).astype(np.float32)
    bias = rng.standard_normal(d1).astype(np.float32)
    layers = [synth.Layer(synth.DENSE, W, bias, (d0, 1, 1), (d1, 1, 1))]
    x0 = rng.uniform(0, 1, (P, d0)).astype(np.float32)
    x_lo, x_hi = x0 - 0.1, x0 + 0.1
    C = rng.standard_normal((P, m, d1)).astype(np.float32)
    empty = np.zeros((P, 0), np.float32)
    dp = np.array([0, 1, 1], np.int32)
    pb = BoundProblem(layers, x_lo, x_hi, C, empty, empty, dp, np.zeros(4, np.int64), [], [], [])
    a, b = pb.alpha_init(), pb.zeros_beta()
    lb_p, ub_p, sat_p = (t.cpu().numpy() for t in pb.upper(a, b))
    pb.set_sound(1)
    lb_s, ub_s, sat_s = (t.cpu().numpy() for t in pb.upper(a, b))
    net64 = bc.dense_net(layers)
    for d in range(3):
        p = dp[d]
        ref = bc.bound(net64, x_lo[p].astype(np.float64), x_hi[p].astype(np.float64), C[p].astype(np.float64),
                       [], [], [], [], [])
        assert (lb_s[d] <= ref).all(), (lb_s[d], ref)
        assert guarded_rel(lb_s[d], ref).max() <= SOUND_TOL
        assert guarded_rel(ub_s[d], ref).max() <= TOL
    assert np.array_equal(ub_s, ub_p) and (sat_s == 1).all() and (sat_p == 1).all()
    assert np.array_equal(lb_p, ub_p)
    pb.close()


@pytest.mark.parametrize("name", ["mlp_deep"])
def test_full_size_sampled(name):
    """The benchmark's workload at full size; sampled subdomains checked one by one."""
    say("full size", name)
    wl, orc, pb = problem(name, full=True)
    pb.autotune()
    a = pb.alpha_init()
    b = pb.zeros_beta()
    lb0 = pb.eval(a, b).cpu().numpy()
    best, last = pb.optimize(a, b)
    best = best.cpu().numpy()
    a0 = orc.default_alpha_flat()
    z = np.zeros(orc.nnz * orc.m)
    e0, e1 = [], []
    for d in sample_doms(orc, 12):
        e0.append(guarded_rel(lb0[d], orc.eval(d, a0, z)).max())
        rbest, *_ = orc.optimize(d, a0, z)
        e1.append(guarded_rel(best[d], rbest).max())
    say(name, "full-size eval err", max(e0), "opt err", max(e1))
    assert max(e0) <= TOL and max(e1) <= TOL


@pytest.mark.parametrize("name", ["cnn_base", "cnn_wide", "cnn_deep"])
def test_full_size_sampled_cnn(name):
    """The CNN workloads at full size, in the bench's launch configuration
    (concurrent sub-batches): sampled subdomains of the properties that carry
    the oracle's root bounds, checked one by one (plain evaluation at CROWN's
    alpha, and the 20-step optimisation)."""
    from paper_2103_06624_amd.api import BoundProblem
    say("full size", name)
    wl, lo, up, orc, props = cases.full_case_props(name)
    pb = BoundProblem.from_workload(wl, lo, up)
    a = pb.alpha_init()
    b = pb.zeros_beta()
    lb0 = pb.eval(a, b).cpu().numpy()
    best, _ = pb.optimize(a, b)
    best = best.cpu().numpy()
    a0 = orc.default_alpha_flat()
    z = np.zeros(orc.nnz * orc.m)
    cand = [d for d in range(orc.B) if int(orc.dom_prop[d]) in props]
    rng = np.random.default_rng(3)
    e0, e1 = [], []
    for d in sorted(rng.choice(cand, size=min(6, len(cand)), replace=False).tolist()):
        e0.append(guarded_rel(lb0[d], orc.eval(d, a0, z)).max())
        rbest, *_ = orc.optimize(d, a0, z)
        e1.append(guarded_rel(best[d], rbest).max())
    say(name, "rows", pb.n_rows, "full-size eval err", max(e0), "opt err", max(e1))
    assert max(e0) <= TOL and max(e1) <= TOL


@pytest.mark.parametrize("n_dom", [600, 1500, 2000])
def test_chain_row_blocks(n_dom):
    """Batch sizes that give the fused chain 2 and 3 row blocks per workgroup,
    the latter with more workgroups than compute units; sampled subdomains
    checked."""
    say("chain row blocks", n_dom)
    from paper_2103_06624_amd.api import BoundProblem
    wl, lo, up, _, _, orc = cases.case("mlp_deep", n_dom=n_dom)
    pb = BoundProblem.from_workload(wl, lo, up)
    pb.set_plan(1, 1)
    alpha, beta = cases.random_vars(orc, seed=9)
    lb = pb.eval(dev(alpha), dev(beta)).cpu().numpy()
    lbg, ga, gb = pb.grad(dev(alpha), dev(beta))
    lbg, ga = lbg.cpu().numpy(), ga.cpu().numpy()
    for d in sample_doms(orc, 6, seed=n_dom):
        g, ra, _ = orc.grad(d, alpha, beta)
        assert guarded_rel(lb[d], g).max() <= TOL
        assert guarded_rel(lbg[d], g).max() <= TOL
        ok = kink_free_rows(orc, d, alpha, beta)
        U = ra.shape[0] // orc.m
        a_gpu = ga[orc.alpha_off[d]:orc.alpha_off[d + 1]].reshape(orc.m, U)
        a_ref = ra.reshape(orc.m, U)
        for k in np.nonzero(ok)[0]:
            scale = max(1.0, np.abs(a_ref[k]).max(initial=0))
            assert np.abs(a_gpu[k] - a_ref[k]).max(initial=0) / scale <= TOL


def test_grad_matches_central_fd_of_oracle():
    """GPU gradient entries against central finite differences (h = 1e-3) of
    the FP64 oracle's bound, on 8 subdomains of the deep MLP.  A coordinate
    is compared where the bound is smooth across the step (the h and h/2
    differences agree), i.e. no sign decision flips inside [x - h, x + h]."""
    say("grad vs central FD")
    wl, orc, pb = problem("mlp_deep")
    alpha, beta = cases.random_vars(orc, seed=11)
    alpha = alpha.astype(np.float64)
    beta = beta.astype(np.float64)
    _, ga, gb = pb.grad(dev(alpha), dev(beta))
    ga, gb = ga.cpu().numpy().astype(np.float64), gb.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(12)
    compared = tried = 0
    worst = 0.0
    for d in sample_doms(orc, 8, seed=13):
        U = (orc.alpha_off[d + 1] - orc.alpha_off[d]) // orc.m
        coords = [("a", int(orc.alpha_off[d] + rng.integers(orc.alpha_off[d + 1] - orc.alpha_off[d])))
                  for _ in range(6)]
        nb = int(orc.ptr[d + 1] - orc.ptr[d])
        coords += [("b", int((orc.ptr[d] + rng.integers(nb)) * orc.m + rng.integers(orc.m))) for _ in range(3)]
        for kind, i in coords:
            x = alpha if kind == "a" else beta
            row = (i - orc.alpha_off[d]) // U if kind == "a" else i % orc.m

            def f(delta):
                y = x.copy()
                y[i] += delta
                return (orc.eval(d, y, beta) if kind == "a" else orc.eval(d, alpha, y))[row]

            h = 1e-3
            fd1 = (f(h) - f(-h)) / (2 * h)
            fd2 = (f(h / 2) - f(-h / 2)) / h
            tried += 1
            if abs(fd1 - fd2) > 1e-6 * max(1.0, abs(fd1)):
                continue  # a kink inside the step
            g = (ga if kind == "a" else gb)[i]
            worst = max(worst, abs(g - fd1) / max(1.0, abs(fd1)))
            compared += 1
    say("FD coordinates compared", compared, "of", tried, "worst", worst)
    assert compared >= tried // 2
    assert worst <= TOL


@pytest.mark.parametrize("nparts", [1, 2, 3])
def test_optimize_parts_and_resume(nparts):
    """The optimiser over concurrent sub-batches matches the oracle, and a run
    resumed from explicit Adam state (10 + 10 steps) equals a 20-step run."""
    say("optimize parts", nparts)
    wl, orc, pb = problem("mlp_deep")
    pb.set_parts(nparts)
    a0 = pb.alpha_init()
    b0 = pb.zeros_beta()
    a, b = a0.clone(), b0.clone()
    best, _ = pb.optimize(a, b, iters=20)
    best = best.cpu().numpy()
    a64 = orc.default_alpha_flat()
    z = np.zeros(orc.nnz * orc.m)
    errs = [guarded_rel(best[d], orc.optimize(d, a64, z)[0]).max() for d in sample_doms(orc, 8, seed=nparts)]
    say("parts", nparts, "opt max rel err", max(errs))
    assert max(errs) <= TOL
    # resume: explicit moments, 10 steps then 10 more from step 10
    st = torch.zeros(2 * pb.n_alpha + 2 * pb.n_beta, device="cuda")
    a2, b2 = a0.clone(), b0.clone()
    best1, _ = pb.optimize(a2, b2, iters=10, adam_state=st)
    best1 = best1.clone()
    best2, last2 = pb.optimize(a2, b2, iters=10, adam_state=st, step0=10)
    a3, b3 = a0.clone(), b0.clone()
    st3 = torch.zeros_like(st)
    best3, last3 = pb.optimize(a3, b3, iters=20, adam_state=st3)
    assert torch.allclose(a2, a3, rtol=0, atol=1e-6) and torch.allclose(b2, b3, rtol=0, atol=1e-6)
    assert torch.allclose(last2, last3, rtol=1e-6, atol=1e-5)
    assert torch.allclose(torch.maximum(best1, best2), best3, rtol=1e-6, atol=1e-5)


def test_parts_rejects_bad_values():
    from paper_2103_06624_amd.binding import CvError
    wl, orc, pb = problem("mlp_small")
    for bad in (0, 5, -1):
        with pytest.raises(CvError):
            pb.set_parts(bad)
    pb.set_parts(4)  # more parts than needed is fine; 16 subdomains

