"""The allocation-free gradient entry point against cv_bound_grad, through
the C ABI: two calls in a row on one GPU (the second on a smaller batch, so
that the shared static workspace holds the first call's contents), each
equal to the ordinary entry point's output; and a batch beyond the static
workspace is rejected with CV_ENOMEM."""
import sys

import numpy as np
import pytest

from tests import cases

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _grads_both(pb, alpha, beta):
    a, b = torch.from_numpy(alpha).cuda(), torch.from_numpy(beta).cuda()
    lb, ga, gb = pb.grad(a, b)
    lb2 = torch.full((pb.n_rows,), float("nan"), device="cuda")
    ga2 = torch.full((max(pb.n_alpha, 1),), float("nan"), device="cuda")[:pb.n_alpha]
    gb2 = torch.full((max(pb.n_beta, 1),), float("nan"), device="cuda")[:pb.n_beta]
    pb.grad_noalloc(a, b, lb2, ga2, gb2)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in (lb, ga, gb, lb2, ga2, gb2)]


@pytest.mark.parametrize("names", [("cnn_base", "mlp_small"), ("mlp_deep", "cnn_odd")])
def test_noalloc_grad_matches_grad_on_two_calls(names):
    from paper_2103_06624_amd.api import BoundProblem
    assert torch.cuda.is_available()
    for i, name in enumerate(names):  # the second batch is the smaller one
        wl, lo, up, _, _, orc = cases.small_case(name)
        say("noalloc grad", name, "call", i + 1, "rows", orc.B * orc.m)
        pb = BoundProblem.from_workload(wl, lo, up)
        alpha, beta = cases.random_vars(orc, seed=31 + i)
        lb, ga, gb, lb2, ga2, gb2 = _grads_both(pb, alpha, beta)
        assert np.array_equal(lb.reshape(-1), lb2.reshape(-1)), name
        assert np.array_equal(ga, ga2) and np.array_equal(gb, gb2), name
        # and the oracle's bound at the same variables (the parity bar)
        ref = np.stack([orc.eval(b, alpha, beta) for b in range(orc.B)])
        assert cases.guarded_rel(lb2.reshape(orc.B, orc.m), ref).max() <= 1e-4
        pb.close()


def test_noalloc_grad_sound_and_l2_modes():
    """Sound mode and l2-ball input sets carve their extra partials too."""
    from paper_2103_06624_amd.api import BoundProblem
    wl, lo, up, x0, eps, orc = cases.small_l2_case("cnn_odd")
    pb = BoundProblem.from_workload(wl, lo, up)
    pb.set_input_l2(x0, eps)
    pb.set_sound(1)
    alpha, beta = cases.random_vars(orc, seed=41)
    lb, ga, gb, lb2, ga2, gb2 = _grads_both(pb, alpha, beta)
    assert np.array_equal(lb.reshape(-1), lb2.reshape(-1))
    assert np.array_equal(ga, ga2) and np.array_equal(gb, gb2)
    pb.close()


def test_noalloc_grad_rejects_a_batch_beyond_the_workspace():
    from paper_2103_06624_amd.api import BoundProblem
    from paper_2103_06624_amd.binding import CV_ENOMEM, CvError
    from paper_2103_06624_amd import api, synth
    wl = synth.make("mlp_deep")  # 9216 rows: dense x* alone is 29 MB, past the 32 MiB array with the rest
    lo, up = api.root_bounds(wl.net.layers, wl.x_lo, wl.x_hi)
    synth.attach_splits(wl, lo, up)
    pb = BoundProblem.from_workload(wl, lo, up)
    a, b = pb.alpha_init(), pb.zeros_beta()
    lb = torch.empty(pb.n_rows, device="cuda")
    ga = torch.empty(pb.n_alpha, device="cuda")
    gb = torch.empty(pb.n_beta, device="cuda")
    with pytest.raises(CvError) as ei:
        pb.grad_noalloc(a, b, lb, ga, gb)
    assert ei.value.code == CV_ENOMEM and "workspace" in str(ei.value)
    pb.close()
