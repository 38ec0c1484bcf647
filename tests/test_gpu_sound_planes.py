"""Sound mode on convolution planes of 128, 64 and 32 positions.

The float64 conv pass blocks a thread's outputs over channels 256 / (h w)
apart when the plane size h w divides 256 (channel strides 2, 4 and 8 here;
the bench networks' 16x16 planes reach only stride 1), with input channel
counts that leave the blocked weight layout padded.  Same bar as the other
sound-mode parity tests: every bound at or below the FP64 oracle's bound at
the same variables, no tolerance, and within SOUND_TOL of it; likewise the
optimiser's final iterate.
"""
import sys

import numpy as np
import pytest

from oracle import batch as ob
from oracle import beta_crown as bc
from paper_2103_06624_amd import synth
from tests.cases import guarded_rel, random_vars

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

SOUND_TOL = 1e-6  # the float64 evaluation's margin plus one float ulp, relative to max(|bound|, 1)

# (input shape, convs (c_out, k, s, p), dense widths)
NETS = {
    # planes 16x8 (128 positions: stride 2, into the input and the first
    # hidden layer) and 8x4 (32 positions: stride 8, into the second)
    "planes_128_32": ((2, 16, 8), [(4, 3, 1, 1), (5, 4, 2, 1), (6, 3, 1, 1)], [12, 10]),
    # 8x8 planes (64 positions: stride 4, into the input and a hidden layer)
    "planes_64": ((3, 8, 8), [(4, 3, 1, 1), (4, 3, 1, 1)], [10, 10]),
}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def problem(name, seed=31):
    from paper_2103_06624_amd.api import BoundProblem
    in_shape, convs, fcs = NETS[name]
    w_ss, c_ss, s_ss = np.random.SeedSequence(seed).spawn(3)
    wr, cr, sr = (np.random.default_rng(s) for s in (w_ss, c_ss, s_ss))
    net = synth.cnn(wr, in_shape, convs, fcs)
    P = 2
    x0 = cr.uniform(0.0, 1.0, size=(P, net.dims[0])).astype(np.float32)
    eps = 2.0 / 255.0
    lo_x, hi_x = synth.box(x0, eps)
    C = np.stack([synth.margin_spec(int(np.argmax(synth.forward(net, x0[p]))), net.dims[-1])
                  for p in range(P)]).astype(np.float32)
    wl = synth.Workload(name, net, lo_x, hi_x, x0, float(eps), C, np.array([9, 7], np.int64), (1, 6),
                        int(sr.integers(0, 2**31 - 1)))
    net64 = bc.dense_net(wl.net.layers)
    lo64, up64 = ob.root_bounds_all(net64, wl.x_lo, wl.x_hi)
    lo, up = bc.outward_f32(lo64, up64)
    sp = synth.attach_splits(wl, lo, up)
    orc = ob.OracleProblem(wl.net.layers, wl.x_lo, wl.x_hi, wl.C, lo, up, sp.dom_prop, sp.split_ptr, sp.layer,
                           sp.neuron, sp.side, net64=net64)
    return orc, BoundProblem.from_workload(wl, lo, up)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda()


@pytest.mark.parametrize("name", sorted(NETS))
def test_sound_mode_on_blocked_planes(name):
    say("sound mode, blocked planes", name)
    orc, pb = problem(name)
    alpha, beta = random_vars(orc, seed=13)
    pb.set_sound(1)
    lb = pb.eval(dev(alpha), dev(beta)).cpu().numpy()
    ref = np.stack([orc.eval(b, alpha, beta) for b in range(orc.B)])
    gap = guarded_rel(lb, ref)
    say(name, "rows", lb.size, "sound excess", float(np.maximum(lb - ref, 0).max()), "gap max", float(gap.max()))
    assert (lb <= ref).all()
    assert gap.max() <= SOUND_TOL
    a, b = pb.alpha_init(), pb.zeros_beta()
    best, last = pb.optimize(a, b, iters=5)
    a_h, b_h = a.cpu().numpy(), b.cpu().numpy()
    ref_last = np.stack([orc.eval(d, a_h, b_h) for d in range(orc.B)])
    last = last.cpu().numpy()
    assert (last <= ref_last).all()
    assert guarded_rel(last, ref_last).max() <= SOUND_TOL
    assert (best.cpu().numpy() >= last).all()
    pb.close()
