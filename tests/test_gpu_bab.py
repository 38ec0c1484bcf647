"""The library's branch and bound (paper_2103_06624_amd.bab) against the
oracle's (oracle.bab) and the exact minimum of tiny networks (activation
patterns enumerated), through the C ABI.  Sound mode on, so every lower
bound the GPU driver reports is rigorous."""
import numpy as np
import pytest

from tests.test_bab_oracle import exact_min, shifted, tiny_net

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def as_layers(net):
    from paper_2103_06624_amd import synth
    return [synth.Layer(synth.DENSE, np.asarray(W, np.float32), np.asarray(b, np.float32), (W.shape[1], 1, 1),
                        (W.shape[0], 1, 1)) for W, b in net]


@pytest.mark.parametrize("warm", [False, True])
@pytest.mark.parametrize("seed", range(6))
def test_bab_matches_oracle_and_exact_minimum(seed, warm):
    from oracle import bab as ob
    from oracle import beta_crown as bc
    from paper_2103_06624_amd import bab as gb
    net, x_lo, x_hi, lo, up = tiny_net(seed + 500)
    C = np.ones((1, 1))
    fstar, n_uns = exact_min(net, C, x_lo, x_hi, lo, up)
    if n_uns > 9 or n_uns < 2:
        pytest.skip("enumeration size")
    # both drivers on the same float32 data: network, box and root bounds
    net32 = [(W.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)) for W, b in net]
    lo32, up32 = bc.outward_f32(np.concatenate(lo), np.concatenate(up))
    dims = [l.shape[0] for l in lo]
    lo_l = np.split(lo32.astype(np.float64), np.cumsum(dims)[:-1])
    up_l = np.split(up32.astype(np.float64), np.cumsum(dims)[:-1])
    fstar, _ = exact_min(net32, C, x_lo.astype(np.float32).astype(np.float64),
                         x_hi.astype(np.float32).astype(np.float64), lo_l, up_l)
    cfg = bc.AdamConfig(iters=60, lr_alpha=0.1, lr_beta=0.2)
    for t in (fstar - 0.05 * max(1.0, abs(fstar)), fstar + 0.05 * max(1.0, abs(fstar))):
        n_t = shifted(net32, t)
        n_t = [(W, b.astype(np.float32).astype(np.float64)) for W, b in n_t]
        target = fstar - t
        ro = ob.bab(n_t, x_lo.astype(np.float32).astype(np.float64), x_hi.astype(np.float32).astype(np.float64), C,
                    lo_l, up_l, batch=4, max_rounds=400, cfg=cfg, warm=warm)
        rg = gb.bab(as_layers(n_t), x_lo, x_hi, C, lo32, up32, batch=4, max_rounds=400, iters=60, lr_alpha=0.1,
                    lr_beta=0.2, sound=True, warm=warm)
        print(seed, warm, round(float(target), 4), "oracle", ro["verdict"], ro["rounds"], ro["domains"], "gpu",
              rg["verdict"], rg["rounds"], rg["domains"], flush=True)
        assert rg["lb"] <= target and rg["ub"] >= target - 1e-5 * max(1.0, abs(target)), (rg, target)
        assert rg["verdict"] == ro["verdict"], (rg, ro)
        if target > 0:
            assert rg["verdict"] == "verified"
        else:
            assert rg["verdict"] in ("falsified", "unknown")


def test_bab_delta_exit_matches_oracle():
    """Alg. 1's f-bar - f-underbar <= delta exit: both drivers stop at the same
    round on the same tiny problem (half the root's gap)."""
    from oracle import bab as ob
    from oracle import beta_crown as bc
    from paper_2103_06624_amd import bab as gb
    for seed in range(500, 520):
        net, x_lo, x_hi, lo, up = tiny_net(seed)
        C = np.ones((1, 1))
        fstar, n_uns = exact_min(net, C, x_lo, x_hi, lo, up)
        if 3 <= n_uns <= 9:
            break
    net32 = [(W.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)) for W, b in net]
    lo32, up32 = bc.outward_f32(np.concatenate(lo), np.concatenate(up))
    dims = [l.shape[0] for l in lo]
    lo_l = np.split(lo32.astype(np.float64), np.cumsum(dims)[:-1])
    up_l = np.split(up32.astype(np.float64), np.cumsum(dims)[:-1])
    x_lo64, x_hi64 = x_lo.astype(np.float32).astype(np.float64), x_hi.astype(np.float32).astype(np.float64)
    fstar, _ = exact_min(net32, C, x_lo64, x_hi64, lo_l, up_l)
    cfg = bc.AdamConfig(iters=60, lr_alpha=0.1, lr_beta=0.2)
    n_t = shifted(net32, fstar - 0.05 * max(1.0, abs(fstar)))
    n_t = [(W, b.astype(np.float32).astype(np.float64)) for W, b in n_t]
    root = ob.bab(n_t, x_lo64, x_hi64, C, lo_l, up_l, batch=1, max_rounds=0, cfg=cfg)
    delta = 0.5 * (root["ub"] - root["lb"])
    ro = ob.bab(n_t, x_lo64, x_hi64, C, lo_l, up_l, batch=1, max_rounds=400, cfg=cfg, delta=delta)
    rg = gb.bab(as_layers(n_t), x_lo, x_hi, C, lo32, up32, batch=1, max_rounds=400, iters=60, lr_alpha=0.1,
                lr_beta=0.2, sound=True, delta=delta)
    print("delta", delta, "oracle", ro, "gpu", rg["verdict"], rg["rounds"], rg["domains"], flush=True)
    assert (rg["verdict"], rg["rounds"], rg["domains"]) == (ro["verdict"], ro["rounds"], ro["domains"])
