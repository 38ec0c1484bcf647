"""Host checks of the parity-case helpers (no GPU)."""
import numpy as np

from oracle import beta_crown as bc
from paper_2103_06624_amd import synth
from tests import cases


def test_interval_bounds_enclose_sampled_preactivations():
    """The interval bounds used for the properties not compared at full size
    contain every pre-activation at points sampled in the box (corners
    included)."""
    wl = synth.make("cnn_base", n_props=1, n_dom=4)
    net64 = bc.dense_net(wl.net.layers)
    lo, up = cases.interval_bounds(net64, wl.x_lo[0], wl.x_hi[0])
    rng = np.random.default_rng(0)
    xl, xu = wl.x_lo[0].astype(np.float64), wl.x_hi[0].astype(np.float64)
    pts = [xl, xu] + [xl + (xu - xl) * rng.uniform(size=xl.shape) for _ in range(64)]
    pts += [np.where(rng.uniform(size=xl.shape) < 0.5, xl, xu) for _ in range(64)]
    for x in pts:
        h, z = x, []
        for i, (W, b) in enumerate(net64[:-1]):
            zz = W @ h + b
            z.append(zz)
            h = np.maximum(zz, 0)
        z = np.concatenate(z)
        assert np.all(z >= lo - 1e-9) and np.all(z <= up + 1e-9)
