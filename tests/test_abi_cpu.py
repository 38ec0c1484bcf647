"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, and rejects invalid inputs in its host-side validation (which runs
before any device call)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2103_06624_amd import binding as B
from paper_2103_06624_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "cvbound.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cv_[a-z_]+)\s*\(", src)))


def test_header_declares_the_abi():
    names = declared_functions()
    for n in ["cv_bound_init", "cv_bound_eval", "cv_bound_grad", "cv_bound_optimize", "cv_bound_destroy",
              "cv_last_error", "cv_bound_alpha_init", "cv_bound_root_bounds"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = B.lib()
    for n in declared_functions():
        assert hasattr(lib, n), n
        assert n in B.SIGNATURES, n


def _tiny():
    wl = synth.make("tiny2d")
    P = wl.n_props
    nd = sum(wl.net.dims[1:-1])
    lo = np.full((P, nd), -1.0, np.float32)
    up = np.full((P, nd), 1.0, np.float32)
    lo[:, 0] = 0.5  # neuron (1,0) is active at the root
    return wl, lo, up


def _init(wl, lo, up, dom_prop, ptr, layer, neuron, side, layers=None):
    from paper_2103_06624_amd.api import make_layers
    arr, keep = make_layers(layers or wl.net.layers)
    h = ctypes.c_void_p()
    a = lambda x, t: np.ascontiguousarray(x, t)
    args = [a(wl.x_lo, np.float32), a(wl.x_hi, np.float32), a(wl.C, np.float32), a(lo, np.float32),
            a(up, np.float32), a(dom_prop, np.int32), a(ptr, np.int64), a(layer, np.int32), a(neuron, np.int32),
            a(side, np.int8)]
    p = [ctypes.c_void_p(x.ctypes.data) for x in args]
    rc = B.cv_bound_init(ctypes.byref(h), arr, len(arr), wl.n_props, p[0], p[1], wl.m, p[2], p[3], p[4],
                         len(dom_prop), p[5], p[6], p[7], p[8], p[9], None)
    return rc, B.cv_last_error().decode()


@pytest.mark.parametrize("bad,code,msg", [
    (dict(layer=[0]), B.CV_ESPLIT, "layer"),
    (dict(layer=[3]), B.CV_ESPLIT, "layer"),
    (dict(neuron=[6]), B.CV_ESPLIT, "neuron"),
    (dict(neuron=[0]), B.CV_ESPLIT, "root-unstable"),
    (dict(side=[0]), B.CV_ESPLIT, "side"),
    (dict(layer=[1, 1], neuron=[2, 2], side=[1, -1], ptr=[0, 2]), B.CV_ESPLIT, "twice"),
    (dict(dom_prop=[5]), B.CV_EINVAL, "property"),
])
def test_invalid_splits_are_rejected(bad, code, msg):
    wl, lo, up = _tiny()
    kw = dict(dom_prop=[0], ptr=[0, 1], layer=[1], neuron=[2], side=[1])
    kw.update(bad)
    rc, err = _init(wl, lo, up, kw["dom_prop"], kw["ptr"], kw["layer"], kw["neuron"], kw["side"])
    assert rc == code and msg in err, (rc, err)


def test_non_finite_bounds_rejected():
    wl, lo, up = _tiny()
    lo[0, 3] = np.nan
    rc, err = _init(wl, lo, up, [0], [0, 0], [], [], [])
    assert rc == B.CV_EINVAL and "non-finite" in err


def test_shape_mismatch_rejected():
    wl, lo, up = _tiny()
    layers = list(wl.net.layers)
    bad = synth.Layer(0, np.zeros((2, 5), np.float32), np.zeros(2, np.float32), (5, 1, 1), (2, 1, 1))
    layers[-1] = bad
    rc, err = _init(wl, lo, up, [0], [0, 0], [], [], [], layers=layers)
    assert rc == B.CV_ESHAPE and "does not match" in err


def test_conv_last_layer_rejected():
    rng = np.random.default_rng(0)
    net = synth.cnn(rng, (3, 16, 16), [(8, 4, 2, 1)], [10])
    net.layers.append(synth.conv(rng, (10, 1, 1), 2, 1, 1, 0))
    wl, lo, up = _tiny()
    rc, err = _init(wl, lo, up, [0], [0, 0], [], [], [], layers=net.layers)
    assert rc in (B.CV_ESHAPE,)


@pytest.mark.parametrize("shape,msg", [
    (((40, 16, 16), [(8, 4, 2, 1)]), "at most 128"),      # 4 * 40 back-substitution columns
    (((64, 32, 32), [(64, 3, 1, 1)]), "fit in LDS"),       # a 64 x 32 x 32 row does not fit on chip
])
def test_conv_limits_rejected_before_any_device_call(shape, msg):
    """The conv implicit GEMMs' limits are checked on the host, so init fails
    cleanly (no device needed)."""
    rng = np.random.default_rng(0)
    net = synth.cnn(rng, shape[0], shape[1], [10])
    wl, lo, up = _tiny()
    rc, err = _init(wl, lo, up, [0], [0, 0], [], [], [], layers=net.layers)
    assert rc == B.CV_ESHAPE and msg in err, (rc, err)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the built library every entry point raises: the product path
    has no CPU fallback."""
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "libcvbound.so"))
    monkeypatch.setattr(B, "_lib", None)
    with pytest.raises(RuntimeError, match="is missing"):
        B.lib()
    for name in B.SIGNATURES:
        with pytest.raises(RuntimeError, match="is missing"):
            getattr(B, name)()
