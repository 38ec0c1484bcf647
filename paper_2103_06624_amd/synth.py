"""Seeded synthetic workloads shaped like the paper's verification benchmarks.

This module only draws inputs: network weights, input boxes, specification
matrices and branch-and-bound split sets.  It contains none of the bound
arithmetic of the method; both the GPU library and the FP64 oracle consume
what it produces.

Network notation follows Sec. 2.1 of the paper: layer i maps
z(i) = W(i) zhat(i-1) + b(i), zhat(i) = ReLU(z(i)) for i = 1..L-1, and the
last layer L is linear.  The specification C is a linear map of the logits
(Sec. 2.1 treats it as an extra linear layer).  Split sets Z+ / Z- of a
subdomain (Sec. 2.3) are stored in CSR form: side +1 means the constraint
z >= 0, side -1 means z < 0.

Workload recipe (stated in full so that the tests and the benchmark build the
same inputs):
  * weights He-normal N(0, 2/fan_in), biases N(0, 0.01^2); drawn in float64 and
    cast once to float32;
  * input centres x0 ~ U[0,1]^d0, box [max(x0-eps,0), min(x0+eps,1)];
  * MLP eps: the smallest eps (60-step bisection on [0,1]) for which at least
    round(0.3*d1) first-layer neurons have interval bounds straddling zero;
    CNN eps = 2/255;
  * spec rows e_y - e_j (j != y), m = 9; y = 0 for the MLPs, y = argmax f(x0)
    for the CNNs;
  * subdomains: a property, a depth, that many distinct root-unstable neurons
    drawn uniformly from all ReLU layers pooled, each with a uniform side.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

DENSE = 0
CONV = 1


@dataclasses.dataclass
class Layer:
    """One affine layer.  Dense: weight [out, in].  Conv: weight OIHW."""

    kind: int
    weight: np.ndarray
    bias: np.ndarray
    in_shape: tuple  # (C, H, W); dense layers use (in, 1, 1)
    out_shape: tuple
    kernel: int = 1
    stride: int = 1
    pad: int = 0

    @property
    def d_in(self) -> int:
        return int(np.prod(self.in_shape))

    @property
    def d_out(self) -> int:
        return int(np.prod(self.out_shape))


@dataclasses.dataclass
class Network:
    layers: List[Layer]

    @property
    def dims(self) -> List[int]:
        return [self.layers[0].d_in] + [ly.d_out for ly in self.layers]

    @property
    def n_relu(self) -> int:
        return len(self.layers) - 1


@dataclasses.dataclass
class Splits:
    """CSR split sets: subdomain b owns entries split_ptr[b]:split_ptr[b+1]."""

    dom_prop: np.ndarray  # int32 [B]
    split_ptr: np.ndarray  # int64 [B+1]
    layer: np.ndarray  # int32 [nnz], 1-based ReLU layer index
    neuron: np.ndarray  # int32 [nnz]
    side: np.ndarray  # int8 [nnz], +1: z >= 0, -1: z < 0

    @property
    def n_dom(self) -> int:
        return int(self.dom_prop.shape[0])

    @property
    def nnz(self) -> int:
        return int(self.split_ptr[-1])

    def of(self, b: int):
        s, e = int(self.split_ptr[b]), int(self.split_ptr[b + 1])
        return [(int(self.layer[t]), int(self.neuron[t]), int(self.side[t])) for t in range(s, e)]


@dataclasses.dataclass
class Workload:
    name: str
    net: Network
    x_lo: np.ndarray  # float32 [P, d0]
    x_hi: np.ndarray  # float32 [P, d0]
    x0: np.ndarray  # float32 [P, d0]
    eps: float
    C: np.ndarray  # float32 [P, m, dL]
    n_dom_per_prop: np.ndarray  # int64 [P]
    depth_range: tuple
    split_seed: int
    splits: Optional[Splits] = None

    @property
    def n_props(self) -> int:
        return int(self.x_lo.shape[0])

    @property
    def m(self) -> int:
        return int(self.C.shape[1])


# ----------------------------------------------------------------------------
# networks


def _he(rng, shape, fan_in):
    w = rng.standard_normal(shape) * math.sqrt(2.0 / fan_in)
    return w.astype(np.float32)


def _bias(rng, n):
    return (rng.standard_normal(n) * 0.01).astype(np.float32)


def dense(rng, d_in, d_out) -> Layer:
    return Layer(DENSE, _he(rng, (d_out, d_in), d_in), _bias(rng, d_out), (d_in, 1, 1), (d_out, 1, 1))


def conv(rng, in_shape, c_out, k, s, p) -> Layer:
    c, h, w = in_shape
    ho = (h + 2 * p - k) // s + 1
    wo = (w + 2 * p - k) // s + 1
    return Layer(CONV, _he(rng, (c_out, c, k, k), c * k * k), _bias(rng, c_out), (c, h, w), (c_out, ho, wo), k, s, p)


def mlp(rng, widths: Sequence[int]) -> Network:
    return Network([dense(rng, widths[i], widths[i + 1]) for i in range(len(widths) - 1)])


def cnn(rng, in_shape, convs, fcs) -> Network:
    """convs: list of (c_out, k, stride, pad); fcs: hidden widths then logits."""
    layers = []
    shape = in_shape
    for c_out, k, s, p in convs:
        ly = conv(rng, shape, c_out, k, s, p)
        layers.append(ly)
        shape = ly.out_shape
    d = int(np.prod(shape))
    for w in fcs:
        layers.append(dense(rng, d, w))
        d = w
    return Network(layers)


def forward(net: Network, x: np.ndarray) -> np.ndarray:
    """Plain float64 forward pass (Sec. 2.1), used to pick the label y."""
    h = np.asarray(x, dtype=np.float64)
    for i, ly in enumerate(net.layers):
        if ly.kind == DENSE:
            h = ly.weight.astype(np.float64) @ h.reshape(-1) + ly.bias
        else:
            c, hh, ww = ly.in_shape
            xin = np.pad(h.reshape(c, hh, ww), ((0, 0), (ly.pad, ly.pad), (ly.pad, ly.pad)))
            co, ho, wo = ly.out_shape
            out = np.empty((co, ho, wo))
            wt = ly.weight.astype(np.float64)
            for oy in range(ho):
                for ox in range(wo):
                    patch = xin[:, oy * ly.stride: oy * ly.stride + ly.kernel, ox * ly.stride: ox * ly.stride + ly.kernel]
                    out[:, oy, ox] = np.tensordot(wt, patch, axes=([1, 2, 3], [0, 1, 2]))
            h = (out + ly.bias.astype(np.float64)[:, None, None]).reshape(-1)
        if i < len(net.layers) - 1:
            h = np.maximum(h, 0.0)
    return h


# ----------------------------------------------------------------------------
# boxes and specifications


def box(x0: np.ndarray, eps: float):
    lo = np.maximum(x0.astype(np.float64) - eps, 0.0).astype(np.float32)
    hi = np.minimum(x0.astype(np.float64) + eps, 1.0).astype(np.float32)
    return lo, hi


def first_layer_unstable(net: Network, lo: np.ndarray, hi: np.ndarray) -> int:
    """Number of layer-1 neurons whose interval range over the box straddles 0.

    Used only to choose eps for the MLP workloads (plain interval arithmetic of
    one affine map).
    """
    ly = net.layers[0]
    assert ly.kind == DENSE
    w = ly.weight.astype(np.float64)
    c = (lo.astype(np.float64) + hi) / 2
    r = (hi.astype(np.float64) - lo) / 2
    mid = w @ c + ly.bias
    rad = np.abs(w) @ r
    return int(np.sum((mid - rad < 0) & (mid + rad > 0)))


def bisect_eps(net: Network, x0: np.ndarray, frac: float = 0.3, steps: int = 60) -> float:
    target = int(round(frac * net.layers[0].d_out))
    a, b = 0.0, 1.0
    for _ in range(steps):
        mid = 0.5 * (a + b)
        lo, hi = box(x0, mid)
        if first_layer_unstable(net, lo, hi) >= target:
            b = mid
        else:
            a = mid
    return b


def margin_spec(y: int, n_cls: int) -> np.ndarray:
    rows = []
    for j in range(n_cls):
        if j == y:
            continue
        r = np.zeros(n_cls, np.float32)
        r[y] = 1.0
        r[j] = -1.0
        rows.append(r)
    return np.stack(rows)


# ----------------------------------------------------------------------------
# split sets


def sample_splits(seed: int, dims: Sequence[int], lo_root, up_root, dom_prop: np.ndarray,
                  depth_range: tuple) -> Splits:
    """Draw split sets given per-property root bounds.

    lo_root / up_root: float arrays [P, sum(d_1..d_{L-1})] (ReLU layers only,
    layer-major).  A neuron is root-unstable when lo < 0 < up.  Subdomain b
    draws from its own stream (seed, b): a depth, then one key and one side
    per neuron; it splits the `depth` root-unstable neurons with the smallest
    keys.  A neuron whose stability differs between two sets of root bounds
    therefore only changes the subdomains that would have picked it.
    """
    relu_dims = list(dims[1:-1])
    nd = int(sum(relu_dims))
    offs = np.concatenate([[0], np.cumsum(relu_dims)])
    ptr = [0]
    lay, neu, side = [], [], []
    unstable = [np.nonzero((lo_root[p] < 0) & (up_root[p] > 0))[0] for p in range(lo_root.shape[0])]
    for b in range(dom_prop.shape[0]):
        rng = np.random.default_rng([seed, b])
        depth = int(rng.integers(depth_range[0], depth_range[1] + 1))
        keys = rng.random(nd)
        sides = rng.integers(0, 2, size=nd) * 2 - 1
        unst = unstable[int(dom_prop[b])]
        depth = min(depth, unst.shape[0])
        pick = np.sort(unst[np.argsort(keys[unst], kind="stable")[:depth]])
        for flat in pick:
            i = int(np.searchsorted(offs, flat, side="right"))  # 1-based layer
            lay.append(i)
            neu.append(int(flat - offs[i - 1]))
            side.append(int(sides[flat]))
        ptr.append(len(lay))
    return Splits(dom_prop.astype(np.int32), np.asarray(ptr, np.int64), np.asarray(lay, np.int32),
                  np.asarray(neu, np.int32), np.asarray(side, np.int8))


def attach_splits(wl: Workload, lo_root, up_root) -> Splits:
    """Draw the workload's subdomains (random order across properties).

    Deterministic for a workload: repeated calls give the same subdomains."""
    rng = np.random.default_rng(wl.split_seed)
    dom_prop = np.repeat(np.arange(wl.n_props, dtype=np.int32), wl.n_dom_per_prop)
    rng.shuffle(dom_prop)
    wl.splits = sample_splits(wl.split_seed, wl.net.dims, lo_root, up_root, dom_prop, wl.depth_range)
    return wl.splits


# ----------------------------------------------------------------------------
# the five workloads


def _ragged_counts(rng, n_props, lo, hi, total):
    c = np.exp(rng.uniform(math.log(lo), math.log(hi), size=n_props))
    c = np.clip(np.round(c * total / c.sum()), lo, hi).astype(np.int64)
    # fix the total by nudging the largest / smallest entries within range
    while c.sum() != total:
        if c.sum() < total:
            j = int(np.argmin(np.where(c < hi, c, np.iinfo(np.int64).max)))
            c[j] += 1
        else:
            j = int(np.argmax(np.where(c > lo, c, -1)))
            c[j] -= 1
    return c


def make(name: str, n_props: Optional[int] = None, n_dom: Optional[int] = None) -> Workload:
    """Build a named workload without its split sets (those need root bounds).

    n_props / n_dom shrink a workload for quick tests while keeping its
    network and input distribution.
    """
    specs = {
        "mlp_small": dict(seed=1),
        "mlp_deep": dict(seed=2),
        "cnn_base": dict(seed=3),
        "cnn_wide": dict(seed=4),
        "cnn_deep": dict(seed=5),
        "tiny2d": dict(seed=11),
        "cnn_odd": dict(seed=12),
    }
    if name not in specs:
        raise KeyError(name)
    ss = np.random.SeedSequence(specs[name]["seed"])
    w_ss, c_ss, s_ss = ss.spawn(3)
    wr, cr, sr = (np.random.default_rng(s) for s in (w_ss, c_ss, s_ss))
    if name == "mlp_small":
        net = mlp(wr, [784, 100, 100, 10])
        P, per, depth = 1, [16], (4, 4)
    elif name == "mlp_deep":
        net = mlp(wr, [784] + [200] * 6 + [10])
        P, per, depth = 1, [1024], (1, 8)
    elif name == "cnn_base":
        net = cnn(wr, (3, 32, 32), [(8, 4, 2, 1), (16, 4, 2, 1)], [100, 10])
        P, per, depth = 1, [2048], (1, 12)
    elif name == "cnn_wide":
        net = cnn(wr, (3, 32, 32), [(16, 4, 2, 1), (32, 4, 2, 1)], [100, 10])
        P, per, depth = 8, [512] * 8, (1, 16)
    elif name == "cnn_deep":
        net = cnn(wr, (3, 32, 32), [(8, 4, 2, 1), (8, 3, 1, 1), (8, 3, 1, 1), (8, 4, 2, 1)], [100, 10])
        P, per, depth = 64, None, (1, 16)
    elif name == "cnn_odd":  # non-square planes, odd kernels and sizes that fill no tile or word evenly
        net = cnn(wr, (3, 11, 13), [(5, 3, 2, 1), (7, 3, 1, 0)], [20, 10])
        P, per, depth = 2, [10, 9], (1, 6)
    else:  # tiny2d: 2-D input, used by the brute-force pins
        net = mlp(wr, [2, 6, 6, 2])
        P, per, depth = 1, [4], (1, 3)
    if n_props is not None:
        P = n_props
    d0 = net.dims[0]
    x0 = cr.uniform(0.0, 1.0, size=(P, d0)).astype(np.float32)
    if name.startswith("mlp"):
        eps = bisect_eps(net, x0[0])
    elif name == "tiny2d":
        eps = 0.25
    else:
        eps = 2.0 / 255.0
    lo, hi = box(x0, eps)
    n_cls = net.dims[-1]
    Cs = []
    for p in range(P):
        y = 0 if (name.startswith("mlp") or name == "tiny2d") else int(np.argmax(forward(net, x0[p])))
        Cs.append(margin_spec(y, n_cls))
    C = np.stack(Cs).astype(np.float32)
    if name == "cnn_deep":
        counts = _ragged_counts(sr, P, 16, 512, 8192 if n_props is None else P * 128)
    else:
        counts = np.asarray((per * P)[:P] if n_props is not None else per, np.int64)
    if n_dom is not None:
        counts = np.maximum(1, np.round(counts * n_dom / counts.sum())).astype(np.int64)
    split_seed = int(sr.integers(0, 2**31 - 1))
    return Workload(name, net, lo, hi, x0, float(eps), C, counts, depth, split_seed)


WORKLOADS = ("mlp_small", "mlp_deep", "cnn_base", "cnn_wide", "cnn_deep")
