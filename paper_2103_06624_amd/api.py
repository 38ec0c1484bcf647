"""Torch-facing wrapper of libcvbound (device memory and streams only).

`BoundProblem` owns a library handle; its methods pass torch tensors' device
pointers and the current HIP stream to the C ABI.  `BetaCrownBound` is a
torch.autograd.Function whose forward is cv_bound_eval and whose backward is
cv_bound_grad scaled by the incoming per-row gradient.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import binding as B


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _dptr(t):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous() and t.dtype == torch.float32, "expected contiguous float32 device tensor"
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def make_layers(layers):
    """cv_layer array (+ host arrays kept alive) from synth.Layer-like objects."""
    keep = []
    arr = (B.cv_layer * len(layers))()
    for i, ly in enumerate(layers):
        w = np.ascontiguousarray(ly.weight, dtype=np.float32)
        b = np.ascontiguousarray(ly.bias, dtype=np.float32)
        keep += [w, b]
        ci, hi, wi = ly.in_shape
        co, ho, wo = ly.out_shape
        arr[i] = B.cv_layer(B.CV_LAYER_DENSE if ly.kind == 0 else B.CV_LAYER_CONV2D, ci, hi, wi, co, ho, wo,
                            ly.kernel, ly.stride, ly.pad, w.ctypes.data, b.ctypes.data)
    return arr, keep


def root_bounds(layers, x_lo, x_hi, sound=False, opt_iters=0, lr_alpha=0.1, decay=0.98):
    """Per-layer CROWN intermediate bounds on the GPU: (l, u) float32 [P, sum d_i];
    sound: evaluated in float64 with a rigorous rounding margin and rounded
    outward (sound mode); opt_iters > 0:
    each bound maximised over its own alpha' by that many Adam steps."""
    arr, keep = make_layers(layers)
    x_lo = np.ascontiguousarray(x_lo, np.float32)
    x_hi = np.ascontiguousarray(x_hi, np.float32)
    P = x_lo.shape[0]
    nd = sum(ly.d_out for ly in layers[:-1])
    lo = np.zeros((P, nd), np.float32)
    up = np.zeros((P, nd), np.float32)
    if opt_iters > 0:
        B.check(B.cv_bound_root_bounds_opt(arr, len(layers), P, _ptr(x_lo), _ptr(x_hi), opt_iters, lr_alpha, decay,
                                           int(sound), _ptr(lo), _ptr(up), _stream()))
    else:
        fn = B.cv_bound_root_bounds_sound if sound else B.cv_bound_root_bounds
        B.check(fn(arr, len(layers), P, _ptr(x_lo), _ptr(x_hi), _ptr(lo), _ptr(up), _stream()))
    return lo, up


class BoundProblem:
    def __init__(self, layers, x_lo, x_hi, C, lo, up, dom_prop, split_ptr, split_layer, split_neuron, split_side):
        arr, keep = make_layers(layers)
        self._keep = keep
        x_lo = np.ascontiguousarray(x_lo, np.float32)
        x_hi = np.ascontiguousarray(x_hi, np.float32)
        C = np.ascontiguousarray(C, np.float32)
        lo = np.ascontiguousarray(lo, np.float32)
        up = np.ascontiguousarray(up, np.float32)
        dom_prop = np.ascontiguousarray(dom_prop, np.int32)
        split_ptr = np.ascontiguousarray(split_ptr, np.int64)
        split_layer = np.ascontiguousarray(split_layer, np.int32)
        split_neuron = np.ascontiguousarray(split_neuron, np.int32)
        split_side = np.ascontiguousarray(split_side, np.int8)
        self.P, self.m = C.shape[0], C.shape[1]
        self.nd = sum(ly.d_out for ly in layers[:-1])
        self.B = dom_prop.shape[0]
        self._ucount = ((lo < 0) & (up > 0)).sum(axis=1).astype(np.int64)
        self._dom_prop = dom_prop
        self._split_ptr = split_ptr
        self._maps = None
        h = ctypes.c_void_p()
        B.check(B.cv_bound_init(ctypes.byref(h), arr, len(layers), self.P, _ptr(x_lo), _ptr(x_hi), self.m, _ptr(C),
                                _ptr(lo), _ptr(up), self.B, _ptr(dom_prop), _ptr(split_ptr), _ptr(split_layer),
                                _ptr(split_neuron), _ptr(split_side), _stream()))
        self.h = h
        na, nb, nr = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        B.check(B.cv_bound_sizes(h, ctypes.byref(na), ctypes.byref(nb), ctypes.byref(nr)))
        self.n_alpha, self.n_beta, self.n_rows = na.value, nb.value, nr.value

    def update(self, dom_prop, split_ptr, split_layer, split_neuron, split_side):
        """A new batch of subdomains on this handle (cv_bound_update): same
        network, properties, specifications and root bounds; the alpha / beta
        layouts and sizes follow the new batch."""
        dom_prop = np.ascontiguousarray(dom_prop, np.int32)
        split_ptr = np.ascontiguousarray(split_ptr, np.int64)
        split_layer = np.ascontiguousarray(split_layer, np.int32)
        split_neuron = np.ascontiguousarray(split_neuron, np.int32)
        split_side = np.ascontiguousarray(split_side, np.int8)
        B.check(B.cv_bound_update(self.h, dom_prop.shape[0], _ptr(dom_prop), _ptr(split_ptr), _ptr(split_layer),
                                  _ptr(split_neuron), _ptr(split_side), _stream()))
        self.B = dom_prop.shape[0]
        self._dom_prop = dom_prop
        self._split_ptr = split_ptr
        self._maps = None
        na, nb, nr = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        B.check(B.cv_bound_sizes(self.h, ctypes.byref(na), ctypes.byref(nb), ctypes.byref(nr)))
        self.n_alpha, self.n_beta, self.n_rows = na.value, nb.value, nr.value

    @classmethod
    def from_workload(cls, wl, lo, up, splits=None):
        sp = splits if splits is not None else wl.splits
        return cls(wl.net.layers, wl.x_lo, wl.x_hi, wl.C, lo, up, sp.dom_prop, sp.split_ptr, sp.layer, sp.neuron,
                   sp.side)

    def close(self):
        if getattr(self, "h", None):
            B.cv_bound_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _f(self, n):
        return torch.empty(max(n, 1), dtype=torch.float32, device="cuda")[:n]

    def alpha_offset(self, dom, row, layer, neuron):
        return B.cv_bound_alpha_offset(self.h, dom, row, layer, neuron)

    def alpha_init(self):
        a = self._f(self.n_alpha)
        B.check(B.cv_bound_alpha_init(self.h, _dptr(a), _stream()))
        return a

    def zeros_beta(self):
        return torch.zeros(self.n_beta, dtype=torch.float32, device="cuda")

    def eval(self, alpha, beta, out=None):
        lb = out if out is not None else self._f(self.n_rows)
        B.check(B.cv_bound_eval(self.h, _dptr(alpha), _dptr(beta), _dptr(lb), _stream()))
        return lb.view(self.B, self.m)

    def grad(self, alpha, beta):
        lb = self._f(self.n_rows)
        ga = self._f(self.n_alpha)
        gb = self._f(self.n_beta)
        B.check(B.cv_bound_grad(self.h, _dptr(alpha), _dptr(beta), _dptr(lb), _dptr(ga), _dptr(gb), _stream()))
        return lb.view(self.B, self.m), ga, gb

    def grad_noalloc(self, alpha, beta, lb, g_alpha, g_beta):
        """cv_bound_grad into caller-provided outputs, with the library's
        static workspace instead of the handle's (no device allocation)."""
        B.check(B.cv_bound_grad_noalloc(self.h, _dptr(alpha), _dptr(beta), _dptr(lb), _dptr(g_alpha), _dptr(g_beta),
                                        _stream()))
        return lb.view(self.B, self.m), g_alpha, g_beta

    def upper(self, alpha, beta, with_lb=True):
        """(lb, ub, sat) [B, m]: the bound, the network at each row's box
        minimiser x*, and whether x* meets the subdomain's splits."""
        lb = self._f(self.n_rows) if with_lb else None
        ub = self._f(self.n_rows)
        sat = torch.empty(self.n_rows, dtype=torch.int32, device="cuda")
        B.check(B.cv_bound_upper(self.h, _dptr(alpha), _dptr(beta), _dptr(lb), _dptr(ub), ctypes.c_void_p(sat.data_ptr()),
                                 _stream()))
        return (lb.view(self.B, self.m) if with_lb else None), ub.view(self.B, self.m), sat.view(self.B, self.m)

    def optimize(self, alpha, beta, iters=20, lr_alpha=0.01, lr_beta=0.05, decay=0.98, adam_state=None, step0=0,
                 lb_best=None, lb_last=None):
        """In-place projected Adam on alpha, beta; returns (best, last) bounds [B, m]."""
        best = lb_best if lb_best is not None else self._f(self.n_rows)
        last = lb_last if lb_last is not None else self._f(self.n_rows)
        B.check(B.cv_bound_optimize(self.h, iters, lr_alpha, lr_beta, decay, _dptr(alpha), _dptr(beta),
                                    _dptr(adam_state), step0, _dptr(best), _dptr(last), _stream()))
        return best.view(self.B, self.m), last.view(self.B, self.m)

    def optimize_joint(self, alpha, beta, iters=20, lr_alpha=0.01, lr_beta=0.05, decay=0.98, bounds=False):
        """In-place projected Adam on alpha, beta jointly with every subdomain's
        intermediate bounds (cv_bound_optimize_joint); returns (best, last)
        bounds [B, m], and with bounds=True also the final iterate's
        intermediate bounds (l, u) [B, sum d_i]."""
        best = self._f(self.n_rows)
        last = self._f(self.n_rows)
        lo = self._f(self.B * self.nd) if bounds else None
        up = self._f(self.B * self.nd) if bounds else None
        B.check(B.cv_bound_optimize_joint(self.h, iters, lr_alpha, lr_beta, decay, _dptr(alpha), _dptr(beta),
                                          _dptr(best), _dptr(last), _dptr(lo), _dptr(up), _stream()))
        out = (best.view(self.B, self.m), last.view(self.B, self.m))
        if bounds:
            out += (lo.view(self.B, self.nd), up.view(self.B, self.nd))
        return out

    def joint_vars(self, layer):
        """(alpha', beta', their gradients) of intermediate layer `layer` after
        the last optimize_joint (cv_bound_joint_vars layouts), device tensors."""
        na, nb = ctypes.c_int64(), ctypes.c_int64()
        B.check(B.cv_bound_joint_sizes(self.h, layer, ctypes.byref(na), ctypes.byref(nb)))
        out = [self._f(na.value), self._f(nb.value), self._f(na.value), self._f(nb.value)]
        B.check(B.cv_bound_joint_vars(self.h, layer, *[_dptr(t) for t in out], _stream()))
        return tuple(out)

    def row_maps(self):
        """(row of each alpha entry, row of each beta entry) as device index tensors."""
        if self._maps is None:
            rows = np.arange(self.B * self.m)
            ra = np.repeat(rows, np.repeat(self._ucount[self._dom_prop], self.m))
            dom = np.repeat(np.arange(self.B), np.diff(self._split_ptr))
            rb = (dom[:, None] * self.m + np.arange(self.m)[None, :]).reshape(-1)
            self._maps = (torch.from_numpy(ra).cuda(), torch.from_numpy(rb).cuda())
        return self._maps

    def autotune(self):
        B.check(B.cv_bound_autotune(self.h, _stream()))

    @staticmethod
    def num_tilings():
        return int(B.cv_bound_num_tilings())

    def set_tiling(self, tiling):
        """Force one GEMM tiling on every dense layer (-1: the tuned choice)."""
        B.check(B.cv_bound_set_tiling(self.h, tiling))

    @staticmethod
    def num_conv_variants():
        return int(B.cv_bound_num_conv_variants())

    def set_conv_variant(self, variant):
        """Force one conv kernel variant on every conv layer (-1: the tuned choice)."""
        B.check(B.cv_bound_set_conv_variant(self.h, variant))

    def conv_variant(self, layer, direction):
        """Variant conv layer `layer` (1..L) runs: direction 0 back-substitution, 1 adjoint."""
        return int(B.cv_bound_conv_variant(self.h, layer, direction))

    def set_sound(self, on):
        """Lower every reported bound by a rigorous float32 rounding-error margin."""
        B.check(B.cv_bound_set_sound(self.h, int(on), _stream()))

    def set_input_l2(self, x0, eps):
        """Input sets {x : ||x - x0_p||_2 <= eps_p} per property (x0 [P, d0], eps [P],
        host arrays) in place of the boxes; x0=None returns to the boxes."""
        if x0 is None:
            B.check(B.cv_bound_set_input_l2(self.h, None, None, _stream()))
            return
        x0 = np.ascontiguousarray(x0, dtype=np.float32)
        eps = np.ascontiguousarray(np.broadcast_to(np.asarray(eps, np.float32), (x0.shape[0],)))
        B.check(B.cv_bound_set_input_l2(self.h, _ptr(x0), _ptr(eps), _stream()))

    def set_input_lp(self, x0, eps, p):
        """Input sets {x : ||x - x0_k||_p <= eps_k} per property, p in [4/3, inf)
        (x0 [P, d0], eps [P], host arrays); x0=None returns to the boxes."""
        if x0 is None:
            B.check(B.cv_bound_set_input_lp(self.h, None, None, 2.0, _stream()))
            return
        x0 = np.ascontiguousarray(x0, dtype=np.float32)
        eps = np.ascontiguousarray(np.broadcast_to(np.asarray(eps, np.float32), (x0.shape[0],)))
        B.check(B.cv_bound_set_input_lp(self.h, _ptr(x0), _ptr(eps), float(p), _stream()))

    def set_parts(self, nparts):
        """Concurrent sub-batches (streams) of optimize(); 1 disables the split."""
        B.check(B.cv_bound_set_parts(self.h, nparts))

    def set_plan(self, chain_bwd, chain_fwd):
        """Fused dense chain (1) or one kernel per layer (0), per direction."""
        B.check(B.cv_bound_set_plan(self.h, chain_bwd, chain_fwd))

    def profile(self, alpha, beta, reps=5):
        out = (B.cv_kernel_stat * 64)()
        n = ctypes.c_int32()
        B.check(B.cv_bound_profile(self.h, _dptr(alpha), _dptr(beta), reps, out, 64, ctypes.byref(n), _stream()))
        res = []
        for i in range(min(n.value, 64)):
            s = out[i]
            res.append(dict(name=s.name.decode(), launches=s.launches, total_ms=s.total_ms, reps=reps, flops=s.flops,
                            bytes=s.bytes))
        return res


class BetaCrownBound(torch.autograd.Function):
    """lb = g(alpha, beta) per row [B, m].  forward is cv_bound_eval (the bound
    alone); backward is cv_bound_grad at the saved variables, scaled by the
    incoming per-row gradient (each variable belongs to exactly one row), so a
    forward with no backward pays for the bound only."""

    @staticmethod
    def forward(ctx, alpha, beta, problem):
        a, b = alpha.detach().contiguous(), beta.detach().contiguous()
        lb = problem.eval(a, b)
        ctx.problem = problem
        ctx.save_for_backward(a, b)
        return lb.clone()

    @staticmethod
    def backward(ctx, grad_lb):
        a, b = ctx.saved_tensors
        pb = ctx.problem
        _, ga, gb = pb.grad(a, b)
        g = grad_lb.reshape(-1).contiguous()
        ra, rb = pb.row_maps()
        return ga * g[ra], gb * g[rb], None
