"""Joint optimisation of intermediate-layer bounds, FP64.  TEST INFRASTRUCTURE ONLY.

Sec. 3.3, Eq. (opt_non_convex): the bound g of Theorem 3.1 depends on the
pre-activation bounds l(i), u(i) of every ReLU layer through the relaxation of
its unstable neurons.  Those bounds are themselves beta-CROWN bounds -- l(i)_j
is Theorem 3.1's bound of the objective z(i)_j on the sub-network of layers
1..i, u(i)_j minus that of -z(i)_j -- each with variables alpha', beta' of its
own, independent of the final objective's alpha, beta.  All of them are
optimised together, the gradient of g reaching alpha', beta' through l and u.
The paper shares alpha' and beta' among the neurons of one layer (O(L^2 d)
variables instead of O(L^2 d^2)); here that sharing is per (layer i, bound
side): every lower bound of layer i uses one alpha'_(i,lo) (one entry per
neuron of every layer below i) and one beta'_(i,lo) (one entry per split
neuron below i), the upper bounds another pair.

Readings where the paper is silent (each listed in the design notes):
  * layer 1's bounds are the root's: they are exact over the box (a linear
    function), with no variables;
  * a subdomain's bound of layer i is the larger (l) / smaller (u) of the
    root bound and the jointly computed one -- both are sound for the
    subdomain, a subset of the root's input set; the gradient reaches alpha',
    beta' through the computed bound unless it is looser than the root bound
    by more than a relative 1e-4 (`clip_lower`: at the start, with no splits,
    the two tie exactly, and either is a valid subgradient choice);
  * a split neuron's relaxation follows its split (z >= 0: identity, z < 0:
    zero) whatever its bounds say; they can contradict the split only when
    the subdomain is empty;
  * alpha' starts at CROWN's adaptive slope of the root bounds, beta' at 0;
    the optimiser is the same projected Adam as the final variables' (lr_alpha
    for alpha and alpha', lr_beta for beta and beta', decay per iteration),
    ascending sum_rows g; the reported bound is the best of the iters + 1
    evaluated iterates, row by row.

Gradients come from torch's float64 autograd over the same arithmetic; the
bound itself is Theorem 3.1's recursion written out in torch.
"""
from __future__ import annotations

import numpy as np
import torch

from . import beta_crown as bc

_F = torch.float64


def _t(x):
    return torch.as_tensor(np.asarray(x, np.float64), dtype=_F)


def bound_t(net, x_lo, x_hi, C, lo, up, split, alpha, beta):
    """Theorem 3.1's bound of C f(x) over the box, as a torch function of
    alpha, beta, lo and up (all float64 tensors).

    net: [(W(i), b(i))] tensors for layers 1..n; C [m, d_n]; lo, up, split,
    alpha [m, d_k], beta [m, d_k] per ReLU layer k = 1..n-1 (list index k-1).
    Same recursion as the NumPy oracle: A(n-1) = C W(n), c = C b(n); for
    k = n-1..1: Lambda = A D(k) + beta S(k), c += A lowerb(k) + Lambda b(k),
    A(k-1) = Lambda W(k); g = sum_j min(A(0)_j x_lo_j, A(0)_j x_hi_j) + c.
    Returns g [m]."""
    n = len(net)
    W, b = net[n - 1]
    A = C @ W
    c = C @ b
    for k in range(n - 1, 0, -1):
        W, b = net[k - 1]
        l, u, s = lo[k - 1], up[k - 1], split[k - 1]
        act = (s > 0) | ((s == 0) & (l >= 0))
        ina = (s < 0) | ((s == 0) & ~(l >= 0) & (u <= 0))
        uns = ~act & ~ina
        den = torch.where(uns, u - l, torch.ones_like(u))
        slope = torch.where(uns, u / den, torch.zeros_like(u))
        icpt = torch.where(uns, -u * l / den, torch.zeros_like(u))
        pos = A >= 0
        D = torch.where(act, torch.ones_like(A),
                        torch.where(ina, torch.zeros_like(A), torch.where(pos, alpha[k - 1], slope.expand_as(A))))
        lowb = torch.where(uns & ~pos, icpt.expand_as(A), torch.zeros_like(A))
        sgn = torch.where(s > 0, -torch.ones_like(u), torch.where(s < 0, torch.ones_like(u), torch.zeros_like(u)))
        Lam = A * D + beta[k - 1] * sgn
        c = c + (A * lowb).sum(dim=1) + Lam @ b
        A = Lam @ W
    return torch.minimum(A * x_lo, A * x_hi).sum(dim=1) + c


class JointVars:
    """alpha'_(i,side), beta'_(i,side) for layers i = 2..L-1 and side 0 (lower
    bounds) / 1 (upper bounds): ap[i][side] and bp[i][side] are lists over
    the layers k = 1..i-1 of [d_k] tensors."""

    def __init__(self, ap, bp):
        self.ap, self.bp = ap, bp

    def leaves(self):
        out = []
        for i in sorted(self.ap):
            for side in (0, 1):
                out += self.ap[i][side] + self.bp[i][side]
        return out


def init_vars(net64, lo_root, up_root):
    """alpha' at CROWN's adaptive slope of the root bounds, beta' = 0."""
    L = len(net64)
    ap, bp = {}, {}
    for i in range(2, L):
        ap[i] = [[_t(bc.default_alpha(lo_root[k], up_root[k])) for k in range(i - 1)] for _ in (0, 1)]
        bp[i] = [[torch.zeros(lo_root[k].shape[0], dtype=_F) for k in range(i - 1)] for _ in (0, 1)]
    return JointVars(ap, bp)


TIE = 1e-4  # relative width of a tie between a computed bound and the root bound


def clip_lower(new, root):
    """The larger of a computed lower bound and the root one, as used; its
    gradient follows the computed bound unless that is looser than the root
    bound by more than TIE max(1, |root|) (at a tie either bound is a valid
    choice of subgradient; this one keeps the computed bound's variables
    moving, and the margin makes the choice the same in any precision)."""
    use = new >= root - TIE * torch.clamp(root.abs(), min=1.0)
    return torch.where(use, new + (torch.maximum(new, root) - new).detach(), root)


def joint_bound(net64, x_lo, x_hi, C, lo_root, up_root, split, alpha, beta, jv):
    """(g [m], lo, up): the final bound with every intermediate bound of
    layers 2..L-1 computed from jv, as torch tensors (differentiable in
    alpha, beta and jv's leaves).  alpha, beta: per ReLU layer [m, d_k]."""
    L = len(net64)
    net = [(_t(W), _t(b)) for W, b in net64]
    xl, xu = _t(x_lo), _t(x_hi)
    sp = [torch.as_tensor(np.asarray(s, np.int64)) for s in split]
    lo = [_t(lo_root[0])]
    up = [_t(up_root[0])]
    for i in range(2, L):
        d = net64[i - 1][0].shape[0]
        rows = []
        for side in (0, 1):
            Ci = (1.0 if side == 0 else -1.0) * torch.eye(d, dtype=_F)
            a_rows = [a.expand(d, -1) for a in jv.ap[i][side]]
            b_rows = [bb.expand(d, -1) for bb in jv.bp[i][side]]
            rows.append(bound_t(net[:i], xl, xu, Ci, lo, up, sp[:i - 1], a_rows, b_rows))
        lo.append(clip_lower(rows[0], _t(lo_root[i - 1])))
        up.append(-clip_lower(rows[1], -_t(up_root[i - 1])))
    g = bound_t(net, xl, xu, _t(C), lo, up, sp, alpha, beta)
    return g, lo, up


def _adam(x, g, m, v, t, lr, cfg, lo, hi):
    """Projected Adam ascent step (Kingma & Ba), in place on tensors."""
    m.mul_(cfg.b1).add_((1 - cfg.b1) * g)
    v.mul_(cfg.b2).add_((1 - cfg.b2) * g * g)
    mh = m / (1 - cfg.b1 ** t)
    vh = v / (1 - cfg.b2 ** t)
    x.add_(lr * mh / (torch.sqrt(vh) + cfg.eps))
    x.clamp_(lo, hi)


def joint_optimize(net64, x_lo, x_hi, C, lo_root, up_root, split, alpha0, beta0, cfg=None):
    """Projected Adam on (alpha, beta, alpha', beta') ascending sum_rows g of
    Eq. (opt_non_convex).  alpha0, beta0: per ReLU layer [m, d_k] NumPy
    arrays (the final objective's start).  Iterates t = 0..iters-1 evaluate
    g with fresh intermediate bounds, take its gradient and step with
    lr * decay**t, projecting alpha, alpha' onto [0, 1] and beta, beta' onto
    [0, inf); the final iterate is evaluated once more.  Returns (best g [m]
    over the iters + 1 iterates, final alpha, final beta (NumPy lists), g of
    the final iterate, lo, up of the final iterate (NumPy lists, layers
    1..L-1))."""
    cfg = cfg or bc.AdamConfig()
    alpha = [_t(a).clone().requires_grad_(True) for a in alpha0]
    beta = [_t(b).clone().requires_grad_(True) for b in beta0]
    jv = init_vars(net64, lo_root, up_root)
    for x in jv.leaves():
        x.requires_grad_(True)
    groups = [(alpha, cfg.lr_alpha, 1.0), (beta, cfg.lr_beta, np.inf)]
    for i in sorted(jv.ap):
        for side in (0, 1):
            groups += [(jv.ap[i][side], cfg.lr_alpha, 1.0), (jv.bp[i][side], cfg.lr_beta, np.inf)]
    mom = [[(torch.zeros_like(x), torch.zeros_like(x)) for x in xs] for xs, _, _ in groups]
    best = None
    for t in range(cfg.iters):
        g, _, _ = joint_bound(net64, x_lo, x_hi, C, lo_root, up_root, split, alpha, beta, jv)
        gv = g.detach().numpy().copy()
        best = gv if best is None else np.maximum(best, gv)
        params = [x for xs, _, _ in groups for x in xs]
        grads = torch.autograd.grad(g.sum(), params, allow_unused=True)
        it = iter(grads)
        with torch.no_grad():
            for (xs, lr, hi), ms in zip(groups, mom):
                for x, (m1, m2) in zip(xs, ms):
                    gr = next(it)
                    if gr is None:
                        gr = torch.zeros_like(x)
                    _adam(x, gr, m1, m2, t + 1, lr * cfg.decay ** t, cfg, 0.0, hi)
    with torch.no_grad():
        g, lo, up = joint_bound(net64, x_lo, x_hi, C, lo_root, up_root, split, alpha, beta, jv)
    gv = g.numpy().copy()
    best = gv if best is None else np.maximum(best, gv)
    return (best, [a.detach().numpy().copy() for a in alpha], [b.detach().numpy().copy() for b in beta], gv,
            [x.numpy().copy() for x in lo], [x.numpy().copy() for x in up])
