"""Batch driver of the FP64 oracle.  TEST INFRASTRUCTURE ONLY.

Subdomains and specification rows are independent (Sec. 3.4 batches them only
for throughput), so the batch result is the concatenation of per-subdomain
results of `beta_crown`.  This module also converts between the library's
documented variable layouts and the oracle's per-layer dense arrays:

  * alpha: per subdomain b, an [m, U_p] block where U_p counts the root-unstable
    neurons (l < 0 < u) of b's property p in layer-major, index order; blocks are
    concatenated in subdomain order;
  * beta: [nnz, m] in CSR split order;
  * bounds: [B, m].
"""
from __future__ import annotations

import numpy as np

from . import beta_crown as bc
from . import joint as jt


def root_bounds_all(net64, x_lo, x_hi):
    """Per-property root bounds, float64 [P, sum d_i] each (layer-major)."""
    los, ups = [], []
    for p in range(x_lo.shape[0]):
        lo, up = bc.root_bounds(net64, np.asarray(x_lo[p], np.float64), np.asarray(x_hi[p], np.float64))
        los.append(np.concatenate(lo))
        ups.append(np.concatenate(up))
    return np.stack(los), np.stack(ups)


class OracleProblem:
    """The batched problem as the library sees it, evaluated in float64."""

    def __init__(self, layers, x_lo, x_hi, C, lo, up, dom_prop, split_ptr, split_layer, split_neuron, split_side,
                 net64=None):
        self.net64 = net64 if net64 is not None else bc.dense_net(layers)
        self.dims = [self.net64[0][0].shape[1]] + [W.shape[0] for W, _ in self.net64]
        self.relu_dims = self.dims[1:-1]
        self.offs = np.concatenate([[0], np.cumsum(self.relu_dims)]).astype(np.int64)
        self.x_lo = np.asarray(x_lo, np.float64)
        self.x_hi = np.asarray(x_hi, np.float64)
        self.C = np.asarray(C, np.float64)
        self.lo = np.asarray(lo, np.float64)
        self.up = np.asarray(up, np.float64)
        self.dom_prop = np.asarray(dom_prop)
        self.ptr = np.asarray(split_ptr, np.int64)
        self.s_layer = np.asarray(split_layer)
        self.s_neuron = np.asarray(split_neuron)
        self.s_side = np.asarray(split_side)
        self.m = self.C.shape[1]
        self.B = self.dom_prop.shape[0]
        # compact alpha layout
        self.unstable = [np.nonzero((self.lo[p] < 0) & (self.up[p] > 0))[0] for p in range(self.lo.shape[0])]
        sizes = np.array([self.m * self.unstable[int(p)].shape[0] for p in self.dom_prop], np.int64)
        self.alpha_off = np.concatenate([[0], np.cumsum(sizes)])
        self.l2 = None  # (x0 [P, d0], eps [P], p) when the input set is an l_p ball per property

    def set_l2(self, x0, eps, p=2.0):
        """Input set of property k: the l_p ball (default l2) of radius eps[k]
        around x0[k] (x0 None: back to the box)."""
        self.l2 = None if x0 is None else (np.asarray(x0, np.float64), np.asarray(eps, np.float64), float(p))

    def _ball(self, p):
        return None if self.l2 is None else (self.l2[0][p], float(self.l2[1][p]), self.l2[2])

    @property
    def n_alpha(self):
        return int(self.alpha_off[-1])

    @property
    def nnz(self):
        return int(self.ptr[-1])

    def _layers(self, vec):
        return [vec[self.offs[i]:self.offs[i + 1]] for i in range(len(self.relu_dims))]

    def domain(self, b):
        p = int(self.dom_prop[b])
        split = [np.zeros(d, np.int8) for d in self.relu_dims]
        for t in range(self.ptr[b], self.ptr[b + 1]):
            split[int(self.s_layer[t]) - 1][int(self.s_neuron[t])] = int(self.s_side[t])
        return p, self._layers(self.lo[p]), self._layers(self.up[p]), split

    # ---- layout conversion -------------------------------------------------
    def alpha_to_layers(self, b, alpha_flat):
        p = int(self.dom_prop[b])
        u = self.unstable[p]
        blk = np.asarray(alpha_flat[self.alpha_off[b]:self.alpha_off[b + 1]], np.float64).reshape(self.m, u.shape[0])
        dense = np.zeros((self.m, self.offs[-1]))
        dense[:, u] = blk
        return [dense[:, self.offs[i]:self.offs[i + 1]] for i in range(len(self.relu_dims))]

    def alpha_from_layers(self, b, alpha_layers):
        p = int(self.dom_prop[b])
        dense = np.concatenate(alpha_layers, axis=1)
        return dense[:, self.unstable[p]].reshape(-1)

    def beta_to_layers(self, b, beta_flat):
        beta = [np.zeros((self.m, d)) for d in self.relu_dims]
        bf = np.asarray(beta_flat, np.float64).reshape(-1, self.m)
        for t in range(self.ptr[b], self.ptr[b + 1]):
            beta[int(self.s_layer[t]) - 1][:, int(self.s_neuron[t])] = bf[t]
        return beta

    def beta_from_layers(self, b, beta_layers):
        out = np.zeros((int(self.ptr[b + 1] - self.ptr[b]), self.m))
        for k, t in enumerate(range(self.ptr[b], self.ptr[b + 1])):
            out[k] = beta_layers[int(self.s_layer[t]) - 1][:, int(self.s_neuron[t])]
        return out

    # ---- evaluation --------------------------------------------------------
    def default_alpha_flat(self):
        out = np.zeros(self.n_alpha)
        for b in range(self.B):
            p = int(self.dom_prop[b])
            u = self.unstable[p]
            a = bc.default_alpha(self.lo[p][u], self.up[p][u])
            out[self.alpha_off[b]:self.alpha_off[b + 1]] = np.tile(a, self.m)
        return out

    def eval(self, b, alpha_flat, beta_flat):
        p, lo, up, split = self.domain(b)
        return bc.bound(self.net64, self.x_lo[p], self.x_hi[p], self.C[p], lo, up, split,
                        self.alpha_to_layers(b, alpha_flat), self.beta_to_layers(b, beta_flat), ball=self._ball(p))

    def upper(self, b, alpha_flat, beta_flat):
        """(g [m], ub [m], sat [m], margin [m]) of subdomain b (beta_crown.upper_bound)."""
        p, lo, up, split = self.domain(b)
        return bc.upper_bound(self.net64, self.x_lo[p], self.x_hi[p], self.C[p], lo, up, split,
                              self.alpha_to_layers(b, alpha_flat), self.beta_to_layers(b, beta_flat), self._ball(p))

    def grad(self, b, alpha_flat, beta_flat):
        """(g [m], dalpha in the compact block of b, dbeta [depth_b, m])."""
        p, lo, up, split = self.domain(b)
        g, ga, gb = bc.bound_and_grad(self.net64, self.x_lo[p], self.x_hi[p], self.C[p], lo, up, split,
                                      self.alpha_to_layers(b, alpha_flat), self.beta_to_layers(b, beta_flat),
                                      self._ball(p))
        return g, self.alpha_from_layers(b, ga), self.beta_from_layers(b, gb)

    def optimize(self, b, alpha_flat, beta_flat, cfg=None):
        """(best g [m], final alpha block, final beta [depth_b, m], final g)."""
        p, lo, up, split = self.domain(b)
        best, a, bt, g = bc.optimize(self.net64, self.x_lo[p], self.x_hi[p], self.C[p], lo, up, split,
                                     self.alpha_to_layers(b, alpha_flat), self.beta_to_layers(b, beta_flat), cfg,
                                     self._ball(p))
        return best, self.alpha_from_layers(b, a), self.beta_from_layers(b, bt), g

    def joint_optimize(self, b, alpha_flat, beta_flat, cfg=None):
        """Eq. (opt_non_convex) for subdomain b (oracle.joint.joint_optimize):
        (best g [m], final alpha block, final beta [depth_b, m], final g,
        lo, up of the final iterate, each [sum d_i] layer-major)."""
        if self.l2 is not None:
            raise ValueError("joint optimisation is over boxes")
        p, lo, up, split = self.domain(b)
        best, a, bt, g, l_j, u_j = jt.joint_optimize(self.net64, self.x_lo[p], self.x_hi[p], self.C[p], lo, up, split,
                                                     self.alpha_to_layers(b, alpha_flat),
                                                     self.beta_to_layers(b, beta_flat), cfg)
        return (best, self.alpha_from_layers(b, a), self.beta_from_layers(b, bt), g, np.concatenate(l_j),
                np.concatenate(u_j))

    # ---- joint optimisation: the library's shared alpha' / beta' layouts ---
    def joint_layout(self, b, i):
        """Entries of subdomain b in the shared variables of layer i: the
        root-unstable neurons of its property below layer i (nd-axis index,
        layer-major) and its splits below layer i (CSR entries, in order)."""
        u = self.unstable[int(self.dom_prop[b])]
        us = u[u < self.offs[i - 1]]
        ts = [t for t in range(self.ptr[b], self.ptr[b + 1]) if int(self.s_layer[t]) < i]
        return us, ts

    def joint_offsets(self, i):
        """Start of each subdomain's block in layer i's shared alpha' and beta'."""
        oa, ob = [0], [0]
        for b in range(self.B):
            us, ts = self.joint_layout(b, i)
            oa.append(oa[-1] + 2 * len(us))
            ob.append(ob[-1] + 2 * len(ts))
        return oa, ob

    def joint_vars(self, b, flat):
        """oracle.joint.JointVars of subdomain b from the library's shared
        arrays flat = {layer i: (alpha' [sum 2 uc], beta' [nnz_i * 2])}."""
        ap, bp = {}, {}
        for i, (ash, bsh) in flat.items():
            oa, ob = self.joint_offsets(i)
            us, ts = self.joint_layout(b, i)
            a = np.asarray(ash[oa[b]:oa[b + 1]], np.float64).reshape(2, len(us))
            bb = np.asarray(bsh[ob[b]:ob[b + 1]], np.float64).reshape(len(ts), 2)
            ap[i], bp[i] = [], []
            for side in (0, 1):
                dense = np.zeros(self.offs[i - 1])
                dense[us] = a[side]
                ap[i].append([jt._t(dense[self.offs[k]:self.offs[k + 1]]) for k in range(i - 1)])
                dense = np.zeros(self.offs[i - 1])
                for n, t in enumerate(ts):
                    dense[self.offs[int(self.s_layer[t]) - 1] + int(self.s_neuron[t])] = bb[n, side]
                bp[i].append([jt._t(dense[self.offs[k]:self.offs[k + 1]]) for k in range(i - 1)])
        return jt.JointVars(ap, bp)

    def joint_eval(self, b, alpha_flat, beta_flat, jv, grad=False):
        """(g [m], lo, up [sum d_i]) of Eq. (opt_non_convex)'s bound for
        subdomain b at the final objective's alpha, beta (library layouts)
        and the intermediate variables jv; with grad, also d(sum g)/d(jv) in
        the library's shared layouts {layer i: (g alpha' block, g beta' block)}."""
        p, lo, up, split = self.domain(b)
        leaves = jv.leaves()
        if grad:
            for x in leaves:
                x.requires_grad_(True)
        g, l_j, u_j = jt.joint_bound(self.net64, self.x_lo[p], self.x_hi[p], self.C[p], lo, up, split,
                                     [jt._t(a) for a in self.alpha_to_layers(b, alpha_flat)],
                                     [jt._t(x) for x in self.beta_to_layers(b, beta_flat)], jv)
        out = (g.detach().numpy().copy(), np.concatenate([x.detach().numpy() for x in l_j]),
               np.concatenate([x.detach().numpy() for x in u_j]))
        if not grad:
            return out
        gr = jt.torch.autograd.grad(g.sum(), leaves, allow_unused=True)
        gmap = {id(x): (jt.torch.zeros_like(x) if y is None else y) for x, y in zip(leaves, gr)}
        gflat = {}
        for i in jv.ap:
            us, ts = self.joint_layout(b, i)
            ga = np.zeros((2, len(us)))
            gb = np.zeros((len(ts), 2))
            for side in (0, 1):
                dense = np.concatenate([gmap[id(x)].numpy() for x in jv.ap[i][side]])
                ga[side] = dense[us]
                dense = np.concatenate([gmap[id(x)].numpy() for x in jv.bp[i][side]])
                for n, t in enumerate(ts):
                    gb[n, side] = dense[self.offs[int(self.s_layer[t]) - 1] + int(self.s_neuron[t])]
            gflat[i] = (ga.reshape(-1), gb.reshape(-1))
        return out + (gflat,)

    def joint_start(self, b):
        """oracle.joint.init_vars for subdomain b (alpha' at CROWN's slopes of
        its property's root bounds, beta' = 0)."""
        p, lo, up, _ = self.domain(b)
        return jt.init_vars(self.net64, lo, up)
