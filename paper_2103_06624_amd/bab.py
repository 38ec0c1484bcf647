"""Batched branch and bound over the library's bound (App. B.1, Alg. 1).

One property at a time.  The objective of a subdomain is min_k (C f(x))_k over
its specification rows: the property holds when every row is >= 0.  The pool
of unverified subdomains lives on the host as arrays (a subdomain is its
split decisions); every round takes the `batch` subdomains with the lowest
lower bounds (batch_pick_out), splits each on its next neuron into a z >= 0 and a
z < 0 child (batch_split) and bounds all children in one batch on the GPU:
cv_bound_optimize from CROWN's default alpha and beta = 0, then cv_bound_upper
at the final iterate for the network at the box minimiser x* (the upper
bound).  Children whose lower bound is >= 0 are dropped (Domain_Filter), the
rest go back to the pool.  The global lower bound is the pool's smallest, the
global upper bound the smallest network value seen.  The loop stops when the
property is proved (empty pool), a counter-example is found (upper bound
< 0), the global bounds are within `delta` (Alg. 1's f-bar - f-underbar <=
delta), no pooled subdomain can be split further, the pool reaches
`max_pool`, or after `max_rounds` rounds.

One handle serves every round: each round re-targets it to the round's
children (cv_bound_update), so the network, the tables of the property and
the device buffers are built once.  With warm=True a child's optimisation
starts from its parent's final alpha and beta (the new split's beta at 0,
the Adam moments fresh) instead of CROWN's default and 0 -- the paper does
not say where it starts; the pool keeps each open subdomain's final
variables on the device for that.  Intermediate bounds stay those of the root; a
split neuron's own bounds become l >= 0 or u <= 0 (App. B.1 remark).

Branching rule (the paper cites BaBSR and FSB without defining them, so the
rule is this project's own): root-unstable neurons in decreasing order of the
intercept -l u / (u - l) of their upper chord, ties by layer then index; a
subdomain splits the first neuron of that order it has not split yet.

sound=True runs the bounds in sound mode (cv_bound_set_sound): every lower
bound is then evaluated in float64 with a rigorous rounding margin and
rounded down to float, so a 'verified' verdict is a proof (given sound root
bounds, e.g. api.root_bounds(..., sound=True)).
"""
from __future__ import annotations

import time

import numpy as np

from .api import BoundProblem


def branch_order(lo, up, relu_dims):
    """[(layer (1-based), neuron)] of the root-unstable neurons of one property,
    largest chord intercept first.  lo, up: [sum d_i] (layer-major)."""
    lo = np.asarray(lo, np.float64)
    up = np.asarray(up, np.float64)
    items = []
    off = 0
    for i, d in enumerate(relu_dims):
        l, u = lo[off:off + d], up[off:off + d]
        for j in np.nonzero((l < 0) & (u > 0))[0]:
            items.append((l[j] * u[j] / (u[j] - l[j]), i + 1, int(j)))
        off += d
    items.sort()
    return [(i, j) for _, i, j in items]


def bab(layers, x_lo, x_hi, C, lo, up, batch=1024, max_rounds=64, max_pool=1 << 20, iters=20, lr_alpha=0.01,
        lr_beta=0.05, decay=0.98, sound=False, warm=False, delta=0.0):
    """x_lo, x_hi [d0]; C [m, dL]; lo, up [sum d_i] root bounds of this property.
    Returns a dict: verdict ('verified' | 'falsified' | 'unknown'), lb (the
    smallest lower bound over the leaves of the search tree), ub, rounds,
    domains (subdomains bounded, the root included), seconds, and per_round:
    (children bounded, seconds, seconds in cv_bound_optimize) of each round.

    Every subdomain splits the neurons of the branching order in turn, so it
    is its depth d (it has split order[0..d-1]) and the d sides it took; the
    pool is held as arrays (lower bound, sequence number, depth, sides) and,
    with warm, the final variables of each pooled subdomain as device tensors
    (alpha [pool, m U], beta [pool, width, m])."""
    import torch

    t_start = time.perf_counter()
    x_lo = np.asarray(x_lo, np.float32)[None]
    x_hi = np.asarray(x_hi, np.float32)[None]
    C = np.asarray(C, np.float32)[None]
    lo = np.asarray(lo, np.float32)[None]
    up = np.asarray(up, np.float32)[None]
    m = C.shape[1]
    relu_dims = [ly.d_out for ly in layers[:-1]]
    order = branch_order(lo[0], up[0], relu_dims)
    o_lay = np.array([i for i, _ in order], np.int32)
    o_neu = np.array([j for _, j in order], np.int32)
    width = max(1, min(len(order), max_rounds))  # no subdomain is deeper than the rounds run
    opt = dict(iters=iters, lr_alpha=lr_alpha, lr_beta=lr_beta, decay=decay)
    state = {}

    def solve(depth, sides, a_start=None, b_start=None):
        """(lower, upper) bound per subdomain (depth [n], sides [n, width]) and
        the final alpha [n, m U], beta [n, width, m] (device)."""
        n = depth.shape[0]
        ptr = np.zeros(n + 1, np.int64)
        np.cumsum(depth, out=ptr[1:])
        rep = np.repeat(np.arange(n), depth)
        pos = np.arange(ptr[-1]) - ptr[rep]
        args = (np.zeros(n, np.int32), ptr, o_lay[pos], o_neu[pos], sides[rep, pos])
        pb = state.get("pb")
        if pb is None:
            pb = state["pb"] = BoundProblem(layers, x_lo, x_hi, C, lo, up, *args)
            if sound:
                pb.set_sound(1)
        else:
            pb.update(*args)
        a = a_start.reshape(-1).contiguous() if a_start is not None else pb.alpha_init()
        if b_start is not None:
            mask = torch.from_numpy(np.arange(width)[None, :] < depth[:, None]).cuda()
            bt = b_start[mask].reshape(-1).contiguous()
        else:
            bt = pb.zeros_beta()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        best, _ = pb.optimize(a, bt, **opt)
        torch.cuda.synchronize()
        state["t_opt"] = time.perf_counter() - t0
        _, ub, _ = pb.upper(a, bt, with_lb=False)
        a_fin = a.view(n, pb.n_alpha // n)
        b_fin = torch.zeros((n, width, m), dtype=torch.float32, device="cuda")
        if pb.n_beta:
            mask = torch.from_numpy(np.arange(width)[None, :] < depth[:, None]).cuda()
            b_fin[mask] = bt.view(-1, m)
        return best.min(dim=1).values.cpu().numpy(), ub.min(dim=1).values.cpu().numpy(), a_fin, b_fin

    try:
        lb0, ub0, a0, b0 = solve(np.zeros(1, np.int32), np.zeros((1, width), np.int8))
        # the pool: lower bound, sequence number (ties), depth, sides, final variables
        p_lb = np.array([lb0[0]], np.float64) if lb0[0] < 0 else np.zeros(0)
        p_seq = np.zeros(p_lb.shape[0], np.int64)
        p_dep = np.zeros(p_lb.shape[0], np.int32)
        p_sid = np.zeros((p_lb.shape[0], width), np.int8)
        p_a, p_b = (a0[:p_lb.shape[0]], b0[:p_lb.shape[0]]) if warm else (None, None)
        f_lb = float(lb0[0]) if p_lb.size else np.inf
        f_ub = float(ub0[0])
        done_lb = np.inf if p_lb.size else float(lb0[0])
        rounds, domains, seq = 0, 1, 1
        per_round = []
        while (f_lb < 0 <= f_ub and f_ub - f_lb > delta and p_lb.size and p_lb.size < max_pool
               and rounds < max_rounds):
            t_round = time.perf_counter()
            srt = np.lexsort((p_seq, p_lb))  # lowest lower bound first, then the oldest
            can = srt[p_dep[srt] < min(len(order), width)]
            pick = can[:batch]
            if pick.size == 0:
                break
            keep = np.ones(p_lb.size, bool)
            keep[pick] = False
            # children: each picked subdomain splits order[depth], z >= 0 child first
            nc = 2 * pick.size
            c_dep = np.repeat(p_dep[pick] + 1, 2)
            c_sid = np.repeat(p_sid[pick], 2, axis=0)
            c_sid[np.arange(nc), c_dep - 1] = np.tile(np.array([1, -1], np.int8), pick.size)
            if warm:
                ip = torch.from_numpy(np.repeat(pick, 2)).cuda()
                lbs, ubs, a_c, b_c = solve(c_dep, c_sid, p_a[ip], p_b[ip])  # the new split's beta row is 0
            else:
                lbs, ubs, a_c, b_c = solve(c_dep, c_sid)
            domains += nc
            f_ub = min(f_ub, float(ubs.min()))
            c_seq = seq + np.arange(nc, dtype=np.int64)
            seq += nc
            open_ = lbs < 0
            if (~open_).any():
                done_lb = min(done_lb, float(lbs[~open_].min()))
            p_lb = np.concatenate([p_lb[keep], lbs[open_].astype(np.float64)])
            p_seq = np.concatenate([p_seq[keep], c_seq[open_]])
            p_dep = np.concatenate([p_dep[keep], c_dep[open_]])
            p_sid = np.concatenate([p_sid[keep], c_sid[open_]])
            if warm:
                ik = torch.from_numpy(np.nonzero(keep)[0]).cuda()
                io = torch.from_numpy(np.nonzero(open_)[0]).cuda()
                p_a = torch.cat([p_a[ik], a_c[io]])
                p_b = torch.cat([p_b[ik], b_c[io]])
            f_lb = float(p_lb.min()) if p_lb.size else np.inf
            rounds += 1
            per_round.append((nc, time.perf_counter() - t_round, state["t_opt"]))
    finally:
        if state.get("pb") is not None:
            state["pb"].close()
    verdict = "falsified" if f_ub < 0 else ("verified" if f_lb >= 0 else "unknown")
    return {"verdict": verdict, "lb": min(f_lb, done_lb), "ub": f_ub, "rounds": rounds, "domains": domains,
            "seconds": time.perf_counter() - t_start, "per_round": per_round}
