"""Batched branch and bound over the beta-CROWN bound (App. B.1, Alg. 1) in
float64.  TEST INFRASTRUCTURE ONLY: only the tests may import it.

The objective of a subdomain is min_k (C f(x))_k over its rows (the property
holds when every row is >= 0).  Each round takes the `batch` unverified
subdomains with the lowest lower bounds (batch_pick_out), splits each on one
root-unstable neuron it has not split yet into z >= 0 and z < 0 children
(batch_split), bounds every child by the projected-Adam optimisation of
`beta_crown.optimize` from CROWN's default alpha and beta = 0, takes the
network at the box minimiser of the final iterate as its upper bound
(`beta_crown.upper_bound`), drops the children whose lower bound is >= 0
(Domain_Filter) and returns the rest to the pool.  The global lower bound is
the pool's smallest, the global upper bound the smallest upper bound seen.
It stops when the property is proved (empty pool), a counter-example is found
(upper bound < 0), the global upper and lower bounds are within `delta` of
each other (Alg. 1's f-bar - f-underbar <= delta), no pooled subdomain can be
split further, the pool exceeds `max_pool`, or after `max_rounds` rounds.
Intermediate bounds stay those of the root, split neurons taking l >= 0 /
u <= 0 (App. B.1 remark).

Children's starting point: CROWN's default alpha and beta = 0, or with
warm=True their parent's final alpha and beta (the new split's beta at 0,
the Adam moments fresh) -- the paper does not say where a child's
optimisation starts; any start gives a sound bound.

Branching rule: the paper names BaBSR and FSB only by citation, so a simple
rule of this project is used, the same in the library's driver: neurons in
decreasing order of the intercept -l u / (u - l) of their upper chord (the
height of the triangle relaxation), ties by layer then index; each subdomain
splits the first neuron of that order it has not split.
"""
from __future__ import annotations

import numpy as np

from . import beta_crown as bc


def branch_order(lo, up):
    """[(layer index i (0-based ReLU layer), neuron j)] of every root-unstable
    neuron, largest chord intercept first."""
    items = []
    for i, (l, u) in enumerate(zip(lo, up)):
        for j in np.nonzero((l < 0) & (u > 0))[0]:
            items.append((l[j] * u[j] / (u[j] - l[j]), i, int(j)))  # = -intercept: ascending sort
    items.sort()
    return [(i, j) for _, i, j in items]


def bab(net64, x_lo, x_hi, C, lo, up, batch=8, max_rounds=64, max_pool=4096, cfg=None, warm=False, delta=0.0):
    """Returns a dict: verdict ('verified' | 'falsified' | 'unknown'), lb (the
    smallest lower bound over the leaves of the search tree, a lower bound of
    the minimum), ub (the smallest upper bound seen), rounds, domains
    (subdomains bounded, the root included)."""
    cfg = cfg or bc.AdamConfig()
    m = C.shape[0]
    order = branch_order(lo, up)
    a_root = [np.tile(bc.default_alpha(l, u), (m, 1)) for l, u in zip(lo, up)]
    b_root = [np.zeros((m, l.shape[0])) for l in lo]

    def solve(split, start):
        a0, b0 = start if warm and start is not None else (a_root, b_root)
        best, a, b, _ = bc.optimize(net64, x_lo, x_hi, C, lo, up, split, a0, b0, cfg)
        _, ub, _, _ = bc.upper_bound(net64, x_lo, x_hi, C, lo, up, split, a, b)
        return float(best.min()), float(ub.min()), (a, b)

    def next_neuron(split):
        for i, j in order:
            if split[i][j] == 0:
                return i, j
        return None

    root = [np.zeros(l.shape[0], np.int8) for l in lo]
    lb, ub, var = solve(root, None)
    pool = [(lb, 0, root, var)] if lb < 0 else []  # (lower bound, insertion number, split, final alpha / beta)
    f_lb = lb if pool else np.inf
    f_ub = ub
    done_lb = np.inf if pool else lb  # smallest lower bound among the dropped (proved) leaves
    rounds, domains, seq = 0, 1, 1
    while f_lb < 0 <= f_ub and f_ub - f_lb > delta and pool and len(pool) < max_pool and rounds < max_rounds:
        pool.sort(key=lambda t: (t[0], t[1]))
        picked, rest = [], []
        for t in pool:
            (picked if len(picked) < batch and next_neuron(t[2]) is not None else rest).append(t)
        if not picked:
            break
        pool = rest
        for _, _, split, var in picked:
            i, j = next_neuron(split)
            for side in (1, -1):
                child = [s.copy() for s in split]
                child[i][j] = side
                lb_c, ub_c, var_c = solve(child, var)
                domains += 1
                f_ub = min(f_ub, ub_c)
                if lb_c < 0:
                    pool.append((lb_c, seq, child, var_c))
                else:
                    done_lb = min(done_lb, lb_c)
                seq += 1
        f_lb = min(t[0] for t in pool) if pool else np.inf
        rounds += 1
    verdict = "falsified" if f_ub < 0 else ("verified" if f_lb >= 0 else "unknown")
    # reported lower bound: over every leaf of the tree, proved ones included
    return {"verdict": verdict, "lb": min(f_lb, done_lb), "ub": f_ub, "rounds": rounds, "domains": domains}
