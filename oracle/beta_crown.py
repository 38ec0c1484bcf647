"""FP64 CPU oracle of the beta-CROWN bound.  TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never calls it, and it shares no code
with the GPU library: the only common module is the seeded input generator.

Everything here is plain float64 NumPy, one subdomain at a time, with the m
specification rows of a subdomain carried as the rows of a matrix (each row is
an independent objective with its own alpha and beta; the rows never mix).

Paper references (Wang et al., "Beta-CROWN", NeurIPS 2021):
  * network and verification problem: Sec. 2.1, Eq. (nn_verify);
  * ReLU relaxation: Lemma 2.1 and its appendix form (D, lowerb);
  * split encoding S: Eq. (S) in Sec. 3.1;
  * the bound: Theorem 3.1, appendix form with Eq. (definition_D),
    (definition_lowerb), (definition_A) and the constant terms of the
    induction proof (the c' update: A D b + A lowerb at every ReLU layer, plus
    beta^T S b through Lambda = A D + beta^T S);
  * concretisation over the input set: Eq. (beta_crown_lp), written here for a
    general box (min over each coordinate), which equals the Hoelder form
    -eps*||a||_1 + a^T x0 on an unclipped L-inf ball;
  * alpha/beta optimisation: Eq. (opt_alpha_beta), Adam with 20 iterations and
    a 0.98 per-iteration learning-rate decay (experimental setup, App. C.1);
  * intermediate bounds: computed once at the root (App. B.1 remark) by
    per-layer CROWN, i.e. this same bound with beta = 0 and a specification
    of +-I on the layer in question (Sec. 3.3 with no splits).

Readings where the paper is silent (each also listed in the design notes):
  * default alpha (CROWN's adaptive choice): 1 if u >= -l else 0;
  * tie-breaks: l = 0 counts as active, u = 0 as inactive, A_j = 0 takes the
    alpha branch, and the box minimiser at A_j = 0 is the box centre;
  * alpha and beta are per (subdomain, specification row);
  * Adam constants beta1 = 0.9, beta2 = 0.999, eps = 1e-8, ascent form, with
    the learning rate at step t (0-based) equal to lr * decay**t.
"""
from __future__ import annotations

import numpy as np

DENSE = 0
CONV = 1

# ----------------------------------------------------------------------------
# the network as dense float64 matrices (Sec. 2.1: z(i) = W(i) zhat(i-1) + b(i))


def conv_as_matrix(weight, in_shape, out_shape, stride, pad):
    """Dense matrix of a 2-D cross-correlation with zero padding.

    Output (co, oy, ox) reads input (ci, oy*stride - pad + ky, ox*stride - pad + kx)
    with weight[co, ci, ky, kx]; taps that fall in the padding contribute 0.
    """
    w = np.asarray(weight, dtype=np.float64)
    co_n, ci_n, kh, kw = w.shape
    ci_, h, wd = in_shape
    co_, ho, wo = out_shape
    assert ci_ == ci_n and co_ == co_n
    M = np.zeros((co_n * ho * wo, ci_n * h * wd))
    oy, ox = np.meshgrid(np.arange(ho), np.arange(wo), indexing="ij")
    for co in range(co_n):
        rows = (co * ho + oy) * wo + ox
        for ky in range(kh):
            for kx in range(kw):
                iy = oy * stride - pad + ky
                ix = ox * stride - pad + kx
                ok = (iy >= 0) & (iy < h) & (ix >= 0) & (ix < wd)
                for ci in range(ci_n):
                    cols = (ci * h + iy) * wd + ix
                    M[rows[ok], cols[ok]] += w[co, ci, ky, kx]
    return M


def dense_net(layers):
    """List of (W, b) in float64 for a list of synth.Layer-like objects."""
    out = []
    for ly in layers:
        if ly.kind == DENSE:
            W = np.asarray(ly.weight, dtype=np.float64)
        else:
            W = conv_as_matrix(ly.weight, ly.in_shape, ly.out_shape, ly.stride, ly.pad)
        b = np.asarray(ly.bias, dtype=np.float64)
        if ly.kind == CONV:
            b = np.repeat(b, ly.out_shape[1] * ly.out_shape[2])
        out.append((W, b))
    return out


# ----------------------------------------------------------------------------
# ReLU relaxation (Lemma 2.1; Eq. definition_D and definition_lowerb)


def default_alpha(l, u):
    """CROWN's adaptive lower slope: 1 where u >= -l, else 0."""
    return np.where(u >= -l, 1.0, 0.0)


def neuron_kind(l, u, split):
    """Boolean masks (active, inactive, unstable) for one ReLU layer.

    A Z+ split is treated as l >= 0 and a Z- split as u <= 0 (proof of
    Theorem 3.1); otherwise l >= 0 is active, u <= 0 inactive.
    """
    act = (l >= 0) | (split > 0)
    ina = ~act & ((u <= 0) | (split < 0))
    uns = ~act & ~ina
    return act, ina, uns


def relax(A, l, u, split, alpha):
    """D (diagonal, as a matrix of row-wise entries) and lowerb for rows A.

    A: [m, d] coefficients of the objective with respect to zhat(i);
    alpha: [m, d] lower slopes (used only where unstable and A >= 0).
    Returns (D, lowerb), both [m, d].
    """
    act, ina, uns = neuron_kind(l, u, split)
    den = np.where(uns, u - l, 1.0)
    slope = np.where(uns, u / den, 0.0)  # upper chord slope u/(u-l)
    icpt = np.where(uns, -u * l / den, 0.0)  # its intercept -u l/(u-l)
    pos = A >= 0
    D = np.where(act, 1.0, np.where(ina, 0.0, np.where(pos, alpha, slope)))
    lowerb = np.where(uns & ~pos, icpt, 0.0)
    return D, lowerb


def split_sign(split):
    """Diagonal of S(i) (Eq. S): -1 for z >= 0 splits, +1 for z < 0, 0 otherwise."""
    return np.where(split > 0, -1.0, np.where(split < 0, 1.0, 0.0))


# ----------------------------------------------------------------------------
# the bound at fixed (alpha, beta)


def ball_parts(ball):
    """(x0, eps, q) of an l_p ball given as (x0, eps) (p = 2) or (x0, eps, p),
    1 < p < inf; q = p / (p - 1) is the dual exponent (1/p + 1/q = 1)."""
    if len(ball) == 2:
        x0, eps = ball
        p = 2.0
    else:
        x0, eps, p = ball
    return x0, eps, p / (p - 1.0)


def concretise(A0, x_lo, x_hi, ball=None):
    """min over the input set of A0 x, row by row (Eq. beta_crown_lp): over
    the box, sum_j min(A0_j x_lo_j, A0_j x_hi_j); over the l_p ball
    ||x - x0||_p <= eps, A0 x0 - eps ||A0||_q (Hoelder's inequality with the
    dual exponent q; q = 2 for the l2 ball)."""
    if ball is None:
        return np.minimum(A0 * x_lo, A0 * x_hi).sum(axis=1)
    x0, eps, q = ball_parts(ball)
    return A0 @ x0 - eps * np.linalg.norm(A0, ord=q, axis=1)


def minimiser(A0, x_lo, x_hi, ball=None):
    """x* of min A0 x over the input set, row by row: `box_minimiser`, or on
    the l_p ball x0 - eps sign(A0) |A0|^(q-1) / ||A0||_q^(q-1), the point of
    equality in Hoelder's inequality (x0 where A0 = 0); for p = 2 this is
    x0 - eps A0 / ||A0||_2."""
    if ball is None:
        return box_minimiser(A0, x_lo, x_hi)
    x0, eps, q = ball_parts(ball)
    nrm = np.linalg.norm(A0, ord=q, axis=1, keepdims=True)
    dirn = np.sign(A0) * np.abs(A0) ** (q - 1.0)
    scale = nrm ** (q - 1.0)
    return x0[None, :] - eps * np.divide(dirn, scale, out=np.zeros_like(A0), where=scale > 0)


def bound(net64, x_lo, x_hi, C, lo, up, split, alpha, beta, keep=False, ball=None):
    """Lower bounds of C f(x) over the box under split constraints.

    net64: [(W(1), b(1)), ..., (W(L), b(L))]; ReLU after layers 1..L-1.
    x_lo, x_hi: [d0] box.  C: [m, dL] specification rows.
    lo, up, split, alpha, beta: per ReLU layer i = 1..L-1 (list index i-1):
      lo/up [d_i] pre-activation bounds, split [d_i] in {+1, -1, 0},
      alpha [m, d_i] in [0, 1], beta [m, d_i] >= 0 (read only where split).
    Returns g [m] (and the per-layer trace used by the adjoint when keep).
    ball = (x0, eps) or (x0, eps, p): the input set is the l2 (or l_p) ball
    instead of the box.

    Recursion (Eq. definition_A with the spec merged into the last layer):
      A(L-1) = C W(L),  c = C b(L);
      for i = L-1 .. 1:  Lambda = A D(i) + beta(i)^T S(i),
                         c += A lowerb(i) + Lambda b(i),
                         A(i-1) = Lambda W(i);
      g = sum_j min(A(0)_j x_lo_j, A(0)_j x_hi_j) + c.
    """
    L = len(net64)
    W, b = net64[L - 1]
    A = C @ W
    c = C @ b
    trace = [None] * (L - 1)
    for i in range(L - 1, 0, -1):
        W, b = net64[i - 1]
        D, lowb = relax(A, lo[i - 1], up[i - 1], split[i - 1], alpha[i - 1])
        Lam = A * D + beta[i - 1] * split_sign(split[i - 1])
        c = c + (A * lowb).sum(axis=1) + Lam @ b
        if keep:
            trace[i - 1] = (A, D, lowb)
        A = Lam @ W
    g = concretise(A, x_lo, x_hi, ball) + c
    if keep:
        return g, A, trace
    return g


def box_minimiser(A0, x_lo, x_hi):
    """x* of min_x A0 x over the box: x_lo where A0 > 0, x_hi where A0 < 0,
    the centre where A0 = 0 (a subgradient choice; the value is unaffected)."""
    return np.where(A0 > 0, x_lo, np.where(A0 < 0, x_hi, 0.5 * (x_lo + x_hi)))


def bound_and_grad(net64, x_lo, x_hi, C, lo, up, split, alpha, beta, ball=None):
    """g and its (super)gradient with respect to alpha and beta.

    Chain rule through the recursion of `bound`: the adjoint of A(0) is the box
    minimiser x*, and the adjoint of Lambda(i) is zbar(i) = W(i) zhat(i-1) +
    b(i), with zhat(0) = x* and zhat(i) = D(i) zbar(i) + lowerb(i) -- the
    network evaluated forward through the relaxation chosen by the bound (the
    minimiser of Eq. beta_crown_linear, App. B.1 footnote).  Hence
      dg/dalpha(i)_j = zbar(i)_j A(i)_j  (unstable, unsplit, A(i)_j >= 0),
      dg/dbeta(i)_j  = S(i)_jj zbar(i)_j (split neurons),
    and zero elsewhere.  D and lowerb are piecewise constant in A, so within a
    sign pattern this is the exact gradient.
    """
    L = len(net64)
    g, A0, trace = bound(net64, x_lo, x_hi, C, lo, up, split, alpha, beta, keep=True, ball=ball)
    zhat = minimiser(A0, x_lo, x_hi, ball)
    galpha, gbeta = [], []
    for i in range(1, L):
        W, b = net64[i - 1]
        zbar = zhat @ W.T + b
        A, D, lowb = trace[i - 1]
        _, _, uns = neuron_kind(lo[i - 1], up[i - 1], split[i - 1])
        galpha.append(np.where(uns & (A >= 0), zbar * A, 0.0))
        gbeta.append(split_sign(split[i - 1]) * zbar)
        zhat = D * zbar + lowb
    return g, galpha, gbeta


# ----------------------------------------------------------------------------
# the primal side: an upper bound from the box minimiser (Alg. 1 and its
# footnote; infeasibility check of the appendix on infeasible subdomains)


def upper_bound(net64, x_lo, x_hi, C, lo, up, split, alpha, beta, ball=None):
    """The lower bound g, and for each specification row the network itself
    evaluated at that row's box minimiser x* (the x that minimises the final
    linear function A(0) x + c over the box, Eq. beta_crown_linear).

    x* lies in the box, so ub = (C f(x*))_k bounds min over the box of
    (C f(x))_k from above (Alg. 1 takes f(x*) as the subdomain's upper bound;
    ub < 0 is a counter-example).  sat_k says whether x* also meets every split
    of the subdomain -- z(i)_j(x*) >= 0 for a z >= 0 split, <= 0 for a z < 0
    split (the strict inequality closed, as in the LP) -- in which case ub
    also bounds the subdomain's own minimum from above, so g <= ub; a
    subdomain whose optimised g exceeds an upper bound that its minimum must
    meet is infeasible (the appendix on infeasibility).  margin_k is the
    smallest |z(i)_j(x*)| over the split neurons (inf without splits): how far
    sat_k is from a tie.  Returns (g [m], ub [m], sat [m] bool, margin [m]).
    """
    L = len(net64)
    g, A0, _ = bound(net64, x_lo, x_hi, C, lo, up, split, alpha, beta, keep=True, ball=ball)
    xs = minimiser(A0, x_lo, x_hi, ball)
    m = C.shape[0]
    ub = np.zeros(m)
    sat = np.ones(m, bool)
    margin = np.full(m, np.inf)
    for k in range(m):
        h = xs[k]
        for i in range(1, L):
            W, b = net64[i - 1]
            z = W @ h + b
            sp = split[i - 1]
            broken = ((sp > 0) & (z < 0)) | ((sp < 0) & (z > 0))
            if broken.any():
                sat[k] = False
            if (sp != 0).any():
                margin[k] = min(margin[k], np.abs(z[sp != 0]).min())
            h = np.maximum(z, 0.0)
        W, b = net64[L - 1]
        ub[k] = C[k] @ (W @ h + b)
    return g, ub, sat, margin


# ----------------------------------------------------------------------------
# intermediate bounds at the root (per-layer CROWN, beta = 0, no splits)


def root_bounds(net64, x_lo, x_hi):
    """Pre-activation bounds l(i), u(i) for i = 1..L-1.

    Layer i's bounds are this module's bound on the sub-network of layers
    1..i with specification [I; -I]: l = g[:d], u = -g[d:].  Earlier layers'
    bounds are those already computed, alpha is the CROWN default.
    """
    L = len(net64)
    lo, up = [], []
    for i in range(1, L):
        d = net64[i - 1][0].shape[0]
        C = np.vstack([np.eye(d), -np.eye(d)])
        split = [np.zeros(net64[k][0].shape[0], np.int8) for k in range(i - 1)]
        alpha = [np.broadcast_to(default_alpha(lo[k], up[k]), (2 * d, lo[k].shape[0])) for k in range(i - 1)]
        beta = [np.zeros((2 * d, lo[k].shape[0])) for k in range(i - 1)]
        g = bound(net64[:i], x_lo, x_hi, C, lo, up, split, alpha, beta)
        lo.append(g[:d].copy())
        up.append(-g[d:].copy())
    return lo, up


def root_bounds_opt(net64, x_lo, x_hi, cfg=None):
    """Intermediate bounds with their own optimised variables (Sec. 3.3: each
    intermediate neuron's bound l(i)_j = max over its own alpha' of the bound
    of z(i)_j, u(i)_j likewise for -z(i)_j), at the root (no splits, so beta'
    plays no part).  Layer by layer as `root_bounds`: the specification
    [I; -I] on layer i gives each of the 2 d_i bounds its own rows, hence its
    own alpha' for every unstable neuron below (the unshared form), optimised
    by `optimize` from CROWN's default; later layers use the optimised bounds
    of earlier ones.  The reported bound is the best iterate."""
    cfg = cfg or AdamConfig()
    L = len(net64)
    lo, up = [], []
    for i in range(1, L):
        d = net64[i - 1][0].shape[0]
        C = np.vstack([np.eye(d), -np.eye(d)])
        split = [np.zeros(net64[k][0].shape[0], np.int8) for k in range(i - 1)]
        alpha = [np.tile(default_alpha(lo[k], up[k]), (2 * d, 1)) for k in range(i - 1)]
        beta = [np.zeros((2 * d, lo[k].shape[0])) for k in range(i - 1)]
        best, *_ = optimize(net64[:i], x_lo, x_hi, C, lo, up, split, alpha, beta, cfg)
        lo.append(best[:d].copy())
        up.append(-best[d:].copy())
    return lo, up


def outward_f32(lo, up):
    """Round bounds to float32 outward (l down, u up) so they stay sound."""
    lo32 = np.asarray(lo, dtype=np.float32)
    up32 = np.asarray(up, dtype=np.float32)
    lo32 = np.where(lo32.astype(np.float64) > lo, np.nextafter(lo32, np.float32(-np.inf)), lo32)
    up32 = np.where(up32.astype(np.float64) < up, np.nextafter(up32, np.float32(np.inf)), up32)
    return lo32.astype(np.float32), up32.astype(np.float32)


# ----------------------------------------------------------------------------
# projected Adam ascent on (alpha, beta) (Eq. opt_alpha_beta; App. C.1)


class AdamConfig:
    def __init__(self, iters=20, lr_alpha=0.01, lr_beta=0.05, decay=0.98, b1=0.9, b2=0.999, eps=1e-8):
        self.iters, self.lr_alpha, self.lr_beta, self.decay = iters, lr_alpha, lr_beta, decay
        self.b1, self.b2, self.eps = b1, b2, eps


def adam_ascent_step(theta, grad, m, v, t, lr, cfg):
    """One Adam step (Kingma & Ba), ascent form; t is 1-based."""
    m = cfg.b1 * m + (1 - cfg.b1) * grad
    v = cfg.b2 * v + (1 - cfg.b2) * grad * grad
    mhat = m / (1 - cfg.b1 ** t)
    vhat = v / (1 - cfg.b2 ** t)
    return theta + lr * mhat / (np.sqrt(vhat) + cfg.eps), m, v


def optimize(net64, x_lo, x_hi, C, lo, up, split, alpha0, beta0, cfg=None, ball=None):
    """Projected Adam ascent; returns (best g over all evaluated iterates,
    final alpha, final beta, g of the final iterate).

    Iterates t = 0..iters-1 evaluate g and its gradient at (alpha_t, beta_t),
    keep the best g so far, take an Adam step with lr * decay**t and project
    alpha onto [0, 1] and beta onto [0, inf).  The final iterate is evaluated
    once more.  Every iterate is a sound bound (Sec. 3.1), so the best of the
    iters + 1 evaluated values is reported.
    """
    cfg = cfg or AdamConfig()
    alpha = [a.astype(np.float64).copy() for a in alpha0]
    beta = [b.astype(np.float64).copy() for b in beta0]
    ma = [np.zeros_like(a) for a in alpha]
    va = [np.zeros_like(a) for a in alpha]
    mb = [np.zeros_like(b) for b in beta]
    vb = [np.zeros_like(b) for b in beta]
    best = None
    for t in range(cfg.iters):
        g, ga, gb = bound_and_grad(net64, x_lo, x_hi, C, lo, up, split, alpha, beta, ball)
        best = g.copy() if best is None else np.maximum(best, g)
        for i in range(len(alpha)):
            a, ma[i], va[i] = adam_ascent_step(alpha[i], ga[i], ma[i], va[i], t + 1, cfg.lr_alpha * cfg.decay ** t, cfg)
            alpha[i] = np.clip(a, 0.0, 1.0)
            bb, mb[i], vb[i] = adam_ascent_step(beta[i], gb[i], mb[i], vb[i], t + 1, cfg.lr_beta * cfg.decay ** t, cfg)
            beta[i] = np.maximum(bb, 0.0)
    g = bound(net64, x_lo, x_hi, C, lo, up, split, alpha, beta, ball=ball)
    best = g.copy() if best is None else np.maximum(best, g)
    return best, alpha, beta, g
