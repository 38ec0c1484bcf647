"""Independent checkers used to pin the FP64 oracle (no GPU, no oracle code).

Each checker here computes a quantity the paper or plain mathematics fixes by
a route other than the oracle's back-substitution:
  * brute-force grid minimum of the true network over a 2-D box;
  * vertex enumeration of a fully split (hence piecewise-affine) subdomain;
  * the LP of Eq. (lp_verify_split) solved by HiGHS, with its duals;
  * the dual propagation form of Theorem 3.2 (nu, nu-hat recursion);
  * the explicit form (a, P, q, c) of Theorem 3.1 built from Omega products;
  * alpha-CROWN (Lemma 2.1 applied layer by layer, no beta) with splits
    expressed as modified bounds (l := 0 for z >= 0, u := 0 for z < 0).
"""
from __future__ import annotations

import itertools

import numpy as np
from scipy.optimize import linprog


def random_net(rng, widths, scale=1.0):
    net = []
    for a, b in zip(widths[:-1], widths[1:]):
        net.append((rng.standard_normal((b, a)) * scale / np.sqrt(a) * 1.5, rng.standard_normal(b) * 0.3))
    return net


def forward_all(net, X):
    """Pre-activations of every ReLU layer and the logits for points X [n, d0]."""
    h = X
    zs = []
    for i, (W, b) in enumerate(net):
        z = h @ W.T + b
        if i < len(net) - 1:
            zs.append(z)
            h = np.maximum(z, 0.0)
        else:
            return zs, z
    return zs, None


def grid(x_lo, x_hi, n):
    g0 = np.linspace(x_lo[0], x_hi[0], n)
    g1 = np.linspace(x_lo[1], x_hi[1], n)
    G0, G1 = np.meshgrid(g0, g1, indexing="ij")
    return np.stack([G0.ravel(), G1.ravel()], axis=1)


def grid_min(net, C, x_lo, x_hi, split, n=801):
    """min over grid points satisfying the split constraints of C f(x); +inf if
    no grid point satisfies them."""
    X = grid(x_lo, x_hi, n)
    zs, out = forward_all(net, X)
    ok = np.ones(X.shape[0], bool)
    for i, s in enumerate(split):
        for j in np.nonzero(s)[0]:
            ok &= (zs[i][:, j] >= 0) if s[j] > 0 else (zs[i][:, j] <= 0)
    vals = out @ C.T
    if not ok.any():
        return np.full(C.shape[0], np.inf)
    return vals[ok].min(axis=0)


# ----------------------------------------------------------------------------
# LP of Eq. (lp_verify_split)


def lp_verify_split(net, x_lo, x_hi, c_row, lo, up, split):
    """HiGHS solution of the triangle-relaxation LP with split constraints.

    Variables: x, then (z(i), zhat(i)) for i = 1..L-1.  Returns (p*, result,
    index maps) so callers can read the duals.
    """
    L = len(net)
    d0 = net[0][0].shape[1]
    dims = [W.shape[0] for W, _ in net[:-1]]
    nz = [0] * L
    nzh = [0] * L
    off = d0
    for i in range(1, L):
        nz[i] = off
        nzh[i] = off + dims[i - 1]
        off += 2 * dims[i - 1]
    nvar = off
    cost = np.zeros(nvar)
    WL, bL = net[-1]
    cvec = c_row @ WL
    cost[nzh[L - 1]:nzh[L - 1] + dims[L - 2]] = cvec
    const = float(c_row @ bL)
    A_eq, b_eq, A_ub, b_ub, tags = [], [], [], [], []

    def row():
        return np.zeros(nvar)

    for i in range(1, L):
        W, b = net[i - 1]
        prev = (0, d0) if i == 1 else (nzh[i - 1], dims[i - 2])
        for j in range(dims[i - 1]):
            r = row()
            r[nz[i] + j] = 1.0
            r[prev[0]:prev[0] + prev[1]] -= W[j]
            A_eq.append(r)
            b_eq.append(b[j])
        for j in range(dims[i - 1]):
            l, u, s = lo[i - 1][j], up[i - 1][j], split[i - 1][j]
            zj, hj = nz[i] + j, nzh[i] + j
            if s > 0 or (s == 0 and l >= 0):
                r = row(); r[hj] = 1.0; r[zj] = -1.0
                A_eq.append(r); b_eq.append(0.0)
                if s > 0:
                    r = row(); r[zj] = -1.0
                    A_ub.append(r); b_ub.append(0.0); tags.append(("beta", i, j))
            elif s < 0 or (s == 0 and u <= 0):
                r = row(); r[hj] = 1.0
                A_eq.append(r); b_eq.append(0.0)
                if s < 0:
                    r = row(); r[zj] = 1.0
                    A_ub.append(r); b_ub.append(0.0); tags.append(("beta", i, j))
            else:
                r = row(); r[hj] = -1.0
                A_ub.append(r); b_ub.append(0.0); tags.append(("mu", i, j))
                r = row(); r[zj] = 1.0; r[hj] = -1.0
                A_ub.append(r); b_ub.append(0.0); tags.append(("gamma", i, j))
                sl = u / (u - l)
                r = row(); r[hj] = 1.0; r[zj] = -sl
                A_ub.append(r); b_ub.append(-sl * l); tags.append(("lambda", i, j))
    bounds = [(x_lo[k], x_hi[k]) for k in range(d0)] + [(None, None)] * (nvar - d0)
    res = linprog(cost, A_ub=np.array(A_ub) if A_ub else None, b_ub=np.array(b_ub) if b_ub else None,
                  A_eq=np.array(A_eq), b_eq=np.array(b_eq), bounds=bounds, method="highs")
    p = res.fun + const if res.status == 0 else (np.inf if res.status == 2 else np.nan)
    return p, res, tags


def duals_to_alpha_beta(res, tags, dims):
    """alpha = gamma/(mu+gamma), beta = split multipliers (Cor. 3.2.1 proof)."""
    lam = -np.asarray(res.ineqlin.marginals)  # Lagrange multipliers of A_ub x <= b_ub
    mu = [np.zeros(d) for d in dims]
    ga = [np.zeros(d) for d in dims]
    beta = [np.zeros(d) for d in dims]
    for v, (kind, i, j) in zip(lam, tags):
        if kind == "mu":
            mu[i - 1][j] = v
        elif kind == "gamma":
            ga[i - 1][j] = v
        elif kind == "beta":
            beta[i - 1][j] = v
    alpha = [np.where(m + g > 0, g / np.where(m + g > 0, m + g, 1.0), 0.0) for m, g in zip(mu, ga)]
    return alpha, beta


# ----------------------------------------------------------------------------
# fully split subdomains: the network is affine on the subdomain


def affine_preacts(net, lo, up, split):
    """For a pattern with every unstable neuron split, z(i) = M_i x + v_i."""
    d0 = net[0][0].shape[1]
    M, v = np.eye(d0), np.zeros(d0)
    out = []
    for i, (W, b) in enumerate(net):
        Mz, vz = W @ M, W @ v + b
        if i == len(net) - 1:
            return out, (Mz, vz)
        out.append((Mz, vz))
        on = (split[i] > 0) | ((split[i] == 0) & (lo[i] >= 0))
        off = (split[i] < 0) | ((split[i] == 0) & (up[i] <= 0))
        assert np.all(on | off), "pattern not fully split"
        M, v = Mz * on[:, None], vz * on
    return out, None


def vertex_min_2d(net, C, x_lo, x_hi, lo, up, split, tol=1e-9):
    """Exact min of C f over box & split half-planes (2-D input) by enumerating
    pairwise intersections of the constraint lines; +inf when infeasible."""
    pre, (Mo, vo) = affine_preacts(net, lo, up, split)
    lines = [(np.array([1.0, 0.0]), -x_lo[0], 1), (np.array([1.0, 0.0]), -x_hi[0], -1),
             (np.array([0.0, 1.0]), -x_lo[1], 1), (np.array([0.0, 1.0]), -x_hi[1], -1)]
    for i, s in enumerate(split):
        for j in np.nonzero(s)[0]:
            lines.append((pre[i][0][j], pre[i][1][j], int(s[j])))  # s*(a.x + c) >= 0
    best = np.full(C.shape[0], np.inf)
    for (a1, c1, _), (a2, c2, _) in itertools.combinations(lines, 2):
        Mx = np.array([a1, a2])
        if abs(np.linalg.det(Mx)) < 1e-12:
            continue
        x = np.linalg.solve(Mx, -np.array([c1, c2]))
        if all(s * (a @ x + c) >= -tol for a, c, s in lines):
            best = np.minimum(best, C @ (Mo @ x + vo))
    return best


def max_over_beta_lp(bound_fn, nbeta, x_lo, x_hi):
    """max_{beta >= 0} of g(beta) = sum_j min(A_j xl_j, A_j xu_j) + c when
    A(beta) and c(beta) are affine (fully split: D is fixed).  bound_fn(beta)
    returns (A0 [d0], c).  Solved as an LP in (beta, t) with t >= |A|."""
    A0, c0 = bound_fn(np.zeros(nbeta))
    P = np.zeros((A0.shape[0], nbeta))
    q = np.zeros(nbeta)
    for s in range(nbeta):
        e = np.zeros(nbeta); e[s] = 1.0
        A1, c1 = bound_fn(e)
        P[:, s] = A1 - A0
        q[s] = c1 - c0
    ctr = 0.5 * (x_lo + x_hi)
    rad = 0.5 * (x_hi - x_lo)
    d0 = A0.shape[0]
    # maximise (A0 + P b).ctr + c0 + q.b - rad.t  -> minimise negative
    cost = np.concatenate([-(P.T @ ctr + q), rad])
    A_ub = np.block([[P, -np.eye(d0)], [-P, -np.eye(d0)]])
    b_ub = np.concatenate([-A0, A0])
    bounds = [(0, None)] * nbeta + [(None, None)] * d0
    res = linprog(cost, A_ub=A_ub, b_ub=b_ub, bounds=bounds, method="highs")
    if res.status == 3:
        return np.inf
    return -(res.fun) + A0 @ ctr + c0


# ----------------------------------------------------------------------------
# Theorem 3.2 dual propagation form (L-inf ball around x0 with radius eps)


def dual_nu_bound(net, x0, eps, c_row, lo, up, split, alpha, beta, with_input=False, q=1):
    """g from nu(L) = -c, nu-hat(i-1) = W(i)^T nu(i) and the per-neuron rules of
    the dual problem (inactive 0, active nu-hat, unstable
    u/(u-l)[nu-hat]^+ - alpha [nu-hat]^-, z<0 split -beta, z>=0 split beta + nu-hat).
    Returns (g, list of nu-hat per ReLU layer), and with with_input also
    nu-hat(0) = W(1)^T nu(1), whose negation is the coefficient of x in the
    dual objective."""
    L = len(net)
    nu = -np.asarray(c_row, float)
    obj = 0.0
    lterm = 0.0
    nuhats = [None] * (L - 1)
    for i in range(L, 0, -1):
        W, b = net[i - 1]
        obj -= nu @ b
        nh = W.T @ nu
        if i == 1:
            break
        k = i - 1
        nuhats[k - 1] = nh
        l, u, s = lo[k - 1], up[k - 1], split[k - 1]
        new = np.zeros_like(nh)
        for j in range(nh.shape[0]):
            if s[j] < 0:
                new[j] = -beta[k - 1][j]
            elif s[j] > 0:
                new[j] = beta[k - 1][j] + nh[j]
            elif u[j] <= 0:
                new[j] = 0.0
            elif l[j] >= 0:
                new[j] = nh[j]
            else:
                pos, neg = max(nh[j], 0.0), max(-nh[j], 0.0)
                new[j] = u[j] / (u[j] - l[j]) * pos - alpha[k - 1][j] * neg
                lterm += l[j] * max(new[j], 0.0)
        nu = new
    # the input set is the l_p ball around x0 with 1/p + 1/q = 1: q = 1 for l_inf, q = 2 for l_2
    g = obj - nh @ x0 - np.linalg.norm(nh, ord=q) * eps + lterm
    return (g, nuhats, nh) if with_input else (g, nuhats)


def explicit_bound(net, x_lo, x_hi, c_row, Ds, lbs, split, beta):
    """Theorem 3.1's explicit a, P, q, c (Omega products), for given per-layer
    diagonals D(i) and offsets lowerb(i) (vectors), evaluated at beta."""
    L = len(net)
    Ws = [None] + [W for W, _ in net]
    bs = [None] + [b for _, b in net]
    Ws[L] = c_row[None, :] @ Ws[L]
    bs[L] = np.array([c_row @ bs[L]])
    D = [None] + [np.diag(d) for d in Ds]
    lb = [None] + list(lbs)
    S = [None] + [np.diag(np.where(s > 0, -1.0, np.where(s < 0, 1.0, 0.0))) for s in split]

    def omega(k, i):
        M = np.eye(Ws[i].shape[0])
        for t in range(i, k):
            M = Ws[t + 1] @ D[t] @ M
        return M

    a = (omega(L, 1) @ Ws[1]).ravel()
    c = sum((omega(L, i) @ bs[i]).item() for i in range(1, L + 1))
    c += sum((omega(L, i) @ Ws[i] @ lb[i - 1]).item() for i in range(2, L + 1))
    Pb = np.zeros_like(a)
    qb = 0.0
    for i in range(1, L):
        Pi = S[i] @ omega(i, 1) @ Ws[1]
        qi = sum(S[i] @ omega(i, k) @ bs[k] for k in range(1, i + 1))
        qi = qi + sum((S[i] @ omega(i, k) @ Ws[k] @ lb[k - 1] for k in range(2, i + 1)), np.zeros(Ws[i].shape[0]))
        Pb += Pi.T @ beta[i - 1]
        qb += qi @ beta[i - 1]
    A = a + Pb
    return np.minimum(A * x_lo, A * x_hi).sum() + qb + c


# ----------------------------------------------------------------------------
# alpha-CROWN with splits as modified bounds (Lemma 2.1, no beta)


def alpha_crown_modified_bounds(net, x_lo, x_hi, c_row, lo, up, split, alpha):
    L = len(net)
    lo = [np.where(s > 0, 0.0, l) for l, s in zip(lo, split)]
    up = [np.where(s < 0, 0.0, u) for u, s in zip(up, split)]
    W, b = net[-1]
    w = W.T @ c_row
    const = float(c_row @ b)
    for i in range(L - 2, -1, -1):
        W, b = net[i]
        v = np.zeros_like(w)
        for j in range(w.shape[0]):
            l, u = lo[i][j], up[i][j]
            if l >= 0:
                v[j] = w[j]
            elif u <= 0:
                v[j] = 0.0
            elif w[j] >= 0:
                v[j] = alpha[i][j] * w[j]
            else:
                v[j] = u / (u - l) * w[j]
                const += w[j] * (-u * l / (u - l))
        const += v @ b
        w = W.T @ v
    return const + sum(wj * (x_lo[j] if wj >= 0 else x_hi[j]) for j, wj in enumerate(w))
