"""Dense numpy helpers for pinning the oracle on tiny meshes.

Built straight from the LDU definition A[own,nb] = upper, A[nb,own] = lower,
A[i,i] = diag (paper Sec. 2.1), independently of the oracle's face loops.
"""
import numpy as np


def dense(n, owner, neighbour, diag, upper, lower):
    A = np.zeros((n, n))
    A[np.arange(n), np.arange(n)] = diag
    A[owner, neighbour] = upper
    A[neighbour, owner] = lower
    return A


def dense_case(case):
    return dense(case.n_cells, case.owner, case.neighbour, case.diag,
                 case.upper, case.lower)


def prolongation(agg, nc):
    P = np.zeros((agg.size, nc))
    P[np.arange(agg.size), agg] = 1.0
    return P


def splitmix64_out(z):
    """SplitMix64 output function (Steele, Lea & Flood 2014), Python ints."""
    m = (1 << 64) - 1
    z = (z + 0x9E3779B97F4A7C15) & m
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
    return z ^ (z >> 31)


def tie_key(i, j):
    lo, hi = (i, j) if i < j else (j, i)
    return splitmix64_out((lo << 32) | hi)


def strength2(owner, neighbour, upper, lower, diag):
    """Squared coupling strength of each face relative to the diagonals."""
    s = 0.5 * (np.abs(upper) + np.abs(lower))
    return (s * s) / (np.abs(diag[owner]) * np.abs(diag[neighbour]))


def greedy_matching(n, owner, neighbour, upper, lower, diag):
    """Sequential greedy matching: scan edges by (weight, tie key) descending
    and take an edge when both ends are free.  With a strict total order on
    edges this is the unique fixed point of repeated locally-dominant
    (handshake) matching rounds."""
    w = strength2(owner, neighbour, upper, lower, diag)
    keys = [(-w[f], -tie_key(int(owner[f]), int(neighbour[f])), f)
            for f in range(owner.size)]
    keys.sort()
    partner = -np.ones(n, np.int64)
    for _, _, f in keys:
        i, j = int(owner[f]), int(neighbour[f])
        if partner[i] < 0 and partner[j] < 0:
            partner[i] = j
            partner[j] = i
    return partner


def closed_form_1d(n, h, kind):
    """Eigenpairs of the 1D three-point operator -(u_{i-1} - 2u_i + u_{i+1})/h^2.

    kind "neumann": zero gradient at both ends.
    kind "dirichlet0": half-cell Dirichlet at the left end (boundary
    coefficient 2/h^2), zero gradient at the right end.
    kind "dirichlet_node": u_{-1} = u_n = 0 (constant diagonal 2/h^2).
    Returns (lam [n], V [n, n]) with the k-th eigenvector in column k."""
    i = np.arange(n)
    k = np.arange(n)
    if kind == "neumann":
        lam = (2 - 2 * np.cos(k * np.pi / n)) / h ** 2
        V = np.cos(np.outer(i + 0.5, k) * np.pi / n)
    elif kind == "dirichlet0":
        lam = (2 - 2 * np.cos((k + 0.5) * np.pi / n)) / h ** 2
        V = np.sin(np.outer(i + 0.5, k + 0.5) * np.pi / n)
    elif kind == "dirichlet_node":
        lam = (2 - 2 * np.cos((k + 1) * np.pi / (n + 1))) / h ** 2
        V = np.sin(np.outer(i + 1, k + 1) * np.pi / (n + 1))
    else:
        raise ValueError(kind)
    return lam, V


def pairwise_aggregation(n, owner, neighbour, upper, lower, diag):
    """One pairwise agglomeration from its definition: greedy matching, then
    each unmatched cell joins the aggregate of its strongest matched
    neighbour (ties by tie key, then smaller index), else stays alone;
    aggregates are numbered by their smallest seed cell.  Returns (agg, nc)."""
    partner = greedy_matching(n, owner, neighbour, upper, lower, diag)
    w = strength2(owner, neighbour, upper, lower, diag)
    best = {}
    for f in range(owner.size):
        i, j = int(owner[f]), int(neighbour[f])
        for a, b in ((i, j), (j, i)):
            if partner[a] < 0 and partner[b] >= 0:
                key = (w[f], tie_key(a, b), -b)
                if a not in best or key > best[a][0]:
                    best[a] = (key, b)
    seeds = sorted(i for i in range(n)
                   if (partner[i] >= 0 and i < partner[i]) or (partner[i] < 0 and i not in best))
    rank = {s: k for k, s in enumerate(seeds)}
    agg = np.empty(n, np.int64)
    for i in range(n):
        if partner[i] >= 0:
            agg[i] = rank[min(i, int(partner[i]))]
        elif i not in best:
            agg[i] = rank[i]
    for i, (_, j) in best.items():
        agg[i] = rank[min(j, int(partner[j]))]
    return agg, len(seeds)


def galerkin_ldu(n, owner, neighbour, diag, upper, lower, agg, nc):
    """P^T A P in LDU form, formed densely: coarse faces are the aggregate
    pairs a < b joined by a fine face, in (a, b) order."""
    A = dense(n, owner, neighbour, diag, upper, lower)
    P = prolongation(agg, nc)
    Ac = P.T @ A @ P
    adj = np.zeros((n, n), bool)
    adj[owner, neighbour] = True
    adj[neighbour, owner] = True
    pat = (P.T @ adj @ P) > 0
    co, cn = np.nonzero(np.triu(pat, 1))
    return co, cn, np.diag(Ac).copy(), Ac[co, cn], Ac[cn, co]


def handshake_rounds(n, owner, neighbour, weight, rounds):
    """Handshake matching from its definition, round by round: in each round
    every unmatched cell picks its unmatched neighbour of largest weight, and
    two cells that picked each other become partners; stop after `rounds`
    rounds or after a round that pairs nobody.  The weights of any cell's
    candidate faces must be distinct (no tie rule is applied here)."""
    nbrs = [[] for _ in range(n)]
    for f in range(owner.size):
        i, j = int(owner[f]), int(neighbour[f])
        nbrs[i].append((float(weight[f]), j))
        nbrs[j].append((float(weight[f]), i))
    for i in range(n):
        ws = [w for w, _ in nbrs[i]]
        assert len(set(ws)) == len(ws), "tied candidate weights"
    partner = -np.ones(n, np.int64)
    for _ in range(rounds):
        pick = -np.ones(n, np.int64)
        for i in range(n):
            if partner[i] < 0:
                cand = [(w, j) for w, j in nbrs[i] if partner[j] < 0]
                if cand:
                    pick[i] = max(cand)[1]
        new = [i for i in range(n) if pick[i] >= 0 and pick[pick[i]] == i]
        if not new:
            break
        for i in new:
            partner[i] = pick[i]
    return partner


def pcg32_inner_steps(n, owner, neighbour, diag, upper, lower, rhat, steps):
    """The FP32 inner CG of the mixed-precision solve for a fixed number of
    steps from d = 0, from its definition: coefficients, vectors, products,
    divisions and axpys in float32; the dot products accumulated in float64
    in index order; alpha and beta formed in float64 and rounded to float32.
    The product visits the diagonal, then each face in order (lower into the
    neighbour's row, then upper into the owner's row), each step in float32."""
    f32 = np.float32
    d32 = np.asarray(diag, np.float64).astype(f32)
    u32 = np.asarray(upper, np.float64).astype(f32)
    l32 = np.asarray(lower, np.float64).astype(f32)

    def dot64(a, b):
        s = 0.0
        for ai, bi in zip(a.tolist(), b.tolist()):
            s += float(ai) * float(bi)
        return s

    def amul32(x):
        y = d32 * x
        for f in range(owner.size):
            o, b = int(owner[f]), int(neighbour[f])
            y[b] = f32(y[b] + f32(l32[f] * x[o]))
            y[o] = f32(y[o] + f32(u32[f] * x[b]))
        return y

    r = np.asarray(rhat, f32).copy()
    d = np.zeros(n, f32)
    z = r / d32
    p = z.copy()
    rho = dot64(r, z)
    for k in range(steps):
        q = amul32(p)
        alpha = f32(rho / dot64(p, q))
        d = d + alpha * p
        r = r - alpha * q
        if k == steps - 1:
            break
        z = r / d32
        rho_new = dot64(r, z)
        beta = f32(rho_new / rho)
        rho = rho_new
        p = z + beta * p
    return d
