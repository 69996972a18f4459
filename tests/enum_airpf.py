"""Exact enumeration of AIRPF on the binary toy HMM (Section 4.1).

Test helper, written from Algorithm 1 independently of the C oracle: it
propagates the exact probability distribution of the filter's state
(particles, island weights) through every random choice, in rational
arithmetic, and returns the exact law of the estimate Zhat_T = gamma^N_T(1).

Model: x in {0,1}, x_0 uniform, stay with probability 3/4, y = x with
probability 3/4.  Systematic internal resampling with exact weights: the
offset is continuous uniform on [0, G), G = sum_i g_i; slot j takes
min{i : N C_i > U + j G}.  Multinomial internal resampling (the i.i.d.
draws of Algorithm 1 as written): slot j takes i with probability g_i / G,
independently.  Stage s pairs k with k xor 2^(s-1); interaction
iff ENF < tau; a block is taken from the partner with probability
W_p/(W_k + W_p); the island weights become the pair mean.
"""
from collections import defaultdict
from fractions import Fraction as Fr
from itertools import product

G_MATCH, G_MISS, P_STAY = Fr(3, 4), Fr(1, 4), Fr(3, 4)


def g_of(x, y):
    return G_MATCH if x == y else G_MISS


def forward_algorithm(y):
    """Exact marginal likelihood p(y_0..y_{T-1}) of the toy HMM."""
    a = {0: Fr(1, 2) * g_of(0, y[0]), 1: Fr(1, 2) * g_of(1, y[0])}
    for yn in y[1:]:
        a = {x1: sum(a[x0] * (P_STAY if x0 == x1 else 1 - P_STAY) for x0 in (0, 1)) * g_of(x1, yn)
             for x1 in (0, 1)}
    return a[0] + a[1]


def systematic_outcomes(g, N):
    """[(ancestors tuple, probability)] for weights g (Fractions)."""
    G = sum(g)
    C, acc = [], Fr(0)
    for v in g:
        acc += v
        C.append(acc)
    pts = {Fr(0), G}
    for i in range(N):
        for j in range(N):
            b = N * C[i] - j * G
            if 0 < b < G:
                pts.add(b)
    pts = sorted(pts)
    out = defaultdict(Fr)
    for lo, hi in zip(pts[:-1], pts[1:]):
        U = (lo + hi) / 2
        anc = tuple(min(i for i in range(N) if N * C[i] > U + j * G) for j in range(N))
        out[anc] += (hi - lo) / G
    return list(out.items())


def multinomial_outcomes(g, N):
    """[(ancestors tuple, probability)]: N independent draws with P(i) = g_i / G."""
    G = sum(g)
    out = []
    for anc in product(range(N), repeat=N):
        pr = Fr(1)
        for a in anc:
            pr *= g[a] / G
        if pr:
            out.append((anc, pr))
    return out


def enf(W):
    m = len(W)
    s1, s2 = sum(W), sum(w * w for w in W)
    if s2 == 0:
        return None
    return (s1 / m) ** 2 / (s2 / m)


def law_of_zhat(y, m, N, tau, scheme="systematic"):
    """Exact law {Zhat: probability} of the AIRPF estimate after len(y) weightings."""
    outcomes = systematic_outcomes if scheme == "systematic" else multinomial_outcomes
    tau = Fr(tau)
    S = m.bit_length() - 1
    T = len(y)
    # state: (x flat tuple of length m*N, W tuple of length m)
    dist = defaultdict(Fr)
    for xs in product((0, 1), repeat=m * N):
        dist[(xs, (Fr(1),) * m)] += Fr(1, 2 ** (m * N))
    law = defaultdict(Fr)
    for n in range(T):
        # island weighting (and, at the last step, the estimate)
        nd = defaultdict(Fr)
        for (xs, W), p in dist.items():
            W2 = tuple(W[k] * sum(g_of(xs[k * N + i], y[n]) for i in range(N)) / N for k in range(m))
            nd[(xs, W2)] += p
        dist = nd
        if n == T - 1:
            for (xs, W), p in dist.items():
                law[sum(W) / m] += p
            break
        # internal resampling
        nd = defaultdict(Fr)
        for (xs, W), p in dist.items():
            per_island = [outcomes([g_of(xs[k * N + i], y[n]) for i in range(N)], N)
                          for k in range(m)]
            for combo in product(*per_island):
                pr = p
                nx = []
                for k, (anc, q) in enumerate(combo):
                    pr *= q
                    nx.extend(xs[k * N + a] for a in anc)
                nd[(tuple(nx), W)] += pr
        dist = nd
        # stages
        for s in range(1, S + 1):
            nd = defaultdict(Fr)
            b = 1 << (s - 1)
            for (xs, W), p in dist.items():
                e = enf(W)
                if e is None or not (e < tau):
                    nd[(xs, W)] += p
                    continue
                choices = []
                for k in range(m):
                    pk = k ^ b
                    tot = W[k] + W[pk]
                    pp = W[pk] / tot if tot > 0 else Fr(0)
                    choices.append([(k, 1 - pp), (pk, pp)])
                W2 = tuple((W[k] + W[k ^ b]) / 2 for k in range(m))
                for combo in product(*choices):
                    pr = p
                    nx = []
                    for k, (src, q) in enumerate(combo):
                        pr *= q
                        nx.extend(xs[src * N:(src + 1) * N])
                    if pr:
                        nd[(tuple(nx), W2)] += pr
            dist = nd
        # mutation
        nd = defaultdict(Fr)
        for (xs, W), p in dist.items():
            for flips in product((0, 1), repeat=m * N):
                pr = p
                nx = []
                for x, f in zip(xs, flips):
                    pr *= (1 - P_STAY) if f else P_STAY
                    nx.append(1 - x if f else x)
                nd[(tuple(nx), W)] += pr
        dist = nd
    return dict(law)
