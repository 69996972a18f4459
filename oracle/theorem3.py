"""Exact second moment of the AIRPF marginal-likelihood estimate on the binary
toy HMM, by the collision formula of Section 3.3 (Theorem 3, proved through
its two lemmas), with multinomial internal resampling.

TEST INFRASTRUCTURE ONLY (a checker, like the rest of oracle/): the tests and
the variance study's CPU side use it; the product path never does.

What is computed.  For a fixed interaction scheme (every stage interacting,
alpha_s = A_s = I (x) (1/2)1_2 (x) I, or none, alpha_s = I: m independent
filters; a single filter when m = 1) Theorem 3 writes
    E[(sum_i W^i_{n,0} phi(xi^i_{n,0}))^2]
as a sum over the island paths (i_{q,s}), (j_{q,s}) of two tagged islands
traced back through the stages of every step, weighted by the products of
the interaction matrices' entries, of pi_0^{(x)2M} C H_0 ... H_{n-1} applied to
phi^{(x)2}, with H_q = R_q C K_{q+1}^{(x)2} C: C the collision operator (the two
tagged blocks are one block when the paths meet), K the block mutation, R_q
the weighting by the island likelihoods gbar_q(xi) gbar_q(xi') and the
multinomial internal resampling of both blocks.  Consecutive steps share
the island index between the last stage of a step and the first of the next
(the lemma is applied step after step).

How.  The sum over paths is organised backwards as a recursion over the xor
distance d of the two tagged islands (at stage s island k pairs with
k xor 2^(s-1), and A_s sends a tag to itself or to its partner with
probability 1/2 each, independently for the two tags), carrying for each d a
function of the pair of blocks.  With phi = 1 every function involved is
symmetric in the particles of a block, so a block is represented by its
number of particles in state 1 (0..M): pi_0 is Binomial(M, 1/2), the
multinomial resampling of a block with c ones gives Binomial(M, p_c) ones,
p_c = c g(1) / (c g(1) + (M - c) g(0)), and the mutation flips each particle
with probability 1/4.  Every quantity is an exact rational.

The estimate Zhat = gamma^N_T(1) = m^-1 sum_k W^k_T and phi = 1 give
sum_i W^i phi(xi^i) = M m Zhat (each of the N = mM particles carries its
island's weight), so E[Zhat^2] is the formula divided by (mM)^2 (pinned
exactly against the rational enumeration of the filter's law).
"""
from fractions import Fraction as Fr
from math import comb

P_STAY = Fr(3, 4)
G_MATCH, G_MISS = Fr(3, 4), Fr(1, 4)


def _g(x, y):
    return G_MATCH if x == y else G_MISS


def _binom(n, p):
    return [comb(n, k) * p ** k * (1 - p) ** (n - k) for k in range(n + 1)]


def _mutation(M):
    """K[c][e]: a block with c ones has e ones after every particle flips
    with probability 1 - P_STAY."""
    f = 1 - P_STAY
    K = [[Fr(0)] * (M + 1) for _ in range(M + 1)]
    for c in range(M + 1):
        down, up = _binom(c, f), _binom(M - c, f)
        for a, pa in enumerate(down):          # a ones become zeros
            for b, pb in enumerate(up):        # b zeros become ones
                K[c][c - a + b] += pa * pb
    return K


def _pair_apply(A, B, f):
    """(A (x) B) f: sum_{e,e'} A[c][e] B[c'][e'] f[e][e']."""
    n = len(f)
    tmp = [[sum(B[c2][e2] * f[e][e2] for e2 in range(n)) for c2 in range(n)] for e in range(n)]
    return [[sum(A[c][e] * tmp[e][c2] for e in range(n)) for c2 in range(n)] for c in range(n)]


def _collide(f):
    """C_1: both tagged blocks are the first one."""
    n = len(f)
    return [[f[c][c] for _ in range(n)] for c in range(n)]


def _add(acc, f, w):
    n = len(f)
    for c in range(n):
        for c2 in range(n):
            acc[c][c2] += w * f[c][c2]


def second_moment_sum(y, m, M, interact):
    """The right-hand side of Theorem 3 for phi = 1 after len(y) weightings:
    E[(sum_{i=1}^{mM} W^i_T)^2]."""
    S = m.bit_length() - 1
    assert 1 << S == m
    n = M + 1
    K = _mutation(M)
    phi2 = [[Fr(M * M)] * n for _ in range(n)]
    F = {d: [[m * v for v in row] for row in phi2] for d in range(m)}   # m ordered pairs per distance
    for yq in reversed(y):
        gbar = [(c * _g(1, yq) + (M - c) * _g(0, yq)) / M for c in range(n)]
        R = [_binom(M, (c * _g(1, yq)) / (c * _g(1, yq) + (M - c) * _g(0, yq))) for c in range(n)]
        newF = {d: [[Fr(0)] * n for _ in range(n)] for d in range(m)}
        for d_after, G in F.items():
            h = _collide(G) if d_after == 0 else G
            h = _pair_apply(K, K, h)
            # the two tags' sources through stages S, ..., 1: (distance before stage 1, collided) -> weight
            paths = {(d_after, False): Fr(1)}
            for s in range(S, 0, -1):
                b = 1 << (s - 1)
                nxt = {}
                for (d, col), w in paths.items():
                    moves = ((0, 0), (0, b), (b, 0), (b, b)) if interact else ((0, 0),)
                    for mi, mj in moves:
                        d2 = d ^ mi ^ mj
                        key = (d2, col or d2 == 0)
                        nxt[key] = nxt.get(key, Fr(0)) + w / len(moves)
                paths = nxt
            for (d1, col), w in paths.items():
                hh = _collide(h) if col else h
                r = _pair_apply(R, R, hh)
                r = [[gbar[c] * gbar[c2] * r[c][c2] for c2 in range(n)] for c in range(n)]
                _add(newF[d1], r, w)
        F = newF
    pi0 = _binom(M, Fr(1, 2))
    tot = Fr(0)
    for d, f in F.items():
        ff = _collide(f) if d == 0 else f
        tot += sum(pi0[c] * pi0[c2] * ff[c][c2] for c in range(n) for c2 in range(n))
    return tot


def second_moment_zhat(y, m, M, interact=True):
    """E[Zhat^2] of the estimate after len(y) weightings (exact rational)."""
    return second_moment_sum(y, m, M, interact) / (m * M) ** 2


def likelihood(y):
    """p(y_0..y_{T-1}) by the forward algorithm (exact rational)."""
    a = {0: Fr(1, 2) * _g(0, y[0]), 1: Fr(1, 2) * _g(1, y[0])}
    for yn in y[1:]:
        a = {x1: sum(a[x0] * (P_STAY if x0 == x1 else 1 - P_STAY) for x0 in (0, 1)) * _g(x1, yn)
             for x1 in (0, 1)}
    return a[0] + a[1]


def relative_variance(y, m, M, interact, m_ref=1):
    """Var Zhat of the (m, M) filter over Var Zhat of one bootstrap filter of
    m M particles (both with multinomial resampling), exact."""
    Z = likelihood(y)
    v = second_moment_zhat(y, m, M, interact) - Z * Z
    vb = second_moment_zhat(y, m_ref, m * M // m_ref, True) - Z * Z
    return v / vb
