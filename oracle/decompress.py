"""Oracle: decompression -- ReconstIdx (Alg. 1), Reconst (Alg. 4), Decomp (Alg. 6).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Given w = C v (the power sums w_j = sum over matched indices i of i^j,
Lemma 2) and e_c = C d_c for each value column:
1. Newton's identity (Lemma 1) turns the power sums into the coefficients of
   f(X) = prod over the multiset J (matched indices padded with zeros to s
   elements) of (X - i): a_0 = 1, a_k = k^-1 sum_{i=1..k} (-1)^(i-1) a_{k-i} w_i,
   f = sum_k (-1)^k a_k X^(s-k)  (Alg. 1, step 1);
2. strip the factors X (the zero padding) and find the roots (Alg. 1, step 2).
   The paper suggests Cantor-Zassenhaus; this oracle instead evaluates the
   polynomial at every candidate index 1..N_group, which is slower but
   obviously complete;
3. solve C_hat x = e_c, C_hat the s x l matrix of the columns of C at the l
   roots (Alg. 4). The first l rows form a nonsingular scaled Vandermonde
   matrix (distinct nonzero nodes below p); they are solved by Gaussian
   elimination mod p and the remaining s - l rows are checked.
A decoding failure (root count different from the degree, or an
inconsistent system) raises DecodeError: more than s matches, or a corrupted
input.
"""
import numpy as np


class DecodeError(ValueError):
    pass


def newton_coefficients(w, p):
    """a_0..a_s from power sums w_1..w_s (Alg. 1 step 1)."""
    s = len(w)
    a = [1]
    for k in range(1, s + 1):
        acc = 0
        for i in range(1, k + 1):
            term = a[k - i] * int(w[i - 1])
            acc += term if (i - 1) % 2 == 0 else -term
        a.append(acc % p * pow(k, -1, p) % p)
    return a


def f_coefficients(w, p):
    """Coefficients of f, highest degree first: (-1)^k a_k for X^(s-k)."""
    a = newton_coefficients(w, p)
    return [(x if k % 2 == 0 else -x) % p for k, x in enumerate(a)]


def strip_x(coeffs_high_first):
    """Divide by X while X divides (the constant term is zero)."""
    c = list(coeffs_high_first)
    while len(c) > 1 and c[-1] == 0:
        c.pop()
    return c


def roots_brute_force(coeffs_high_first, p, N):
    """All alpha in [1, N] with g(alpha) = 0 mod p (Horner, vectorised)."""
    x = np.arange(1, N + 1, dtype=np.int64) % p
    acc = np.zeros(N, dtype=np.int64)
    for c in coeffs_high_first:
        acc = (acc * x + int(c)) % p
    return [int(i) for i in np.nonzero(acc == 0)[0] + 1]


def reconst_idx(w, p, N):
    """Alg. 1: index set (ascending, 1-based) from w."""
    g = strip_x(f_coefficients(w, p))
    deg = len(g) - 1
    roots = roots_brute_force(g, p, N)
    if len(roots) != deg:
        raise DecodeError("root count %d != degree %d" % (len(roots), deg))
    return roots


def solve_mod_p(A, b, p):
    """Solve A x = b mod p for square nonsingular A (Gaussian elimination)."""
    A = np.array(A, dtype=np.int64) % p
    b = np.array(b, dtype=np.int64) % p
    l = A.shape[0]
    M = np.concatenate([A, b.reshape(l, -1)], axis=1)
    for col in range(l):
        piv = col + int(np.nonzero(M[col:, col])[0][0]) if M[col:, col].any() else None
        if piv is None:
            raise DecodeError("singular system")
        if piv != col:
            M[[col, piv]] = M[[piv, col]]
        M[col] = M[col] * pow(int(M[col, col]), -1, p) % p
        f = M[:, col].copy()
        f[col] = 0
        M = (M - np.outer(f, M[col])) % p
    return M[:, l:]


def reconst(e, idx, p):
    """Alg. 4: values at the indices idx from e = C d."""
    s, l = len(e), len(idx)
    if l == 0:
        if any(int(x) % p for x in e):
            raise DecodeError("nonzero e with an empty index set")
        return []
    nodes = np.array(idx, dtype=np.int64) % p
    C_hat = np.empty((s, l), dtype=np.int64)
    row = nodes.copy()
    for j in range(s):       # row j holds the (j+1)-th powers
        C_hat[j] = row
        row = row * nodes % p
    x = solve_mod_p(C_hat[:l], np.array(e[:l], dtype=np.int64), p)[:, 0]
    check = (C_hat @ x % p) if l < 32 else np.array(
        [int(sum(int(C_hat[j, k]) * int(x[k]) for k in range(l)) % p) for j in range(s)])
    if any(int(check[j]) % p != int(e[j]) % p for j in range(s)):
        raise DecodeError("inconsistent system")
    return [int(v) for v in x]


def decompress_group(p, N_group, w, es):
    """Alg. 6 for one group: returns (indices 1-based, [values per column])."""
    idx = reconst_idx(w, p, N_group)
    vals = [reconst(e, idx, p) for e in es]
    return idx, vals
