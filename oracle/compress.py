"""Oracle: the homomorphic compression map Comp, SIMD-aware (Sec. 3, Sec. 5.2).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

What is computed (Alg. 7, steps 2-3; Eq. (1); Sec. 5.2):
* Mask: ctxt(d_c) = ctxt(v) boxtimes DB_c for every value column c;
* Comp: ctxt(C v) and ctxt(C d_c), C the s x N matrix with C[j, i] = i^j mod p
  (j = 1..s, i = 1..N, Eq. (1)), evaluated as a short-matrix product over the
  slots (Sec. 5.2): both rows of a ciphertext carry one block u = [a; b] of two
  vectors, the product by each s x (n/2) block of C is the sum of plaintext
  "diagonals" times row rotations of u, the blocks are summed and a single
  rotate-and-sum follows.

Readings where the paper is silent (each fixed so that a ciphertext is fully
determined by the inputs and the key seeds):
* s = 2^ceil(log2 t_bound) so that s divides n/2;
* records are split into G = ceil(n_ct / ((p-1)/n)) balanced groups of whole
  ciphertexts, so each group has at most p-1 records and C's columns stay
  distinct and nonzero mod p; a record's column index is its 1-based position
  inside its group;
* streams: the vectors [v, d_1, ..., d_ncol] taken in pairs (a, b); a missing b
  leaves row 1 of the block empty;
* the u-block of group-local ciphertext i, row r covers the group-local records
  [(2i + r) n/2, (2i + r + 1) n/2). For row 0 it is
  A*[1;0] + Rot_col(B*[1;0]), for row 1 Rot_col(A*[0;1]) + B*[0;1]
  (the paper's u_1, u_2 of Sec. 5.2, applied per ciphertext);
* block products use baby step/giant step with B the power of two in [1, s]
  minimising k (B-1) + (s/B - 1) (k = blocks in the group), ties to the larger
  B. Baby-step rotations Rot_row(u; b), b < B, are hoisted (one ModUp per
  block); giant-step, rotate-and-sum, Rot_col and merge rotations are not. The
  giant-step rotations of one block product are summed before ModDown: their
  key products are added over PQ and brought down once (bfv.rotate_sum);
* pre-rotated diagonal for block beta, giant index g, baby index b, slot m of
  either row: alpha(beta, (m + b) mod n/2) ^ (((m - g B) mod s) + 1) mod p with
  alpha(beta, c) = beta n/2 + c + 1;
* rotate-and-sum: y <- y + Rot_row(y; s 2^i) for i = 0, 1, ... while s 2^i < n/2;
* bands: band g * (#streams) + sigma holds group g, stream sigma. With one band
  the output is that band as is; otherwise every band is multiplied by the
  mask of slots [0, s) and band beta' is rotated by -beta' s before summing;
  the bands must fit: bands * s <= n/2;
* smaller parameters for the answer (Sec. 5.3; Sec. 6.2 counts the answer as
  one ciphertext modulo a single 54-bit prime): after the merge the output may
  be modulus-switched once more, to its first `out_level` primes, by the same
  division by the dropped primes (out_level in compress; default: no switch);
* smaller parameters for Comp (Sec. 5.3 switches to a smaller ring after
  Mask): here the modulus is switched instead. After Mask, the index-vector
  and masked ciphertexts drop to the first `level` ciphertext primes, and
  everything after (u-packing, the block products, rotate-and-sum, merge) runs
  there with the top-level Galois keys restricted to those primes. The default
  level is the smallest multiple of the digit size that is at least 2 primes
  (comp_level in compress); level = L keeps the full modulus.
"""
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np

from . import bfv


class ScheduleError(ValueError):
    pass


@dataclass
class Group:
    ct_start: int   # first ciphertext of the group (query-global index)
    ct_count: int
    rec_start: int  # first record (query-global, 0-based)
    n_rec: int      # records in the group
    k: int          # u-blocks
    B: int          # baby-step count


@dataclass
class Schedule:
    n: int
    p: int
    N: int
    n_ct: int
    ncol: int
    s: int
    groups: List[Group]
    streams: List[Tuple[int, Optional[int]]]  # vector ids: 0 = v, c = d_c
    keys: List[int] = field(default_factory=list)  # Galois elements, ascending

    @property
    def nh(self):
        return self.n // 2

    @property
    def bands(self):
        return len(self.groups) * len(self.streams)


def sparsity_bound(t_bound):
    s = 1
    while s < t_bound:
        s *= 2
    return s


def choose_B(s, k):
    best = None
    B = 1
    while B <= s:
        cost = k * (B - 1) + (s // B - 1)
        if best is None or cost <= best[0]:
            best = (cost, B)
        B *= 2
    return best[1]


def make_schedule(n, p, N, ncol, t_bound) -> Schedule:
    nh = n // 2
    if N < 1 or t_bound < 1 or ncol < 0:
        raise ScheduleError("empty query")
    s = sparsity_bound(t_bound)
    if s > nh:
        raise ScheduleError("sparsity bound exceeds the slots of one row")
    n_ct = -(-N // n)
    per_group = (p - 1) // n
    G = -(-n_ct // per_group)
    groups = []
    ct = 0
    for g in range(G):
        cnt = n_ct // G + (1 if g < n_ct % G else 0)
        rec_start = ct * n
        n_rec = min(N, (ct + cnt) * n) - rec_start
        k = -(-n_rec // nh)
        groups.append(Group(ct, cnt, rec_start, n_rec, k, choose_B(s, k)))
        ct += cnt
    vecs = list(range(ncol + 1))
    streams = [(vecs[i], vecs[i + 1] if i + 1 < len(vecs) else None)
               for i in range(0, len(vecs), 2)]
    sched = Schedule(n, p, N, n_ct, ncol, s, groups, streams)
    if sched.bands * s > nh:
        raise ScheduleError("bands do not fit in one row")
    sched.keys = sorted(required_keys(sched))
    return sched


def rot(n, r):
    return pow(3, r % (n // 2), 2 * n)


def required_keys(sched):
    n, s, nh = sched.n, sched.s, sched.nh
    keys = set()
    for g in sched.groups:
        for b in range(1, g.B):
            keys.add(rot(n, b))
        for gi in range(1, s // g.B):
            keys.add(rot(n, gi * g.B))
        if g.k >= 2 or any(b is not None for _, b in sched.streams):
            keys.add(2 * n - 1)
    sh = s
    while sh < nh:
        keys.add(rot(n, sh))
        sh *= 2
    for band in range(1, sched.bands):
        keys.add(rot(n, -band * s))
    return keys


# ---------------------------------------------------------------------------
# plaintext slot matrices used by the map

def row_mask(nh, row):
    m = np.zeros((2, nh), dtype=np.uint64)
    m[row, :] = 1
    return m


def prefix_mask(nh, s):
    m = np.zeros((2, nh), dtype=np.uint64)
    m[:, :s] = 1
    return m


def diagonal_slots(p, nh, s, B, beta, gi, b):
    """Slots of the diagonal for block beta, giant index gi, baby index b."""
    m = np.arange(nh, dtype=np.int64)
    alpha = (beta * nh + (m + b) % nh + 1) % p
    expo = (m - gi * B) % s + 1
    row = powmod_vec(alpha, expo, p).astype(np.uint64)
    return np.stack([row, row])


def powmod_vec(base, expo, p):
    """base^expo mod p element-wise (p < 2^31, so products fit in int64)."""
    base = np.asarray(base, dtype=np.int64) % p
    expo = np.asarray(expo, dtype=np.int64).copy()
    out = np.ones_like(base)
    while expo.any():
        odd = (expo & 1).astype(bool)
        out = np.where(odd, out * base % p, out)
        base = base * base % p
        expo >>= 1
    return out


def db_slots(db_col, n, ct_index):
    """Slot matrix of the database values in the slots of ciphertext ct_index: the
    records [ct_index n, (ct_index + 1) n) of the column (0 beyond its end). A query
    over the first N records of a longer database uses the database's values in the
    unused slots of its last ciphertext; its index vector is 0 there."""
    vals = np.zeros(n, dtype=np.uint64)
    lo = ct_index * n
    hi = min(len(db_col), lo + n)
    if hi > lo:
        vals[:hi - lo] = np.asarray(db_col[lo:hi], dtype=np.uint64)
    return vals.reshape(2, n // 2)


# ---------------------------------------------------------------------------
# the map

class KeySet:
    def __init__(self, gks: Dict[int, "bfv.GaloisKey"]):
        self.gks = gks

    def __getitem__(self, k):
        if k not in self.gks:
            raise KeyError("missing Galois key %d" % k)
        return self.gks[k]


def mask(pr, ct_v, db_col, ct_index):
    """ctxt(d) = ctxt(v) boxtimes DB (Alg. 7 step 2) for one ciphertext."""
    return bfv.mul_plain(pr, ct_v, bfv.plain_poly(pr, db_slots(db_col, pr.n, ct_index)))


def u_blocks(pr, sched, grp, A_cts, B_cts, keys):
    """u-blocks of one (group, stream): A_cts / B_cts are the group's ciphertexts."""
    nh = pr.nh
    m0 = bfv.plain_poly(pr, row_mask(nh, 0))
    m1 = bfv.plain_poly(pr, row_mask(nh, 1))
    us = []
    for beta in range(grp.k):
        i, row = divmod(beta, 2)
        A = A_cts[i]
        Bc = B_cts[i] if B_cts is not None else None
        if row == 0:
            u = bfv.mul_plain(pr, A, m0)
            if Bc is not None:
                u = u + bfv.rotate(pr, bfv.mul_plain(pr, Bc, m0), keys[2 * pr.n - 1])
        else:
            u = bfv.rotate(pr, bfv.mul_plain(pr, A, m1), keys[2 * pr.n - 1])
            if Bc is not None:
                u = u + bfv.mul_plain(pr, Bc, m1)
        us.append(u)
    return us


def block_product(pr, sched, grp, us, keys):
    """Sum over blocks of C_beta u_beta, before rotate-and-sum (Sec. 5.2)."""
    n, s, B = pr.n, sched.s, grp.B
    baby = []
    for u in us:
        rs = [u]
        if B > 1:
            rs += bfv.rotate_hoisted(pr, u, [keys[rot(n, b)] for b in range(1, B)])
        baby.append(rs)
    accs = []
    for gi in range(s // B):
        acc = None
        for beta in range(grp.k):
            for b in range(B):
                d = diagonal_slots(pr.p, pr.nh, s, B, beta, gi, b)
                term = bfv.mul_plain(pr, baby[beta][b], bfv.plain_poly(pr, d))
                acc = term if acc is None else acc + term
        accs.append(acc)
    # giant steps: y = A_0 + sum_{g >= 1} Rot_row(A_g; g B), one ModDown for the sum
    y = accs[0]
    if len(accs) > 1:
        y = y + bfv.rotate_sum(pr, accs[1:], [keys[rot(n, gi * B)] for gi in range(1, len(accs))])
    return y


def rotate_and_sum(pr, sched, y, keys):
    sh = sched.s
    while sh < pr.nh:
        y = y + bfv.rotate(pr, y, keys[rot(pr.n, sh)])
        sh *= 2
    return y


def default_level(pr):
    """Smallest multiple of the digit size that is at least 2 primes (at most L)."""
    lvl = pr.alpha * -(-2 // pr.alpha)
    return min(lvl, pr.L)


def compress(pr, sched, cts_v, db, gks, level=None, out_level=None, given=None):
    """Comp of Alg. 7 step 3 on ciphertexts of v (and Mask, step 2).

    cts_v: n_ct ciphertexts of the index vector; db: ncol value columns of
    length N; gks: Galois keys by element; level: ciphertext primes kept for
    Comp (None: default_level); out_level: primes of the answer (None: the Comp
    level; fewer: the merged output is modulus-switched down to them). Returns
    one ciphertext at out_level. given: instead of masking db, the ciphertexts of
    every value vector d_c directly ([ncol][n_ct], at the full modulus; Alg. 5)."""
    out = _compress(pr, sched, cts_v, db, gks, level, given)
    lvl = len(out.c0.mods)
    if out_level is None or out_level == lvl:
        return out
    if not 0 < out_level < lvl:
        raise ScheduleError("out_level must be in [1, Comp level]")
    return bfv.mod_switch(bfv.at_level(pr, lvl), out, out_level)


def _compress(pr, sched, cts_v, db, gks, level, given=None):
    if given is not None:
        if len(cts_v) != sched.n_ct or len(given) != sched.ncol or any(len(g) != sched.n_ct for g in given):
            raise ScheduleError("inputs do not match the schedule")
        masked = [list(g) for g in given]
    else:
        if len(cts_v) != sched.n_ct or len(db) != sched.ncol or any(len(col) < sched.N for col in db):
            raise ScheduleError("inputs do not match the schedule")
        masked = [[mask(pr, cts_v[i], db[c], i) for i in range(sched.n_ct)]
                  for c in range(sched.ncol)]
    level = default_level(pr) if level is None else level
    if level < pr.L:
        cts_v = [bfv.mod_switch(pr, ct, level) for ct in cts_v]
        masked = [[bfv.mod_switch(pr, ct, level) for ct in row] for row in masked]
        gks = {k: bfv.key_at_level(pr, gk, level) for k, gk in gks.items()}
        pr = bfv.at_level(pr, level)
    keys = KeySet(gks)

    def vec_cts(vid, grp):
        src = cts_v if vid == 0 else masked[vid - 1]
        return src[grp.ct_start:grp.ct_start + grp.ct_count]

    bands = []
    for grp in sched.groups:
        for a, b in sched.streams:
            us = u_blocks(pr, sched, grp, vec_cts(a, grp),
                          vec_cts(b, grp) if b is not None else None, keys)
            y = block_product(pr, sched, grp, us, keys)
            bands.append(rotate_and_sum(pr, sched, y, keys))
    if len(bands) == 1:
        return bands[0]
    ms = bfv.plain_poly(pr, prefix_mask(pr.nh, sched.s))
    out = bfv.mul_plain(pr, bands[0], ms)
    for beta in range(1, len(bands)):
        t = bfv.mul_plain(pr, bands[beta], ms)
        out = out + bfv.rotate(pr, t, keys[rot(pr.n, -beta * sched.s)])
    return out


# ---------------------------------------------------------------------------
# the unencrypted-database form (Sec. 5.2, remark on an unencrypted database)
#
# With the database in the clear, C (DB * v) = (C diag(DB)) v, so the server can
# fold the values into the matrix, D_c = C diag(DB_c), and compute [C; D_1; ...] v
# directly on the index vector: no Mask, and no per-stream packing. Reading used here
# (the remark gives no slot layout): the stream pairs are the same as above, (C, D_1),
# (D_2, D_3), ..., and band g * (#streams) + sigma again holds group g's products,
# row 0 = M_a v and row 1 = M_b v, so the answer decrypts exactly like the
# encrypted-database form. Each input ciphertext X_i = [x_(2i); x_(2i+1)] (its two
# slot rows hold the group-local record blocks 2i and 2i+1) gives two u-blocks, X_i and
# Y_i = Rot_col(X_i) = [x_(2i+1); x_(2i)], shared by every stream; a diagonal now
# differs between the rows: in row r of a u-block holding record block beta_r it
# carries M_r's entries for that block,
#   alpha(beta_r, c)^(((m - g B) mod s) + 1) * DB_(col_r)[record(beta_r, c)] mod p,
#   c = (m + b) mod n/2,
# with the DB factor 1 for the matrix C. Records past the database's end count as 0.
# k = 2 (ciphertexts in the group) u-blocks per group, B by the same rule; baby steps
# are hoisted once per u-block for all streams; the block products, giant steps,
# rotate-and-sum, merge and the answer's switch follow the encrypted form. The inputs
# are switched to the Comp level first (no Mask runs at the top level).

def plain_db_blocks(grp):
    """(beta_0, beta_1) of the u-blocks of a group: X_i, then Y_i, per ciphertext i."""
    out = []
    for i in range(grp.ct_count):
        out.append((2 * i, 2 * i + 1))
        out.append((2 * i + 1, 2 * i))
    return out


def plain_db_schedule(sched):
    """The schedule of the unencrypted-database form: same groups, streams and s, with
    k = 2 (ciphertexts in the group) and B chosen for that k."""
    import copy
    s2 = copy.deepcopy(sched)
    for g in s2.groups:
        g.k = 2 * g.ct_count
        g.B = choose_B(s2.s, g.k)
    s2.keys = sorted(required_keys(s2) | {2 * s2.n - 1})
    return s2


def diagonal_slots_db(p, nh, s, B, blocks, gi, b, cols, db, rec_start):
    """Slots of the unencrypted-database diagonal: row r for record block blocks[r]
    and matrix cols[r] (0: C; c >= 1: C diag(DB_c)), giant gi, baby b."""
    m = np.arange(nh, dtype=np.int64)
    c = (m + b) % nh
    expo = (m - gi * B) % s + 1
    rows = []
    for r in range(2):
        beta = blocks[r]
        alpha = (beta * nh + c + 1) % p
        val = powmod_vec(alpha, expo, p)
        col = cols[r]
        if col is not None and col > 0:
            col_vals = np.asarray(db[col - 1], dtype=np.int64)
            rec = rec_start + beta * nh + c
            fac = np.where(rec < len(col_vals), col_vals[np.minimum(rec, len(col_vals) - 1)] % p, 0)
            val = val * fac % p
        elif col is None:
            val = np.zeros_like(val)
        rows.append(val.astype(np.uint64))
    return np.stack(rows)


def compress_plain_db(pr, sched, cts_v, db, gks, level=None, out_level=None):
    """Comp in the unencrypted-database form (see above): the same answer layout as
    compress, computed as [C; D_1; ...] v without Mask. sched: make_schedule's
    schedule of the query (its groups, streams and s; k and B follow
    plain_db_schedule)."""
    if len(cts_v) != sched.n_ct or len(db) != sched.ncol or any(len(col) < sched.N for col in db):
        raise ScheduleError("inputs do not match the schedule")
    sc = plain_db_schedule(sched)
    level = default_level(pr) if level is None else level
    top = pr
    if level < pr.L:
        cts_v = [bfv.mod_switch(pr, ct, level) for ct in cts_v]
        gks = {k: bfv.key_at_level(pr, gk, level) for k, gk in gks.items()}
        pr = bfv.at_level(pr, level)
    keys = KeySet(gks)
    n, s = pr.n, sc.s
    bands = []
    for grp in sc.groups:
        blocks = plain_db_blocks(grp)
        us = []
        for i in range(grp.ct_count):
            X = cts_v[grp.ct_start + i]
            us.append(X)
            us.append(bfv.rotate(pr, X, keys[2 * n - 1]))
        B = grp.B
        baby = []
        for u in us:
            rs = [u]
            if B > 1:
                rs += bfv.rotate_hoisted(pr, u, [keys[rot(n, b)] for b in range(1, B)])
            baby.append(rs)
        for a, bcol in sc.streams:
            accs = []
            for gi in range(s // B):
                acc = None
                for beta in range(grp.k):
                    for b in range(B):
                        d = diagonal_slots_db(pr.p, pr.nh, s, B, blocks[beta], gi, b, (a, bcol), db,
                                              grp.rec_start)
                        term = bfv.mul_plain(pr, baby[beta][b], bfv.plain_poly(pr, d))
                        acc = term if acc is None else acc + term
                accs.append(acc)
            y = accs[0]
            if len(accs) > 1:
                y = y + bfv.rotate_sum(pr, accs[1:], [keys[rot(n, gi * B)] for gi in range(1, len(accs))])
            bands.append(rotate_and_sum(pr, sc, y, keys))
    if len(bands) == 1:
        out = bands[0]
    else:
        ms = bfv.plain_poly(pr, prefix_mask(pr.nh, s))
        out = bfv.mul_plain(pr, bands[0], ms)
        for beta in range(1, len(bands)):
            t = bfv.mul_plain(pr, bands[beta], ms)
            out = out + bfv.rotate(pr, t, keys[rot(pr.n, -beta * s)])
    lvl = len(out.c0.mods)
    if out_level is None or out_level == lvl:
        return out
    if not 0 < out_level < lvl:
        raise ScheduleError("out_level must be in [1, Comp level]")
    return bfv.mod_switch(bfv.at_level(top, lvl), out, out_level)


# ---------------------------------------------------------------------------
# plain definition of what the compressed ciphertext decrypts to

def vandermonde_product(p, s, vec):
    """(C x)_j = sum_i i^j x_i mod p, j = 1..s, i = 1..len(vec)  (Eq. (1))."""
    x = np.asarray(vec, dtype=np.int64) % p
    idx = np.arange(1, len(x) + 1, dtype=np.int64) % p
    out = []
    powv = idx.copy()
    for _ in range(s):
        out.append(int((powv * x % p).sum() % p))
        powv = powv * idx % p
    return out


def vandermonde_product_sparse(p, s, vec):
    """vandermonde_product restricted to the nonzero entries of vec (the zero
    entries add nothing to any sum): for long, sparse vectors."""
    x = np.asarray(vec, dtype=np.int64) % p
    nz = np.nonzero(x)[0]
    idx = (nz + 1) % p
    xv = x[nz]
    out = []
    powv = idx.copy()
    for _ in range(s):
        out.append(int((powv * xv % p).sum() % p))
        powv = powv * idx % p
    return out


def expected_bands(sched, v, db):
    """For each band, (row0, row1): the first s slots it must decrypt to."""
    p, s = sched.p, sched.s
    vecs = [np.asarray(v, dtype=np.int64)[:sched.N] % p]
    for c in range(sched.ncol):
        vecs.append(vecs[0] * (np.asarray(db[c][:sched.N], dtype=np.int64) % p) % p)
    out = []
    for grp in sched.groups:
        sl = slice(grp.rec_start, grp.rec_start + grp.n_rec)
        for a, b in sched.streams:
            r0 = vandermonde_product_sparse(p, s, vecs[a][sl])
            r1 = vandermonde_product_sparse(p, s, vecs[b][sl]) if b is not None else [0] * s
            out.append((r0, r1))
    return out


def band_slots(sched, slots, band):
    """Extract (row0, row1) of a band from a decrypted slot matrix."""
    off = band * sched.s if sched.bands > 1 else 0
    return ([int(x) for x in slots[0][off:off + sched.s]],
            [int(x) for x in slots[1][off:off + sched.s]])
