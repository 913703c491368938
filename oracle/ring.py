"""Oracle: polynomials of Z_M[X]/(X^n+1) in RNS form, M a product of primes.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

A `Poly` holds canonical residues (0 <= x < m_i) of one ring element, one row
per prime m_i, always in the coefficient domain. Products go through the
exact negacyclic convolution in oracle/ring.c; everything else is written
out here with Python integers.
"""
import ctypes
import os

import numpy as np

from . import build_oracle

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = build_oracle.build(force=False)
        _lib = ctypes.CDLL(path)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        u64 = ctypes.c_uint64
        _lib.o_ntt.argtypes = [u64p, u64, u64, u64]
        _lib.o_intt.argtypes = [u64p, u64, u64, u64]
        _lib.o_negacyclic_mul.argtypes = [u64p, u64p, u64p, u64, u64, u64]
        _lib.o_vec_mul.argtypes = [u64p, u64p, u64p, u64, u64]
        _lib.o_vec_scale.argtypes = [u64p, u64p, u64, u64, u64]
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


_PSI = {}


def psi_for(n, q):
    """A primitive 2n-th root of unity mod q: g^((q-1)/2n) for the least g >= 2
    for which that power has order exactly 2n (its n-th power is -1)."""
    key = (n, q)
    if key not in _PSI:
        g = 2
        while True:
            x = pow(g, (q - 1) // (2 * n), q)
            if pow(x, n, q) == q - 1:
                break
            g += 1
        _PSI[key] = x
    return _PSI[key]


def negacyclic_mul_limb(a, b, q):
    """(a * b) mod (X^n + 1, q) for one limb; a, b uint64 arrays of residues."""
    n = a.shape[0]
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    out = np.empty(n, dtype=np.uint64)
    lib().o_negacyclic_mul(_ptr(out), _ptr(a), _ptr(b), n, q, psi_for(n, q))
    return out


def vec_mul(a, b, q):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    out = np.empty_like(a)
    lib().o_vec_mul(_ptr(out), _ptr(a), _ptr(b), a.shape[0], q)
    return out


def vec_scale(a, c, q):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    out = np.empty_like(a)
    lib().o_vec_scale(_ptr(out), _ptr(a), int(c) % q, a.shape[0], q)
    return out


def ntt_limb(a, q):
    """Evaluations (a(psi^1), a(psi^3), ...) -- oracle-internal ordering."""
    a = np.array(a, dtype=np.uint64)
    lib().o_ntt(_ptr(a), a.shape[0], q, psi_for(a.shape[0], q))
    return a


def intt_limb(a, q):
    a = np.array(a, dtype=np.uint64)
    lib().o_intt(_ptr(a), a.shape[0], q, psi_for(a.shape[0], q))
    return a


class Poly:
    """One ring element in RNS form over the primes `mods` (coefficient domain)."""

    __slots__ = ("mods", "c")

    def __init__(self, mods, c):
        self.mods = list(mods)
        self.c = c  # uint64 array [len(mods)][n]

    @property
    def n(self):
        return self.c.shape[1]

    @staticmethod
    def zero(mods, n):
        return Poly(mods, np.zeros((len(mods), n), dtype=np.uint64))

    @staticmethod
    def from_ints(mods, coeffs):
        """Reduce signed integer coefficients (any size) into every limb."""
        coeffs = np.asarray(coeffs, dtype=object)
        c = np.empty((len(mods), coeffs.shape[0]), dtype=np.uint64)
        for i, m in enumerate(mods):
            c[i] = (coeffs % m).astype(np.uint64)
        return Poly(mods, c)

    def copy(self):
        return Poly(self.mods, self.c.copy())

    def limbs(self, idx):
        return Poly([self.mods[i] for i in idx], self.c[list(idx)].copy())

    # Residues are below 2^62, so a + b and a + m - b fit in uint64 exactly.
    def __add__(self, o):
        assert self.mods == o.mods
        out = np.empty_like(self.c)
        for i, m in enumerate(self.mods):
            out[i] = (self.c[i] + o.c[i]) % np.uint64(m)
        return Poly(self.mods, out)

    def __sub__(self, o):
        assert self.mods == o.mods
        out = np.empty_like(self.c)
        for i, m in enumerate(self.mods):
            out[i] = (self.c[i] + np.uint64(m) - o.c[i]) % np.uint64(m)
        return Poly(self.mods, out)

    def __neg__(self):
        out = np.empty_like(self.c)
        for i, m in enumerate(self.mods):
            out[i] = (np.uint64(m) - self.c[i]) % np.uint64(m)
        return Poly(self.mods, out)

    def __mul__(self, o):
        """Ring product (negacyclic convolution, limb by limb)."""
        assert self.mods == o.mods
        out = np.empty_like(self.c)
        for i, m in enumerate(self.mods):
            out[i] = negacyclic_mul_limb(self.c[i], o.c[i], m)
        return Poly(self.mods, out)

    def scale(self, consts):
        """Multiply limb i by the integer consts[i] (or one integer for all limbs)."""
        if not isinstance(consts, (list, tuple)):
            consts = [consts] * len(self.mods)
        out = np.empty_like(self.c)
        for i, m in enumerate(self.mods):
            out[i] = vec_scale(self.c[i], consts[i], m)
        return Poly(self.mods, out)

    def __eq__(self, o):
        return self.mods == o.mods and np.array_equal(self.c, o.c)


def automorphism(poly: Poly, k: int) -> Poly:
    n = poly.n
    idx = (np.arange(n, dtype=np.int64) * k) % (2 * n)
    wrap = idx >= n
    dest = np.where(wrap, idx - n, idx)
    out = np.zeros_like(poly.c)
    for i, m in enumerate(poly.mods):
        src = poly.c[i]
        out[i, dest] = np.where(wrap, (np.uint64(m) - src) % np.uint64(m), src)
    return Poly(poly.mods, out)
