"""CPU oracle for SIMD-aware homomorphic compression (arXiv 2408.17063).

THIS PACKAGE IS TEST INFRASTRUCTURE. Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import or run it; the library
(paper_2408_17063_amd) never does, and shares no code, tables or constants
with it. It is a plain, slow, exact implementation of what the library
computes, written from the paper:

* params.py     -- primes, scaling factor and slot root (readings of Sec. 6.1)
* rng.py        -- seeded SHAKE-128 framing and the samplers
* ring.py       -- RNS polynomials; ring products via ring.c (exact 128-bit)
* slots.py      -- the SIMD slot map Z_p[X]/(X^n+1) = Z_p^(2 x n/2) (Sec. 5.1)
* bfv.py        -- BFV with hybrid key switching, plain and hoisted rotations
* compress.py   -- Mask and Comp (Alg. 7; Eq. (1); Sec. 5.2), plus the plain
                   Vandermonde product that a compressed ciphertext decrypts to
* decompress.py -- ReconstIdx (Alg. 1), Reconst (Alg. 4), Decomp (Alg. 6)

Parity status: the decrypted output, the decompressed sparse vector and every
building block are pinned by tests against definitions that do not go through
this code (brute-force convolution, closed-form slot evaluation, exact CRT,
the Vandermonde product, brute-force subsets). The ciphertext bits themselves
are fixed only by the readings listed in each module: the paper prints no
ciphertext, so beyond those readings they are "parity unpinned".
"""
