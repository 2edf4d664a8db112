"""CPU oracle for the ciphertext branch of bi-CryptoNets (arXiv 2402.01296).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import or call anything here; the
product path never does.

The oracle is written for obviousness, not speed: polynomials are Python lists
of exact integers, every ring operation is its textbook definition (a
negacyclic product over Z computed with one big-integer multiplication by
Kronecker substitution), and every rounding is an exact nearest-integer
rounding on rationals.  It shares no code with the GPU path; the only shared
module is ``synthetic`` (seeded random inputs, no scheme arithmetic).

The paper runs CKKS inside SEAL (Experiments section; appendix "CKKS
Scheme").  The workloads here are integer-quantised and need
decryptions that *equal* the integer network, so the oracle implements the
exact-arithmetic sibling of that scheme, BFV with CRT batching, using the same
operation set the appendix lists: E, D, Add(c,u), Add(c1,c2), Mult(c,u),
Mult(c1,c2), Rot(c,r).

Modules
-------
nt        number theory: primes, roots of unity, CRT
ring      Z[X]/(X^N+1) arithmetic, automorphisms, NTT by its definition
encoder   CRT batching (slot vectors <-> plaintext polynomials mod t)
bfv       keys, encryption, decryption, noise budget, homomorphic operations
network   the integer-quantised network Dec(Eval(.)) must equal
programs  the homomorphic programs of the three workloads
params    the parameter sets

Parity status: every function is pinned by a test in ``tests/test_oracle_*``
except where its docstring says "parity unpinned".
"""
