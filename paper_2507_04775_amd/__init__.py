"""MI355X (gfx950) RNS-CKKS key-switching library.

- ``build``  : compiles csrc/ into the in-tree shared library libckks.so.
- ``ckks``   : Python binding of the C ABI in include/ckks.h (imports fail when
               the library is not built; there is no CPU fallback).
- ``inputs`` : seeded synthetic inputs (primes, residues, slots).
"""
