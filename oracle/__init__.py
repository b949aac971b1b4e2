"""CPU oracle for the exact multi-modular integer matrix product and the Smith
normal form.

TEST INFRASTRUCTURE ONLY.  This package is plain, slow and written to be
checked by eye against the paper's definitions.  Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
product path (the HIP library and its Python binding) never does, and shares
no code, header, table or constant generator with it.

Contents
--------
primes.py  -- the basis: the largest primes below a bound (Section 3.1,
              "Exact double-precision accumulation").
rns.py     -- residue reduction, modular matrix product, CRT reconstruction,
              the exact integer product, two's-complement word encoding
              (Section 3.1).
smith.py   -- exact determinant (fraction-free elimination) and the Smith
              normal form by gcd elimination modulo the determinant
              (Section 1, the definition of S).
modmatmul_ref.c -- the same modular and exact products as plain C loops, for
              sizes Python cannot reach (built by ``oracle.native``).

Every function states which passage it follows.  Where the paper is silent
the reading taken is written next to the code.
"""
