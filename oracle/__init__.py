"""CPU oracle for fast polynomial evaluation through evaluation trees.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct CPU
implementation of what the GPU library computes.  Only the test-suite, the
smoke check of the package entry point and the CPU-baseline leg of the
benchmark may import, call, link or execute anything in it; the product path
never does, and shares no code with it.

Contents (each function cites the passage of the paper it follows):

* ``schemes``  the function schemes D, H, E and B (Section 1.1, 1.2).
* ``tree``     an independent builder of the evaluation tree T_p^f, its
               recursive value (Section 1, Definition of evaluation tree), the
               lazy height (Section 1.3) and the coefficient walk (Section 2.1).
* ``exact``    the plain definition p(x) = sum c_m x^m: exact rationals,
               exact residues mod p, double-double Hörner, fsum closed forms.
* ``compose``  exact composition p(q(x)) over Z/pZ by schoolbook expansion.
* ``interval`` the tree's value over a box with exact interval operations
               (the interval coefficient type of the Abstract).
* ``bigint``   p(x) over the natural numbers at big-integer points (the
               Benchmarks section's workload), with 16-bit limb conversion.
* ``native``   the same definitions in plain C for full-size samples and for
               the timed CPU baseline (built by ``oracle/build_native.sh``).

Parity unpinned: the Estrin lazy height printed in the example of Section 1.3
(the text and the definition disagree; the definition is pinned).
"""
