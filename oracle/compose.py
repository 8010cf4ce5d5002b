"""Exact composition p(q(x)) over Z/pZ (the title problem; Section 1.2 notes
that divide-and-conquer schemes suit elements, such as polynomials, whose size
grows linearly with each multiplication).

The oracle expands the definition p(q(x)) = sum_k p_k q(x)^k by Hörner's rule
in Z/pZ[x] with Python integers (schoolbook products), and evaluates it at a
point t as p(q(t)) for Schwartz-Zippel checks.
"""
from __future__ import annotations


def poly_mul(a, b, p: int):
    out = [0] * (len(a) + len(b) - 1)
    for i, ai in enumerate(a):
        if ai == 0:
            continue
        for j, bj in enumerate(b):
            out[i + j] = (out[i + j] + ai * bj) % p
    return out


def compose(pc, qc, p: int):
    """Coefficients (index = exponent) of p(q(x)) mod p, length deg p * deg q + 1."""
    pc = [int(v) % p for v in pc]
    qc = [int(v) % p for v in qc]
    r = [pc[-1]]
    for k in range(len(pc) - 2, -1, -1):
        r = poly_mul(r, qc, p)
        r[0] = (r[0] + pc[k]) % p
    want = (len(pc) - 1) * (len(qc) - 1) + 1
    r = r + [0] * (want - len(r))
    return r[:want]


def horner_at(coeffs, t: int, p: int) -> int:
    acc = 0
    for c in reversed(list(coeffs)):
        acc = (acc * t + int(c)) % p
    return acc


def compose_at(pc, qc, t: int, p: int) -> int:
    """p(q(t)) mod p."""
    return horner_at(pc, horner_at(qc, t, p), p)
