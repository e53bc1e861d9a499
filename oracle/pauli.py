"""Letter <-> mask encoding of Pauli strings (oracle side).

Supplementary Methods, "Pauli-string bit representation": an n-qubit string
is two integers (p1, p2); bit q of p1 is set iff the letter on qubit q is X
or Y (not diagonal), bit q of p2 iff it is Y or Z.  Qubits run from least to
most significant ("Software implementation"), so the first tensor factor is
qubit 0 / bit 0.  In this package p1 is called x and p2 is called z.
"""
from __future__ import annotations


def label_to_masks(label: str):
    """Masks (x, z) of a string of letters; character q acts on qubit q."""
    x = z = 0
    for q, ch in enumerate(label.upper()):
        if ch in "XY":
            x |= 1 << q
        if ch in "YZ":
            z |= 1 << q
        if ch not in "IXYZ":
            raise ValueError(f"bad Pauli letter {ch!r}")
    return x, z


def masks_to_label(x: int, z: int, n: int) -> str:
    out = []
    for q in range(n):
        xb, zb = (x >> q) & 1, (z >> q) & 1
        out.append("IZXY"[xb * 2 + zb])
    return "".join(out)
