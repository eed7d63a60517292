"""Integral blocks in every occupied/virtual orientation.  TEST INFRASTRUCTURE.

The generator stores six canonical blocks of <pq||rs> (oooo, ooov, oovv,
ovvo, ovvv, vvvv).  Every other block follows from the two symmetries of the
two-body part of the Hamiltonian (Eq. ham2q): antisymmetry within the bra
pair and within the ket pair, and Hermiticity <rs||pq> = conj(<pq||rs>).
"""
from __future__ import annotations

import numpy as np


def _herm(x):
    """<rs||pq> from <pq||rs>: swap bra and ket pairs and conjugate."""
    return np.conj(x.transpose(2, 3, 0, 1))


class Integrals:
    """Holds the canonical blocks; ``get('vvvo')`` returns <ab||ci>."""

    def __init__(self, blocks: dict, o: int, v: int):
        self.o, self.v = o, v
        self._c = blocks

    @classmethod
    def from_system(cls, sysm):
        return cls({b: sysm.block(b) for b in ("oooo", "ooov", "oovv", "ovvo", "ovvv", "vvvv")},
                   sysm.o, sysm.v)

    def get(self, spaces: str) -> np.ndarray:
        c = self._c
        if spaces in c:
            return c[spaces]
        if spaces == "oovo":      # <ij||ak> = -<ij||ka>
            return -c["ooov"].transpose(0, 1, 3, 2)
        if spaces == "ovoo":      # <ia||jk> = conj(<jk||ia>)
            return _herm(c["ooov"])
        if spaces == "vooo":      # <ai||jk> = -<ia||jk>
            return -self.get("ovoo").transpose(1, 0, 2, 3)
        if spaces == "ovov":      # <ia||jb> = -<ia||bj>
            return -c["ovvo"].transpose(0, 1, 3, 2)
        if spaces == "voov":      # <ai||jb> = <ia||bj>
            return c["ovvo"].transpose(1, 0, 3, 2)
        if spaces == "vovo":      # <ai||bj> = -<ia||bj>
            return -c["ovvo"].transpose(1, 0, 2, 3)
        if spaces == "vvoo":      # <ab||ij> = conj(<ij||ab>)
            return _herm(c["oovv"])
        if spaces == "vovv":      # <ai||bc> = -<ia||bc>
            return -c["ovvv"].transpose(1, 0, 2, 3)
        if spaces == "vvov":      # <ab||ic> = conj(<ic||ab>)
            return _herm(c["ovvv"])
        if spaces == "vvvo":      # <ab||ci> = -<ab||ic>
            return -self.get("vvov").transpose(0, 1, 3, 2)
        raise KeyError(spaces)
