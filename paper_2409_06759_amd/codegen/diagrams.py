"""Enumeration of distinct coupled-cluster diagrams.

A diagram of the projection <Phi_k| (H_N exp(T))_connected |Phi_0> (k-fold
excited bra, Eq. eq:amp) is fixed by

* the piece of the normal-ordered Hamiltonian: a one- or two-body vertex
  with `pd` particle and `hd` hole lines below it, contracted with cluster
  vertices, and `body - hd` particle and `body - pd` hole lines above it,
  open towards the bra;
* an unordered set of cluster vertices T_m, each given by the triple
  (m, cp, ch): excitation level m and the numbers of its particle and hole
  lines that end on the Hamiltonian vertex (cp + ch >= 1: connected).

All lines below the Hamiltonian vertex must be contracted (a normal-ordered
operator annihilates the reference otherwise), and the open lines must
supply exactly k particles and k holes.  Two diagrams are the same when
their Hamiltonian piece and sorted triples coincide, which is the
uniqueness condition of the integer-string representation (Kallay &
Surjan, J. Chem. Phys. 115, 2945 (2001); paper, Fig. "algo:gen": the
l-tuples of (level, connections, particle connections), mutually sorted).
The number of cluster vertices is at most four, the number of lines below
a two-body vertex.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, List, Sequence, Tuple


@dataclass(frozen=True, order=True)
class HPiece:
    body: int   # 1 (Fock) or 2 (antisymmetrised integrals)
    pd: int     # particle lines below (annihilated particles, contracted)
    hd: int     # hole lines below (annihilated holes, contracted)

    @property
    def pu(self) -> int:  # particle lines above (created particles, open)
        return self.body - self.hd

    @property
    def hu(self) -> int:  # hole lines above (created holes, open)
        return self.body - self.pd


@dataclass(frozen=True, order=True)
class TVertex:
    m: int   # excitation level of the cluster operator
    cp: int  # particle lines ending on the Hamiltonian vertex
    ch: int  # hole lines ending on the Hamiltonian vertex


@dataclass(frozen=True, order=True)
class Diagram:
    k: int                      # excitation level of the bra
    h: HPiece
    t: Tuple[TVertex, ...]      # sorted ascending

    def string(self) -> Tuple[int, ...]:
        """Integer string: projection level, Hamiltonian piece, then the
        (level, connections, particle connections) triples."""
        s = [self.k, self.h.body, self.h.pd, self.h.hd]
        for v in self.t:
            s += [v.m, v.cp + v.ch, v.cp]
        return tuple(s)


def hamiltonian_pieces() -> List[HPiece]:
    return [HPiece(body, pd, hd) for body in (1, 2) for pd in range(body + 1) for hd in range(body + 1)]


def enumerate_diagrams(k: int, levels: Sequence[int], max_vertices: int = 4) -> List[Diagram]:
    """All distinct connected diagrams of the k-fold projection with cluster
    operators of the given excitation levels.  Vertices are chosen in
    ascending order (multisets), each consuming at least one of the
    Hamiltonian vertex's lower lines, so at most pd + hd <= 4 of them."""
    verts = sorted(TVertex(m, cp, ch) for m in levels for cp in range(m + 1) for ch in range(m + 1)
                   if cp + ch >= 1)
    out = []

    def grow(h: HPiece, start: int, chosen: List[TVertex], rp: int, rh: int):
        if rp == 0 and rh == 0:
            if (h.pu + sum(v.m - v.cp for v in chosen) == k and h.hu + sum(v.m - v.ch for v in chosen) == k):
                out.append(Diagram(k, h, tuple(chosen)))
            return
        if len(chosen) == max_vertices:
            return
        for q in range(start, len(verts)):
            v = verts[q]
            if v.cp <= rp and v.ch <= rh:
                chosen.append(v)
                grow(h, q, chosen, rp - v.cp, rh - v.ch)
                chosen.pop()

    for h in hamiltonian_pieces():
        grow(h, 0, [], h.pd, h.hd)
    return out


METHODS = {"ccd": (2,), "ccsd": (1, 2), "ccsdt": (1, 2, 3), "ccsdtq": (1, 2, 3, 4), "ccsdtqp": (1, 2, 3, 4, 5)}


def method_diagrams(method: str) -> Dict[int, List[Diagram]]:
    """Diagrams of the energy (k = 0) and of every amplitude equation of the
    method; CCD has no singles equation."""
    levels = METHODS[method]
    ks = [0] + list(levels) if method != "ccd" else [0, 2]
    return {k: enumerate_diagrams(k, levels) for k in ks}


def diagram_count(method: str) -> int:
    return sum(len(v) for v in method_diagrams(method).values())
