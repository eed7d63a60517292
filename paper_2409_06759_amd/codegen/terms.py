"""Interpretation of diagrams into explicit tensor terms.

For a diagram (see `diagrams`) one Goldstone representative is built as a
directed line graph:

* the two-body vertex <pq||rs> is split into half-vertices (p out, r in)
  and (q out, s in), the one-body vertex f_pq is one half-vertex (p out,
  q in); out-slots carry first the open particle lines, then the
  contracted hole lines; in-slots first the contracted particle lines, then
  the open hole lines;
* the cluster vertex t_{i1..im}^{a1..am} is split into half-vertices
  (a_s out, i_s in); its first cp particle lines and first ch hole lines
  end on the Hamiltonian vertex, matched to its slots in vertex order;
* each open particle line a_k and open hole line i_k of the bra are joined
  in a node of their own (the line starting in i_k ends in a_k: the pairing
  of Phi_{i1..ik}^{a1..ak} = a+_a1 .. a+_ak a_ik .. a_i1 |Phi_0>).

Every node then has one incoming and one outgoing line, the lines form a
permutation, and its cycles are the loops.  The term is

    sign * weight * A[ H x prod_v t_v ] / stab,

sign = (-1)^(hole lines + loops); weight = prod_v 1/(cp_v! ch_v!) (equivalent
lines between a cluster vertex and the Hamiltonian vertex) times
1/n! for each set of n identical cluster vertices; A antisymmetrises over
the open particle labels and over the open hole labels; stab = prod over
vertices of (open particle lines)! (open hole lines)!, the permutations
that only reorder open lines of one vertex, so that A/stab is the sum of
the distinct permutation-operator images (P(ij), P(ab), ...).  These are
the textbook interpretation rules (e.g. Shavitt & Bartlett, Many-Body
Methods in Chemistry and Physics, ch. 9-10), written out for one
representative; the antisymmetry of integrals and amplitudes makes every
representative give the same term.
"""
from __future__ import annotations

import itertools
import math
from collections import Counter
from dataclasses import dataclass, field
from fractions import Fraction
from typing import Dict, List, Tuple

from .diagrams import Diagram, method_diagrams

EXT_P, EXT_H = "abcdefgh", "ijklmnop"
INT_P, INT_H = "ABCDEFGHIJKL", "MNOPQRSTUVWX"


@dataclass
class Tensor:
    name: str    # "f", "v" or "t<m>"
    block: str   # f/v: space of each slot ('o' hole, 'v' particle); t: ""
    idx: str     # index letters in slot order (t: holes then particles)


@dataclass
class Term:
    diagram: Diagram
    coeff: Fraction            # sign * weight
    tensors: List[Tensor]
    ext_h: str                 # open hole labels, output order
    ext_p: str                 # open particle labels, output order
    stab: int
    loops: int = 0
    holes: int = 0
    perms: List[Tuple[int, Tuple[int, ...], Tuple[int, ...]]] = field(default_factory=list)

    def einsum(self) -> str:
        return ",".join(t.idx for t in self.tensors) + "->" + self.ext_h + self.ext_p

    def text(self) -> str:
        """Readable form: coefficient, the number of distinct permutation
        images summed (P<n>, as P(ij), P(ab), ... would), then the tensors.
        Upper-case letters are summed."""
        c = self.coeff
        s = ("-" if c < 0 else "+") + ("" if abs(c) == 1 else f"{abs(c)} ")
        k = len(self.ext_h)
        images = math.factorial(k) ** 2 // self.stab if k else 1
        if images > 1:
            s += f"P{images} "
        parts = []
        for t in self.tensors:
            if t.name == "v":
                parts.append(f"<{t.idx[0]}{t.idx[1]}||{t.idx[2]}{t.idx[3]}>")
            elif t.name == "f":
                parts.append(f"f_{t.idx[0]}{t.idx[1]}")
            else:
                m = len(t.idx) // 2
                parts.append(f"t_{t.idx[:m]}^{t.idx[m:]}")
        return s + " ".join(parts)


def _letters(pool: str, n: int, start: int) -> List[str]:
    if start + n > len(pool):
        raise ValueError("not enough index letters")
    return list(pool[start:start + n])


def interpret(d: Diagram) -> Term:
    h, k = d.h, d.k
    ip = ih = 0
    # ---- slots of the Hamiltonian vertex --------------------------------
    out_slots: List[Tuple[str, int]] = [("P", -1)] * h.pu + [("h", -1)] * h.hd   # open particle / contracted hole
    in_slots: List[Tuple[str, int]] = [("p", -1)] * h.pd + [("H", -1)] * h.hu    # contracted particle / open hole
    # ---- contracted lines: cluster vertex slots in vertex order ------------
    cp_list = [(v, s) for v, tv in enumerate(d.t) for s in range(tv.cp)]
    ch_list = [(v, s) for v, tv in enumerate(d.t) for s in range(tv.ch)]
    assert len(cp_list) == h.pd and len(ch_list) == h.hd
    # line records: letter, kind ('p'/'h'), from-node, to-node
    lines: Dict[str, Tuple[str, Tuple, Tuple]] = {}
    t_a: Dict[Tuple[int, int], str] = {}
    t_i: Dict[Tuple[int, int], str] = {}
    h_out: List[str] = [""] * h.body
    h_in: List[str] = [""] * h.body
    for n, (v, s) in enumerate(cp_list):        # particle: T(v,s) -> H in-slot
        L = INT_P[ip]; ip += 1
        slot = n
        lines[L] = ("p", ("T", v, s), ("H", slot))
        t_a[(v, s)] = L
        h_in[slot] = L
    for n, (v, s) in enumerate(ch_list):        # hole: H out-slot -> T(v,s)
        L = INT_H[ih]; ih += 1
        slot = h.pu + n
        lines[L] = ("h", ("H", slot), ("T", v, s))
        t_i[(v, s)] = L
        h_out[slot] = L
    # ---- open lines and their labels -------------------------------------
    p_src: List[Tuple] = [("H", s) for s in range(h.pu)]
    p_src += [("T", v, s) for v, tv in enumerate(d.t) for s in range(tv.cp, tv.m)]
    h_dst: List[Tuple] = [("H", h.pd + s) for s in range(h.hu)]
    h_dst += [("T", v, s) for v, tv in enumerate(d.t) for s in range(tv.ch, tv.m)]
    assert len(p_src) == k and len(h_dst) == k
    for kk, node in enumerate(p_src):
        L = EXT_P[kk]
        lines[L] = ("p", node, ("X", kk))
        if node[0] == "H":
            h_out[node[1]] = L
        else:
            t_a[(node[1], node[2])] = L
    for kk, node in enumerate(h_dst):
        L = EXT_H[kk]
        lines[L] = ("h", ("X", kk), node)
        if node[0] == "H":
            h_in[node[1]] = L
        else:
            t_i[(node[1], node[2])] = L
    # ---- loops: follow out-lines node to node ------------------------------
    out_of: Dict[Tuple, str] = {}
    for L, (_, frm, _) in lines.items():
        assert frm not in out_of
        out_of[frm] = L
    seen, loops = set(), 0
    for start in out_of:
        if start in seen:
            continue
        loops += 1
        node = start
        while node not in seen:
            seen.add(node)
            node = lines[out_of[node]][2]
    holes = sum(1 for kind, _, _ in lines.values() if kind == "h")
    sign = -1 if (holes + loops) % 2 else 1
    # ---- weight -----------------------------------------------------------
    w = Fraction(1)
    for tv in d.t:
        w /= math.factorial(tv.cp) * math.factorial(tv.ch)
    for _, n in Counter(d.t).items():
        w /= math.factorial(n)
    # ---- tensors ------------------------------------------------------------
    space = lambda L: "o" if L in EXT_H or L in INT_H else "v"  # noqa: E731
    tensors = []
    if h.body == 2:
        idx = h_out[0] + h_out[1] + h_in[0] + h_in[1]
        tensors.append(Tensor("v", "".join(space(c) for c in idx), idx))
    else:
        idx = h_out[0] + h_in[0]
        tensors.append(Tensor("f", "".join(space(c) for c in idx), idx))
    for v, tv in enumerate(d.t):
        idx = "".join(t_i[(v, s)] for s in range(tv.m)) + "".join(t_a[(v, s)] for s in range(tv.m))
        tensors.append(Tensor(f"t{tv.m}", "", idx))
    # ---- antisymmetriser normalisation -----------------------------------------
    stab = math.factorial(h.pu) * math.factorial(h.hu)
    for tv in d.t:
        stab *= math.factorial(tv.m - tv.cp) * math.factorial(tv.m - tv.ch)
    perms = []
    for sp in itertools.permutations(range(k)):
        for sh in itertools.permutations(range(k)):
            perms.append((_parity(sp) * _parity(sh), sh, sp))
    return Term(d, Fraction(sign) * w, tensors, EXT_H[:k], EXT_P[:k], stab, loops, holes, perms)


def _parity(p) -> int:
    p = list(p)
    s = 1
    for i in range(len(p)):
        while p[i] != i:
            j = p[i]
            p[i], p[j] = p[j], p[i]
            s = -s
    return s


def equations(method: str) -> Dict[int, List[Term]]:
    """Terms of the energy (key 0) and of each amplitude equation."""
    return {k: [interpret(d) for d in ds] for k, ds in method_diagrams(method).items()}
