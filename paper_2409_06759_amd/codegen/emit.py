"""Binary contraction lists for the engine from the derived equations.

Each derived singles/doubles term is a product of one Hamiltonian tensor
and cluster amplitudes.  It is evaluated as a sequence of binary
contractions (the order with the fewest floating-point operations at the
given o, v, found by trying every pairing), writing intermediates G<n> and
finally accumulating into the engine's residual accumulators: R1 for the
singles, and for the doubles XP / Xij / Xab / Xr according to which
antisymmetriser the term carries (none, P(ij), P(ab), both).  Integral
blocks are mapped onto the six stored orientations with antisymmetry
(<pq||rs> = -<qp||rs> = -<pq||sr>) and Hermiticity (<pq||rs> = conj <rs||pq>).
Intermediates formed identically by several terms are computed once.
The text is the input of cc_plan_create_ops.
"""
from __future__ import annotations

import itertools
from typing import Dict, List, Optional, Tuple

from .terms import Term, equations

STORED = ("oooo", "ooov", "oovv", "ovvo", "ovvv", "vvvv")
OCC, VIR = "ijklmn", "abcdefgh"


def _space(c: str) -> str:
    return "o" if c in OCC else "v"


def map_integral(block: str, idx: str) -> Tuple[str, str, int, bool]:
    """(stored block, labels in its slot order, sign, conjugate) for <idx>
    of the given block."""
    p, q, r, s = idx
    forms = []
    for herm in (False, True):
        a, b, c, d = (r, s, p, q) if herm else (p, q, r, s)
        for sw1 in (False, True):
            for sw2 in (False, True):
                x, y = (b, a) if sw1 else (a, b)
                z, w = (d, c) if sw2 else (c, d)
                sign = (-1) ** (int(sw1) + int(sw2))
                forms.append((x + y + z + w, sign, herm))
    for labels, sign, herm in forms:
        sp = "".join(_space(c) for c in labels)
        if sp in STORED:
            return sp, labels, sign, herm
    raise ValueError(f"no stored orientation for {block}")


def map_fock(block: str, idx: str) -> Tuple[str, str, bool]:
    if block == "vo":  # f_ai = conj f_ia
        return "fov", idx[1] + idx[0], True
    return {"oo": "foo", "ov": "fov", "vv": "fvv"}[block], idx, False


def _rename(term: Term) -> Dict[str, str]:
    """Engine labels: open lines keep i, j / a, b; summed holes k..n, summed
    particles c..h."""
    used = set(term.ext_h + term.ext_p)
    free_h = [c for c in OCC if c not in used]
    free_p = [c for c in VIR if c not in used]
    m = {c: c for c in used}
    for t in term.tensors:
        for c in t.idx:
            if c in m:
                continue
            pool = free_h if c.isupper() and c >= "M" else free_p
            if not pool:
                raise ValueError("too many summed indices for the engine's labels")
            m[c] = pool.pop(0)
    return m


def _target(term: Term) -> Tuple[str, str]:
    k = len(term.ext_h)
    if k == 1:
        return "R1", "ia"
    if k == 3:
        return "Y3", "ijkabc"  # R3 = full antisymmetriser of Y3 (terms pre-divided by stab)
    if k != 2:
        raise ValueError("the engine evaluates up to triples")
    same_p = any("a" in t.idx and "b" in t.idx for t in term.tensors)
    same_h = any("i" in t.idx and "j" in t.idx for t in term.tensors)
    if same_p and same_h:
        return "XP", "ijab"
    if same_p:
        return "Xij", "ijab"
    if same_h:
        return "Xab", "ijab"
    return "Xr", "ijab"


def _best_order(ops: List[str], out: str, dims: Dict[str, int]):
    """Cheapest sequence of pairwise merges: list of (i, j, labels) over a
    shrinking operand list; returns (flops, steps)."""
    best = [None]

    def rec(cur: List[str], steps, flops):
        if best[0] is not None and flops >= best[0][0]:
            return
        if len(cur) == 1:
            best[0] = (flops, list(steps))
            return
        for i, j in itertools.combinations(range(len(cur)), 2):
            rest = [cur[q] for q in range(len(cur)) if q not in (i, j)]
            keep = set(out) | set("".join(rest))
            union = []
            for c in cur[i] + cur[j]:
                if c not in union:
                    union.append(c)
            res = "".join(c for c in union if c in keep)
            if len(rest) == 0:
                res = out
            if len(res) > 6:  # the engine's tensors have rank <= 6
                continue
            f = 2
            for c in union:
                f *= dims[c]
            rec(rest + [res], steps + [(i, j, res)], flops + f)

    rec(list(ops), [], 0)
    return best[0]


def _canon(*label_strings: str) -> Tuple[str, ...]:
    """Relabel jointly by first appearance, holes to i, j, ... and particles
    to a, b, ..., so that equal contractions get equal keys."""
    m: Dict[str, str] = {}
    nh = npart = 0
    out = []
    for ls in label_strings:
        r = []
        for c in ls:
            if c not in m:
                if c in OCC:
                    m[c] = OCC[nh]
                    nh += 1
                else:
                    m[c] = VIR[npart]
                    npart += 1
            r.append(m[c])
        out.append("".join(r))
    return tuple(out)


def op_list(method: str, o: int = 32, v: int = 160, share: bool = True) -> str:
    """The cc_plan_create_ops text of the method's singles and doubles
    (and triples, accumulated into Y3, for CCSDT).
    With `share`, an intermediate that an earlier term already formed (the
    same operands contracted the same way, up to relabelling) is reused."""
    formed: Dict[Tuple, str] = {}
    eq = equations(method)
    dims = {c: o for c in OCC}
    dims.update({c: v for c in VIR})
    work: List[str] = []
    ops: List[str] = []
    ng = 0
    for k in sorted(eq):
        if k == 0:
            continue  # the engine computes the energy itself
        for n, term in enumerate(eq[k]):
            ren = _rename(term)
            coeff = float(term.coeff)
            operands = []  # (name, labels, conj)
            for t in term.tensors:
                idx = "".join(ren[c] for c in t.idx)
                if t.name == "v":
                    name, lab, sign, conj = map_integral(t.block, idx)
                    coeff *= sign
                    operands.append((name, lab, conj))
                elif t.name == "f":
                    name, lab, conj = map_fock(t.block, idx)
                    operands.append((name, lab, conj))
                else:
                    if t.name not in ("t1", "t2", "t3"):
                        raise ValueError("the engine stores t1, t2 and t3 only")
                    operands.append((t.name, idx, False))
            target, tl = _target(term)
            if target == "Y3":
                coeff /= term.stab
            tag = f"g{k}_{n}"
            if len(operands) == 1:
                name, lab, conj = operands[0]
                ops.append(f"op {tag} {target} {tl} {coeff!r} {name} {lab} - -" + (" conjA" if conj else ""))
                continue
            best = _best_order([x[1] for x in operands], tl, dims)
            if best is None:
                raise ValueError(f"no contraction order within rank 6 for {term.text()}")
            flops, steps = best
            cur = list(operands)
            for s_i, (i, j, res) in enumerate(steps):
                a, b = cur[i], cur[j]
                last = s_i == len(steps) - 1
                if last:
                    cname, alpha = target, coeff
                    res = tl
                else:
                    k1 = (a[0], a[2], b[0], b[2]) + _canon(a[1], b[1], res)
                    k2 = (b[0], b[2], a[0], a[2]) + _canon(b[1], a[1], res)
                    key = min(k1, k2)
                    if share and key in formed:
                        cur = [cur[q] for q in range(len(cur)) if q not in (i, j)] + [(formed[key], res, False)]
                        continue
                    ng += 1
                    cname, alpha = f"G{ng}", 1.0
                    formed[key] = cname
                    work.append(f"work {cname} {''.join(_space(c) for c in res)}")
                flags = (" conjA" if a[2] else "") + (" conjB" if b[2] else "")
                ops.append(f"op {tag}{'' if last else '_' + str(s_i)} {cname} {res} {alpha!r} "
                           f"{a[0]} {a[1]} {b[0]} {b[1]}{flags}")
                cur = [cur[q] for q in range(len(cur)) if q not in (i, j)] + [(cname, res, False)]
    head = [f"# {method.upper()} singles and doubles from the diagram generator ({len(ops)} ops)"]
    return "\n".join(head + work + ops) + "\n"
