"""NumPy evaluation of the diagram generator's derived terms.  TEST CODE.

Used by the tests only, to check the derivation and the GPU execution of
generated contraction lists against the terms they came from.
"""
from __future__ import annotations

from typing import Callable, Dict, List

import numpy as np

from paper_2409_06759_amd.codegen.terms import Term


def evaluate(terms: List[Term], fock: Callable[[str], np.ndarray], ints: Callable[[str], np.ndarray],
             amps: Dict[int, np.ndarray]) -> np.ndarray:
    """Sum of the terms of one equation.  `fock(block)` returns f restricted
    to a two-letter block of 'o'/'v' (e.g. 'vo' = f_ai), `ints(block)` the
    antisymmetrised integrals <pq||rs> of a four-letter block, `amps[m]`
    the amplitudes t_{i1..im}^{a1..am} (holes first).  Returns a scalar for
    the energy, else R[i1..ik, a1..ak]."""
    total = None
    for t in terms:
        ops = []
        for x in t.tensors:
            if x.name == "f":
                ops.append(fock(x.block))
            elif x.name == "v":
                ops.append(ints(x.block))
            else:
                m = int(x.name[1:])
                if m not in amps or amps[m] is None:
                    break
                ops.append(amps[m])
        else:
            t0 = np.einsum(t.einsum(), *ops, optimize=True)
            k = len(t.ext_h)
            if k == 0:
                val = t0
            else:
                acc = np.zeros_like(t0)
                for sgn, sh, sp in t.perms:
                    acc = acc + sgn * np.transpose(t0, list(sh) + [k + q for q in sp])
                val = acc / t.stab
            val = float(t.coeff) * val
            total = val if total is None else total + val
    return total
