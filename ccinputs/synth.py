"""Seeded synthetic coupled-cluster inputs: antisymmetrised two-electron
integrals and a diagonal Fock operator over o occupied and v virtual spin
orbitals.

The paper's molecular workloads (relativistic X2C integrals of H2O, LiH,
UF6 and CO) are not reproducible without their integral files, so random
integrals of the same algebraic structure stand in for them:

* <pq||rs> is antisymmetric under p<->q and under r<->s, and Hermitian
  under the exchange of the bra pair with the ket pair,
  <rs||pq> = conj(<pq||rs>)  (real case: plain pq<->rs symmetry).  These are
  the symmetries of the Hamiltonian's two-body part (Sec. "Electronic
  Hamiltonian", Eq. ham2q).  No further permutational symmetry is imposed.
* Every canonical element (p<q, r<s, pair(pq) <= pair(rs)) is an independent
  N(0, sigma^2) draw (complex: real and imaginary parts N(0, sigma^2/2) each,
  and the pair-diagonal elements <pq||pq> stay real).
* Orbital energies: occupied uniform in [-2, -0.5], virtual uniform in
  [0.5, 3], each sorted ascending; the Fock operator is diagonal.

Random draws are counter based, so any block of the integral tensor can be
produced on its own and agrees with every other block element for element:
the value of a canonical element is a function of (seed, canonical pair
indices) alone.  The counter hash is SplitMix64 (Steele, Lea & Flood,
OOPSLA 2014) and the normal deviates come from the Box-Muller transform
(Box & Muller, 1958).

Orbital numbering: occupied orbitals are 0..o-1 and virtual orbitals are
o..o+v-1 (the paper orders spaces by rising orbital energy).
"""
from __future__ import annotations

import concurrent.futures as _cf
import dataclasses
import os
from typing import Dict, Optional

import numpy as np

# NumPy releases the GIL inside its array loops, so row chunks of a block are
# filled concurrently; the values do not depend on the number of threads.
_THREADS = max(1, min(16, os.cpu_count() or 1))


def _parallel_rows(nrows: int, rows_per_chunk: int, fn) -> None:
    starts = list(range(0, nrows, rows_per_chunk))
    if _THREADS == 1 or len(starts) == 1:
        for r0 in starts:
            fn(r0)
        return
    with _cf.ThreadPoolExecutor(_THREADS) as ex:
        list(ex.map(fn, starts))

BASE_SEED = 240906759
SIGMA = 0.01

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_C1 = np.uint64(0xBF58476D1CE4E5B9)
_C2 = np.uint64(0x94D049BB133111EB)


def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 output function applied to state ``x`` (uint64 array)."""
    with np.errstate(over="ignore"):
        z = np.asarray(x, dtype=np.uint64) + _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _C1
        z = (z ^ (z >> np.uint64(27))) * _C2
        return z ^ (z >> np.uint64(31))


def _unit(z: np.ndarray) -> np.ndarray:
    """Top 53 bits of a uint64 mapped to the open interval (0, 1)."""
    return ((z >> np.uint64(11)).astype(np.float64) + 0.5) * (1.0 / 9007199254740992.0)


def _seed_key(seed: int) -> np.uint64:
    return splitmix64(np.array([seed], dtype=np.uint64))[0]


def pair_gaussian(seed: int, counter: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Two independent standard normal deviates per uint64 counter value."""
    key = _seed_key(seed)
    c2 = np.asarray(counter, dtype=np.uint64) * np.uint64(2)
    with np.errstate(over="ignore"):
        u1 = _unit(splitmix64(c2 + key))
        u2 = _unit(splitmix64(c2 + np.uint64(1) + key))
    r = np.sqrt(-2.0 * np.log(u1))
    ang = 2.0 * np.pi * u2
    return r * np.cos(ang), r * np.sin(ang)


def orbital_energies(o: int, v: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    rng = np.random.Generator(np.random.PCG64(seed))
    eo = np.sort(rng.uniform(-2.0, -0.5, size=o))
    ev = np.sort(rng.uniform(0.5, 3.0, size=v))
    return eo, ev


def _space(o: int, v: int, s: str) -> np.ndarray:
    if s == "o":
        return np.arange(o)
    if s == "v":
        return np.arange(o, o + v)
    if s == "g":
        return np.arange(o + v)
    raise ValueError(f"unknown orbital space {s!r}")


def _pairs(n: int, P: np.ndarray, Q: np.ndarray):
    """Canonical global pair index, sign, and a compact local numbering.

    For every (p, q) of the grid P x Q: the index of the unordered pair
    {p, q} in the lexicographic list of p<q pairs over n orbitals, the sign
    (+1 if p<q, -1 if p>q, 0 if p==q) and the position of that pair in the
    sorted list of distinct pairs met in this grid.
    """
    p = P[:, None]
    q = Q[None, :]
    lo = np.minimum(p, q).astype(np.int64)
    hi = np.maximum(p, q).astype(np.int64)
    g = lo * n - (lo * (lo + 1)) // 2 + (hi - lo - 1)
    sign = np.sign(q - p).astype(np.float64)
    g = np.where(sign == 0, -1, g).ravel()
    uniq, inv = np.unique(g, return_inverse=True)
    return uniq, inv.astype(np.int64), sign.ravel()


def _pair_matrix(seed: int, n: int, gl: np.ndarray, gr: np.ndarray, is_complex: bool, sigma: float):
    """G[x, y] = <pair gl[x] || pair gr[y]> for canonically ordered pairs."""
    NP = np.uint64(n * (n - 1) // 2)
    out_dtype = np.complex128 if is_complex else np.float64
    G = np.empty((gl.size, gr.size), dtype=out_dtype)
    a = gl[:, None]
    rows = max(1, (1 << 20) // max(1, gr.size))

    def fill(r0):
        aa = a[r0:r0 + rows]
        lo = np.minimum(aa, gr[None, :]).astype(np.uint64)
        hi = np.maximum(aa, gr[None, :]).astype(np.uint64)
        n1, n2 = pair_gaussian(seed, lo * NP + hi)
        if is_complex:
            diag = aa == gr[None, :]
            val = np.where(diag, n1 * sigma, n1 * (sigma / np.sqrt(2.0))) + 1j * np.where(
                diag, 0.0, n2 * (sigma / np.sqrt(2.0))
            )
            val = np.where(aa > gr[None, :], np.conj(val), val)
        else:
            val = n1 * sigma
        G[r0:r0 + rows] = val

    _parallel_rows(gl.size, rows, fill)
    # pairs that do not exist (p == q) carry index -1 and sign 0; zero them
    if gl.size and gl[0] < 0:
        G[0, :] = 0
    if gr.size and gr[0] < 0:
        G[:, 0] = 0
    return G


def integral_block(o: int, v: int, spaces: str, seed: int, is_complex: bool = False,
                   sigma: float = SIGMA, out: Optional[np.ndarray] = None) -> np.ndarray:
    """Dense block <pq||rs> with p in spaces[0], q in spaces[1], r in
    spaces[2], s in spaces[3] ('o', 'v' or 'g' for all orbitals), stored
    row-major as [p][q][r][s]."""
    n = o + v
    S = [_space(o, v, s) for s in spaces]
    gl, invl, sl = _pairs(n, S[0], S[1])
    gr, invr, sr = _pairs(n, S[2], S[3])
    G = _pair_matrix(seed, n, gl, gr, is_complex, sigma)
    shape = (S[0].size, S[1].size, S[2].size, S[3].size)
    dt = np.complex128 if is_complex else np.float64
    if out is None:
        out = np.empty(shape, dtype=dt)
    flat = out.reshape(S[0].size * S[1].size, S[2].size * S[3].size)
    rows = max(1, (1 << 22) // max(1, flat.shape[1]))

    def fill(r0):
        r1 = min(flat.shape[0], r0 + rows)
        blk = G[invl[r0:r1]][:, invr]
        blk *= sl[r0:r1, None]
        blk *= sr[None, :]
        flat[r0:r1] = blk

    _parallel_rows(flat.shape[0], rows, fill)
    return out


BLOCKS = ("oooo", "ooov", "oovv", "ovvo", "ovvv", "vvvv")


@dataclasses.dataclass
class CCSystem:
    """One synthetic system.  Integral blocks are generated on first use.

    Block conventions (row-major): oooo[i][j][k][l] = <ij||kl>,
    ooov[i][j][k][a] = <ij||ka>, oovv[i][j][a][b] = <ij||ab>,
    ovvo[i][a][b][j] = <ia||bj>, ovvv[i][a][b][c] = <ia||bc>,
    vvvv[a][b][c][d] = <ab||cd>.
    """
    o: int
    v: int
    seed: int
    is_complex: bool = False
    sigma: float = SIGMA
    f_oo: np.ndarray = None
    f_ov: np.ndarray = None
    f_vv: np.ndarray = None
    _blocks: Dict[str, np.ndarray] = dataclasses.field(default_factory=dict)

    @property
    def dtype(self):
        return np.complex128 if self.is_complex else np.float64

    def block(self, name: str) -> np.ndarray:
        if name not in self._blocks:
            self._blocks[name] = integral_block(self.o, self.v, name, self.seed,
                                                self.is_complex, self.sigma)
        return self._blocks[name]

    def drop(self, name: str) -> None:
        self._blocks.pop(name, None)

    def full_integrals(self) -> np.ndarray:
        """All of <pq||rs> over the o+v orbitals (small systems only)."""
        return integral_block(self.o, self.v, "gggg", self.seed, self.is_complex, self.sigma)

    def fock(self) -> np.ndarray:
        """Full (o+v) x (o+v) Fock matrix."""
        n = self.o + self.v
        F = np.zeros((n, n), dtype=self.dtype)
        F[:self.o, :self.o] = self.f_oo
        F[:self.o, self.o:] = self.f_ov
        F[self.o:, :self.o] = np.conj(self.f_ov.T)
        F[self.o:, self.o:] = self.f_vv
        return F


def make_system(o: int, v: int, seed: int = BASE_SEED, is_complex: bool = False,
                sigma: float = SIGMA) -> CCSystem:
    eo, ev = orbital_energies(o, v, seed)
    dt = np.complex128 if is_complex else np.float64
    return CCSystem(o=o, v=v, seed=seed, is_complex=is_complex, sigma=sigma,
                    f_oo=np.diag(eo).astype(dt), f_ov=np.zeros((o, v), dtype=dt),
                    f_vv=np.diag(ev).astype(dt))


def batch_shapes(count: int, seed: int = BASE_SEED + 1000, o_range=(4, 16), v_range=(20, 60)):
    """(o, v, seed) for a batch of independent systems: o and v integer
    uniform over the closed ranges; system s uses seed + s."""
    rng = np.random.Generator(np.random.PCG64(seed))
    os_ = rng.integers(o_range[0], o_range[1] + 1, size=count)
    vs_ = rng.integers(v_range[0], v_range[1] + 1, size=count)
    return [(int(a), int(b), seed + s) for s, (a, b) in enumerate(zip(os_, vs_))]


def random_amplitudes(o: int, v: int, seed: int, scale: float = 0.01, is_complex: bool = False):
    """Test amplitudes (not a coupled-cluster solution): t1[i][a] and
    t2[i][j][a][b] with independent N(0, scale^2) entries (complex: real and
    imaginary parts each N(0, scale^2)), t2 then made antisymmetric in (i, j)
    and in (a, b) by t2 <- P(ij) P(ab) x.  Drawn from PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))

    def draw(shape):
        x = rng.standard_normal(size=shape) * scale
        if is_complex:
            x = x + 1j * (rng.standard_normal(size=shape) * scale)
        return x

    t1 = draw((o, v))
    t2 = draw((o, o, v, v))
    t2 = t2 - t2.transpose(1, 0, 2, 3)
    t2 = t2 - t2.transpose(0, 1, 3, 2)
    return t1, t2
