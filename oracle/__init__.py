"""CPU oracle for the coupled-cluster residual path.  TEST INFRASTRUCTURE.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark
may import anything from this package.  The device library never calls it
and shares no code with it; the only thing both sides use is the seeded
input generator in ``ccinputs``.

Contents
* ``integrals``  -- orientation of the six stored integral blocks into any
  of the sixteen occupied/virtual blocks of <pq||rs> (Hermiticity and
  antisymmetry of the two-body operator, Eq. ham2q).
* ``cc``         -- the unfactorised spin-orbital CCD (11 terms) and CCSD
  (48 terms) energy and amplitude equations, Eq. eq:amp, one einsum per
  diagram; the Jacobi iteration and the residual norm.
* ``projection`` -- brute force: <Phi_l| exp(-T) H_N exp(T) |Phi_0> in the
  determinant basis for tiny systems (the plain definition of Eq. eq:amp).
* ``mlp``        -- FP64 forward/backward of the amplitude-guess network.

All arithmetic is float64 / complex128.
"""
