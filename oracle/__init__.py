"""CPU FP64 oracle for the multi-shifted BiCG resonant-spectrum path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import anything from this package.  The
HIP library never calls it and shares no code with it; the two sides meet only
through the seeded inputs of ``workloads``.

Everything here is a plain, slow, obviously-checkable transcription of the
paper's definitions in float64 / complex128 with NumPy and SciPy:

* ``hubbard``  -- fixed-(N_up, N_dn) basis and the Hubbard / core-hole
  Hamiltonians of Eqs. ``Hubbard`` and ``intermediate_H``, built by applying
  fermion operators to occupation bit strings with Jordan-Wigner signs.
* ``groundstate`` -- (E_G, |G>) by dense diagonalisation or Lanczos with full
  reorthogonalisation.
* ``solve`` -- the intermediate state of Eq. ``intermediateState`` by direct
  solves per shift, and the multi-shift COCG recurrence of Appendix D
  (Algorithm 1) in the corrected reading.
* ``spectrum`` -- the Kramers-Heisenberg intensity of Eq. ``kramers1`` by the
  Lehmann sum, by a Lanczos continued fraction, and by correction vectors.
* ``mlp`` -- float64 forward/backward, Adam and the ensemble fallback rule of
  the surrogate network of the learned form (textbook definitions; the paper
  has no network), with an option that applies the GPU's bfloat16 roundings.

Parity status of each function is stated in its docstring; every function is
pinned by ``tests/test_oracle_*.py`` against closed forms, invariants or brute
force, except where a docstring says "parity unpinned".
"""
from . import hubbard, groundstate, solve, spectrum, mlp  # noqa: F401
