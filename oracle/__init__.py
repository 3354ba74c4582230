"""Oracle: a plain, slow, obviously correct complex128 CPU state-vector simulator.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  The
product library (``paper_2203_08826_amd``) never imports, links or calls it, and
the two share no code: no kernels, headers, helpers, gate tables or constant
generators.  The only code both sides use is the seeded input generators in
``workloads/``, which hold none of the simulation arithmetic.

What is here, each written from the paper's statement of the problem:

* ``sim.c`` (built to ``_build/liboracle.so`` by ``oracle.build``): Eq. 1 of
  the paper's introduction as an out-of-place loop over output amplitudes.
* ``gates``: gate matrices from their textbook definitions.
* ``statevec``: circuits, probabilities, norms, inner products, infidelity,
  the transverse-field Ising energy, and the full Kronecker-product checker.
* ``fusion``: greedy gate fusion as described in the gate-fusion section of
  the benchmarks (Sec. 3.2), with the gate/depth counts of the paper's table of
  benchmark circuits.
* ``adjoint``: adjoint-method gradients, parameter shift, finite differences.
* ``mlp``: float64 numpy forward/backward/Adam of the fusion cost model.
* ``measure``: collapse and re-normalisation onto a measurement outcome,
  inverse-CDF shot sampling and Metropolis shot frequencies (Sec. 2).
* ``evolution``: adiabatic evolution by exponentiating the dense Hamiltonian
  at every step (Sec. 3.3).
* ``density``: density matrices, U rho U^dagger with full operators, Kraus
  channels, probabilities of the diagonal (Sec. 2).

Every function states the passage it follows.  Functions with nothing but the
code itself to check them against say "parity unpinned".
"""
