"""Plain CPU oracle (complex128 / float64) for the TeD-Q hot path.

TEST INFRASTRUCTURE ONLY. Nothing in the product path imports, calls or links this
package; only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use it. It shares no code with the HIP path: its gate matrices,
network construction, contraction order and reductions are written here. The only
shared module is ``paper_2301_05451_amd.workloads`` (seeded circuit structure and
random draws, none of the simulation arithmetic).

Modules:

* :mod:`oracle.sv`   -- state-vector evolution, Z-string expectation values, brute-force
  full unitaries, parameter-shift and central finite-difference gradients.
* :mod:`oracle.tn`   -- doubled (ket + bra) tensor network of a circuit expectation
  value, pairwise einsum contraction with and without slicing, QAOA light cones.
* :mod:`oracle.mlp`  -- float64 MLP forward, manual backward and Adam (parity unpinned
  by the paper; pinned by finite differences, Adam's closed-form first step and forward
  invariants: odd symmetry, the small-weight linear limit, biases as weights on a constant
  unit, an affine output layer, independent rows).
"""
