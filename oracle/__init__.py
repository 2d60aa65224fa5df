"""CPU oracle for the lifted layer-splitting step -- TEST INFRASTRUCTURE ONLY.

Plain, slow, FP64 NumPy/SciPy implementation of what the hot path computes,
written from Wang, Chen, Zhou & Zhou, "Layer-splitting methods for
time-dependent Schroedinger equations of incommensurate systems"
(arXiv 2103.14897).  Only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import it; the product path (the HIP library and its
Python binding) never does and shares no code with it.

Modules
-------
lifted       lattices, reciprocal lattices, the lifted index set I, fibres,
             and the dense lifted matrices D, V^1, V^2 (Secs. 2-3, eqs. 3.4-3.6)
splitting    fibre Hamiltonians, exact fibre propagators via eigh, the kinetic
             phase, and the Lie / Strang layer-splitting compositions
             (Sec. 4.2, App. A)
observables  mass (eq. 2.3 via orthonormality 3.1), energy (eq. 2.4), fibre masses
reference    brute-force exponentials of the full lifted Hamiltonian and a
             direct commensurate-supercell computation used to pin the rest
multilayer   index set, fibres, fibre Hamiltonians and Lie / Strang / Yoshida layer
             splitting for L >= 2 layers (the generalisation of Secs. 2-4), with exact,
             backward-Euler or Crank-Nicolson fibre sub-steps
blocks       lifted systems whose layers share index blocks (Example 3 of Sec. 5:
             a direction periodic for every layer), split like `multilayer`
stochastic   semi-implicit (Alg. 1) and random batch (Alg. 4) steps, stochastic
             layer splitting with an importance-sampling proposal, the proposal
             network (MLP forward/backward), its variance objective and Adam

Parity status
-------------
Every function here is pinned by tests in ``tests/test_oracle_pins.py``,
``tests/test_stochastic_pins.py``, ``tests/test_multilayer_pins.py`` and
``tests/test_blocks_pins.py`` against
closed forms, brute force, invariants or an independent supercell computation,
except where a function's docstring says "parity unpinned".
"""

from . import lifted, splitting, observables, reference, stochastic, multilayer, blocks  # noqa: F401
