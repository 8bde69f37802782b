"""FP64 CPU oracle for the filtered (LES) lattice-Boltzmann MHD method of
Flint & Vahala, "A large eddy lattice Boltzmann simulation of MHD turbulence"
(arXiv 1705.09807).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
definition that the HIP path is checked against.  It shares no code, tables or
constants with the HIP path and must never be imported by the product: only
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use it.

Modules
-------
lbmhd_oracle
    The method step by step in the paper's order (moments, filtered
    equilibria with the subgrid closure, collision in moment space, streaming
    in population space), the Kelvin-Helmholtz initial state and the scalar
    diagnostics.
linear
    A brute-force Fourier-space linearisation of one timestep about a uniform
    equilibrium.  Its eigenvalues give the exact discrete decay rates and
    frequencies of small-amplitude waves, used to pin the oracle.
learned
    The learned closure: Gaussian filtering and subsampling of a fine-grid
    state, the exact subgrid terms of the filtered products, the analytic
    closure in the same four components, the network's input patches, a
    two-hidden-layer network with the GPU's bfloat16 roundings, its loss
    gradients and Adam.  ``Oracle(closure_correction=...)`` adds a correction
    to the analytic closure, evaluated every step or, with
    ``correction_every=K``, every K-th step and held in between.
spectra
    Radially binned kinetic and magnetic energy spectra.

Parity status: every function of ``lbmhd_oracle`` is pinned by the CPU tests
(printed matrices and tables, closed forms, invariants, brute force) except the
closure's macroscopic effect on the nonlinear Kelvin-Helmholtz dynamics, which
has no closed form: "parity unpinned" beyond the pins listed in the tests.
"""

from .lbmhd_oracle import Oracle  # noqa: F401
