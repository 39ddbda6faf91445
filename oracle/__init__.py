"""FP64 CPU oracle for the D3Q19 BGK + implicit-IBM time step.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
GPU path is checked against.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the solver library never
does, and it shares no code, tables or helpers with the HIP path.

Everything is NumPy/SciPy in float64, written to be read against the paper:

* ``lattice``  - equilibrium (Eq. 4), BGK collision (Eq. 1), Guo forcing
                 (Eqs. 7-9), moments (Eq. 2, Eq. 11) and streaming with the
                 boundary rules of Sec. 2.1 (velocity inlet, pressure outlet,
                 half-way bounce-back walls, periodic span).
* ``ibm``      - the 4-point cosine delta kernel (Eq. 14), marker placement on
                 the elliptic foils, kinematics (Eqs. 20-21, 23), delta
                 interpolation (Eq. 17), spreading (Eq. 15), the no-slip
                 system A X = B (Eqs. 18-19) and force integration (Eq. 26).
* ``params``   - mapping of (Re, J, f) to lattice units (Eqs. 3, 22, 24).
* ``sim``      - the time loop of Sec. 2.2 tying these together.

Readings of the paper where it is 2D, silent or garbled are listed in the
docstrings of the functions that implement them.  Parity pins for every part
live in tests/test_oracle_*.py.  The force histories of the clap & fling
workload itself are "parity unpinned": the paper prints them only as figures.
"""
