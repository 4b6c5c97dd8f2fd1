"""Plain FP64 CPU oracle of the coupled Maxwell-Schroedinger step.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously-correct
reference that the HIP library is checked against.  Only the test suite, the
smoke check and the benchmark's CPU-baseline leg may import it; the product
path never does.  It shares no code with the HIP library: it reads the shared
seeded inputs from ``workloads`` and implements every step itself with NumPy /
SciPy in float64 / complex128.

Modules
-------
molecule  - two-state ro-vibrational wavepacket step (Eqs. (3)-(5)),
            split-operator with FFT, angular DVR for the dipole coupling.
fdtd      - Yee leap-frog of Eq. (1) with the Drude current of Eq. (2),
            periodic x/y, CPML in z, soft current-sheet source, flux monitor.
maps      - SplitMix64 molecule placement -> cell index -> CSR of cells.
coupled   - the self-consistent step: field gather, molecular step,
            mean-field polarisation current, E update.
tangent   - forward-mode (tangent-linear) derivative of the coupled run,
            the reference for the hand-written adjoint.
"""
