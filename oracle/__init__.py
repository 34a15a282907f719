"""CPU oracle for the PAGD-solved fully implicit PFC / FCH steps.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) imports, calls or links anything here; only the test-suite,
the smoke check and the CPU-baseline leg of the benchmark do.

Everything is plain NumPy in float64, written from the definitions in
Park, Salgado & Wise, "Benchmark computations of the phase field crystal and
functionalized Cahn-Hilliard equations via fully implicit, Nesterov
accelerated schemes" (arXiv 2204.07247):

* ``spectral``  grid, wavenumbers and the Fourier-collocation operators
                (Sec. 3.2, eq. def:frac-Lap, eq. def:neg-norm).
* ``models``    PFC / FCH energies and chemical potentials
                (Sec. 2, eqs. obj:PFC-egy, eqn:PFCsystem, obj:FCHegy).
* ``schemes``   BDF2 / backward Euler / implicit-midpoint coefficients and the
                two-level extrapolation (Sec. 3.1, eqs. obj:BDF2, obj:MP).
* ``pagd``      objective G_N, projected gradient (eq. obj:G'), averaged-Newton
                preconditioner (Sec. 3.4.1) and PGD / PAGD (Alg. 1, Alg. 2).
* ``driver``    fixed-step time marching (Alg. 3 without step adaptation).
* ``imex``      linear IMEX steps LBDF2 / LMP (Sec. 3.1.1,
                eq. eqn:FCH-semidis-simplicit).
* ``adaptive``  AM3 / midAB2 error estimators and the step-size controller
                of Alg. 3 (Sec. 3.1.2).
* ``dft``       brute-force O(P^2) DFT sums, used only to pin ``spectral``.
* ``newton``    dense Newton solve of the step equation, used only to pin the
                PAGD fixed point on tiny grids.
* ``fno``       float64 Fourier-neural-operator forward / backward, the
                reference for the learned warm start's gradient checks.
"""
