"""Plain FP64 CPU oracle for the low-rank Lindblad readout integrator.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the test-suite, the package's smoke check and the
CPU-baseline leg of the benchmark use it.  It shares no code with the HIP
library; the two meet only at the seeded inputs of
``paper_2508_18114_amd.inputs``, which hold none of the method's arithmetic.

Modules
  pulses   -- drive coefficient d(t) (envelopes of supplement S2.C, as read
              for the lab-frame Duffing model)
  lowrank  -- the low-rank equation of motion (supplement S1.A, eq. "nosse"
              with the dissipator map O[m] and the Moore-Penrose inverse),
              classic RK4, observables
  dense    -- brute-force dense operators (Kronecker products) and the full
              Lindblad master equation (eq. "master_equation"), the reference
              the low-rank path is pinned against on tiny Hilbert spaces
  loss     -- readout figures of merit (supplement S3.A-B: SNR, separation
              and decay errors, ionisation penalty, loss)
  validity -- spectrum p_1 >= ... >= p_M of the low-rank rho, the control
              quantity p_M / p_1 and the purity (supplement S1.B)
  adaptive -- adaptive-step integration of the low-rank equation (the
              Dormand-Prince 5(4) pair with an error-norm step controller)
  papermodel -- the paper's mode basis: charge-basis transmon levels and charge
              operator (supplement S2.A), resonator-filter normal modes and
              their coupling coefficients (supplement S2.D)

Every function is written in the notation of the paper, step by step, with
numpy/scipy library primitives (matmul, Cholesky, triangular solve, erfc) as
the only building blocks.  Pins: tests/test_oracle_pins.py.
"""
