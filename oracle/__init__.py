"""CPU FP64 oracle for the SPCG hot path (test infrastructure only).

This package is the independent, slow, plainly written reference that the
HIP library is checked against.  It is NOT part of the product: only the
test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  It shares no code with the GPU library (no
kernels, headers, tables or helpers); both sides only consume the seeded
inputs produced by the separate ``workloads`` package.

Modules and the part of the paper each one follows
(Chen, Xie, Yang, Zheng, "Sequential Preconditioned Conjugate Gradient
Method for Linear Statistical Models"):

* ``philox``   - Philox4x64-10 counter-based generator (Salmon et al., SC'11),
                 the randomness behind the SRHT's D, P and sampled rows (Sec. 2.1).
* ``feistel``  - keyed Feistel bijections on L-bit integers: the random
                 permutation P and the nested row sets I_1 c ... c I_K (Sec. 2.2).
* ``fwht``     - unnormalised Walsh-Hadamard transform (the H of the SRHT, Sec. 2.1).
* ``sketch``   - nested SRHT: (Z_X, Z_Y) = (HDPX, HDPY) once, prefix row sets
                 for S_i and an independent row set for S-hat (Sec. 2.2).
* ``countsketch`` - nested CountSketch of the SPCG-CS variant (Sec. 4.3):
                 bucket map, signs, folding of nested sizes, independent S-hat.
* ``linalg``   - Householder QR and triangular solves (preconditioner
                 "applied through a QR factorization", Sec. 4).
* ``pcg``      - PCG(A, b, H-hat, beta_init, a) in normal-equation form (Sec. 2.2).
* ``spcg``     - Algorithm 1 (Stage I / Stage II) and full-data PCG.
* ``ols``      - the OLS estimator of eq. (ols) by Householder QR / TSQR.
* ``theory``   - closed forms of Theorems 3.3 and 3.4 and the FLOP counts.
* ``mlp``      - FP64 reference forward/backward of the schedule MLP.

Parity pins for every module live in ``tests/test_oracle_*.py``.
"""
