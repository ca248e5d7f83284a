"""Plain FP64 CPU oracle for multilevel BDDC (test infrastructure only).

This package is the checker the GPU library is compared against.  It is
slow and sequential on purpose: each step follows the definitions of
Sistek, Mandel, Sousedik, Burda, "Parallel implementation of Multilevel BDDC"
(section 2, equations (1) and (2), Algorithms 1 and 2) with sparse LU
factorizations of the full saddle-point matrices.  It shares no code with the
GPU library and must only be imported by tests, the smoke check and the CPU
baseline leg of the benchmark -- never by the product path.

Modules
-------
fem     : element matrices, loads and global assembly of the model problems.
dd      : one level of the decomposition: subdomain matrices, interface, globs,
          constraints, weights, coarse basis and coarse matrices (Eq. (1)).
bddc    : the multilevel preconditioner apply (Eq. (2), Algorithm 2).
krylov  : preconditioned conjugate gradients and the Lanczos estimate.
direct  : direct solves used as ground truth.
grad    : compliance gradient with respect to element log-moduli.
"""
