"""CPU ORACLE for the GP-FVM hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never links,
imports or calls it, and it imports nothing from the product library.

What it computes, plainly and in float64 (paper Sec. 2.1 eq. lin-cond-mean /
lin-cond-cov, Sec. 2.2, Sec. 3, Sec. 4):

* 1-D factors ``F^{pq}``, ``Q^{pq}``, ``P^{pq}`` by adaptive Gauss-Kronrod
  quadrature of the kernel's pointwise derivatives (``quad.c``), with no
  antiderivatives or closed forms;
* the dense IBVP Gram ``G = L k L' + Sigma`` by summing, over every pair of
  operator terms (alpha, alpha'), Kronecker products of those factors
  (Sec. 3.2 eq. LkL and Sec. 4.1 eq. kronecker-structure);
* the posterior mean and variance by LAPACK Cholesky (Sec. 4, representer
  weights);
* for problems whose dense Gram does not fit: the same quantities matrix-free,
  with the IC/BC block conditioned exactly by Cholesky first and the volume
  observations integrated by IterGP with CG actions (Sec. 4.1 and Sec. 4.2;
  IterGP's recurrences as published by Wenger et al. 2022).

Parity status of each function is listed in ``oracle.gpfvm_oracle``'s header.
"""
from .gpfvm_oracle import *  # noqa: F401,F403
