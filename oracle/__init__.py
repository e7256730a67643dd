"""FP64 CPU oracle for the hp-FEM ADI screened-Poisson solver.

This package is TEST INFRASTRUCTURE. It is a plain, slow, FP64 NumPy/SciPy
implementation of what the GPU library computes, written from the paper
(Knook, Olver and Papadopoulos, "Quasi-optimal complexity hp-FEM for the
Poisson equation on a rectangle", arXiv 2402.11299). Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it. The product (``paper_2402_11299_amd``) never imports it, and it never
imports the product: the two share no code. The only shared module is
``workloads`` (seeded input generators, no method arithmetic).

Modules
-------
basis     1D operators K, M, T = R^T M_P in the degree-major hat+bubble basis
          (Sec. 2, App. A), plus an independent Gauss-quadrature assembly.
cholesky  Reverse Cholesky of B^3-arrowhead matrices (Sec. 4, Alg. 1) and the
          O(N) solve (Sec. 4, corollary).
spectrum  Spectral interval of the pencil (A_Y, M) (Sec. 5, Alg. 2
          precomputation; Lemma "Spectrum").
shifts    Iteration count J and Zolotarev ADI shifts (Sec. 5, Alg. 2).
adi       Generalised ADI (Sec. 5, Alg. 2), exact reference solves, the
          error metric, FP64 residual and mixed-precision refinement.

Parity pins live in ``tests/test_oracle_*.py``; every function states the
passage it follows.
"""
