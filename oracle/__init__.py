"""FP64 CPU oracle for the nonoverlapping DDM-ELM (test infrastructure only).

This package is the plain, slow, obviously-correct reference that the GPU
library is checked against.  It is test infrastructure: only the tests, the
smoke check and the CPU-baseline leg of the benchmark may import it.  The
product path (the HIP library and its binding) never imports or calls it.

Everything is NumPy/SciPy float64, written step by step after the paper:

* layout.py  -- subdomains, collocation/boundary/interface points, interface
                numbering and outward normals (Section 3, points x_i, x_b, x_Gamma).
* ddm.py     -- features and operator rows (Section 4.1), local blocks
                K^s, A^s, B^s, F^s (eq. nonoverlap_discrete), the Schur
                complement system (eq. schur) built from per-subdomain
                Householder QR factors, its solution by dense Cholesky or by
                CG (Section 3), the local back-solve K^T K c = K^T (F - B u)
                (Algorithm 1), and evaluation of the network solution.
* literal.py -- tiny-problem brute force: the global matrices K, A, B, F of
                eq. discrete-simple with a dense pseudo-inverse, the
                eliminated least-squares system (eq. eliminated / LS_system)
                and the least squares of the original system; used only to
                pin ddm.py.

Parity status: every function is pinned by the CPU tests (finite
differences, closed-form manufactured solutions, the single-domain ELM
least squares, the literal pseudo-inverse form of eq. schur, and the
monolithic eliminated system).
"""
