"""Plain FP64 CPU oracle for the spin-projected MPS (SP-MPS) hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything under ``oracle/``: only the tests, the smoke check and the
CPU-baseline leg of the benchmark do.  It shares no code with the HIP library
(the only common module is the seeded input generator ``workloads``, which
holds none of the method's arithmetic).

Modules, each following the paper (Li & Chan, SP-MPS):

* ``quadrature`` -- Gauss-Legendre nodes (Golub-Welsch), Wigner small-d,
  projector coefficients and the exact-point count (Sec. 2.2).
* ``local_ops``  -- Jordan-Wigner local matrices, spatial-orbital spin
  matrices and the local rotation r(beta) (Secs. 2.1, 2.2).
* ``mpo``        -- Hubbard, S^2 and identity MPOs in the operator-valued
  matrix form of Sec. 2.1, plus MPO -> dense contraction for tiny chains.
* ``ed``         -- exact diagonalisation in occupation-number form with an
  exact S^2 projector (the plain definition of the projected energy).
* ``mps``        -- the SP-MPS sweep: environments for every quadrature point,
  H_eff x and N_eff x, the diagonal, the Davidson local solve and the
  canonical gauge moves (Sec. 2.3).
* ``slater``     -- closed-form energies of one or two occupation-number
  determinants of the ab-initio Hamiltonian (Slater-Condon rules), with the
  spin projector for an open-shell pair: exact values at any orbital count.

Functions whose result is not pinned by a test against a closed form, a
library routine, brute force or a printed value of the paper say
"parity unpinned" in their docstring.  At present every function is pinned.
"""
