"""CPU FP64 oracle for block Krylov solves of the O(a)-improved Wilson-Dirac
equation (Sakurai, Tadano, Kuramashi, arXiv:0903.4936).

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
link this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (``paper_0903_4936_amd``); its inputs come from ``synthetic``.

Modules
-------
gamma     the Euclidean gamma matrices exactly as printed in Sec. 2, and
          sigma_{mu nu} = [gamma_mu, gamma_nu] / 2.
dirac     geometry, clover leaves, F_{mu nu}, the 12x12 site-local term and
          D_W of Eq. (1) on fields of shape (Lt, Lz, Ly, Lx, 4, 3, L); the
          adjoint; dense assembly.
solvers   BiCGSTAB, block BiCGSTAB and the new block method (Block BiCGGR)
          of Sec. 3, the true residual of Sec. 4.3.
spectrum  critical hopping parameter probe.
gradients gradients of a solve with respect to B, kappa, c_SW and the links
          (adjoint formulas derived from Eq. (1)).
correlators pion and rho two-point functions contracted from the 12
          point-source solutions (textbook Wick contraction).
evenodd   the Schur complement of D_W on the even sites (every extent even):
          the even-site operator, right-hand side and odd-site reconstruction.
deflation restarted Block BiCGGR that leaves out converged columns and solves
          only an independent subset of the others (pivoted Cholesky of the
          normalised Gram matrix), mapping the correction back.
native    ctypes loader of dirac_sites.c: the operator of ``dirac`` written
          out in plain C (FP64, OpenMP over sites) for whole-lattice residual
          checks at full size; pinned against ``dirac`` and the same closed
          forms.

Every function is written for a reader who checks it against the paper by
eye; nothing is blocked, fused or reordered.  Readings of points the paper
leaves open are listed in the repository's design notes and repeated where
they are used.  Parity status: every function here is pinned by a test in
``tests/test_oracle_*.py`` against a closed form, an invariant, a library
routine or a number printed in the paper.
"""
from . import gamma, dirac, solvers, spectrum, gradients, evenodd, deflation  # noqa: F401
