"""CPU FP64 oracle for the FMM-BEM preconditioned Helmholtz solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library, its
Python binding, the autograd wrapper) may import, call or link anything in
this package.  Only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.

The oracle is written from the paper (Ibeid, Yokota, Keyes, "A Matrix-free
Preconditioner for the Helmholtz Equation based on the Fast Multipole
Method"), in plain numpy/scipy FP64, with no blocking or fusion beyond what
the definitions state:

* ``kernel``   -- the 2-D free-space kernel G = (i/4) H0(k r) and its normal
                  derivative dG/dn (Sec. 5.2) and the direct N-body sums
                  (Sec. 5.1, the N-body sum equation).
* ``fmm``      -- a reference FMM (Sec. 5.1.2: P2M, M2M, M2L, L2L, L2P, P2P on
                  the quad-tree of Sec. 5.1.1) written with Graf's addition
                  theorem, so that "the oracle's own FMM error at order p" has
                  a meaning.
* ``fmm3``     -- the same flow on the oct-tree with the 3-D kernel
                  exp(i k r) / (4 pi r) (Sec. 5.1.1, Sec. 5.2), with
                  spherical-harmonic expansions and Gaunt-coefficient
                  translations.
* ``helm3``    -- the 3-D model problem of Sec. 7 on a 7-point grid and its
                  free-space volume-potential preconditioner (cell self
                  term by pyramid quadrature).
* ``bem``      -- the dense BEM preconditioner of Sec. 5.2-5.3 (Dirichlet
                  boundary equation, interior equation, constant elements and
                  the analytic singular diagonal), and the solution with
                  inhomogeneous Dirichlet data (double layer and 1/2 delta).
* ``fd``       -- the 5-point finite-difference Helmholtz matrix.
* ``fgmres``   -- right-preconditioned restarted flexible GMRES (Sec. 3-4).
* ``bicgstab`` -- right-preconditioned BiCGSTAB, the short-recurrence
                  alternative of Sec. 3.
* ``adjoint``  -- the adjoint gradient dJ/dk^2 by sparse direct solves.

Every function names the passage it follows.  Readings of passages where the
paper is silent or ambiguous are stated at the function.
"""

from . import kernel, fmm, fmm3, helm3, bem, fd, fgmres, bicgstab, adjoint  # noqa: F401
