"""Plain FP64 CPU oracle for the deflated-PCG / three-level-BDDC solver.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import anything from here.  The
product path (``paper_2412_17543_amd``) never imports, links or calls it, and
this package never imports the product path.  The two share no code; the only
common module is ``workload`` (seeded input generators, no solver arithmetic).

Everything is written for clarity, not speed: scipy sparse LU for the local
problems, explicit formation of every small matrix, Python loops over
subdomains.  Each function cites the passage of Hanek, Papez & Sistek,
"Speeding up an unsteady flow simulation by adaptive BDDC and Krylov subspace
recycling" (arXiv 2412.17543) that it follows.

Modules:
  q1           -- Q1 element matrices and global assembly (Section 2, eq. of the
                  algebraic systems; the Q1 pressure space of the Taylor-Hood pair)
  substructure -- interior/interface split, interface Schur complement,
                  condensation and interior recovery (Section 3.1, eq. Sug)
  bddc         -- globs, coarse DOFs, weights, two- and three-level BDDC
                  (Section 3.2, eqs. averaging_subdomain_solves, coarse_problem,
                  localCorr; multilevel paragraph)
  dpcg         -- deflated PCG (Section 4.1, Algorithm 1; stopping rules of
                  Section 5, eqs. stopping_residual and stopping_rhs)
  recycle      -- deflation-basis construction B1..B4 with harmonic Ritz
                  vectors (Section 4.2, eqs. harmonicRitz, harmritzstopcrit)
  sequence     -- a right-hand-side sequence solved with recycling
  adjoint      -- adjoint gradient of a least-squares loss w.r.t. log-coefficients
  block        -- the adjoint systems solved as one block (block deflated PCG,
                  breakdown-free form; an extension, not in the paper)
  adaptive     -- adaptive face constraints (Section 3.3), levels 1 and 2

Parity status of each piece (what pins it) is listed in the tests and in the
design notes; the three-level iteration counts are pinned only by the
lambda_min >= 1 bound and by identities, not by any printed value.
"""
