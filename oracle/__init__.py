"""FP64 CPU oracle for the multilevel linearized buckling analysis.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import anything from here; the
product library never calls it and shares no code with it.

The oracle is a plain, slow, obviously-correct transcription of what the paper
computes (Ferrari & Sigmund, "Towards solving large-scale topology optimization
problems with buckling constraints at the cost of linear analyses"):

  * ``fem``        element matrices and assembled sparse K[x], G[x, u]
                   (Sec. 2, eq. interpolationSIMP2-SIMP; element choice Q4/H8)
  * ``levels``     nested grids, interpolation/restriction and Galerkin
                   coarse operators (Sec. 2.1 step 1; Alg. 2, hierarchy and Galerkin steps)
  * ``lba``        linear analysis, coarse eigenproblem, prolongation, fine
                   block solve, Rayleigh-Ritz (Alg. 1; Sec. 2.1 steps 1-4)
  * ``sens``       compliance and buckling-factor sensitivities with the
                   adjoint system (eqs. SensitivityLambda and AdjointSystem)
  * ``mg``         the multigrid V-cycle, the preconditioned inverse
                   iteration on the fine modes (App. A, eqs.
                   PInvIt-GeneralInteration and errorEstimate) and the
                   intermediate-level Kaczmarz smoothing and Ritz steps of
                   Alg. 2

Every function cites the passage it follows.  Readings of passages that are
silent or garbled are listed in each module header.
"""
