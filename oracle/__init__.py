"""Plain FP64 CPU oracle of the space-time FE slab problem and its GMRES-GMG solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the C-ABI library and
its Python binding) imports, links or executes anything in this package; only
the test-suite, the smoke check and the CPU-baseline leg of the benchmark do.

The oracle follows the paper (Anselmann, Bause, Margenberg, Shamko: "An
energy-efficient GMRES-Multigrid solver for space-time finite element
computation of dynamic poro- and thermoelasticity", arXiv:2303.06742):

* ``timedg``   -- right Gauss-Radau rule and dG(k) Lagrange time basis (Sec. 2, Eq:GF, Eq:TimeExp).
* ``fem``      -- tensor Lagrange elements Q_r^d / Q_{r-1} and the broken P_{r-1}^disc,
                   the forms Def:ACB, Def:ab (SIPG B_gamma for the discontinuous pressure).
* ``problem``  -- Problem 3.1 (or Problem B.1) assembled into the algebraic slab system of Problem 4.1.
* ``gmg``      -- grid transfers, vertex/cell patches, Def. 4.2 and Alg. 4.1, V-cycle.
* ``fgmres``   -- flexible (right-preconditioned) restarted GMRES.
* ``norms``    -- the discrete error norms of Sec. 5.1.

Everything is written for clarity, not speed, in float64 throughout.

What pins it (tests/test_oracle_*.py, all CPU):
  time rule and matrices  -- Gauss-Radau exactness, known nodes, the (k,k+1)
                             Pade identity of dG(k)+right Radau, backward Euler;
  element integrals       -- closed forms (mass, rigid motions, uniaxial strain
                             energy, divergence, face terms);
  assembled problem       -- exact reproduction of a solution in the discrete
                             space (row-wise residual ~1e-16), optimal EOC,
                             nodal superconvergence 2k+1, energy decay of
                             Lemma 3.2, symmetry and coercivity (Appendix A);
  discontinuous pressure  -- closed-form cell mass and single SIPG face entries,
                             symmetry and coercivity, exact reproduction, exact
                             transfer, Table 5.1 rows 1-2 (grad u and v errors to
                             0.5 %, rates), Table 5.2 row 1 relation to Taylor-Hood;
  Problem B.1             -- exact reproduction (both pressure pairs, 2D/3D), and the
                             coincidence with Problem 3.1 on Table 5.1 row 1;
  multigrid / Krylov      -- polynomial reproduction of the transfers, the
                             exact-local-solve invariant of Def:VankaOP, the
                             averaging identity of Alg. 4.1, one-level V-cycle =
                             direct solve, agreement with the sparse direct
                             solve, brute-force minimal residual of FGMRES.
Parity unpinned: the magnitudes of Table C.1 and Table 5.2 are not reproduced
digit for digit (rates agree, values differ by 1.4-7x; recorded, not asserted),
nor the pressure errors of Table 5.1 (1.6-1.9x larger; grad u and v match), and GMRES
iteration counts and V-cycle output values have no printed reference.

"""
