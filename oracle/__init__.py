"""CPU oracle for the parametric Lifted-KKT interior-point NMPC solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this package: only the test suite, the smoke check and the CPU-baseline leg of
the benchmark use it.  It is a plain, slow, obviously correct restatement of the
method in NumPy/SciPy (float64 throughout) and shares no code with the HIP
library.

Modules
    distillation  transcribed distillation-column OCP (Section 4.1 family)
    lq            linear-quadratic test family (Riccati closed form pin)
    toy           the one-state example of the re-solve code listing (Section 3.3)
    symbolic      SymCholesky: ordering, elimination tree, column structure,
                  supernodes (Section 3.2.3, eqs. 18-19, Fig. 1)
    ipm           the Lifted-KKT interior-point method (Section 3.2, Algorithm 2)
    kkt           optimality error of the original (unlifted) problem, eq. (8)
    riccati       finite-horizon LQ closed form
    nmpc          the receding-horizon loop (Algorithm 1)
"""
