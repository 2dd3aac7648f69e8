"""Plain, slow CPU FP64 oracle of the SSsNAL method (arXiv 1910.01312).

TEST INFRASTRUCTURE ONLY.  Only `tests/`, `__graft_entry__.smoke()` and the
CPU-baseline leg of `bench.py` may import anything under `oracle/`.  The
product path (the HIP library and its Python binding) never imports it, and
the oracle never imports the product package: the two share nothing except
the seeded input generators in `synth/`.

Modules:
  projection  - Algorithm 2 breakpoint search, Pi_{K∩L}, HS-Jacobian (Thm 3.1)
  ssnal       - Algorithm 1 + Algorithm 3 in omega-space, Newton solvers,
                R_KKT (eq. Def_Rkkt), objective, duality gap
  general     - the same method on the unified problem (P) with Q = B B^T:
                C-SVC and eps-SVR instances, the SVR primal for duality gaps
  features    - random Fourier and Nystroem features of the RBF kernel
                (Section 4), which feed the linear C-SVC unchanged
  kernel      - the C-SVC dual with a nonlinear kernel (explicit Q, small n)
  bruteforce  - 3^n active-set enumeration of the QP and of the projection
  literal     - the paper's n-space Newton system and Proposition 5 verbatim
  mlp         - FP64 forward/backward of the warm-start network
"""
