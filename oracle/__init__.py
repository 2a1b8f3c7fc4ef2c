"""CPU oracle for ExactSim single-source SimRank.

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import, call or
link anything in this package.  It shares no code with the HIP library and
imports nothing from it.

Two parts:

* ``oracle.simrank`` -- exact ground truth in float64 from the plain
  definitions: the SimRank equation (Eq. 1, Section 1), the Power Method
  S = (c P^T S P) v I (Section 2.1, "Other Related Work"), a direct solve of
  the pair equations for tiny graphs, the exact diagonal correction D of the
  linearization S = sum_l c^l (P^l)^T D P^l (Section 2, "Linearization and
  ParSim"), and that linearization evaluated with the exact D.
* ``oracle.exactsim`` -- the randomized estimator of Algorithm 1 (basic
  ExactSim) with the sample allocation of Section 3.2 ("Sampling according
  to pi_i(k)^2"), step by step in the paper's order, with the walk pairs of
  Algorithm 2 simulated by the plain C file ``walks.c``.
* ``oracle.mlp`` -- float64 forward/backward of the small budget network.
"""
