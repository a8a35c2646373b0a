"""Plain FP64 CPU oracle for one GP-augmented chance-constrained MPPI iteration.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The product path (the
HIP library and its Python binding) never imports, links or calls it.

It is written from the paper (arXiv 2411.03289, "Data-Driven Sampling Based
Stochastic MPC for Skid-Steer Mobile Robot Navigation") and the textbook
methods it relies on; every function cites the passage it follows:

  philox.py       control noise: Philox4x32-10 counter-based generator
                  (Salmon et al., SC'11) and the Box-Muller transform
                  -> Alg. 1, Step 1 ("Sample eps^s ~ N(0, Sigma_sim)"), Eq. (8)
  gp.py           exact GP regression (Rasmussen & Williams, Alg. 2.1) with
                  the SE-ARD kernel -> Sec. III-A, Eq. (3), Sec. V-A
  dynamics.py     dynamic unicycle and first-order covariance propagation
                  -> Eqs. (1), (2), (6), (10)
  constraints.py  lane and obstacle chance-constraint tightening
                  -> Eqs. (13)-(16)
  mppi.py         rollout, stage costs, MPPI weights and control update
                  -> Eqs. (5), (11), (12), Alg. 1 Steps 1 and the closed loop

Everything is float64, vectorised over samples with an explicit loop over
the horizon.  Readings of points the paper leaves open are listed in
`mppi.READINGS`.
"""
