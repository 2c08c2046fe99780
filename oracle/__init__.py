"""CPU FP64 oracle for the sketch-and-project ridge solver (RidgeSketch, arXiv 2105.05565).

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or
execute this package: only the test suite, the smoke check and the CPU
baseline leg of the benchmark use it. It shares no code, constants,
headers or helpers with the HIP library; both sides only consume the same
seeded inputs.

What it computes, and where the paper defines it:

* ``problem``  -- the linear system A w = b in primal or dual form
  (Sec. 2.1, eq:linear, eq:duallinear, eq:Axb) and the dual-to-primal map.
* ``philox``   -- the Philox4x64-10 counter-based generator (Salmon et al.,
  SC'11), the source of every random draw the method makes.
* ``sketch``   -- subsample (Def. 4.2, eq:subsample), count (Sec. 4.2) and
  SubCount (Def. 4.3, eq:Sigmacount) sketches, plus a weighted subsample for
  a learned proposal distribution (any distribution D, Sec. 3).
* ``linalg``   -- Cholesky factorisation and triangular solves used as the
  least-norm solution of the sketched system (eq:sketched_system).
* ``solver``   -- Alg. 1 / Alg. 2 (sketch-and-project with momentum,
  eq:res_update_mom) and the momentum schedules of Sec. 6 and Sec. 8.1.
* ``mlp``      -- the small MLP (forward, backward, Adam) that scores
  coordinates for the learned proposal. The paper is silent on it; it is
  pinned by finite differences.

Every floating-point quantity is FP64. Readings of ambiguous passages are
listed in the design notes of the repository.
"""
