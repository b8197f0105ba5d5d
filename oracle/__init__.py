"""FP64 CPU oracle for Log-Averaged Mirror Prox (LAMP, arXiv 2511.11359).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute anything under ``oracle/``: only the tests, the smoke check and the
CPU-baseline leg of the benchmark use it.  It shares no code with the HIP path
(no kernels, headers, helpers, tables or constant generators) and never takes
an input or an expected value from the HIP path.

Every routine is a plain, slow, direct transcription of a definition or of an
algorithm's steps from the paper, in FP64, with the paper's notation:

* ``lamp``   -- cost, dual-to-primal map, mirror maps, clipping, the eta_t
  schedule, Algorithm 2 (LAMP), Algorithm 1 (PDMP), Algorithm 3 (Round), the
  dual functions D and D^eta, the penalised primal, Proposition infeas_bound,
  the envelope gradient.
* ``exact``  -- ground-truth OT values: brute force over permutations, the
  assignment solver, the HiGHS LP, log-domain Sinkhorn for the EOT fixed point.
* ``stream`` -- the same LAMP iteration evaluated in row blocks without ever
  materialising C (for large sizes: timing and sampled parity).
* ``cmax``   -- max_ij ||x_i - y_j||^2 in plain C (exact FP64), for the cost
  normalisation at sizes where NumPy is too slow.
* ``rowpass`` -- one iteration's row log-normalisers on every row and column
  marginals and dual steps on listed columns, in plain C (FP64, OpenMP), for
  parity at the full benchmark sizes.

Parity status of each function is stated in its docstring; functions with no
independent pin say "parity unpinned".
"""
