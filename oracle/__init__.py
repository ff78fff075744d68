"""FP64 CPU oracle for sketched RT3D (SRT3D).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the tests, the smoke check in `__graft_entry__`
and the `cpu_baseline` leg of `bench.py` use it.  It shares no code, table or
constant with the HIP library; both sides consume the same seeded inputs from
`synth`, which holds none of the method's arithmetic.

Modules
  sketch  eq. (2) and eq. (3): sketches of time stamps and of histograms.
  model   eq. (1) and eq. (4): impulse-response spectrum, model sketch,
          the sketched loss of eq. (6)/(8) with W = I and its gradients.
  srt3d   the sketched RT3D iteration of Section 3 (initialisation, step
          sizes, data step, point-cloud and intensity denoisers, background,
          output); the parts the paper leaves open follow the readings listed
          in each function's docstring.
  smle    the pixelwise sketched estimator (SRT3D's data steps alone, per-pixel
          steps, several starts, the lowest loss kept): the comparison system.
  weighted  eq. (6) with W = Sigma^{-1}: the sketch covariance from the characteristic
          function and a two-step weighted fit of each pixel.
  rt3d_full  full-data RT3D: SRT3D's iteration with the data step on the Poisson likelihood of
          each pixel's whole histogram (eq. 1), the quality reference the sketched
          reconstruction is compared with on tiny frames.

Parity status: every function is pinned by the `-m "not gpu"` tests in
`tests/test_oracle_*.py` against closed forms, invariants or brute force.
"""
