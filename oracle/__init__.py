"""FP64 CPU oracle for range analysis of MLP implicit surfaces.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only the tests, the smoke check and the benchmark's CPU
baseline leg use it.  It shares no code with the HIP path.

It follows Sharp & Jacobson, "Spelunking the Deep: Guaranteed Queries on
General Neural Implicit Surfaces via Range Analysis" (ACM TOG 41(4), 2022):

* :mod:`oracle.affine`   -- affine forms (Section 3.2, Appendix A, Tables 2-3),
  condensation policies (Section 3.3), interval arithmetic (Section 3.1);
* :mod:`oracle.mlp`      -- plain evaluation and bound propagation through an MLP;
* :mod:`oracle.queries`  -- RangeBound (Procedure 1), CastRay (Procedure 2),
  BuildSpatialTree in parallel rounds (Procedure 3, Section 4.5), closest point
  (Section 4.10).

Arithmetic is float64 with round-to-nearest and no rounding inflation, as in
the paper (Section 3.4 notes that rounding control is not needed there).
"""
