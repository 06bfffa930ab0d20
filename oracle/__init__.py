"""CPU oracle for the ProbeWalk estimator.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import or run anything in this package.
The product (``paper_2512_05460_amd``) never imports it, and this package never
imports the product: the two share only the seeded inputs from ``synth``.

Contents
  * ``estimator``: Algorithm 1 (section 3) in plain C (``pw_oracle.c``),
    driven through ctypes -- probes, walks, U-statistic, median-of-means.
  * ``planner``: the walk counts B, G, K, R of Algorithm 1 and Theorem 3.8.
  * ``exact``: exact squared biharmonic distance in binary64 -- dense
    pseudoinverse (Definition 2.1), conjugate gradients, the truncated series
    of Lemmas 2.2/2.3.
"""
