"""FP64 CPU oracle for the batched quadrotor step and the ray-cast depth render.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, link or call
anything under ``oracle/``; only the test suite, the package smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP path: the
two meet only at the seeded inputs from ``workloads``.

What it computes (each function cites the passage it follows):
  dynamics   Sec. III-A: Eq. (1) rigid body, Eq. (2) drag, Eq. (3) thrust and
             moment, Eq. (4) first-order rotor lag, the CTBR / SRT controllers
             and RK4 / Euler integration with sub-steps.
  render     Sec. III-B: per-agent depth / triangle id / flat colour by a
             brute-force closest hit over every triangle (Moller-Trumbore in
             FP64, plain C, one loop per ray and triangle), plus the per-pixel
             edge / tie diagnostics that define the comparison mask.
  gradients  Sec. III-A (differentiable dynamics): the rollout loss and its
             central finite differences.

Where the paper is silent or garbled the readings are stated in the module
docstrings.  Every function here is pinned by a ``-m "not gpu"`` test against
closed forms, invariants, exact rational arithmetic or brute force.
"""
