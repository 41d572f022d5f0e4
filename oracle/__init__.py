"""FP64 CPU oracle for the Hessian / OPG hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct NumPy implementation of what the device
library computes, written from the paper ("Efficient Computation of Hessian
Matrices in TensorFlow", Nilsen, Munthe-Kaas, Skaug, Brun).  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import
it.  It shares no code with the device library and imports nothing from it.

Modules
  mlp      model, cost, per-example gradients J, OPG, R-op Hessian-vector
           products and the exact Hessian by basis columns
  eig      leading (algebraically largest) eigenpairs, sign convention
  predvar  logit gradients and the damped curvature (predictive variance) query

Pins: every function is checked in tests/test_oracle_pins.py against values
fixed by the paper or by mathematics (finite differences, complex step,
closed forms, null spaces, textbook routines), never against itself.
"""
from . import mlp, eig, predvar  # noqa: F401
