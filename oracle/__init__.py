"""FP64 oracle for the per-cell DNN chemistry update.

TEST INFRASTRUCTURE.  Only the test-suite, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import,
call or link anything in this package.  It shares no code with the HIP path
in ``paper_2508_18969_amd``: no kernels, headers, helpers, tables or
constants; neither side imports the other.  Both receive the same seeded
inputs from ``synth``.

Contents
--------
``chem``     the chemistry update: Box-Cox, Z-score, MLP with tanh-form
             GELU, inverse transform, FP64 update, renormalisation,
             enthalpy-conserving temperature; exact FP64 and an emulation of
             narrow operand formats (bf16, f16, OCP e4m3) with power-of-two
             per-layer scales.
``prop``     the property networks (PRNet): Z-score of the input fields,
             the same MLP, and the output scaling.
``train``    MLP forward with saved pre-activations, MSE loss, hand-derived
             backward, Adam.
``kinetics`` mass-action kinetics of an ideal-gas constant-pressure
             adiabatic reactor and an ROS2 Rosenbrock integrator (C, built by
             ``__graft_entry__.build``), used to make training labels.

Parity pins for every function live in ``tests/test_oracle_*.py``.
"""
