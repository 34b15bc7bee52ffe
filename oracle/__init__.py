"""CPU oracle (test infrastructure only).

Plain FP64 numpy/scipy implementation of the implicit viscous-plastic momentum
step and its stress-velocity Newton solve.  Only the tests, the smoke check and
the CPU-baseline leg of the benchmark may import this package; the product path
(the HIP library and its binding) never does.
"""
