"""CPU oracle for the InFo-ESRF perturbation update -- TEST INFRASTRUCTURE ONLY.

Plain, slow, FP64 NumPy/SciPy code written from the paper (Armstrong &
Grooms, "Data Assimilation With An Integral-Form Ensemble Square-Root
Filter").  It exists to check the HIP path; it is not part of it.  Only the
test-suite, the package smoke check and the CPU-baseline leg of the
benchmark may import it.  It shares no code with the HIP library and never
imports it; both take their inputs from the ``synthetic`` generators.

Modules
-------
``infoesrf_ref``   ensemble statistics, localized covariance, the exact
                   (eigendecomposition) updates, the quadrature rules, the
                   limited-memory preconditioner and a matrix-free PCG.
``warmstart_ref``  the 1-D convolutional warm-start network: forward,
                   backward, loss and Adam in FP64.
``cycle_ref``      RTPS inflation for the cycled driver.

Parity status of each function is stated in its docstring; functions whose
result has no independent pin say "parity unpinned".
"""
