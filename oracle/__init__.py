"""FP64 CPU oracle for the EnSF analysis step (test infrastructure only).

Plain, slow and written to be checked against the paper by eye.  Only the tests, the
smoke check and the benchmark's CPU-baseline leg may import it; the product path (the
HIP library and its Python binding) never does, and this package imports nothing from
the product either.

Contents
  philox   Philox4x32-10 counter-based generator (Salmon et al., SC'11) and the
           Box-Muller transform (Box & Muller, 1958), from their published definitions.
  ensf     diffusion schedule (Sec. III-A-1, eq. 9), observation densification and the
           likelihood score (eqs. 2, 5), the Monte-Carlo prior score (eqs. 12-16), the
           damped posterior score (eqs. 11, 17), the Euler-Maruyama reverse-SDE analysis
           (eq. 7) and a brute-force loop form of the prior score for tiny inputs.
  linear_gaussian
           the closed-form mean/variance recursion of the same Euler-Maruyama scheme
           for a Gaussian prior with an exact prior score and a linear observation,
           and the Kalman posterior it is compared with.
  conv, sqg
           the convolutional forecast surrogate in FP64 and a pseudo-spectral SQG
           stepper (Sec. II-B) used as truth generator and as the reference forecast.
"""
