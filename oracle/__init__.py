"""Oracle for the beyond-Limber C_l hot path -- TEST INFRASTRUCTURE ONLY.

Plain, slow FP64 CPU code (NumPy / SciPy) that shares no code with the HIP
path.  Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import it; the product package never does.

Modules
  geometry    continuous inputs from samples (natural cubic splines), z(chi),
              clustering, lensing and CMB-lensing radial kernels (Sec. 2.2-2.4 of
              the paper)
  fftlog      the paper's method, step by step in its own notation: FFTLog
              coefficients (Sec. 3.1, eq. FFTLog), the analytic power-law Bessel
              integral (eq. int_jl, corrected), the sum over n per k, the k-sum
  quadrature  the plain definition: windows by direct quadrature of
              j_l(k chi), used to pin the FFTLog oracle (method-error floor)
  limber      the Limber limit (eq. Limber), a high-l check of the quadrature, and the
              rule on the FFTLog chi nodes with its dL/dP through the spline of ln P
  gradients   exact / directional derivatives of C_l for the adjoint tests
  kgrowth     scale-dependent growth D(k, z) (Sec. 3.2): coefficients at N_interp
              k nodes, continued along ln k by a natural cubic spline
The optional terms of Sec. 2.2-2.3 (intrinsic alignment, RSD, magnification bias) live in
geometry (their radial kernels), fftlog (their FFTLog windows) and quadrature (the same windows
by direct integration, j_l'' from the Bessel equation).  CMB lensing (Sec. 2.4) is a third tracer
kind with the kernel of one source plane at the last-scattering surface; it has no HIP path yet.

Readings of the paper that the oracle fixes are listed in each function's
docstring; every one is shared, by statement and not by code, with the HIP
path.
"""
