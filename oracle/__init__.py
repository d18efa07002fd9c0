"""CPU oracle for the KB-NUFFT path: test infrastructure, not product code.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library and never
imports it.

Contents
  ndft       exact FP64 non-uniform DFT (C, OpenMP) and the closed-form
             omega/x Jacobian-vector products derived from it (Sec. II-C,
             II-D, II-G; eq. (e,jac,Ax,v)).
  nufft_ref  FP64 Kaiser-Bessel NUFFT written step by step as the appendix
             describes it (scale, zero-padded K-point FFT, J-tap
             interpolation), plus the window and its Fourier transform.
  points_ref the per-point grid offsets, fractions, tile ids and the stable
             tile order that the index pass must reproduce bit for bit.
  cg         FP64 conjugate-gradient CG-SENSE reconstruction.
  inverse    the regularised inverse (E^H E + lambda T^H T)^{-1} by dense FP64
             solves, and the gradients of the Gram and inverse operators
             (Sec. II-E, II-F).
  field      the off-resonance model of Sec. II-H: the exact operator, the
             segmented form sum_l diag(b_l) A diag(c_l) and its omega-gradients,
             and linear-interpolation time segmentation.
"""
