"""FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the bench's CPU-baseline leg may import
this package.  It shares no code with the GPU library and never calls it.

Parity status per function (what pins it, in tests/test_oracle.py):
  conv / power / power_at   brute force, numpy.convolve, impulse, linearity,
                            convolution theorem, z=0 row
  dft                       numpy.fft, closed forms (impulse, constant, Parseval)
  template_spectrum         zero-padded numpy.fft of h, divided by L
  ols_convolve (Alg. 2)     equals direct convolution for several L, ragged K_t
  ola_convolve (Alg. 1)     equals direct convolution for K' in {8, 64}
  topk                      brute-force sort on small planes
  workload                  Tables 4 and 5 theoretical latency, 13.26 TFLOPS
"""
from .core import (conv, power, power_at, dft, template_spectrum, ols_geometry,  # noqa: F401
                   ols_convolve, ola_convolve, topk, threads)
from . import workload  # noqa: F401
