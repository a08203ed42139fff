"""FP64 CPU oracle for the FDAS correlation (Dimoudi et al. 2018).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links anything here: only the test suite, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg do.  The oracle shares no code with the GPU
library: it computes templates from the closed-form response with scipy's
Fresnel integrals and evaluates the correlation sum directly (no FFT).

Modules:
  templates  closed-form templates R(q, z) and the bank T[K][M]  (Sec. 2, eq. 23)
  direct     numpy FP64 correlation, power plane, loss gradients
  native     the same correlation and gradients in plain C + OpenMP (FP64)
  r2c        the real-to-complex transform of a time series (literal DFT)
  harmonic   harmonic sums of the power plane and peak candidates (FP32 sums
             in a fixed order, so threshold decisions match bit for bit)

Pins (tests marked "not gpu"): quadrature of the defining integral, the
z = 0 template as a Kronecker delta, conjugate symmetry of +/-z templates,
Parseval energy, the paper's 36 % scalloping loss at a half-bin offset,
injected-signal peaks against the sinc^2 limit, an independent time-domain
chirp route, the parallelogram law, brute-force overlap-save by explicit DFT
matrices (Sec. 3, Fig. 1), and central finite differences for the
gradients (exact for a quadratic loss).
"""
from . import templates, direct  # noqa: F401
