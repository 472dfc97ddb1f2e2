"""FP64 CPU oracle of the batched light-path throughput path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow reference used to
check the GPU library.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the library and its Python
binding never do, and this package imports nothing from them.  Its inputs
are the float32 arrays produced by the seeded generators in ``synth``,
upcast to float64.

What it computes (each function cites the passage it follows):

* ``shade.encode`` / ``shade.decode``: the linear codec z = W_enc s,
  s_hat = W_dec z (Eq. 4) and the colour projection T_cmf (Sec. 4.3).
* ``shade.shade_spectral``: per-path product of the light spectrum with the
  weighted reflectance spectra met along the path (the operations listed in
  Sec. 3), projected to XYZ with T_cmf and averaged over a pixel's samples.
* ``shade.shade_latent``: the same in code space, with the element-wise
  product taken blockwise on k = 3B channels (Eq. 6).
* ``codec``: softplus reparameterisation (Eq. 5), the codec-fit loss
  (reconstruction of both spectra plus lambda times the product term, the
  L_rec and L_e2e parts of Eq. 8 without the cosine factor), its analytic
  gradient, and Adam.
* ``records``: the light-path record format read by both forms.
* ``multibounce.chain_xyz``: the cascaded products of the multi-bounce
  evaluation (Eq. 10) in spectral and latent form.
* ``upsample``: the RGB-to-latent upsampling network of Sec. 5 (three fully
  connected layers, width 128, SiLU between them).

Pins: every function here is checked in the CPU test suite against closed
forms, invariants, finite differences, exact rational brute force or
library routines (see tests/test_oracle_*.py).
"""

from . import codec, multibounce, records, shade, upsample  # noqa: F401
