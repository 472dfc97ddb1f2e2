"""Seeded synthetic input generators.

This package produces the inputs that both the CPU oracle and the GPU library
consume: wavelength grids, the colour-matching table, reflectance and
illuminant spectra, Perlin-blended spectral textures, codec matrices and
light-path records.  It holds none of the method's arithmetic (no encoding,
shading, decoding or loss): every array it returns is input data.

The paper measures on Munsell / LSPDD spectra and Mitsuba scenes (Sec. 4.4,
Sec. 6).  None of that data is available here; these generators stand in for
it with the same kinds of spectra (broad Gaussian mixtures for reflectance,
Planckian and narrow-band Gaussian mixtures for light, unit-peak lights as in
Sec. 4.4) at the workload shapes the benchmark uses.
"""

from .spectra import (  # noqa: F401
    wavelengths,
    cmf_fit_cie1931,
    cmf_matrix,
    planck,
    planck_table,
    gaussian_mixture,
    reflectances,
    narrowband,
    illuminant_table,
    codec_uniform,
    codec_init,
    XYZ_TO_LINEAR_SRGB,
)
from .texture import perlin_texture, perlin_weights  # noqa: F401
from .paths import (  # noqa: F401
    mix64,
    rand64,
    stream_key,
    PathSpec,
    gen_paths,
    path_records,
    records_of_pixels,
    chain_records,
    uniform_indices,
)
from .config import config  # noqa: F401
from .workloads import workload  # noqa: F401
