"""FP64 CPU oracle for the real spherical harmonic transform pair.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link anything in this package; only
the test suite, the smoke check and the CPU-baseline leg of the benchmark use
it.  It shares no code with the GPU path.

What it computes (all in float64 / complex128, plain definitions written out):

* ``grids``     -- latitude nodes and quadrature weights (App. B.1,
                   eqs. latlon_grid / latlon_quad_weights, the Clenshaw-Curtis
                   footnote, and Gauss-Legendre nodes).
* ``legendre``  -- orthonormal associated Legendre functions P^_l^m(cos t)
                   (App. B.3, eq. spherical_harmonics) by the three-term
                   recurrence, one order m at a time.
* ``transforms``-- SHT (eq. sht) as a quadrature sum, ISHT (eq. isht), their
                   exact adjoints, and a literal four-fold brute-force sum for
                   tiny grids.
* ``mix``       -- the per-degree complex channel mix (a multi-channel form of
                   the spectral convolution, App. B.4, eq. s2_spectral_conv)
                   and its adjoint.
* ``scores``    -- ensemble CRPS in its integral, rank and spread-skill forms
                   (App. D.4), the spectral and spatial CRPS loss terms
                   (App. E.1) and the angular and zonal power spectral
                   densities (App. F.7).
* ``noise``     -- the spherical diffusion process (App. B.7, eq.
                   spherical_diffusion) with a counter-based Philox4x64-10
                   generator and Box-Muller normals.

Every function is pinned by tests in ``tests/test_oracle_*.py`` against
closed forms, library special cases, invariants and brute force; the
full-size 721x1440 coefficients have no independent closed form
("parity unpinned" beyond those pins, see the test docstrings).
"""
from .grids import (equiangular_nodes, gauss_legendre, clenshaw_curtis_weights,
                    trapezoid_weights, grid)
from .legendre import legendre_order, legendre_table
from .transforms import sht, isht, sht_T, isht_T, sht_bruteforce, isht_bruteforce
from .mix import channel_mix, channel_mix_T, channel_mix_dW, isotropic_filter, isotropic_filter_T, isotropic_filter_dk
from .scores import (crps_integral, crps_sorted, crps_spread_skill, spectral_crps, spatial_crps,
                     psd, zonal_psd, crps_spread_skill_grad, spectral_crps_grad, spatial_crps_grad)
from .noise import philox4x64_10, normal_pairs, diffusion_params, diffusion_step

__all__ = [
    "equiangular_nodes", "gauss_legendre", "clenshaw_curtis_weights",
    "trapezoid_weights", "grid", "legendre_order", "legendre_table",
    "sht", "isht", "sht_T", "isht_T", "sht_bruteforce", "isht_bruteforce",
    "channel_mix", "channel_mix_T", "channel_mix_dW", "isotropic_filter", "isotropic_filter_T", "isotropic_filter_dk",
    "crps_integral", "crps_sorted", "crps_spread_skill", "spectral_crps", "spatial_crps", "psd", "zonal_psd",
    "crps_spread_skill_grad", "spectral_crps_grad", "spatial_crps_grad",
    "philox4x64_10", "normal_pairs", "diffusion_params", "diffusion_step",
]
