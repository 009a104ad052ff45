"""FP64 CPU oracle for the saliency -> Kalman prior -> MRF weight path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's CPU
baseline leg may import this package.  The product (the HIP library and its Python
binding) never calls it, and it shares no code with the product: the only module
both sides use is the seeded input generator, which holds none of this arithmetic.

Plain, slow, obviously correct NumPy in float64, written step by step from the
paper (Sections 3-6) and from the readings taken where the paper is silent:

* saliency.py  -- Itti-style saliency map (Section 3, Section 7.2): colour threshold,
                  features, Gaussian pyramid, Gabor orientation, centre-surround,
                  N(.) normalisation, across-scale sum, conspicuity, weighted sum.
* prior.py     -- observation q_t from the saliency map (Section 5), the Kalman prior
                  update (Section 6, the unnumbered recursion for p-hat and sigma_xi^2),
                  and the MRF capacities (Section 4, Eqs. 1-4).
* adjoint.py   -- the FP64 adjoint of the prior chain with respect to the channel
                  weights and the Kalman variances, plus central finite differences.
* variants.py  -- the variants of the prior: f by distance transform (Section 6), the
                  manual first-frame prior (Section 4, Section 8.1) and the stochastic
                  saliency map (Section 3).
* gmm.py       -- the colour likelihood of the t-links: two RGB Gaussian mixtures fitted
                  by EM with every pixel weighted by the prior (Sections 4, 5, 8.1).
* mincut.py    -- the minimum cut of the MRF (Section 4) on integer capacities: maximum
                  flow and the labelling with the largest object among the minimum cuts.
* pixel_adjoint.py -- the adjoint of the whole chain through the saliency model to the
                  frames' pixels (N, centre-surround, Gabor, pyramid, features).

Parity status: every function is pinned by the CPU tests (constant images, Gabor
closed form, Kalman steady state, brute-force loops, adjoint dot products, gauge
and transpose symmetries, finite differences).  The *quality* of the saliency
model itself (what the paper's private clips would show) is parity unpinned: the
paper prints no saliency or prior values.
"""
from .saliency import (OracleParams, Geometry, geometry, colour_max, features, blur, reduce_level,
                       pyramid, gabor_kernel, gabor, upsample, centre_surround, normalise,
                       saliency)
from .prior import (observation, kalman_gains, prior_clip, mrf_weights, border_mask,
                    run_clip)
from . import gmm, mincut, pixel_adjoint, variants
from .adjoint import (mse_mask_loss, prior_chain_forward, prior_chain_backward, blur_adjoint,
                      upsample_adjoint, finite_difference_grad)

__all__ = [
    "OracleParams", "Geometry", "geometry", "colour_max", "features", "blur", "reduce_level",
    "pyramid", "gabor_kernel", "gabor", "upsample", "centre_surround", "normalise", "saliency",
    "observation", "kalman_gains", "prior_clip", "mrf_weights", "border_mask", "run_clip",
    "mse_mask_loss", "prior_chain_forward", "prior_chain_backward", "blur_adjoint",
    "upsample_adjoint", "finite_difference_grad",
]
