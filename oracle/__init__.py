"""FP64 CPU oracle for saliency-guided progressive hologram generation.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain, obviously-correct
reference that the GPU path is checked against.  Only the test suite, the
smoke check and the benchmark's CPU-baseline leg may import it; the product
library never does, and the two share no code.

What it computes (paper: "Progressive hologram generation based on object
saliency", arXiv 2211.09938):

* ``haar``        -- 3-level (any-level) averaging Haar analysis/synthesis,
                     Mallat layout (Sec. 2, Eq. 2 and algorithm step 1).
* ``saliency``    -- saliency quantisation by block maximum to 1/2, 1/4, 1/8
                     size and the per-level thresholds (step 1, Sec. 3).
* ``fresnel``     -- the point-source object wave of Eq. 1 in its Fresnel
                     (paraxial) form, evaluated as a direct 2D sum over points.
* ``progressive`` -- the progressive hologram: layer split, DWT, detail
                     masking, synthesis, direct sum (Eq. 3 and steps 2-5).
* ``literal``     -- the same hologram computed the way steps 2-5 describe it
                     (image-domain residual maps times shifted block fringes)
                     plus the paper's operator accounting (Sec. 3).
* ``fringe``      -- the 1D block fringes g_lo, g_hi of the Haar basis blocks (the
                     factors of the paper's look-up-table blocks, Sec. 2).
* ``separable``   -- the same hologram over a window as three matrix products
                     (the paraxial kernel factors per axis), for large sizes.
* ``exact``       -- Eq. 1 with the exact distance and 1/r amplitude, to measure
                     the error of the Fresnel form.
* ``quality``     -- SSIM of the stage evaluation (Sec. 3).
* ``angular``     -- angular-spectrum propagation; with z -> -z the inverse
                     method the paper reconstructs its holograms with (Sec. 2).
* ``gradient``    -- the adjoint (gradient of a real loss with respect to the
                     object amplitudes) and the Fresnel back-propagation used
                     for the differentiable form.

All arithmetic is float64 / complex128.  Nothing here is blocked, fused or
reordered beyond the definitions it states.
"""

from . import (haar, saliency, fresnel, progressive, literal, gradient, separable, exact,  # noqa: F401
               quality, angular, fringe)
