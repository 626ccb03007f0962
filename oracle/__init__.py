"""CPU oracle for the differentiable tile rasterizer: TEST INFRASTRUCTURE ONLY.

A plain, slow, FP64 numpy implementation of what the GPU path computes,
written from the paper (Sec. 2.1 forward with compact SnugBox tiles, Eq. 1-2;
Sec. 2.2 backward; Sec. 2.3 neural Gaussians) and from the 3DGS image
formation model the paper builds on (its reference for 3D Gaussian
Splatting, Kerbl et al. 2023).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package. The product path (the HIP library and its Python
binding) never imports it, and this package never imports the product path.
The two share no code: inputs come from the seeded generators, which hold
none of the method's arithmetic.

Modules:
    sh          real spherical-harmonic basis and its gradient
    preprocess  per-Gaussian projection (EWA), SH colour, SnugBox threshold
    binning     compact per-column tile sets, pair list sorted by (tile, depth)
    render      per-pixel front-to-back compositing and its backward
    backward    per-Gaussian chain rule back to the 3D parameters
    adam        the textbook Adam update
"""
