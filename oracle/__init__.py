"""FP64 CPU oracle for lifted (spectral-axis) PROPELLER reconstruction.

TEST INFRASTRUCTURE. This package is the slow, plain reference that the HIP path
is checked against. Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import it; the product path never does, and it imports
nothing from the product package.

Every function follows the paper (Ghosh, Wetzstein, Pilanci, Fridovich-Keil,
"Volumetric Reconstruction Resolves Off-Resonance Artifacts in Static and Dynamic
PROPELLER MRI", CVPR 2024) in complex128 arithmetic; each docstring cites the
section or equation it follows. Points where the paper is silent are fixed by
the readings listed in the module docstring of ``lifted``.
"""

from .lifted import (  # noqa: F401
    Geometry,
    MASK_EPS,
    signed_freq,
    blade_mask,
    blade_masks,
    displacement,
    taps,
    shear,
    shear_transpose,
    knot_weights,
    volume_at,
    project_blade,
    forward_blade,
    forward,
    residual,
    data_loss,
    adjoint,
    tv_value,
    tv_grad,
    l1_value,
    l1_grad,
    objective,
    gradient,
    adam_update,
    gd_update,
    reconstruct,
    splitmix64,
    random_blade,
    render,
    coverage_baseline,
    window_baseline,
    psnr,
    simulate_measurements,
)
