"""Seeded synthetic greyscale test images and batch recipes.

This module is the only code shared by the oracle and the GPU path: it draws
random images and random workload parameters and holds none of the sensing or
reconstruction arithmetic.

The paper evaluates on natural greyscale image sets (256x256 and 512x512,
8-bit, dynamic range [0, 255]; Table 1 note, Figs 4-5) that are not available
here.  These images stand in for them: smooth shading (background + Gaussian
blobs), sharp-edged opaque shapes (filled polygons) and a 1/f texture, which
gives blocks of very different sparsity, the property the adaptive budgets
react to.
"""

from .images import synth_image, synth_batch  # noqa: F401
