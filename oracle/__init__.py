"""CPU oracle for the BioEM posterior: TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct FP64 implementation of what the GPU path
computes, written from the paper (Cossio, Rohr et al., "BioEM:
GPU-accelerated computing of Bayesian inference of electron microscopy
images", Comput. Phys. Commun., arXiv 1609.06634).  It exists so that tests,
the smoke check and the benchmark's CPU-baseline leg have something
independent to compare the GPU library against.  Nothing in the product
package imports it; it imports nothing from the product package.  The only
code it shares with the GPU side is the seeded input generator in
``workloads`` (random numbers, no method arithmetic).

Every function is pinned by CPU tests against facts fixed by the paper or by
mathematics (brute-force integration of the likelihood, exact invariances,
Plancherel, direct-vs-FFT correlation, shift equivariance, parameter
recovery, high-precision log-sum-exp, projection mass and symmetry, CTF
special values; for the ensemble posterior, the cropping real-space variant
and Euler angles: 50-digit sums, zero-padded FFT correlation, a library
rotation).  The absolute level of log P depends on the prior reading
(flat N and mu, Jeffreys lambda, uniform normalised grid priors); the paper
prints no posterior values, so that level is "parity unpinned" beyond the
closed-form integral itself.

``cnn_oracle`` is the FP64 reference of the orientation-proposal network
(forward, backward, cross entropy, top-K), pinned by finite differences and a
library correlation; it is likewise test infrastructure only.
"""
from .bioem_oracle import (  # noqa: F401
    quat_to_matrix, euler_to_matrix, matrix_to_quat, euler_to_quat, project_model, ctf_envelope_table, filtered_projection,
    image_moments, projection_norm, correlation_direct, correlation_fft, correlation_cropped,
    log_likelihood, loglik_at, logsumexp_exact, logpost_oracle, OracleResult, ensemble_logpost,
    render_image, render_images, signed_freq, psf_kernel, psf_convolution, calculated_image,
)
