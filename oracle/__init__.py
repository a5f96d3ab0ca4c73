"""CPU oracle for the 2-D lifting discrete wavelet transform.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or
executes this package: it exists so that tests, the smoke check and the
benchmark's CPU baseline can compare the HIP kernels against a plain, slow,
obviously correct definition written from Barina et al., "Accelerating
Discrete Wavelet Transforms on Parallel Architectures" (WSCG 2017,
arXiv:1704.08657).  It shares no code, constants or helpers with the HIP
library.

Modules
-------
lifting     separable lifting (the scheme of Section "Background", eq. (2) and
            the four 4x4 step matrices T_P^H, T_P^V, S_U^H, S_U^V), FP64 and
            int64, forward / inverse, multi-level Mallat layout.  This is the
            definition every kernel is compared against.
adjoint     the transpose W^T of the forward transform, built from explicit
            sparse 1-D step matrices and their transposes.
nonsep      the paper's fused non-separable lifting steps T_P and S_U
            (Section "Proposed Schemes") and the split P = P0 + P1,
            U = U0 + U1 (Section "Optimization Approach"), written as
            whole-plane 2-D neighbour gathers; used to pin the claim that the
            schemes compute the same values.
filterbank  closed-form CDF filters (roots of the Daubechies half-band
            polynomial) and brute-force separable / non-separable convolution
            on the symmetrically extended image.
polymat     exact Laurent-polynomial 4x4 matrix algebra and the paper's
            operation / step counting rule (Table 1).
window      evaluation of the oracle on crops, for sampled parity checks of
            very large images.
"""
