"""FP64 CPU oracle for APR-native discrete convolution (arXiv 2112.03592).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
statement of what the GPU library computes, used to check it.  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import it;
the product path never does.  It shares no code with the HIP library or its
Python binding, and it imports nothing from them.

Modules (each function cites the passage of the paper it follows):

* ``access``  -- LinearAccess (Algorithm 1), sequential iteration (Algorithm 2),
                 APR tree structure (Section 3.4, Algorithm 3), validity checks.
* ``tree``    -- tree values by average reduction over children (Section 3.4).
* ``stencil`` -- per-level stencils: same, restricted (Eq. restrict_stenc and
                 the averaging rule of Section 4.2), resolution-adaptive
                 (Eq. adapt_grad).
* ``conv``    -- level-l reconstruction (Section 3.5) and APR convolution
                 (Section 4.1); its adjoint (input and weight gradients).
* ``rl``      -- APR Richardson-Lucy deconvolution (Section 6.2).
"""
