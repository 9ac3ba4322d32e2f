"""Oracle: a plain, slow, FP64 CPU reference of the coarsest-level solve.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import or run anything in this package.  The
GPU library never calls it, and it shares no code with the GPU library; both
take their inputs from the seeded generator in `synth`.

Contents (paper: Espinoza-Valverde, Frommer, Ramirez-Hidalgo, Rottmann,
"Coarsest-level improvements in multigrid for lattice QCD on large-scale
computers"):

* `operator`  - the coarse operator D_c as a 9-point block stencil (Sec. 2.2,
                eq. for the coarsest-level structure; Sec. 2.1 twisted mass),
                its apply, adjoint apply, dense / BSR assembly, block-Jacobi
                inverse (Sec. 3.2).
* `krylov`    - Arnoldi (Sec. 3.1, Alg. 1, and the modified Gram-Schmidt
                variant), restarted GMRES(m) with left/right preconditioning.
* `poly`      - harmonic Ritz values, Leja ordering (Alg. 2), the Newton-like
                form of q (Sec. 3.3), polynomially preconditioned GMRES (Alg. 3).
* `gcrodr`    - GCRO-DR with recycling across right-hand sides (Sec. 3.4).
* `mixed`     - FP16 block quantisation with per-block scale and an FP64
                flexible GMRES outer loop around a simulated FP32 inner solve.
* `adjoint`   - adjoint solves and the gradient of x = D_c^{-1} b.
* `lattice`   - periodic neighbour tables.

Every function here favours being checkable by eye against the paper over
speed: no blocking, fusion or reordering beyond what the paper states.
"""
