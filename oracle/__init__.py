"""Plain, slow CPU FP64 oracle of the FODIBM-R + hybrid lattice Boltzmann time step.

TEST INFRASTRUCTURE ONLY. Nothing in the product path (the HIP library and its
Python binding) imports, links or calls anything in this package; only the test
suite, the smoke check and the CPU-baseline leg of the benchmark do.

Written from: Mao, Zhao, Boivin, Favier, "An improved fully one-sided
diffuse-interface immersed boundary method with target-value reconstruction for
compressible flows" (arXiv 2607.07432). Equation numbers follow the paper's
numbering (main text Eqs. (1)-(39), Appendix A Eqs. (A.1)-(A.16)).

Modules
  lattice  velocity sets, weights, Hermite polynomials (Appendix A)
  lbm      hybrid LBM collision, LB-consistent fluxes, MUSCL-Hancock energy
           update, streaming and domain closure (Sec. 2.2, Appendix A)
  ib       DIBM / FODIBM / FODIBM-R geometry, interpolation, target-value
           reconstruction, forces and spreading (Secs. 2.3-2.5)
  loads    drag / lift / Nusselt, boundary-condition errors, residual
           (Secs. 3.2, 3.5; where the paper gives no formula, the reading is
           stated in the function docstring)

Every floating-point value is numpy float64. No blocking, fusion or reordering
beyond what the paper's definitions state.

Parity unpinned by the paper: a^C and the time derivative in Eq. (A.9) (lbm), the absolute
loads (loads), and the network and warm-start helpers (unet, warmstart), which the paper does
not contain; each is pinned by definitions, closed forms or physics tests instead.
"""
