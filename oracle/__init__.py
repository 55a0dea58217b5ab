"""FP64 CPU oracle of the semi-analytical isogeometric thermal model.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check of the package
entry point and the CPU-baseline leg of the benchmark may import this
package.  The HIP library never calls it and shares no code with it; the only
thing both consume is the seeded input generator module of the package
(patches, materials, scan paths), which holds none of the method's
arithmetic.

Everything here is plain, slow and written to be checked against the paper
by eye (Yang, Ji, Moeller, Ayas, "Efficient thermal simulation in metal
additive manufacturing via semi-analytical isogeometric analysis"):

  bspline     Cox-de Boor B-spline basis and NURBS rationalisation (Sec. 2.3)
  iga         geometry map, Gauss quadrature, mass and conductivity matrices
              (Eqs. 16-17), boundary quadrature tables (Eq. 18)
  pointsource point-source kernel and its superposition (Eqs. 7-8)
  solver      transferred boundary data (Eqs. 10-11), load vector (Eq. 18),
              theta-scheme (Eqs. 19-20), reconstruction (Eq. 21)
  mlp         FP64 forward/backward of the far-history network

Readings where the paper is silent or ambiguous are listed in each module.
Every function is pinned by tests under tests/ against closed forms,
library routines, invariants or brute force; none is pinned against the
HIP path.
"""
