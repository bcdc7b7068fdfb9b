"""MI355X-native (gfx950) leapfrog shaped-stencil acoustic wave propagation.

Hot path of Peixoto & Silva, "Arbitrary high order shaped stencils for time
domain finite difference schemes in seismic wave propagation": explicit
leapfrog stepping of u_tt - c^2 lap(u) = f with cross, rhombus and square
Laplacian stencils of any radius, a damping layer, a Ricker source and
receiver traces, plus the exact discrete adjoint (FWI gradient) and batched
ragged multi-shot execution.  The compute runs in hand-written HIP kernels
behind the C ABI declared in include/fdwave.h.
"""
