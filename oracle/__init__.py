"""FP64 CPU oracle for the electrokinetic lattice-Boltzmann / MD time step.

This package is test infrastructure.  Only the test-suite, the smoke check and
the CPU-baseline leg of the benchmark import it; the product path (the HIP
library and its Python binding) never does, and shares no code with it.

Every function is plain NumPy in float64, written from the paper's statement
of the method (Sec. II): the D3Q19 kinetic scheme with BGK relaxation and a
second-order forcing term (Eqs. kernelf, kernelf2, kernelg), the inter-species
drag (Eq. Fidef), the Poisson equation (Eq. poisson) solved by red-black SOR
with Chebyshev acceleration (Sec. II.C), and Langevin beads coupled by friction
(Sec. II.B).  Where the paper is silent the module docstrings state the reading
taken.

Modules
-------
d3q19    lattice velocities and weights (Sec. II.C)
lb       moments, equilibrium, forcing, drag, collision, streaming
poisson  7-point Laplacian, residual, red-black SOR + Chebyshev schedule
md       trilinear kernels, FENE/WCA/wall forces, friction-coupled substeps
noise    Philox4x32-10 random numbers, the D3Q19 mode basis, the stochastic
         term Delta of the populations and the beads' Langevin noise
step     one full time step in the order of the paper's algorithm (Fig. 1)
unet     float64 reference of the 3-D convolution network used as a warm start
"""
