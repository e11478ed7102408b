"""Plain, slow FP64 CPU oracle of the N-phase conservative Allen-Cahn + Navier-Stokes
lattice Boltzmann step (Zhan, Liu, Chai, Shi, "A comparative study of two Allen-Cahn
models for immiscible N-phase flows by using a consistent and conservative lattice
Boltzmann method", Sec. 2-3).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or link this
package: only the tests, the graft smoke check and the CPU-baseline leg of the bench use
it.  It shares no code with the HIP path; it depends on NumPy only.

Modules
-------
lattice  D2Q9 (the paper's natural moment matrix, Sec. 4 intro) and D3Q19 (raw-moment
         basis of the same construction; the paper only uses D2Q9).
nphase   parameters, initial state, one time step (whole-grid NumPy arrays, literal
         moment-space collisions M^-1 S M), macroscopic fields and per-phase mass.  The
         adjoint tests take central finite differences of losses through it.
nphase_loops
         the same step written a second time, node by node with explicit periodic
         neighbour coordinates and per-node moment-matrix products (tiny grids only);
         it cross-checks the vectorised module.
"""
