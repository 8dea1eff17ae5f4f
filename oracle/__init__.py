"""FP64 CPU oracle for the iHDG method (test infrastructure only).

This package is a plain, slow, deliberately unoptimised restatement of the
upwind HDG discretisation and of the iHDG iteration (Algorithm 1, Section 2)
for the three PDE families the paper analyses: steady scalar transport
(Section 3), the linearised shallow-water system (Section 3) and the
first-order convection-diffusion system (Section 4).

It exists only to check the GPU library.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  It shares no code with the HIP path: the reference element, the
mesh, the local operators and the solvers are all written here again, in
NumPy/SciPy, in the paper's notation.

Modules
-------
reference_element  GLL / Gauss rules and 1-D Lagrange bases.
mesh               uniform box meshes of quads/hexes, faces, neighbours.
transport          transport: local operators, iHDG, direct HDG, downwind
                   block substitution, dense brute force, NPC variant.
shallow_water      linearised shallow water (one Crank-Nicolson step).
convdiff           first-order convection-diffusion, plus GMRES driven by
                   the iHDG sweep.
norms              the fused GLL-weighted norm and the true L2 error.

Every function with no independent pin says "parity unpinned" in its
docstring.
"""
