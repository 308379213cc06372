"""Plain FP64 CPU oracle for the wavelength-adaptive 27-point Helmholtz path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link anything in this package; only
the tests, the smoke check and the CPU-baseline leg of the benchmark do.

It is written from the paper (Aghamiry, Gholami, Combe, Operto: "Accurate 3D
frequency-domain seismic wave modeling with the wavelength-adaptive 27-point
finite-difference stencil") and shares no code with the GPU path:

* ``table``     -- dispersion relation (Sec. 2.2, eq. for the normalised phase
                   velocity), the linear system H w = g and the Tikhonov-smoothed
                   weight table (Sec. 2.2, regularised problem with L = D P).
* ``operator``  -- per-row weight selection by the local G (Sec. 3.1, "GA"),
                   PML stretching (Sec. 2.1) and explicit CSR assembly of the
                   27-point stiffness + consistent mass (Sec. 2.1, weighted sum
                   of stiffness matrices, second consistent-mass form).
* ``solve``     -- point-source right-hand side (Sec. 3.1) and a plain
                   dense / sparse-direct solve of the assembled system.
* ``analytic``  -- homogeneous-medium Green's function and the amplitude factor
                   of the discrete operator, used to pin the oracle.
* ``accuracy``  -- the wavefield accuracy metric (Sec. 3.1, equation err) and
                   the closed-form Green's function of the linear-velocity
                   benchmark (Sec. 3.2).

Every function cites the passage it follows; readings of points the paper
leaves open are listed in each module docstring.
"""
