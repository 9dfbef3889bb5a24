"""FP64 CPU oracle for the lubrication-adapted MFS solver of Broms, Barnett
and Tornberg, "Accurate close interactions of Stokes spheres using
lubrication-adapted image systems" (arXiv 2407.03343).

TEST INFRASTRUCTURE ONLY.  Nothing in the product library may import, link
or execute anything under this directory; only the test suite, the smoke
check and the CPU-baseline leg of the benchmark do.  It shares no code with
the HIP library: geometry, kernels, factorisation, matrix-vector product,
GMRES and post-processing are written here from the paper, in plain NumPy /
SciPy and one plain C pair-sum loop (``pairsum.c``), all in float64.

Modules
  geometry  -- node sets: proxy spheres, image lines, collocation caps,
               left weights, check points (Sections 2.1, 2.3, 5.1).
  kernels   -- Stokeslet, rotlet and potential-dipole tensors (Section 2.3)
               and dense target-from-source blocks.
  pairsum   -- ctypes wrapper of the C direct sum used for big sums.
  mfs       -- one-body preconditioned system: setup, pseudo-inverse apply,
               matrix-vector product, GMRES, force/torque extraction,
               residuals, dense brute-force solve (Sections 2.2, 3).
  brenner   -- Brenner's two-sphere squeeze series (Section 3, eq. Brenner).

Parity status of each function is stated in its docstring: "pinned" means a
CPU test checks it against something other than itself (a closed form, an
exact identity, an asymptotic limit, brute force).
"""
