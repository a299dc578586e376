"""FP64 CPU oracle for the batched docking hot path (TEST INFRASTRUCTURE ONLY).

This package is a plain, slow, obviously-correct restatement of what the
GPU path computes, written from the TRIDS paper (arXiv 2510.24186) and the
readings listed beside each function.  It exists to check the GPU library.
Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import it; the product path never calls it and shares no code with it.

Modules
  params    atom-type table and the two term presets (TRIDS physics, Vina form)
  terms     pair functions phi_k(d) and their derivatives
  atomtype  ligand atom typing
  topology  fragments, torsion tree, root choice, intra-ligand pair list
  fk        forward kinematics of the torsion tree and its Jacobian products
  maps      brute-force receptor grid maps
  score     energy and gradient (grid or direct pairwise), chain rule to DOFs
  optim     Adam and Armijo line-search local steps
  philox    Philox4x32-10 counter-based generator
  sampler   Metropolis Monte Carlo driving the local steps
  best      rank, RMSD clustering, top-N and the screening score
  adjoint   gradients of summed scores w.r.t. map values, weights, coordinates

Parity status: every function here is pinned by a CPU test in tests/ against
closed forms, library routines, brute force or finite differences; none is
marked "parity unpinned".
"""
