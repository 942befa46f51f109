"""Plain FP64 CPU oracle for the circulant-preconditioned voxel JVIE solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) imports, calls or links anything in this package; only
the test-suite, the smoke check and the CPU-baseline leg of the benchmark do.
It shares no code, tables or constants with the HIP path.

Every function follows a passage of Groth, Polimeridis, Tambova & White,
"Circulant preconditioning in the volume integral equation method for
silicon photonics" (arXiv:1903.07884), cited by section / equation:

* ``contrast``   -- local medium operator M = (eps_r - 1)/eps_r (Sec. 2, eq. JVIE)
                    and the three homogenisations of Sec. 5.2.
* ``generator``  -- Galerkin entries N^{ab}_{ij} = <N p_j^b, p_i^a> of the voxel
                    discretisation (Sec. 2, eq. op_N) by piecewise Gauss-Legendre
                    quadrature with a Duffy transform at the singular corner.
* ``matvec``     -- (I - M N) w by explicit summation over all voxel pairs
                    (Sec. 2, eq. discrete_form / sys_mat).
* ``circulant``  -- T. Chan's optimal circulant (Sec. 4, eq. Chan), the
                    Chan-Olkin 1-level block circulant and its inverse
                    (Sec. 4, eqs. Di and the inverse after it), the memory
                    reduction of Sec. 5.1.1 (eqs. proxy1, proxy2) and the
                    blocked (partitioned) preconditioner of Sec. 5.3.
* ``gmres``      -- restarted, right-preconditioned GMRES (Sec. 1).

All arithmetic is complex128.  Precision, GMRES restart/side and the
quadrature of the singular integrals are not fixed by the paper; the readings
taken are listed in each module's header.
"""
