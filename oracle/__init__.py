"""CPU oracle for the parallel heat method for geodesic distance.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link anything under ``oracle/``; only
the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.

The oracle is plain, slow and FP64 (x87 extended precision is not needed: the
diffusion solve is made range-safe by an exact diagonal similarity, see
:mod:`oracle.diffusion`).  It follows Tao et al., "Parallel and Scalable Heat
Methods for Geodesic Distance Computation" (arXiv 1812.06060):

* :mod:`oracle.mesh`       mesh topology: edges, orientation halfedges, face
                           signs (Sec. 4.1, Eq. 20 and Fig. 6)
* :mod:`oracle.assembly`   face areas, cotangent Laplacian, lumped vertex
                           areas, mean edge length (Sec. 3.1, Eqs. 4, 7, 27)
* :mod:`oracle.diffusion`  backward-Euler heat step, Eq. 4; the paper's
                           breadth-first Gauss-Seidel, Eqs. 6-7
* :mod:`oracle.gradient`   face gradients and the normalised field, Eq. 3;
                           edge targets, Eq. 18
* :mod:`oracle.poisson`    the heat method's Poisson step (Sec. 3.2), face
                           form and edge-form variant, Dirichlet at sources
* :mod:`oracle.admm`       face ADMM (Sec. 3.2) and edge ADMM (Sec. 4.1) in
                           the paper's update order
* :mod:`oracle.bfs`        breadth-first vertex sets and pairing (Eq. 6,
                           Sec. 3.3)
* :mod:`oracle.integrate`  integration of face gradients (Eq. 17) and of edge
                           differences (Sec. 4)
* :mod:`oracle.metrics`    E (Eq. 8), epsilon (Eq. 28), E1/E2 (Eqs. 29-30) and
                           the diameter-normalised parity errors
* :mod:`oracle.pipeline`   the whole heat method end to end

Parity pins (what each function is checked against) live in
``tests/test_oracle_*.py``; functions without an independent pin say
"parity unpinned" in their docstring.
"""
