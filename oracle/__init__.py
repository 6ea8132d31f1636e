"""CPU FP64 oracle for multi-shift BiCGstab(l) -- TEST INFRASTRUCTURE ONLY.

A plain, slow NumPy (complex128) statement of what the HIP library computes,
written from the paper (Heybrock, "Double-pass variants for multi-shift
BiCGstab(l)", Lattice 2010) and from the published methods it builds on.  It
shares no code with the HIP path and neither imports the other; both take
their inputs from the seeded generators in ``workloads``.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import or execute anything in this package.  The product
(``paper_1010_2592_amd``) never does.

Modules
  dirac     gamma matrices, the Wilson stencil D_w(mu) (mu as e^{+-mu} on
            the time links), H = gamma5 D_w, A = a H^2 (Section 1, Eq. (1.1) and the
            text after Eq. (1.2)), spectral-radius estimate, dense builders.
  pfe       Neuberger partial-fraction coefficients (Eq. (1.2), Fig. 1).
  krylov    seed BiCGstab(l), multi-shift single-pass, double-pass
            (Section 2 Eqs. (2.1)-(2.2), Section 3 cost table, Section 5).
  backward  gradients of Re<eta, f(A) b> (not in the paper; adjoint solves
            with A^dagger = A(-mu)).
"""
