"""CPU oracle for the TGBA hot path (arXiv 2410.04204).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import anything from here.  The
product path (``paper_2410_04204_amd``) never imports, links or executes the
oracle, and the oracle never imports the product package; the two share no
kernels, headers, helpers or tables.  Only the seeded input generators in
``workloads.py`` (which contain none of the method's arithmetic) serve both.

Everything here is plain double precision, written for legibility:

* ``model``    mode tables and vacuum energies (Example section, eqs. 4-6)
* ``basis``    Gaussian basis enumeration, momentum labels, truncation
* ``brute``    explicit 2^N state vectors and exact diagonalisation (N <= 12)
* ``lanczos``  sparse exact diagonalisation of the zero-momentum sector (N <= 24)
* ``wick``     literal generalized Wick theorem -> Pfaffian (Appendix A)
* ``heff``     the truncated effective Hamiltonian (eq. 2, eq. S4)
* ``spectral`` LAPACK eigensolve and the dynamic structure factor (eq. 8)
* ``quench``   overlaps (eqs. S5-S6), B(t) (eq. 9), <sigma^x>(t), eps (eq. 10)
* ``corr``     sigma^x_1 sigma^x_{j+1} matrices and connected correlators after a
               quench (appendix on correlation functions)
* ``mlp``      plain forward/backward pass of the basis-scoring network

Functions whose result has no independent pin say "parity unpinned" in their
docstring.
"""
