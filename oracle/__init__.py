"""CPU oracle for the determinant-CI Hamiltonian-vector product.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import anything from here.  The
GPU library never links, loads or calls it, and it never imports the GPU
package.  It shares no code with the GPU path.

Two independent tiers follow the paper's second-quantised Hamiltonian
(section 2.1, Eq. (1)):

* ``literal``  - tier A: dense matrices and density matrices by applying every
  operator term a+ / a to occupation bitstrings, in numpy.  Small cases only.
* ``sc``       - tier B: textbook Slater-Condon rules in plain C (``sc.c``),
  one row at a time, scanning the whole space for connected determinants.
* ``davidson`` - block Davidson-Liu over a sigma callback (numpy ``eigh`` for
  the subspace problem).
* ``csf``      - configuration state functions of section 2.3 (genealogical
  spin coupling, Yamanouchi-Kotani phase) written out in determinants, and
  sigma in that basis as T^T H T c.

Pins: every function is checked in ``tests/test_oracle_*.py`` against closed
forms, invariances, brute force and the other tier (see the test docstrings).
"""
