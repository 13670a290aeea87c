"""CPU oracle for compact (linear-storage) multigrid — TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct numpy implementation of what the GPU path
computes, written from the paper ("Multigrid with Linear Storage
Complexity", Bauer, Kohl, McCormick, Tamstorf, arXiv 2511.19036).  Only the
test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it; the product library never does, and this package
imports nothing from the product package.  Inputs come from ``synthetic``.

Modules

* :mod:`oracle.bfp`      block floating point codec (Sec. 6.1.3 "Exponents",
                          precision-change rule of Sec. 4), widening (Sec. 2.2).
* :mod:`oracle.grid`     level grids, finite-difference operators, transfers,
                          smoothers (the multigrid components of Sec. 3.1).
* :mod:`oracle.compact`  compact FMG: residual (Alg. 2), compact V-cycle
                          (Alg. 1 / eq. cfas, generalised to V(nu1, nu2) from a
                          zero initial guess), compact FMG with IR (Alg. 3).
* :mod:`oracle.plain`    plain FP64 FMG with IR and correction-scheme V-cycle
                          (supplement, Alg. SM2), the comparator.
* :mod:`oracle.dense`    dense matrices on tiny grids for the pins.
* :mod:`oracle.adjoint`  adjoint solve and gradient of a least-squares loss with
                          respect to the cell diffusion coefficient.

Functions whose parity is not pinned to anything but the oracle itself say so
in their docstring ("parity unpinned").
"""
