"""Oracle for the BIE-WOS local DtN method -- TEST INFRASTRUCTURE ONLY.

A slow, plain FP64 CPU implementation of what the GPU path computes, written
from the paper (Yan, Cai & Zeng, "A parallel method for solving Laplace
equations with Dirichlet data using local boundary integral equations and
random walks"):

* ``wos``        -- walk on spheres with an epsilon shell (Sec. 2) and the node
                    estimator (Sec. 5.1.2, eq. bw87), in plain C (wos_oracle.c);
* ``patch``      -- hemisphere nodes (eq. bw85 with a trapezoid rule in the
                    azimuth), the whole-ball Green's function with one Kelvin
                    image (Sec. 4), the local BIE K sigma = b (eqs. bw49-bw51)
                    and its piecewise-constant collocation (Sec. 5.2);
* ``potential``  -- the integral representation of u from Dirichlet and
                    Neumann data (eq. bw03).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP library
(``paper_1210_1491_amd``) and imports nothing from it.
"""
