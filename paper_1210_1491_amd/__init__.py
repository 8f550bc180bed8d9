"""MI355X-native library for the local Dirichlet-to-Neumann (BIE-WOS) method.

Yan, Cai & Zeng: walk on spheres for u on local hemispheres, then a
collocation solve of the local boundary integral equation for du/dn.  The
compute path is the HIP library ``libdtn.so`` (C-ABI in ``include/dtn.h``);
``paper_1210_1491_amd.dtn`` is its Python binding.
"""
