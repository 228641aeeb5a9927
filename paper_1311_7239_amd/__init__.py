"""MI355X (gfx950) implementation of the D2Q8 porous MRT lattice Boltzmann hot path of
Liu & He (arXiv:1311.7239): a C-ABI HIP library (``libmrtlbm.so``, include/lbm.h) and
its Python binding (``paper_1311_7239_amd.lbm``). Submodules load lazily so that the
seeded input generators import without a GPU."""
