"""MI355X-native thermal lattice Boltzmann (D2Q37, D2Q17 or D2Q9) with a perfectly matched layer and
open boundaries (arXiv 2504.20169): HIP kernels behind a C ABI (``include/lbm.h``) and a thin
ctypes binding (``paper_2504_20169_amd.lbm``)."""
