"""MI355X-native block-adaptive, moment-encoded D3Q27 lattice Boltzmann step
(after arXiv 2603.14982). The compute path is the HIP library liblbmx.so behind
the C ABI of include/lbm.h; `lbm` is its Python binding."""
