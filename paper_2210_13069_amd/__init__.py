"""MI355X-native tensorized approximation of the long-range two-electron
integrals (arXiv 2210.13069): HIP kernels for gfx950 behind a C-ABI library
(`libtai.so`), with a thin ctypes binding in `tai`.

Importing the package is cheap; `paper_2210_13069_amd.tai` loads the library.
"""
