"""MI355X-native THIIM solver (arXiv:1510.05218): split-field Yee iteration in
complex128 behind a C-ABI library of hand-written HIP kernels for gfx950."""
