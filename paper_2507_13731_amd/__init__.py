"""MI355X (gfx950) implementation of pass-efficient randomized low-rank approximation of
quaternion matrices (arXiv 2507.13731): Alg. 2 (subspace) and Alg. 4 (block Krylov).

The compute path lives in libqlra.so (HIP kernels + C ABI, include/qlra.h); the Python
module `paper_2507_13731_amd.qlra` is its ctypes binding.
"""
