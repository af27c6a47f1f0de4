"""MI355X-native THC-factorized rank-reduced CCSD hot path (arXiv:2111.11473).

The compute path is the HIP library under csrc/ (C ABI declared in include/thc.h);
`paper_2111_11473_amd.thc` is its ctypes binding.  `synth` generates seeded inputs.
Nothing is imported eagerly so that the input generator can be used without the GPU library.
"""
