"""MI355X (gfx950) variational inference for the Bayesian non-negative factorial HMM.

The compute lives in libnfhmm.so (HIP kernels + C ABI, include/nfhmm.h);
``paper_1206_6468_amd.nfhmm`` is its ctypes binding.
"""
