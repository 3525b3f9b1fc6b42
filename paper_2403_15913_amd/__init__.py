"""MI355X-native Newton-step KKT solves (Lifted-KKT and HyKKT) behind the libkkt C ABI.

The numerical work runs in HIP kernels compiled for gfx950 into libkkt.so;
``paper_2403_15913_amd.kkt`` is the ctypes binding.
"""
