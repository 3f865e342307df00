"""MI355X-native Metropolis + parallel tempering for the Trotter-Suzuki 2D
transverse-field Ising spin glass (arXiv:2310.07486).

The compute path is the HIP library ``libtfim.so`` behind the C ABI of
``include/tfim.h``; ``paper_2310_07486_amd.tfim`` is its ctypes binding.
"""
