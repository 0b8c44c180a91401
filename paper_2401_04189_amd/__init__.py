"""Tucker-tensor Fock exchange on MI355X (gfx950).

The compute path lives in the HIP/C++ shared library ``libtxe.so`` built from
``csrc/``; :mod:`paper_2401_04189_amd.txe` is its ctypes binding.
"""
