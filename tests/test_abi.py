"""The C-ABI library: it loads, exports every symbol include/txe.h declares,
and its host-only FP64 setup (the erf closed form of the 1-D convolution
matrices) agrees with the oracle's Gauss-Legendre construction.  No GPU."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from oracle import txe_oracle as O
from paper_2401_04189_amd import txe, workloads as W

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "txe.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(txe_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = txe.lib()
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), f"libtxe.so does not export {n}"
    # and the binding knows the signature of each of them
    assert set(names) == set(txe.SIGNATURES)


def test_abi_version_and_status_strings():
    L = txe.lib()
    hdr = open(HEADER).read()
    ver = int(re.search(r"#define TXE_ABI_VERSION (\d+)", hdr).group(1))
    assert L.txe_abi_version() == ver == 4
    for st in range(7):
        assert len(L.txe_status_string(st)) > 0


@pytest.mark.parametrize("alpha", [0.0, 1.1e-7, 1e-3, 0.3, 30.0, math.exp(8.0)])
def test_conv_matrix_closed_form_vs_oracle(alpha):
    """Library (erf / erfc / expm1 closed form, extended precision) against the
    oracle's composite Gauss-Legendre quadrature."""
    for n, L in ((24, 6.0), (64, 10.0)):
        x = W.uniform_grid(n, L).x[0]
        C_lib = txe.conv_matrix_1d(x, alpha)
        C_or = O.conv_matrix_1d(x, alpha)
        assert np.abs(C_lib - C_or).max() <= 1e-13


def test_conv_matrix_rejects_bad_input():
    x = W.uniform_grid(8, 2.0).x[0]
    with pytest.raises(txe.TxeError):
        txe.conv_matrix_1d(x, -1.0)
    with pytest.raises(txe.TxeError):
        txe.conv_matrix_1d(x[::-1].copy(), 1.0)
    with pytest.raises(txe.TxeError):
        txe.conv_matrix_1d(np.array([0.0, 1.0, 3.0, 4.0]), 1.0)   # not uniform


def test_context_without_gpu_fails_cleanly():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    st = txe.lib().txe_context_create(0, None, ctypes.byref(h))
    assert st != 0
    assert len(txe.lib().txe_last_error()) > 0
