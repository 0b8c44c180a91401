"""The ceiling microbenchmarks behind each roofline's measured denominator:
every kind returns a rate between a fifth of and just above MI355X's
published peak (FP64 MFMA 78.6, FP32 MFMA 157.3, bf16 MFMA 2,516 TFLOP/s;
HBM 8,000 GB/s), and a kind outside [0, 3] is refused on the host."""
import ctypes

import pytest
import torch

from paper_2401_04189_amd import txe

pytestmark = pytest.mark.gpu

PUBLISHED = {"f64": 78.6, "f32": 157.3, "bf16": 2516.0, "hbm": 8000.0}


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = txe.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("kind", ["f64", "f32", "bf16", "hbm"])
def test_ceiling_plausible(ctx, kind):
    v = ctx.ceiling(kind)
    print(f"{kind}: {v:.1f} (published {PUBLISHED[kind]})", flush=True)
    assert PUBLISHED[kind] / 5 <= v <= PUBLISHED[kind] * 1.05


def test_ceiling_bad_kind_refused(ctx):
    v = ctypes.c_double(-1.0)
    for kind in (-1, 4):
        with pytest.raises(txe.TxeError, match="not in"):
            txe._check(txe.lib().txe_measure_ceiling(ctx.h, kind, ctypes.byref(v)))
    assert v.value == -1.0
