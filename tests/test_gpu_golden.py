"""The library's FP64 energies of the 24^3 smoke workload against the stored
oracle values (tests/golden/oracle_24cube.json): E_x, every pair energy and
the exchange-matrix diagonal to 1e-9 relative."""
import json
import os

import numpy as np
import pytest
import torch

from paper_2401_04189_amd import txe, workloads as W

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_24cube.json")


def test_energies_match_the_stored_oracle_values():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gold = json.load(open(GOLD))
    s = W.build_config("cfg1")
    ctx = txe.Context(0)
    sysm = txe.System.from_workload(ctx, s)
    _, ex, ep, eo = txe.apply(ctx, sysm, s.psi.cuda(), compute="f64", want_pairs=True, want_orb=True)
    torch.cuda.synchronize()
    ep, eo = ep.cpu().numpy(), eo.cpu().numpy()
    ref_ep = np.array(gold["e_pairs_upper_row_major"])
    ref_d = np.array(gold["exchange_diagonal"])
    print(f"golden 24^3: E_x {float(ex):.15e} vs {gold['E_x']:.15e}", flush=True)
    assert abs(float(ex) - gold["E_x"]) <= 1e-9 * abs(gold["E_x"])
    assert np.abs(ep - ref_ep).max() <= 1e-9 * np.abs(ref_ep).max()
    assert np.abs(eo - ref_d).max() <= 1e-9 * np.abs(ref_d).max()
    sysm.close()
    ctx.close()
