"""The back-projection forms (streaming, batched loads, LDS-staged) compute
the same products in the same order, so in FP32 compute every form and
c-tile count must give bitwise the same Vx psi and E_x as the default, at
two to eight b tiles, one to three rank tiles, FP32 and FP64 orbitals (with
and without the FP32 copy of the orbitals), symmetric and block mode.  The
default itself is checked against the FP64 path.  FP64 compute: the same
bitwise agreement of the three forms (its default is the LDS-staged form
where its LDS fits one workgroup per CU)."""
import json

import pytest
import torch

from paper_2401_04189_amd import txe, workloads as W

pytestmark = pytest.mark.gpu

CASES = [  # n, L, N, r, K: b tiles = ceil(n / 16)
    (24, 6.0, 4, 12, 8),    # 2 b tiles, 1 rank tile
    (60, 8.0, 3, 20, 8),    # 4 b tiles, 2 rank tiles
    (92, 9.0, 3, 40, 6),    # 6 b tiles, 3 rank tiles
    (120, 10.0, 3, 24, 6),  # 8 b tiles, 2 rank tiles
]
FORMS = [(1, 1), (1, 2), (2, 1), (2, 2), (3, 1), (3, 2)]  # (back_form, back_ncg)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = txe.Context(0)
    yield c
    c.close()


def forced(ctx, sysm, psi, form, ncg, key_path, compute="f32", **kw):
    """Apply with the back form forced through the launch-shape cache."""
    key = next(iter(json.loads(key_path.read_text())))
    ent = dict(ngs_mul=1, proj_gt=4, back_ncg=ncg, grid_cap=2048, back_form=form)
    key_path.write_text(json.dumps({key: ent}))
    assert txe.tune_load(ctx, key_path) == 1
    out = txe.apply(ctx, sysm, psi, compute=compute, **kw)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"n{c[0]}r{c[3]}")
@pytest.mark.parametrize("psi_dtype", ["f32", "f64"])
def test_back_forms_bitwise(ctx, case, psi_dtype, tmp_path, monkeypatch):
    n, L, N, r, K = case
    s = W.make_system(f"bf{n}", n, L, N, 3, (0.4, 2.5), r, K, seed=900 + n, box=0.4 * L)
    psi = s.psi.cuda().to(torch.float32 if psi_dtype == "f32" else torch.float64)
    for mode in ("symmetric", "block"):
        kw = dict(symmetric=True) if mode == "symmetric" else dict(symmetric=False, i0=1, Ni=N - 1)
        c2 = txe.Context(0)  # a fresh context: no tuned shapes
        try:
            sysm = txe.System.from_workload(c2, s)
            v0, e0, _ = txe.apply(c2, sysm, psi, compute="f32", **kw)
            vf, ef, _ = txe.apply(c2, sysm, psi.double(), compute="f64", **kw)
            torch.cuda.synchronize()
            dE = abs(float(e0) - float(ef))
            print(f"[n{n} r{r} {psi_dtype} {mode}] default FP32 vs FP64 |dE| {dE:.2e}", flush=True)
            assert dE <= 1e-5
            # a cache entry with this problem's key, from one short tuning run
            txe.tune(c2, sysm, psi, "f32", reps=1, **kw)
            path = tmp_path / f"k_{mode}.json"
            txe.tune_save(c2, path)
            for form, ncg in FORMS:
                v, e, _ = forced(c2, sysm, psi, form, ncg, path, **kw)
                assert torch.equal(v, v0), f"form {form} ncg {ncg}: Vx psi differs"
                assert float(e) == float(e0), f"form {form} ncg {ncg}: E_x differs"
            if psi_dtype == "f64":
                # a workspace limit below four times the FP32 copy of the orbitals:
                # the copy is dropped and the kernels read FP64 orbitals
                monkeypatch.setenv("TXE_TEST_MAX_WORKSPACE", str(16 * N * n ** 3 - 1))
                for form, ncg in FORMS:
                    v, e, _ = forced(c2, sysm, psi, form, ncg, path, **kw)
                    if form == FORMS[0][0] and ncg == 1:
                        vd, ed = v, e
                    assert torch.equal(v, vd) and float(e) == float(ed)
                monkeypatch.delenv("TXE_TEST_MAX_WORKSPACE")
            sysm.close()
        finally:
            c2.close()


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"n{c[0]}r{c[3]}")
def test_back_forms_bitwise_f64(case, tmp_path):
    n, L, N, r, K = case
    s = W.make_system(f"bf{n}", n, L, N, 3, (0.4, 2.5), r, K, seed=900 + n, box=0.4 * L)
    psi = s.psi.cuda()
    for mode in ("symmetric", "block"):
        kw = dict(symmetric=True) if mode == "symmetric" else dict(symmetric=False, i0=1, Ni=N - 1)
        c2 = txe.Context(0)
        try:
            sysm = txe.System.from_workload(c2, s)
            v0, e0, _ = txe.apply(c2, sysm, psi, compute="f64", **kw)
            torch.cuda.synchronize()
            print(f"[n{n} r{r} f64 {mode}] E_x {float(e0):.15e}", flush=True)
            txe.tune(c2, sysm, psi, "f64", reps=1, **kw)
            path = tmp_path / f"k64_{mode}.json"
            txe.tune_save(c2, path)
            for form, ncg in FORMS:
                v, e, _ = forced(c2, sysm, psi, form, ncg, path, compute="f64", **kw)
                assert torch.equal(v, v0), f"form {form} ncg {ncg}: Vx psi differs"
                assert float(e) == float(e0), f"form {form} ncg {ncg}: E_x differs"
            sysm.close()
        finally:
            c2.close()
