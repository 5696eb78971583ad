"""Per-launch profile records (spchol_profile_launches): one record per timed
launch, levels within the schedule, and per kind the same launch counts and
algorithmic work as the per-kind sums of spchol_profile_read."""
import numpy as np
import pytest

import gen
from conftest import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

torch = pytest.importorskip("torch")
sc = pytest.importorskip("paper_2409_14009_amd")


def test_launch_records_match_kind_sums():
    print("case profile records cfg 1 side 12", flush=True)
    p = gen.make_config(1, side=12)
    S = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm, 0, 8)
    vals = torch.tensor(p.vals, device="cuda")
    F = S.factor(vals)
    nlev = S.info()["nlevels"]
    B = torch.tensor(np.ascontiguousarray(p.B.T), device="cuda")

    def run():
        F.refactor(vals)
        X = B.clone()
        F.solve_(X)
        torch.cuda.synchronize()

    F.profile(True)
    run()
    recs = F.profile_launches()
    F.profile(True)
    run()
    sums = F.profile_read()
    F.profile(False)
    assert recs and F.profile_launches() == []
    for r in recs:
        assert r["kind"] in sums and r["ms"] >= 0.0
        assert -1 <= r["level"] < nlev and r["side"] in (0, 1)
        assert r["side"] == 0 or r["kind"] == "update_ext"
    for kind, s in sums.items():
        mine = [r for r in recs if r["kind"] == kind]
        assert len(mine) == s["launches"], kind
        assert np.isclose(sum(r["flops"] for r in mine), s["flops"]), kind
        assert np.isclose(sum(r["bytes"] for r in mine), s["bytes"]), kind
    # the schedule's launches carry their level, the others -1
    assert {r["level"] for r in recs if r["kind"] in ("factor", "update_ext", "fwd", "bwd")} <= set(range(nlev))
    assert all(r["level"] == -1 for r in recs if r["kind"] in ("fill", "scatter_a", "perm"))


def test_launches_alone_mode():
    """Profiling with every launch alone (mode 2): the same launches per
    kind and the same algorithmic work as the overlapped mode, none on the
    second stream, and the same factor (the atomic adds may land in another
    order: within rounding)."""
    print("case profile alone cfg 1 side 14", flush=True)
    p = gen.make_config(1, side=14)
    S = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm, 0, 8)
    vals = torch.tensor(p.vals, device="cuda")
    F = S.factor(vals)
    F.profile(True)
    F.refactor(vals)
    ov = F.profile_launches()
    L_ov = F.storage().clone()
    F.profile(True, alone=True)
    F.refactor(vals)
    al = F.profile_launches()
    L_al = F.storage().clone()
    F.profile(False)
    assert any(r["side"] == 1 for r in ov), "no far updates on the second stream in this schedule"
    assert all(r["side"] == 0 for r in al)
    for kind in {r["kind"] for r in ov} | {r["kind"] for r in al}:
        a = [r for r in ov if r["kind"] == kind]
        b = [r for r in al if r["kind"] == kind]
        assert len(a) == len(b), kind
        assert np.isclose(sum(r["flops"] for r in a), sum(r["flops"] for r in b)), kind
    assert F.status() == 0
    err = (L_al - L_ov).abs().max().item() / L_ov.abs().max().item()
    assert err <= 1e-12, err
    # a mode other than 0, 1, 2 is an argument error
    with pytest.raises(sc.SpcholError):
        sc._check(sc.capi.lib().spchol_profile(F._h, 3))
