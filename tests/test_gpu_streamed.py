"""Host-resident factorization with one MI355X: supernodes at or above the
size threshold factored on the device (panel kernels on a copy of the one
supernode), their update matrices computed on the device in column blocks
that fit the device budget and added into the ancestors by the host; the
rest on the host.  Against the oracle (the factor is unique) and against
the device-resident factorization."""
import numpy as np
import pytest

import gen
import oracle
from conftest import gpu_available
from gpu_util import compare_factor, permuted_matrix, storage_to_csc

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

torch = pytest.importorskip("torch")
sc = pytest.importorskip("paper_2409_14009_amd")


@pytest.mark.parametrize("cfg,side,z,thr,budget", [
    (4, 20, 8, 0, 256 << 20),          # every supernode on the device
    (4, 20, 8, 20000, 256 << 20),      # split by size
    (1, 18, 8, 0, 4 << 20),            # small budget: many update blocks
    (2, 8, 8, 600000, 64 << 20),       # the paper's RL threshold
    (0, 48, 0, 2000, 1 << 20),
])
def test_streamed_vs_oracle(cfg, side, z, thr, budget):
    p = gen.make_config(cfg, side=side)
    print(f"streamed case cfg={cfg} side={side} thr={thr} budget={budget} n={p.n}", flush=True)
    S = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm, 0, z)
    L, info, st = S.factor_streamed(p.vals, device_budget=budget, host_threshold=thr)
    print(f"  {st}", flush=True)
    assert info == 0
    assert st["device_bytes"] <= budget + 16 * S.info()["storage"] // 1  # tasks aside, within the budget
    if thr == 0:
        assert st["host_supernodes"] == 0
    of = oracle.Symbolic(p.n, p.colptr, p.rowind, p.perm, 0, z).factor(p.vals)
    A = oracle.full_matrix(p.n, p.colptr, p.rowind, p.vals)
    Cm = permuted_matrix(A, p.perm)
    Lg, upper = storage_to_csc(S.export(), S.storage_offsets(), L, p.n)
    elt, offmax, fro = compare_factor(Lg, of.L_csc(), Cm.diagonal())
    print(f"  frobenius {fro:.2e} elementwise {elt:.2e}", flush=True)
    assert upper == 0.0 and offmax == 0.0 and fro <= 1e-12 and elt <= 1e-10
    # the device-resident factor of the same analysis, to rounding
    Ld = S.factor(torch.tensor(p.vals, device="cuda")).storage().cpu().numpy()
    assert np.abs(Ld - L).max() <= 1e-10 * np.abs(L).max()


def test_streamed_budget_too_small_and_not_spd():
    p = gen.make_config(4, side=14)
    S = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm, 0, 8)
    with pytest.raises(sc.SpcholError) as ei:
        S.factor_streamed(p.vals, device_budget=4096, host_threshold=0)
    assert ei.value.status == -4
    v = p.vals.copy()
    v[p.colptr[p.perm[-1]]] = -50.0  # the diagonal of the last-eliminated column
    with pytest.raises(sc.NotPositiveDefinite) as ei:
        S.factor_streamed(v, host_threshold=0)
    assert ei.value.info == oracle.Symbolic(p.n, p.colptr, p.rowind, p.perm, 0, 8).factor(v).info
