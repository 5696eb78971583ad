"""RLB (Sec. II-B) on the GPU: the update applied by block pairs addressed
with one relative index per block, with and without partition refinement,
against the oracle.  The factor is unique for the elimination order the
analysis used (spchol_sym_perm); with partition refinement that order
relabels columns inside supernodes, and the supernodal storage holds the
oracle's structure for it plus explicit zeros, which must come out exactly
zero."""
import numpy as np
import pytest

import gen
import oracle
from conftest import gpu_available
from gpu_util import compare_factor, permuted_matrix, storage_to_csc

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

torch = pytest.importorskip("torch")
sc = pytest.importorskip("paper_2409_14009_amd")

CASES = [(1, 16, 8), (2, 7, 8), (4, 18, 8), (0, 64, 0)]


@pytest.mark.parametrize("cfg,side,z", CASES)
@pytest.mark.parametrize("pr", [False, True])
def test_rlb_factor_vs_oracle(cfg, side, z, pr):
    p = gen.make_config(cfg, side=side)
    print(f"rlb case cfg={cfg} side={side} z={z} pr={pr} n={p.n}", flush=True)
    S = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm, 0, z, update_method="rlb", partition_refinement=pr)
    perm = S.perm()
    vals = torch.tensor(p.vals, device="cuda")
    F = S.factor(vals)
    X = F.solve(torch.tensor(p.B, device="cuda")).cpu().numpy()
    Lst = F.storage().cpu().numpy()
    ld = F.logdet()
    of = oracle.Symbolic(p.n, p.colptr, p.rowind, perm, 0, z).factor(p.vals)
    A = oracle.full_matrix(p.n, p.colptr, p.rowind, p.vals)
    Cm = permuted_matrix(A, perm)
    Lg, upper = storage_to_csc(S.export(), S.storage_offsets(), Lst, p.n)
    elt, offmax, fro = compare_factor(Lg, of.L_csc(), Cm.diagonal())
    eta, _ = oracle.backward_error(A, X, p.B)
    rel_ld = abs(ld - of.logdet()) / abs(of.logdet())
    print(f"  frobenius {fro:.2e} elementwise {elt:.2e} off-structure {offmax} eta {eta.max():.2e} "
          f"logdet {rel_ld:.2e}", flush=True)
    assert upper == 0.0 and offmax == 0.0
    assert fro <= 1e-12 and eta.max() <= 1e-12 and rel_ld <= 1e-12
    # the same factor as the RL update on the same order, to rounding
    S2 = sc.SparseCholesky(p.n, p.colptr, p.rowind, perm, 0, z)
    if not pr:
        L2 = S2.factor(vals).storage().cpu().numpy()
        assert np.abs(L2 - Lst).max() <= 1e-10 * np.abs(Lst).max()


def test_rlb_deterministic_bitwise():
    p = gen.make_config(1, side=18)
    outs = []
    for _ in range(2):
        S = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm, 0, 8, update_method="rlb",
                              partition_refinement=True, deterministic=True)
        outs.append(S.factor(torch.tensor(p.vals, device="cuda")).storage().cpu().numpy())
    assert np.array_equal(outs[0].view(np.uint64), outs[1].view(np.uint64))


def test_rlb_mixed_precision_refined():
    p = gen.make_config(4, side=16)
    S = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm, 0, 8, update_method="rlb", partition_refinement=True)
    vals = torch.tensor(p.vals, device="cuda")
    F = S.factor(vals, precision="f32")
    X, berr, it = F.refine(vals, torch.tensor(p.B, device="cuda"))
    eta, _ = oracle.backward_error(oracle.full_matrix(p.n, p.colptr, p.rowind, p.vals), X.cpu().numpy(), p.B)
    print(f"  rlb f32 updates: {it} corrections, eta {eta.max():.2e}", flush=True)
    assert eta.max() <= 1e-12
