"""GPU: batched factorization of many independent matrices (one block-
diagonal analysis), per-matrix log-determinants, hipGraph capture and
replay, and the panel-width autotuner.

Gates: per matrix, logdet relative difference to the oracle <= 1e-12 and
normwise backward error of the solve <= 1e-12 (fp64); a graph replay equals
the eager computation on the same values to the same bars (update
accumulation order through atomics is not fixed, so bit equality is not
asked), on every replay, with eager work and synchronizations between
replays and with the values changed in place between replays.
"""
import math

import numpy as np
import pytest

import gen
import oracle
from conftest import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

torch = pytest.importorskip("torch")
sc = pytest.importorskip("paper_2409_14009_amd")


def _batch(count, seed=None, nrhs=2, side2=(12, 48), side3=(8, 20)):
    probs = gen.make_batch(count=count, seed=seed, nrhs=nrhs, side2=side2, side3=side3)
    mats = [(p.n, p.colptr, p.rowind, p.perm) for p in probs]
    vals = np.concatenate([p.vals for p in probs])
    Bt = np.concatenate([p.B.T for p in probs], axis=1)  # (nrhs, N)
    return probs, mats, vals, np.ascontiguousarray(Bt)


def _check_per_matrix(probs, co, logdets, X, tol_eta=1e-12, tol_ld=1e-12):
    worst = (0.0, 0.0)
    for b, p in enumerate(probs):
        # the factor is unique: the oracle's supernode partition does not matter
        o = oracle.Symbolic(p.n, p.colptr, p.rowind, p.perm, 0, 0).factor(p.vals)
        assert o.info == 0
        ldo = o.logdet()
        rel = abs(logdets[b] - ldo) / max(abs(ldo), 1.0)
        A = oracle.full_matrix(p.n, p.colptr, p.rowind, p.vals)
        eta, _ = oracle.backward_error(A, X[:, co[b]:co[b + 1]].T, p.B)
        worst = (max(worst[0], rel), max(worst[1], float(eta.max())))
        assert rel <= tol_ld, (b, logdets[b], ldo)
        assert eta.max() <= tol_eta, (b, eta)
    return worst


@pytest.mark.parametrize("count,nb,z", [(24, 64, 0), (40, 32, 8), (64, 64, 8)])
def test_batch_factor_solve_logdet(count, nb, z):
    print(f"case batch count={count} nb={nb} z={z}", flush=True)
    probs, mats, vals, Bt = _batch(count)
    S = sc.BatchCholesky(mats, amalg_max_zeros=z, panel_width=nb)
    cnt, co, no = S.batch_info()
    F = S.factor(torch.tensor(vals, device="cuda"))
    lds = F.logdet_batch().cpu().numpy()
    X = F.solve(torch.tensor(Bt.T.copy(), device="cuda")).cpu().numpy().T  # (nrhs, N)
    w = _check_per_matrix(probs, co, lds, X)
    # the whole-batch logdet is the sum of the blocks'
    assert abs(F.logdet() - lds.sum()) <= 1e-12 * max(1.0, abs(lds).sum())
    print(f"  ok worst logdet {w[0]:.2e} eta {w[1]:.2e}", flush=True)


def test_batch_single_matrix_segments():
    """A plain (non-batch) factor has one segment: logdet_batch == logdet."""
    p = gen.make_config(0)
    S = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm)
    F = S.factor(torch.tensor(p.vals, device="cuda"))
    l1 = F.logdet_batch().cpu().numpy()
    assert l1.shape == (1,)
    assert abs(l1[0] - F.logdet()) <= 1e-12 * abs(l1[0])


def test_graph_replay_matches_eager():
    print("case graph replay count=32", flush=True)
    probs, mats, vals, Bt = _batch(32, nrhs=3)
    S = sc.BatchCholesky(mats, amalg_max_zeros=8)
    cnt, co, no = S.batch_info()
    v = torch.tensor(vals, device="cuda")
    F = S.factor(v)
    eager_ld = F.logdet_batch().cpu().numpy()
    B0 = torch.tensor(Bt, device="cuda")  # (nrhs, N) == column-major N x nrhs
    Xe = B0.clone()
    F.solve_(Xe)
    Xe = Xe.cpu().numpy()

    stream = torch.cuda.Stream()
    Xg = torch.empty_like(B0)
    with torch.cuda.stream(stream):
        G = F.capture(v, Xg, stream=stream)
    scale = [1.0, 2.0, 1.0, 0.5]
    for r, s in enumerate(scale):
        # eager work between replays: change values in place, touch other memory
        with torch.cuda.stream(stream):
            v.copy_(torch.tensor(vals * s, device="cuda"))
            Xg.copy_(B0)
            junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64).sum()
            G.replay(stream)
            lds = F.logdet_batch(stream=stream)
            assert F.status(stream) == 0
        stream.synchronize()
        lds = lds.cpu().numpy()
        Xr = Xg.cpu().numpy()
        # logdet(sA) = logdet(A) + n log s; x(sA) = x(A)/s
        ns = np.diff(co)
        exp_ld = eager_ld + ns * math.log(s)
        assert np.all(np.abs(lds - exp_ld) <= 1e-12 * np.maximum(np.abs(exp_ld), 1.0)), (r, lds - exp_ld)
        ex = np.abs(Xr * s - Xe).max() / np.abs(Xe).max()
        assert ex <= 1e-12, (r, ex)
        torch.cuda.synchronize()
        del junk
    # the graph's result at scale 1 also passes the oracle gates
    with torch.cuda.stream(stream):
        v.copy_(torch.tensor(vals, device="cuda"))
        Xg.copy_(B0)
        G.replay(stream)
    stream.synchronize()
    _check_per_matrix(probs, co, F.logdet_batch().cpu().numpy(), Xg.cpu().numpy())
    G.close()


def test_graph_detects_not_spd():
    p = gen.make_config(0)
    S = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm)
    v = torch.tensor(p.vals, device="cuda")
    F = S.factor(v)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        G = F.capture(v, stream=stream)
        v.neg_()
        G.replay(stream)
        st = F.status(stream)
        assert st >= 1
        v.neg_()
        G.replay(stream)
        assert F.status(stream) == 0
    G.close()


def test_autotune_batch(tmp_path, monkeypatch):
    from paper_2409_14009_amd import autotune
    monkeypatch.setenv("SPCHOL_TUNE_CACHE", str(tmp_path / "tune.json"))
    autotune._mem_cache.clear()
    probs, mats, vals, Bt = _batch(16, nrhs=1)
    v = torch.tensor(vals, device="cuda")
    best, times = autotune.tune_batch(mats, v, reps=2)
    assert best in autotune.CANDIDATES
    assert all(math.isfinite(t) and t > 0 for t in times.values())
    # cached: a second call returns the same choice without timing
    best2, _ = autotune.tune_batch(mats, v, reps=2)
    assert best2 == best
    assert (tmp_path / "tune.json").exists()


def test_solve_only_graph():
    """A graph holding only the solve reuses the current factor; replays
    after an eager refactorization with new values see the new factor."""
    p = gen.make_config(0)
    S = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm)
    v = torch.tensor(p.vals, device="cuda")
    F = S.factor(v)
    Bt = torch.tensor(np.ascontiguousarray(p.B.T), device="cuda")
    X = torch.empty_like(Bt)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        G = F.capture(None, X, stream=stream)
        for s in (1.0, 4.0, 1.0):
            F.refactor(v * s if s != 1.0 else v, stream=stream)
            X.copy_(Bt)
            G.replay(stream)
            stream.synchronize()
            x = X.cpu().numpy().T * s
            A = oracle.full_matrix(p.n, p.colptr, p.rowind, p.vals)
            eta, _ = oracle.backward_error(A, x, p.B)
            assert eta.max() <= 1e-12, (s, eta)
    G.close()
    with pytest.raises(sc.SpcholError):
        F.capture(None, None, stream=stream)


def test_graph_cache_repeated_calls():
    """Repeated refactorizations / solves with the same buffers run eagerly,
    then as a captured graph, then as replays: every call must see the
    current contents of its buffers (values changed in place, new
    right-hand sides), also after the solve workspace grows."""
    p = gen.make_config(1, side=12)
    S = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm, 0, 8)
    v = torch.tensor(p.vals, device="cuda")
    F = S.factor(v)
    A = oracle.full_matrix(p.n, p.colptr, p.rowind, p.vals)
    ld0 = oracle.Symbolic(p.n, p.colptr, p.rowind, p.perm, 0, 8).factor(p.vals).logdet()
    rng = np.random.default_rng(5)
    X = torch.empty((2, p.n), dtype=torch.float64, device="cuda")
    for it, s in enumerate([1.0, 2.0, 0.5, 3.0, 1.0]):
        v.copy_(torch.tensor(p.vals * s, device="cuda"))
        F.refactor(v)
        assert abs(F.logdet() - (ld0 + p.n * np.log(s))) <= 1e-11 * abs(ld0), it
        B = rng.standard_normal((p.n, 2))
        X.copy_(torch.tensor(B.T.copy(), device="cuda"))
        F.solve_(X)
        eta, _ = oracle.backward_error(A, X.cpu().numpy().T * s, B)
        assert eta.max() <= 1e-12, (it, eta)
    # a wider block moves the solve workspace: cached solves must follow
    X4 = torch.tensor(rng.standard_normal((4, p.n)), device="cuda")
    B4 = X4.cpu().numpy().T.copy()
    for _ in range(3):
        Y = X4.clone()
        F.solve_(Y)
        eta, _ = oracle.backward_error(A, Y.cpu().numpy().T, B4)
        assert eta.max() <= 1e-12
        X.copy_(torch.tensor(B[:, :2].T.copy(), device="cuda"))
        F.solve_(X)
        eta, _ = oracle.backward_error(A, X.cpu().numpy().T, B[:, :2])
        assert eta.max() <= 1e-12


def test_graph_replay_fp32_updates():
    """A batch factored with fp32 update products and captured: every
    replay matches the eager fp32 factor and solve (same arithmetic;
    atomics only reorder fp64 sums of the rounded products), and the
    unrefined solve's backward error sits at fp32 level, well above fp64
    rounding (the reduced-precision products are really used)."""
    print("case graph replay fp32 count=24", flush=True)
    probs, mats, vals, Bt = _batch(24, nrhs=2)
    S = sc.BatchCholesky(mats, amalg_max_zeros=8)
    cnt, co, no = S.batch_info()
    v = torch.tensor(vals, device="cuda")
    F = S.factor(v, precision="f32")
    eager_ld = F.logdet_batch().cpu().numpy()
    B0 = torch.tensor(Bt, device="cuda")
    Xe = B0.clone()
    F.solve_(Xe)
    Xe = Xe.cpu().numpy()
    stream = torch.cuda.Stream()
    Xg = torch.empty_like(B0)
    with torch.cuda.stream(stream):
        G = F.capture(v, Xg, stream=stream)
    for r in range(3):
        with torch.cuda.stream(stream):
            Xg.fill_(0.0)
            junk = torch.randn(1 << 18, device="cuda", dtype=torch.float64).sum()
            Xg.copy_(B0)
            G.replay(stream)
            lds = F.logdet_batch(stream=stream)
            assert F.status(stream) == 0
        stream.synchronize()
        lds = lds.cpu().numpy()
        Xr = Xg.cpu().numpy()
        assert np.all(np.abs(lds - eager_ld) <= 1e-10 * np.maximum(np.abs(eager_ld), 1.0)), r
        ex = np.abs(Xr - Xe).max() / np.abs(Xe).max()
        assert ex <= 1e-10, (r, ex)
        del junk
    worst = 0.0
    for b, p in enumerate(probs):
        A = oracle.full_matrix(p.n, p.colptr, p.rowind, p.vals)
        eta, _ = oracle.backward_error(A, Xr[:, co[b]:co[b + 1]].T, p.B)
        worst = max(worst, float(eta.max()))
    print(f"  worst unrefined eta {worst:.2e}", flush=True)
    assert 1e-14 <= worst <= 1e-5
    G.close()


@pytest.mark.parametrize("nrhs", [6, 10])
def test_graph_replay_many_rhs(nrhs):
    """More than four right-hand sides: groups of four solved alternately on
    the caller's stream and the second stream (fork and join inside the
    captured graph).  Every replay, with eager work and a change of values
    in between, matches the eager solve and the oracle's backward-error bar."""
    print(f"case graph replay nrhs={nrhs}", flush=True)
    p = gen.make_config(4, side=14)
    S = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm, 0, 8)
    v = torch.tensor(p.vals, device="cuda")
    F = S.factor(v)
    B = np.random.default_rng(90 + nrhs).standard_normal((nrhs, p.n))
    B0 = torch.tensor(B, device="cuda")
    Xe = B0.clone()
    F.solve_(Xe)
    Xe = Xe.cpu().numpy()
    A = oracle.full_matrix(p.n, p.colptr, p.rowind, p.vals)
    eta, _ = oracle.backward_error(A, Xe.T, B.T)
    assert eta.max() <= 1e-12, eta
    stream = torch.cuda.Stream()
    Xg = torch.empty_like(B0)
    with torch.cuda.stream(stream):
        G = F.capture(v, Xg, stream=stream)
    for r, s in enumerate([1.0, 2.0, 1.0]):
        with torch.cuda.stream(stream):
            v.copy_(torch.tensor(p.vals * s, device="cuda"))
            Xg.copy_(B0)
            junk = torch.randn(1 << 18, device="cuda", dtype=torch.float64).sum()
            G.replay(stream)
            assert F.status(stream) == 0
        stream.synchronize()
        ex = np.abs(Xg.cpu().numpy() * s - Xe).max() / np.abs(Xe).max()
        assert ex <= 1e-12, (r, ex)
        del junk
    G.close()


def test_autotune_batch_config(tmp_path, monkeypatch):
    """The tuner over supernode granularity, panel width and update method:
    its choice lies in the search space, every candidate was timed (or
    skipped by the axis-wise search), the tuned analysis passes the per-matrix
    oracle gates, and the choice is cached per precision."""
    from paper_2409_14009_amd import autotune
    monkeypatch.setenv("SPCHOL_TUNE_CACHE", str(tmp_path / "tune.json"))
    autotune._mem_cache.clear()
    probs, mats, vals, Bt = _batch(16, nrhs=2)
    v = torch.tensor(vals, device="cuda")
    B = torch.tensor(Bt, device="cuda")
    cfg, times = autotune.tune_batch_config(mats, v, B, "f64", reps=1)
    assert tuple(cfg["amalg"]) in [tuple(a) for a in autotune.AMALG_CHOICES]
    assert cfg["panel_width"] in autotune.WIDTH_CHOICES and cfg["update"] in autotune.UPDATE_CHOICES
    assert len(times) == len(autotune.AMALG_CHOICES) + len(autotune.WIDTH_CHOICES) + len(autotune.UPDATE_CHOICES) - 2
    assert all(math.isfinite(t) and t > 0 for t in times.values())
    print(f"  tuned {cfg} from {times}", flush=True)
    S = sc.BatchCholesky(mats, **autotune.config_kwargs(cfg))
    cnt, co, _ = S.batch_info()
    F = S.factor(v)
    Xt = B.clone()
    F.solve_(Xt)
    _check_per_matrix(probs, co, F.logdet_batch().cpu().numpy(), Xt.cpu().numpy())
    cfg2, _ = autotune.tune_batch_config(mats, v, B, "f64", reps=1)
    assert cfg2 == cfg
    cfg3, t3 = autotune.tune_batch_config(mats, v, B, "f32", reps=1)  # a new key: timed again
    assert len(t3) == len(times)
