"""The launch schedules of the symbolic analysis, replayed entry by entry on
the host (tests/plan_check.cpp): every entry of L gets exactly the update
contributions the right-looking method defines before it is factored, no
two tasks of one launch conflict, and the solve rounds respect their
dependencies.  Covers the one-panel lookahead, the inline / row-tile split
of the panel solve, every panel width and amalgamation."""
import os
import subprocess

import numpy as np
import pytest

import gen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("plan") / "plan_check")
    src = [os.path.join(ROOT, "tests", "plan_check.cpp"),
           os.path.join(ROOT, "paper_2409_14009_amd", "csrc", "analyze.cpp")]
    subprocess.run(["g++", "-O2", "-std=c++17", *src, "-o", exe], check=True)
    return exe


def _run(checker, tmp_path, n, cp, ri, perm, mode, z, nb, det=0, rule=0, rlb=0, pr=0, env=None):
    f = tmp_path / "pat.txt"
    perm = np.arange(n) if perm is None else perm
    with open(f, "w") as fh:
        fh.write(f"{n} {len(ri)}\n")
        fh.write(" ".join(map(str, cp)) + "\n")
        fh.write(" ".join(map(str, ri)) + "\n")
        fh.write(" ".join(map(str, perm)) + "\n")
    r = subprocess.run([checker, str(f), str(mode), str(z), str(nb), str(det), str(rule), str(rlb), str(pr)],
                       capture_output=True, text=True, env=None if env is None else dict(os.environ, **env))
    assert r.returncode == 0, r.stdout + r.stderr
    return r.stdout


@pytest.mark.parametrize("nb", [16, 32, 48, 64])
def test_grid2d(checker, tmp_path, nb):
    p = gen.make_config(0)
    _run(checker, tmp_path, p.n, p.colptr, p.rowind, p.perm, 0, 0, nb)


@pytest.mark.parametrize("side,z,nb", [(10, 8, 64), (12, 8, 32), (9, 0, 48), (11, 30, 16), (20, 8, 64)])
def test_grid3d(checker, tmp_path, side, z, nb):
    p = gen.make_config(1, side=side)
    out = _run(checker, tmp_path, p.n, p.colptr, p.rowind, p.perm, 0, z, nb)
    if side == 20:
        # panels with more than 512 rows below: the backward solve's split
        # (lookahead) tasks are part of the replay
        assert int(out.split("split_bwd=")[1].split()[0]) > 0, out
        # supernodes of several panels: two-panel forward tasks
        assert int(out.split("fwd2=")[1].split()[0]) > 0, out
        # levels of few wide supernodes: one launch per panel round
        assert int(out.split("fused_diag=")[1].split()[0]) > 0, out
        # far external updates on the second stream, forked at their level
        assert int(out.split("fork_probes=")[1].split()[0]) > 0, out
        # and the two-launch rounds everywhere instead
        out2 = _run(checker, tmp_path, p.n, p.colptr, p.rowind, p.perm, 0, z, nb, env={"SPCHOL_PANEL_ROUNDS": "2"})
        assert int(out2.split("fused_diag=")[1].split()[0]) == 0, out2
    # the algorithmic bytes the solve plans charge: each sweep reads every
    # stored entry of L below the diagonal blocks once and the lower
    # triangle of each inverted diagonal block once (plus 16 bytes per row
    # for the right-hand side), so both sweeps come to about 8 bytes per
    # stored entry, and to the same amount
    f = {kv.split("=")[0]: float(kv.split("=")[1]) for kv in out.split()[2:] if "=" in kv}
    fr, br = f["fwd_bytes"] / (8 * f["storage"]), f["bwd_bytes"] / (8 * f["storage"])
    assert abs(fr - br) <= 0.05 * br, (fr, br)
    if z >= 8:  # (without amalgamation the 16 bytes per row weigh more)
        assert 0.8 <= fr <= 1.2 and 0.8 <= br <= 1.2, (fr, br)
    # the leaves of the dissection are done by one-wavefront tasks, in the
    # solves too once a level holds enough of them
    assert int(out.split("small=")[1].split()[0]) > 0, out
    if side == 20:
        assert int(out.split("small_solve=")[1].split()[0]) > 0, out


def test_grid3d_root_past_the_window(checker, tmp_path):
    """28^3: a 15-panel root separator, past the window of the one-launch
    panel rounds, its column blocks taking their finished panels in
    ranges when they enter it (several ranges per block)."""
    p = gen.make_config(1, side=28)
    out = _run(checker, tmp_path, p.n, p.colptr, p.rowind, p.perm, 0, 8, 64)
    assert int(out.split("range_tiles=")[1].split()[0]) > 0, out


def test_elasticity(checker, tmp_path):
    p = gen.make_config(2, side=5)
    _run(checker, tmp_path, p.n, p.colptr, p.rowind, p.perm, 0, 8, 16)


@pytest.mark.parametrize("n,nb", [(150, 64), (150, 16), (65, 64), (1, 64), (400, 64), (1200, 64)])
def test_dense(checker, tmp_path, n, nb):
    cp = np.concatenate([[0], np.cumsum(np.arange(n, 0, -1))]).astype(np.int64)
    ri = np.concatenate([np.arange(j, n) for j in range(n)]).astype(np.int64)
    out = _run(checker, tmp_path, n, cp, ri, None, 0, 0, nb)
    if n >= 1200:
        # 19 panels: the column blocks past the rounds' window take their
        # finished panels in ranges when they enter it
        assert int(out.split("range_tiles=")[1].split()[0]) > 0, out
        # the deterministic schedule has no window (one add per entry and
        # launch)
        out = _run(checker, tmp_path, n, cp, ri, None, 0, 0, nb, det=1)
        assert int(out.split("range_tiles=")[1].split()[0]) == 0, out


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_random_patterns(checker, tmp_path, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(60, 300))
    n2, cp, ri, vv = gen.random_spd(n, rng.uniform(0.01, 0.08), rng)
    _run(checker, tmp_path, n2, cp, ri, rng.permutation(n2), int(rng.integers(0, 2)), int(rng.integers(0, 20)),
         int(rng.choice([16, 32, 48, 64])))


def test_batch_union(checker, tmp_path):
    probs = gen.make_batch(count=6, nrhs=1)
    # block-diagonal union, as the batch analysis forms it
    cps, ris, pms, off, nzoff = [], [], [], 0, 0
    for p in probs:
        cps.append(p.colptr[:-1] + nzoff)
        ris.append(p.rowind + off)
        pms.append(p.perm + off)
        off += p.n
        nzoff += p.nnz
    cp = np.concatenate(cps + [[nzoff]]).astype(np.int64)
    _run(checker, tmp_path, off, cp, np.concatenate(ris), np.concatenate(pms), 0, 8, 64)


# (leaf columns, rows of the parent): at and past the limits of the
# one-wavefront supernode (at most 16 columns; padded block + rows below +
# one unit row per column within 64 lanes)
LEAF_SHAPES = [(1, 59, True), (4, 56, True), (4, 57, False), (5, 43, True), (16, 32, True), (16, 33, False),
               (17, 10, False), (3, 0, True), (16, 0, True), (8, 1, True)]


@pytest.mark.parametrize("k,r,small", LEAF_SHAPES)
def test_small_supernode_limits(checker, tmp_path, k, r, small):
    rng = np.random.default_rng(1000 * k + r)
    n, cp, ri, _ = gen.leaf_pair_spd(k, r, rng)
    out = _run(checker, tmp_path, n, cp, ri, None, 0, 0, 64)
    nsmall = int(out.split("small=")[1].split()[0])
    # the two leaves, and the parent block too when it fits
    parent = r > 0 and r <= 16 and (4 if r <= 4 else 16) + r <= 64
    assert nsmall == (2 if small else 0) + (1 if parent else 0), out


@pytest.mark.parametrize("cfg,side,z,nb", [(0, 24, 0, 64), (1, 12, 8, 32), (1, 20, 8, 64), (2, 5, 8, 64)])
def test_deterministic_schedule(checker, tmp_path, cfg, side, z, nb):
    """Deterministic schedule: the same replay, and no launch holds two adds
    into one entry (so atomic adds land in a fixed order); the scatter
    launches are split by a colouring of each level's supernodes, the
    backward solve never splits a panel, and no update runs on the second
    stream."""
    p = gen.make_config(cfg, side=side)
    out = _run(checker, tmp_path, p.n, p.colptr, p.rowind, p.perm, 0, z, nb, det=1)
    assert int(out.split("split_bwd=")[1].split()[0]) == 0, out
    colors = int(out.split("colors=")[1].split()[0])
    assert 2 <= colors <= 64, out
    base = _run(checker, tmp_path, p.n, p.colptr, p.rowind, p.perm, 0, z, nb, det=0)
    nl = lambda o: sum(int(x) for x in o.split("launches=")[1].split()[0].split("+"))
    assert nl(out) > nl(base)
    print(out)


@pytest.mark.parametrize("cfg,side,nb", [(1, 14, 64), (2, 6, 32), (0, 40, 64)])
def test_greedy_amalgamation_with_nd_ordering(checker, tmp_path, cfg, side, nb):
    """The schedule of a graph-ordered, greedily merged structure (the
    general-pattern path: the library's nested dissection and the Sec. IV-A
    merging with a 25 % cap), in both schedules."""
    import paper_2409_14009_amd as sc
    p = gen.make_config(cfg, side=side)
    perm = sc.order_nd(p.n, p.colptr, p.rowind)
    _run(checker, tmp_path, p.n, p.colptr, p.rowind, perm, 0, 0, nb, det=0, rule=1)
    _run(checker, tmp_path, p.n, p.colptr, p.rowind, perm, 0, 0, nb, det=1, rule=1)


@pytest.mark.parametrize("cfg,side,z,nb,pr", [(1, 12, 8, 64, 0), (1, 12, 8, 64, 1), (0, 64, 0, 32, 1),
                                              (2, 5, 8, 64, 1), (4, 14, 8, 64, 1)])
def test_rlb_schedule(checker, tmp_path, cfg, side, z, nb, pr):
    """RLB (Sec. II-B): every block-pair tile's entries, addressed from the
    block's one relative index, are exactly the targets the method defines,
    each received once; with partition refinement the blocks get fewer."""
    p = gen.make_config(cfg, side=side)
    out = _run(checker, tmp_path, p.n, p.colptr, p.rowind, p.perm, 0, z, nb, rlb=1, pr=pr)
    assert int(out.split("rlb_tasks=")[1].split()[0]) > 0, out
    _run(checker, tmp_path, p.n, p.colptr, p.rowind, p.perm, 0, z, nb, det=1, rlb=1, pr=pr)
    if pr:
        plain = _run(checker, tmp_path, p.n, p.colptr, p.rowind, p.perm, 0, z, nb, rlb=1, pr=0)
        b1 = int(out.split("rlb_blocks=")[1].split()[0])
        b0 = int(plain.split("rlb_blocks=")[1].split()[0])
        print(f"blocks without / with partition refinement: {b0} / {b1}")
        assert b1 <= b0


# (leaf columns, rows of the parent, one-wavefront factor tasks expected):
# short one-panel leaves of at most 32 columns not done by the whole-step
# one-wavefront task, up to several 64-row chunks of rows below
# ((16, 32): the leaves are whole-step ones, the 32-column parent is not)
MEDIUM_SHAPES = [(1, 60, 2), (4, 57, 2), (16, 33, 2), (16, 160, 2), (7, 150, 2), (12, 129, 2), (16, 32, 1),
                 (17, 40, 2), (20, 5, 2), (32, 100, 2), (24, 161, 0), (33, 50, 0), (16, 161, 0), (3, 333, 0)]


@pytest.mark.parametrize("k,r,nmed", MEDIUM_SHAPES)
def test_medium_supernodes(checker, tmp_path, k, r, nmed):
    rng = np.random.default_rng(3000 * k + r)
    n, cp, ri, _ = gen.leaf_pair_spd(k, r, rng)
    out = _run(checker, tmp_path, n, cp, ri, None, 0, 0, 64)
    assert int(out.split("medium=")[1].split()[0]) == nmed, out
