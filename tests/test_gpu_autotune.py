"""The launch-shape autotuner: every candidate shape gives the oracle's result (pinned through
table entries), and a first call on a large shape measures and records one."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL = 1e-6


@pytest.fixture(scope="module")
def fk():
    import paper_2509_02649_amd as fk
    return fk


def _arch():
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def _bucket(n):
    v = min(n >> 10, 1 << 30)
    return (0 if v <= 1 else math.ceil(math.log2(v))) + 10


def _pin(fk, tmp_path, key, values):
    p = tmp_path / "table.txt"
    p.write_text(f"{key} = " + " ".join(f"{k}={v}" for k, v in values.items()) + "\n")
    fk.autotune_clear()
    fk.autotune_load(str(p))


def _errors(M, b, Mo, bo, Y):
    eT = np.abs(M - Mo).max() / abs(Mo.ravel()[Mo.size // 2])
    eb = (np.abs(b - bo) / np.abs(Y.astype(np.float64)).mean(axis=1, keepdims=True)).max()
    return eT, eb


@pytest.mark.parametrize("ntgt,n,m", [(16, 2_000_000, 4), (1, 1_500_000, 12)])
def test_every_type1_shape_matches_the_oracle(fk, tmp_path, ntgt, n, m):
    X = synth.uniform_points(301 + ntgt, 2, n)
    Y = synth.batched_targets(X, 301 + ntgt, ntgt=ntgt)
    Xd, Yd = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    Mo = oracle.gram_generator(X.astype(np.float64), m)
    bo = oracle.rhs(X.astype(np.float64), Y.astype(np.float64), m)
    _, _, info = fk.gram(Xd, Yd, m, info=True)
    key = f"{_arch()} t1 d=2 nf={info['nf']} w={info['w']} nw={ntgt} n=2^{_bucket(n)}"
    shapes = [dict(spread_pts=4096, sort_blk=256, sort_slice=32768), dict(spread_pts=32768, sort_blk=1024,
                                                                         sort_slice=131072)]
    if ntgt >= 8:
        shapes += [dict(mb=2, spread_pts=8192, sort_blk=512, sort_slice=65536),
                   dict(mb=4, spread_pts=16384, sort_blk=512, sort_slice=65536)]
    try:
        for sh in shapes:
            _pin(fk, tmp_path, key, sh)
            M, b, inf = fk.gram(Xd, Yd, m, info=True)
            eT, eb = _errors(M.cpu().numpy(), b.cpu().numpy(), Mo, bo, Y)
            print(f"T={ntgt} shape {sh}: eps_T={eT:.2e} eps_b={eb:.2e} bin={inf['bin']}")
            if "mb" in sh:
                assert inf["bin"] == -sh["mb"]
            assert eT <= TOL and eb <= TOL
    finally:
        fk.autotune_clear()


def test_every_dense_shape_solves_the_system(fk, tmp_path):
    # 48 lambdas at m = 24 (Np = 2432): large enough for the dense shapes to be tuned
    m, nlam, n = 24, 48, 300_000
    X = synth.uniform_points(311, 2, n)
    Y = synth.batched_targets(X, 311, ntgt=2)
    Xd, Yd = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    lams = [10.0 ** (-6 + 5 * i / (nlam - 1)) for i in range(nlam)]
    M, b = fk.gram(Xd, Yd, m)
    Mh, bh = M.cpu().numpy(), b.cpu().numpy()
    p = oracle.sobolev_weights(m, 2, 2.0)
    ref = {i: oracle.solve_system(oracle.system_matrix(Mh, m, lams[i], p), bh) for i in (0, nlam - 1)}
    key = f"{_arch()} dense Np=2432 nlam={nlam} ntgt=2"
    try:
        for sh in [dict(pair=0, trsm_wg=256), dict(pair=1, trsm_wg=1024), dict(pair=1, trsm_wg=512),
                   dict(pair=1, trsm_wg=512, diag64=1)]:
            _pin(fk, tmp_path, key, sh)
            th, info = fk.solve(M, b, m, lams, penalty="sobolev", s=2.0, info=True)
            assert info["resid_rel"] <= 1e-10
            for i, r in ref.items():
                e = np.linalg.norm(th[i].cpu().numpy() - r) / np.linalg.norm(r)
                assert e <= 1e-4, (sh, i, e)
    finally:
        fk.autotune_clear()


def test_first_call_measures_and_records_a_shape(fk):
    # a 2-D type-1 stage above the size threshold with no entry: the call tunes, records the
    # fastest shape and returns the oracle's result
    fk.autotune_clear()
    n, m, ntgt = (1 << 22) + 12_345, 4, 16
    X = synth.uniform_points(321, 2, n)
    Y = synth.batched_targets(X, 321, ntgt=ntgt)
    ctx = fk.Context(0, autotune=3)
    try:
        M, b, info = fk.gram(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(), m, ctx=ctx, info=True)
        table = fk.autotune_table()
        print(table)
        key = f"{_arch()} t1 d=2 nf={info['nf']} w={info['w']} nw={ntgt} n=2^{_bucket(n)}"
        line = [ln for ln in table.splitlines() if ln.startswith(key + " = ")]
        assert len(line) == 1 and "spread_pts=" in line[0] and "mb=" in line[0] and "ms=" in line[0]
        Mo = oracle.gram_generator(X.astype(np.float64), m)
        bo = oracle.rhs(X.astype(np.float64), Y.astype(np.float64), m)
        eT, eb = _errors(M.cpu().numpy(), b.cpu().numpy(), Mo, bo, Y)
        assert eT <= TOL and eb <= TOL
    finally:
        fk.autotune_clear()
