"""Parity of the additive model (Sec. 5): block Gram from 1-D and pairwise 2-D type-1
transforms, stacked right-hand side, and the fitted coefficients, against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fk():
    import paper_2509_02649_amd as fk
    return fk


@pytest.mark.parametrize("d,m,n", [(3, 8, 20_000), (10, 32, 200_000), (10, 32, 1_000_000)])
def test_additive_gram_and_fit(fk, d, m, n):
    # the last case is the first 1e6 points of the additive workload (d = 10, m = 32, n = 1e8),
    # every block entry and right-hand side element against the oracle
    w = synth.workload_additive(n=n, d=d)
    X, Y = w["X"], w["Y"]
    Xd, Yd = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    B, b = fk.additive_gram(Xd, Yd, m)
    B = B.cpu().numpy()
    b = b.cpu().numpy()
    X64, Y64 = X.astype(np.float64), Y.astype(np.float64)
    Bo = oracle.additive_blocks(X64, m)
    bo = oracle.additive_rhs(X64, Y64, m)
    eB = np.abs(B - Bo).max()           # every entry is bounded by 1 = B[k,k]
    eb = np.abs(b - bo).max() / np.abs(Y64).mean()
    print(f"additive d={d} m={m} n={n}: eps_B={eB:.2e} eps_b={eb:.2e}")
    assert eB <= 1e-6 and eb <= 1e-6
    # the Gram is Hermitian and its null space (shared constants) has dimension d - 1
    assert np.abs(B - np.conj(B).T).max() <= 1e-12
    lam = float(n) ** (-2.0 / 3.0)
    p = oracle.additive_penalty(m, d, 1.0)
    A = Bo + lam * np.diag(p)
    th = oracle.solve_system(A, bo)
    kappa = oracle.condition_number(A)
    tg = fk.additive_fit(Xd, Yd, m, lam, s=1.0)[0].cpu().numpy()
    e = np.linalg.norm(tg - th) / np.linalg.norm(th)
    print(f"additive fit: rel={e:.2e} kappa={kappa:.2e}")
    assert kappa <= 1e6 and e <= 1e-4
    # the fitted components predict like the oracle's
    Xq = synth.uniform_points(5, d, 500).astype(np.float64)
    f = oracle.predict_additive(tg[0], Xq, m).real
    fo = oracle.predict_additive(th[0], Xq, m).real
    assert np.abs(f - fo).max() <= 1e-4 * np.abs(fo).max()
