"""The allocation-free prediction entry point (fk_predict_noalloc) against fk_predict.

Both run the same kernels on the same inputs, so the outputs must agree bit for bit; each is also
held to the type-2 bar against the FP64 oracle's direct sum on sampled points.  Two calls in a row
on one context, the second with a smaller shape (the library's device array keeps the first call's
contents), an oversized shape that must be refused, and no change of the device's free memory
across a call."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fk():
    import paper_2509_02649_amd as fk
    return fk


def _herm_sets(rng, T, m, d):
    N = (2 * m + 1) ** d
    k = oracle.modes(m, d)
    decay = 1.0 / (1.0 + (k ** 2).sum(1))
    th = (rng.standard_normal((T, N)) + 1j * rng.standard_normal((T, N))) * decay
    return 0.5 * (th + np.conj(th[:, ::-1]))


def _noalloc(fk, ctx, th, Xq, m, out=None):
    # straight through the C ABI: no workspace argument
    ctx.bind_stream()
    d, nq = Xq.shape
    tr = torch.view_as_real(th.contiguous()).contiguous()
    if out is None:
        out = torch.empty((th.shape[0], nq), dtype=torch.float32, device=Xq.device)
    code = ctx.lib.fk_predict_noalloc(ctx.h, d, m, th.shape[0], C.c_void_p(tr.data_ptr()), nq,
                                      0 if Xq.dtype == torch.float32 else 1, C.c_void_p(Xq.data_ptr()),
                                      C.c_void_p(out.data_ptr()))
    return code, out


@pytest.mark.parametrize("order", ["large_then_small"])
def test_noalloc_predict_matches_predict(fk, order):
    ctx, ref = fk.Context(0), fk.Context(0)
    rng = np.random.default_rng(2026)
    cases = [(2, 32, 16, 300_001), (2, 8, 3, 1001), (1, 50, 2, 777)]
    for d, m, T, nq in cases:
        print(f"noalloc predict d={d} m={m} sets={T} nq={nq}", flush=True)
        th = torch.from_numpy(_herm_sets(rng, T, m, d)).cuda()
        Xq = torch.from_numpy(rng.uniform(-np.pi, np.pi, size=(d, nq)).astype(np.float32)).cuda()
        want = fk.predict(th, Xq, m, ctx=ref)
        code, got = _noalloc(fk, ctx, th, Xq, m)
        assert code == 0
        torch.cuda.synchronize()
        assert torch.equal(got, want)
        # the type-2 bar against the FP64 direct sum, on a sample of the points
        idx = rng.choice(nq, size=min(nq, 1500), replace=False)
        fo = oracle.predict(th.cpu().numpy(), Xq.cpu().numpy()[:, idx].astype(np.float64), m).real
        bound = 2e-6 * np.abs(th.cpu().numpy()).sum(axis=1, keepdims=True)
        assert (np.abs(got.cpu().numpy()[:, idx] - fo) <= bound).all()


def test_noalloc_predict_refuses_oversize_and_allocates_nothing(fk):
    ctx = fk.Context(0, eps=1e-6)        # a tolerance no other test uses: its plan is new to the library
    lib = ctx.lib
    cap = lib.fk_predict_noalloc_max_bytes()
    assert cap == (64 << 20) - 1024
    nb = C.c_size_t()
    assert lib.fk_predict_workspace_size(ctx.h, 3, 31, 8, C.byref(nb)) == 0 and nb.value > cap
    th = torch.zeros((8, 63 ** 3), dtype=torch.complex128, device="cuda")
    Xq = torch.zeros((3, 10), dtype=torch.float32, device="cuda")
    code, _ = _noalloc(fk, ctx, th, Xq, 31)
    assert code == 6                     # FK_ENOMEM, nothing enqueued
    rng = np.random.default_rng(5)
    Xq = torch.from_numpy(rng.uniform(-np.pi, np.pi, size=(2, 50_000)).astype(np.float32)).cuda()
    # a first call loads the library's code object (and with it the device array) if nothing has yet
    th0 = torch.from_numpy(_herm_sets(rng, 4, 20, 2)).cuda()
    code, _ = _noalloc(fk, ctx, th0, Xq, 20)
    assert code == 0
    # then a shape whose plan is new to the context: fk_predict would allocate its device table here
    th = torch.from_numpy(_herm_sets(rng, 4, 21, 2)).cuda()
    tr = torch.view_as_real(th.contiguous()).contiguous()
    out = torch.empty((4, 50_000), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info(0)[0]
    code, out = _noalloc(fk, ctx, th, Xq, 21, out=out)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info(0)[0]
    assert code == 0
    assert free1 == free0
    del tr
    want = fk.predict(th, Xq, 21, ctx=fk.Context(0, eps=1e-6))
    assert torch.equal(out, want)
