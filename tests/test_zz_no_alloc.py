"""The allocation-free training step (lbm_mlp_train_step_noalloc) against the
training step with a caller work buffer (lbm_mlp_train_step), both called
through the C ABI: the same kernels, so parameters, Adam moments and loss
must agree bit for bit, on two calls in a row with the second batch smaller
than the first (the shared work array then holds the larger call's partials
beyond what the second one reads)."""

import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_09807_amd import native as N
    return N, N.load()


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _inputs(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(0.0, 0.8, (n, 64)).astype(np.float32)
    X[:, 63] = 0.0
    out_scale = rng.uniform(1e-5, 1e-4, 4).astype(np.float32)
    T = (rng.normal(0.0, 1.0, (n, 4)) * out_scale).astype(np.float32)
    norm = np.zeros(32, dtype=np.float32)
    norm[0:7] = rng.normal(0.0, 0.1, 7)
    norm[8:15] = rng.uniform(0.5, 2.0, 7)
    norm[16:20] = out_scale
    params = (rng.normal(0.0, 1.0, 8580) * 0.1).astype(np.float32)
    params[63 * 64: 64 * 64] = 0.0          # w1's pad row
    return X, T, norm, params


def test_noalloc_train_step_matches_the_work_buffer_step():
    N, lib = _lib()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    n = 20000
    X, T, norm, params = _inputs(n, 5)
    Xd = torch.from_numpy(X).to(dev)
    Td = torch.from_numpy(T).to(dev)
    nd = torch.from_numpy(norm).to(dev)
    pa = torch.from_numpy(params).to(dev)
    ma, va = torch.zeros_like(pa), torch.zeros_like(pa)
    pb, mb, vb = pa.clone(), ma.clone(), va.clone()
    rng = np.random.default_rng(6)
    for step, batch in ((1, 12000), (2, 3000)):
        print(f"noalloc train step {step}, batch {batch}", flush=True)
        idx = torch.from_numpy(rng.integers(0, n, batch).astype(np.int32)).to(dev)
        wb = lib.lbm_mlp_train_work_bytes(batch)
        work = torch.empty(wb, dtype=torch.uint8, device=dev)
        la = torch.full((1,), float("nan"), dtype=torch.float32, device=dev)
        lb = torch.full((1,), float("nan"), dtype=torch.float32, device=dev)
        N.check(lib.lbm_mlp_train_step(_p(pa), _p(ma), _p(va), step, 1e-3, _p(nd), _p(Xd), _p(Td), _p(idx), batch,
                                       _p(work), wb, _p(la), ctypes.c_void_p(stream.cuda_stream)),
                "lbm_mlp_train_step")
        N.check(lib.lbm_mlp_train_step_noalloc(_p(pb), _p(mb), _p(vb), step, 1e-3, _p(nd), _p(Xd), _p(Td), _p(idx),
                                               batch, _p(lb), ctypes.c_void_p(stream.cuda_stream)),
                "lbm_mlp_train_step_noalloc")
        torch.cuda.synchronize(dev)
        assert torch.isfinite(la).all() and la.item() > 0.0
        assert torch.equal(la, lb), (la.item(), lb.item())
        assert torch.equal(pa, pb) and torch.equal(ma, mb) and torch.equal(va, vb)
        assert not torch.equal(pa, torch.from_numpy(params).to(dev))   # the step moved the parameters
        del work
    # a batch beyond the fixed work array is refused before any work is enqueued
    big = N.LBM_MLP_TRAIN_NOALLOC_BATCH + 1
    rc = lib.lbm_mlp_train_step_noalloc(_p(pb), _p(mb), _p(vb), 3, 1e-3, _p(nd), _p(Xd), _p(Td), _p(idx), big,
                                        None, ctypes.c_void_p(stream.cuda_stream))
    assert rc == N.LBM_EINVAL
    torch.cuda.synchronize(dev)
    assert torch.equal(pa, pb)
