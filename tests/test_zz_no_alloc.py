"""The allocation-free network training step (hawkes_mlp_train_step_noalloc)
against the allocating one (hawkes_mlp_train_step) through the C ABI: two
calls in a row from the same state, the second with a smaller batch; the
parameters, the Adam moments and the loss must agree exactly (same kernels,
same summation order), and a batch above the fixed capacity is refused."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda:0")


def test_noalloc_train_step_matches_allocating_step(gpu):
    import torch

    from paper_2103_03348_amd import _lib

    L = _lib.lib()
    s = _lib.stream_handle()
    npar = int(L.hawkes_mlp_num_params())
    cap = int(L.hawkes_mlp_noalloc_max_batch())
    assert cap == 4096
    rng = np.random.default_rng(11)
    n_rows = 6000
    X = _t(rng.standard_normal((n_rows, 12)).astype(np.float32))
    T = _t((rng.standard_normal(n_rows) - 3.0).astype(np.float32))
    p0 = (0.2 * rng.standard_normal(npar)).astype(np.float32)
    state = {}
    for name in ("alloc", "noalloc"):
        state[name] = [_t(p0.copy()), torch.zeros(npar, dtype=torch.float32, device="cuda:0"),
                       torch.zeros(npar, dtype=torch.float32, device="cuda:0")]
    for step, B in ((1, cap), (2, 777)):
        rows = _t(rng.integers(0, n_rows, size=B).astype(np.int32))
        print(f"\n[noalloc] step {step} batch {B}", flush=True)
        # the allocating step with its own workspace and gradient buffers
        work = torch.empty(int(L.hawkes_mlp_workspace_floats(B)), dtype=torch.float32, device="cuda:0")
        grad = torch.empty(npar, dtype=torch.float64, device="cuda:0")
        loss_a = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        err_a = torch.zeros(1, dtype=torch.int32, device="cuda:0")
        pa, ma, va = state["alloc"]
        _lib.check(L.hawkes_mlp_train_step(_lib.ptr(pa), _lib.ptr(ma), _lib.ptr(va), step, ctypes.c_float(1e-2),
                                           _lib.ptr(X), n_rows, _lib.ptr(rows), _lib.ptr(T), B, _lib.ptr(work),
                                           _lib.ptr(grad), _lib.ptr(loss_a), _lib.ptr(err_a), s), "train_step")
        loss_b = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        err_b = torch.zeros(1, dtype=torch.int32, device="cuda:0")
        pb, mb, vb = state["noalloc"]
        _lib.check(L.hawkes_mlp_train_step_noalloc(_lib.ptr(pb), _lib.ptr(mb), _lib.ptr(vb), step,
                                                   ctypes.c_float(1e-2), _lib.ptr(X), n_rows, _lib.ptr(rows),
                                                   _lib.ptr(T), B, _lib.ptr(loss_b), _lib.ptr(err_b), s),
                   "train_step_noalloc")
        torch.cuda.synchronize()
        assert int(err_a.item()) == 0 and int(err_b.item()) == 0
        assert float(loss_a.item()) == float(loss_b.item()), (loss_a.item(), loss_b.item())
        for a, b in zip(state["alloc"], state["noalloc"]):
            assert torch.equal(a, b)
        # the update moved the parameters
        assert not torch.equal(pa, _t(p0))
    # beyond the fixed capacity: refused on the host, nothing enqueued
    rows = _t(np.zeros(cap + 1, dtype=np.int32))
    pb, mb, vb = state["noalloc"]
    before = pb.clone()
    code = L.hawkes_mlp_train_step_noalloc(_lib.ptr(pb), _lib.ptr(mb), _lib.ptr(vb), 3, ctypes.c_float(1e-2),
                                           _lib.ptr(X), n_rows, _lib.ptr(rows), _lib.ptr(T), cap + 1, None, None, s)
    torch.cuda.synchronize()
    assert code == _lib.E_CAPACITY
    assert torch.equal(before, pb)
