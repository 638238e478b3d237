"""The no-allocation gradient entry point against the trainer's gradient.

aco_mlp_gradient_noalloc keeps its scratch in a fixed per-GPU device array
instead of a caller workspace.  It runs the same kernels as
aco_mlp_trainer_gradient, so on the same BF16 parameters, features and
targets both give the same gradient and loss bit for bit.  Two calls in a
row, the second with fewer edges (a ragged count), check that nothing from
the first call's larger input leaks into the second.
"""
import ctypes

import numpy as np
import pytest

import aco_instances as inst
import oracle

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _params(seed):
    rng = np.random.default_rng(seed)
    p = (rng.standard_normal(4481) * 0.2).astype(np.float32)
    p[4480] = -0.5
    return p


def _noalloc(bf16_params, feats, y, grad, loss, stream, count=None):
    from paper_2404_04895_amd._native import check, lib
    check(lib().aco_mlp_gradient_noalloc(
        ctypes.c_void_p(bf16_params.data_ptr()), ctypes.c_void_p(feats.data_ptr()),
        ctypes.c_void_p(y.data_ptr()), feats.shape[0] if count is None else count,
        ctypes.c_void_p(grad.data_ptr()),
        None if loss is None else ctypes.c_void_p(loss.data_ptr()),
        ctypes.c_void_p(stream.cuda_stream)), "aco_mlp_gradient_noalloc")


def test_noalloc_gradient_equals_trainer_gradient():
    torch = _torch()
    from paper_2404_04895_amd import MlpTrainer, mlp_round
    from paper_2404_04895_amd._native import MLP_NOALLOC_MAX_EDGES
    n = 140
    D = inst.distance_matrix(inst.clustered_cities(n, 31, 4, 0.05))
    F = oracle.edge_features(D)
    feats_all = np.ascontiguousarray(F[~np.eye(n, dtype=bool)].reshape(-1, 3))
    rng = np.random.default_rng(5)
    y_all = rng.random(feats_all.shape[0]).astype(np.float32)
    p = _params(3)
    stream = torch.cuda.current_stream()
    pb = mlp_round(p)
    grad = torch.empty(4481, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    # the largest input first, then a smaller ragged one
    for count in (MLP_NOALLOC_MAX_EDGES, 3001):
        feats = torch.from_numpy(feats_all[:count].copy()).cuda()
        y = torch.from_numpy(y_all[:count].copy()).cuda()
        grad.fill_(np.nan)
        loss.fill_(np.nan)
        _noalloc(pb, feats, y, grad, loss, stream)
        t = MlpTrainer(p, batch=count)
        g_ref = t.gradient(feats, y)
        loss_ref = t.loss()
        torch.cuda.synchronize()
        got = grad.cpu().numpy()
        assert np.all(np.isfinite(got)), count
        assert np.array_equal(got.view(np.uint32), g_ref.cpu().numpy().view(np.uint32)), count
        assert loss.item() == loss_ref, count
        t.close()
    # no loss buffer: the gradient is the same
    grad2 = torch.empty_like(grad)
    _noalloc(pb, feats, y, grad2, None, stream)
    torch.cuda.synchronize()
    assert torch.equal(grad2, grad)


def _native_null_grad(pb, feats, y, stream):
    from paper_2404_04895_amd._native import check, lib
    check(lib().aco_mlp_gradient_noalloc(
        ctypes.c_void_p(pb.data_ptr()), ctypes.c_void_p(feats.data_ptr()),
        ctypes.c_void_p(y.data_ptr()), 10, None, None, ctypes.c_void_p(stream.cuda_stream)),
        "aco_mlp_gradient_noalloc")


def test_noalloc_gradient_rejects_sizes_beyond_the_maximum():
    torch = _torch()
    from paper_2404_04895_amd import AcoError
    from paper_2404_04895_amd._native import MLP_NOALLOC_MAX_EDGES
    stream = torch.cuda.current_stream()
    pb = torch.zeros(4481, dtype=torch.float32, device="cuda")
    grad = torch.empty(4481, dtype=torch.float32, device="cuda")
    feats = torch.zeros((MLP_NOALLOC_MAX_EDGES + 1, 3), dtype=torch.float32, device="cuda")
    y = torch.zeros(MLP_NOALLOC_MAX_EDGES + 1, dtype=torch.float32, device="cuda")
    with pytest.raises(AcoError, match="outside"):
        _noalloc(pb, feats, y, grad, None, stream)
    with pytest.raises(AcoError, match="outside"):
        _noalloc(pb, feats, y, grad, None, stream, count=0)
    with pytest.raises(AcoError, match="NULL"):
        _native_null_grad(pb, feats, y, stream)
