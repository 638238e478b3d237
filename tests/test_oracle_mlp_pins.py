"""Pins for the oracle of the learned edge heuristic (features, MLP, gradient, Adam)."""
import math

import numpy as np
import pytest

import aco_instances as inst

OFF_W1, OFF_B1, OFF_W2, OFF_B2, OFF_W3, OFF_B3 = 0, 192, 256, 4352, 4416, 4480


def test_param_count(oracle_lib):
    assert oracle_lib.mlp_param_count() == 3 * 64 + 64 + 64 * 64 + 64 + 64 + 1 == 4481


def test_bf16_round_matches_torch(oracle_lib):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    vals = np.concatenate([
        rng.standard_normal(3000).astype(np.float32) * 10.0 ** rng.integers(-30, 30, 3000),
        np.array([0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 3.4e38,
                  1e-40, -1e-42, np.inf, -np.inf], np.float32),
    ]).astype(np.float32)
    want = torch.from_numpy(vals).to(torch.bfloat16).to(torch.float32).numpy()
    got = np.array([oracle_lib.bf16_round(v) for v in vals], np.float32)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


def _brute_ranks(D):
    n = D.shape[0]
    R = np.zeros((n, n), np.int32)
    for i in range(n):
        for j in range(n):
            if i == j:
                continue
            R[i, j] = 1 + sum(1 for k in range(n) if k != i and k != j and
                              (D[i, k] < D[i, j] or (D[i, k] == D[i, j] and k < j)))
    return R


def test_ranks_against_brute_force_and_hand_values(oracle_lib):
    tri = inst.distance_matrix(np.array([[0, 0], [3, 0], [0, 4]], np.float32))
    assert oracle_lib.edge_ranks(tri).tolist() == [[0, 1, 2], [1, 0, 2], [1, 2, 0]]
    sq = inst.distance_matrix(np.array([[0, 0], [1, 0], [1, 1], [0, 1]], np.float32))
    R = oracle_lib.edge_ranks(sq)
    assert R[0].tolist() == [0, 1, 3, 2]  # tie d01 = d03 = 1 goes to the smaller index
    for seed in range(5):
        D = inst.distance_matrix(inst.clustered_cities(23, seed, 3, 0.05))
        assert np.array_equal(oracle_lib.edge_ranks(D), _brute_ranks(D))
    # grid points produce many exact ties
    g = np.stack(np.meshgrid(np.arange(5), np.arange(4)), -1).reshape(-1, 2).astype(np.float32)
    Dg = inst.distance_matrix(g)
    assert np.array_equal(oracle_lib.edge_ranks(Dg), _brute_ranks(Dg))


def test_features_triangle_by_hand(oracle_lib):
    tri = inst.distance_matrix(np.array([[0, 0], [3, 0], [0, 4]], np.float32))
    # nearest-neighbour distances 3, 3, 4
    assert oracle_lib.mean_nn(tri) == pytest.approx(10.0 / 3.0, rel=1e-15)
    F = oracle_lib.edge_features(tri)
    assert F[0, 1].tolist() == pytest.approx([0.9, 1.0, 1.0], rel=1e-7)
    assert F[0, 2].tolist() == pytest.approx([1.2, math.log2(3), 1.0], rel=1e-7)
    assert F[2, 1].tolist() == pytest.approx([1.5, math.log2(3), math.log2(3)], rel=1e-7)
    assert np.all(F[[0, 1, 2], [0, 1, 2]] == 0)


def _zero_params():
    return np.zeros(4481, np.float64)


def test_forward_closed_forms(oracle_lib):
    feats = np.array([[0.3, 1.0, 2.0], [2.7, 3.0, 1.0], [1.0 / 3.0, 0.5, 0.25]], np.float32)
    p = _zero_params()
    p[OFF_B3] = 0.7
    z, eta = oracle_lib.mlp_forward(p, feats)
    assert np.all(z == 0.69921875)  # the bias itself is rounded to BF16 (0.7 -> 0.69921875) ...
    p[OFF_B3] = 0.75                                 # ... 0.75 is exact in BF16
    z, eta = oracle_lib.mlp_forward(p, feats)
    assert np.all(z == 0.75)
    assert np.allclose(eta, 1 / (1 + math.exp(-0.75)), rtol=1e-15)
    # eta = sigmoid(z)^kappa / f1^lambda
    z, eta = oracle_lib.mlp_forward(p, feats, kappa=0.5, lam=1.0)
    want = (1 / (1 + math.exp(-0.75))) ** 0.5 / feats[:, 0].astype(np.float64)
    assert np.allclose(eta, want, rtol=1e-14)
    # far in the tail sigmoid(z) keeps its relative precision (no cancellation)
    p[OFF_B3] = -60.0
    z, eta = oracle_lib.mlp_forward(p, feats, kappa=1.0, lam=0.0)
    assert np.allclose(eta, math.exp(-60.0), rtol=1e-12)
    # one path: z = W3[0] relu(W2[0,0] bf16(relu(W1[0,0] f1)))
    p = _zero_params()
    p[OFF_W1 + 0] = 1.0
    p[OFF_W2 + 0] = 2.0
    p[OFF_W3 + 0] = -0.5
    z_r, _ = oracle_lib.mlp_forward(p, feats, round_bf16=True)
    z_f, _ = oracle_lib.mlp_forward(p, feats, round_bf16=False)
    for e in range(3):
        f1 = float(feats[e, 0])
        assert z_f[e] == -0.5 * 2.0 * f1
        assert z_r[e] == -0.5 * 2.0 * oracle_lib.bf16_round(f1)
    assert z_r[2] != z_f[2]  # 1/3 is not a BF16 value: the rounding point shows
    # a negative pre-activation is cut by the ReLU
    p[OFF_W1 + 0] = -1.0
    z, _ = oracle_lib.mlp_forward(p, feats)
    assert np.all(z == 0.0)


def test_loss_closed_form(oracle_lib):
    feats = np.zeros((4, 3), np.float32)
    y = np.array([0.0, 1.0, 0.25, 1.0], np.float32)
    p = _zero_params()  # z = 0 everywhere: loss = log 2, dL/db3 = mean(0.5 - y)
    loss, g = oracle_lib.mlp_loss_grad(p, feats, y)
    assert loss == pytest.approx(math.log(2.0), rel=1e-15)
    assert g[OFF_B3] == pytest.approx(np.mean(0.5 - y.astype(np.float64)), rel=1e-15)
    assert np.count_nonzero(g) == 1


def test_gradient_matches_finite_differences(oracle_lib):
    rng = np.random.default_rng(3)
    p = rng.standard_normal(4481) * 0.3
    D = inst.distance_matrix(inst.clustered_cities(12, 4, 3, 0.05))
    F = oracle_lib.edge_features(D)
    idx = [(i, j) for i in range(12) for j in range(12) if i != j][:40]
    feats = np.array([F[i, j] for i, j in idx], np.float32)
    y = rng.random(len(idx)).astype(np.float32)
    _, g = oracle_lib.mlp_loss_grad(p, feats, y, round_bf16=False)
    check = list(rng.choice(4481, 300, replace=False)) + list(range(OFF_W3, 4481))
    h = 1e-6
    fd = []
    for k in check:
        q = p.copy()
        q[k] += h
        lp, _ = oracle_lib.mlp_loss_grad(q, feats, y, round_bf16=False)
        q[k] -= 2 * h
        lm, _ = oracle_lib.mlp_loss_grad(q, feats, y, round_bf16=False)
        fd.append((lp - lm) / (2 * h))
    fd = np.array(fd)
    err = np.linalg.norm(fd - g[check]) / np.linalg.norm(g[check])
    assert err < 1e-6, err
    # every layer's gradient is exercised
    for lo, hi in ((OFF_W1, OFF_B1), (OFF_B1, OFF_W2), (OFF_W2, OFF_B2), (OFF_B2, OFF_W3),
                   (OFF_W3, OFF_B3)):
        assert np.count_nonzero(g[lo:hi]) > 0


def test_adam_first_steps_closed_form(oracle_lib):
    p = np.array([1.0, -2.0, 0.5, 0.0])
    m = np.zeros(4)
    v = np.zeros(4)
    g = np.array([0.1, -3.0, 0.0, 1e-12])
    oracle_lib.adam_step(p, m, v, g, 1, lr=1e-3)
    # step 1: m_hat = g, v_hat = g^2, so the update is -lr g / (|g| + eps)
    want = np.array([1.0, -2.0, 0.5, 0.0]) - 1e-3 * g / (np.abs(g) + 1e-8)
    assert np.allclose(p, want, rtol=1e-14, atol=0)
    # step 2 with the same gradient: m_hat = g, v_hat = g^2 again
    oracle_lib.adam_step(p, m, v, g, 2, lr=1e-3)
    want = want - 1e-3 * g / (np.abs(g) + 1e-8)
    assert np.allclose(p, want, rtol=1e-12, atol=1e-18)


def test_weight_layout_is_out_by_in(oracle_lib):
    """W1[u][c] feeds feature c into unit u; W2[u][k] feeds layer-1 unit k into
    layer-2 unit u (a transposed layout fails these)."""
    feats = np.array([[0.5, 2.0, 3.0]], np.float32)
    p = _zero_params()
    p[OFF_W1 + 3 * 5 + 2] = 1.0     # unit 5 of layer 1 <- f3 = 3
    p[OFF_W2 + 64 * 7 + 5] = 0.25   # unit 7 of layer 2 <- unit 5 of layer 1
    p[OFF_W3 + 7] = 2.0
    z, _ = oracle_lib.mlp_forward(p, feats)
    assert z[0] == 2.0 * 0.25 * 3.0
    p[OFF_B1 + 5] = -4.0            # pre-activation 3 - 4 < 0: the path is cut
    z, _ = oracle_lib.mlp_forward(p, feats)
    assert z[0] == 0.0
    p[OFF_B1 + 5] = 0.0
    p[OFF_B2 + 7] = -1.0            # 0.75 - 1 < 0
    z, _ = oracle_lib.mlp_forward(p, feats)
    assert z[0] == 0.0
