"""Pins of the oracle's dense SPGD (Algorithm 1 on the random dense NNLS of
section "Algorithm efficiency"), CPU only."""
import itertools

import numpy as np
import pytest

import oracle as orc
from synth import make_dense_instance


def test_matches_torch_adagrad_minibatches():
    """Each minibatch's g = B_o^T (B_o q - y_o) is the gradient of
    0.5 ||B_o q - y_o||^2; torch.optim.Adagrad on it, then a clamp at 0, must
    give the oracle's iterates (3 epochs, 5 minibatches each, short tail)."""
    torch = pytest.importorskip("torch")
    B, y, _, perms = make_dense_instance(9, m=23, epochs=3, seed=5)
    y = y - 1.5        # some coordinates hit the bound
    chunk, eta, eps = 5, 0.3, 1e-10
    q, A, hist = orc.dense_spgd(B, y, perms, chunk, eta, eps)
    qt = torch.zeros(9, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adagrad([qt], lr=eta, eps=eps)
    Bt, yt = torch.tensor(B), torch.tensor(y)
    for e in range(3):
        for s0 in range(0, 23, chunk):
            rows = torch.tensor(perms[e, s0:s0 + chunk].astype(np.int64))
            opt.zero_grad()
            loss = 0.5 * ((Bt[rows] @ qt - yt[rows]) ** 2).sum()
            loss.backward()
            opt.step()
            with torch.no_grad():
                qt.clamp_(min=0.0)
        np.testing.assert_allclose(hist[e], float(((Bt @ qt - yt) ** 2).sum().detach()),
                                   rtol=1e-12)
    np.testing.assert_allclose(q, qt.detach().numpy(), rtol=1e-12, atol=1e-14)
    assert np.any(q == 0) and np.any(q > 0)


def brute_force_nnls(B, y):
    """Enumerate supports; the optimum is the feasible least-squares solution
    on a support that satisfies the KKT conditions."""
    n = B.shape[1]
    best = None
    for k in range(n + 1):
        for S in itertools.combinations(range(n), k):
            q = np.zeros(n)
            if S:
                q[list(S)] = np.linalg.lstsq(B[:, S], y, rcond=None)[0]
            if np.any(q < -1e-12):
                continue
            g = B.T @ (B @ q - y)
            if np.all(g[[j for j in range(n) if j not in S]] >= -1e-9):
                val = float(np.sum((B @ q - y) ** 2))
                if best is None or val < best[0]:
                    best = (val, q)
    return best


def test_reaches_brute_force_optimum_fixed_step():
    """Full-batch fixed steps eta = 1/lambda_max(B^T B) converge to the
    enumerated optimum of a problem with active bounds."""
    rng = np.random.default_rng(7)
    B = rng.uniform(0, 1, size=(20, 6))
    y = B @ np.array([1.0, 0.0, 2.0, 0.0, 0.5, 0.0]) + rng.normal(0, 0.3, size=20) - 0.4
    val, q_bf = brute_force_nnls(B, y)
    eta = 1.0 / np.linalg.eigvalsh(B.T @ B)[-1]
    E = 20000
    perms = np.tile(np.arange(20, dtype=np.int32), (E, 1))
    q, _, hist = orc.dense_spgd(B, y, perms, 20, eta, optimizer=1)
    np.testing.assert_allclose(q, q_bf, atol=1e-8)
    np.testing.assert_allclose(hist[-1], val, rtol=1e-10)
    assert np.any(q_bf == 0)


def test_matches_lawson_hanson_and_kkt():
    """scipy's Lawson-Hanson NNLS gives the same optimum; the end point
    satisfies min(q, g) = 0 to 1e-7."""
    scipy_opt = pytest.importorskip("scipy.optimize")
    B, y, _, _ = make_dense_instance(8, m=30, seed=9)
    y = y - 1.0
    x_lh, rn = scipy_opt.nnls(B, y)
    eta = 1.0 / np.linalg.eigvalsh(B.T @ B)[-1]
    E = 40000
    perms = np.tile(np.arange(30, dtype=np.int32), (E, 1))
    q, _, hist = orc.dense_spgd(B, y, perms, 30, eta, optimizer=1)
    np.testing.assert_allclose(q, x_lh, atol=1e-7)
    np.testing.assert_allclose(hist[-1], rn ** 2, rtol=1e-9)
    g = B.T @ (B @ q - y)
    assert np.max(np.abs(np.minimum(q, g))) <= 1e-7


def test_planted_recovery_adagrad():
    """Noiseless, overdetermined, full rank: y = B x* with x* > 0; Adagrad
    minibatches drive the loss to 0 and q to x*."""
    B, y, xs, perms = make_dense_instance(10, m=60, epochs=6000, seed=11)
    q, _, hist = orc.dense_spgd(B, y, perms, 16, 0.2)
    assert hist[-1] <= 1e-24 * float(y @ y)
    np.testing.assert_allclose(q, xs, atol=1e-12)
    assert hist[-1] < hist[0]


def test_first_step_closed_form():
    """From q = 0 the first Adagrad step moves each coordinate by
    eta |g| / (|g| + eps) against the sign of g, then clamps at 0."""
    B, y, _, _ = make_dense_instance(7, m=12, seed=13)
    y = y.copy()
    y[:6] *= -1.0
    perm = np.arange(12, dtype=np.int32)[None, :]
    q, A, _ = orc.dense_spgd(B, y, perm, 12, 0.7)
    g = B.T @ (0 - y)
    expect = np.maximum(-0.7 * g / (np.abs(g) + 1e-10), 0.0)
    np.testing.assert_allclose(q, expect, rtol=1e-14)
    np.testing.assert_allclose(A, g * g, rtol=1e-14)


def test_loss_definition():
    B, y, xs, _ = make_dense_instance(5, seed=17)
    assert orc.dense_loss(B, y, xs) <= 1e-24 * float(y @ y) + 1e-28
    q = xs + 0.1
    np.testing.assert_allclose(orc.dense_loss(B, y, q), np.sum((B @ q - y) ** 2), rtol=1e-13)
