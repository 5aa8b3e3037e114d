"""Algorithm 1 on the dense random NNLS of section "Algorithm efficiency" on
the GPU (dense_spgd_run) against the FP64 oracle: FP64 and FP32, vector and
scalar row paths (n a multiple of the vector width or not), B stored as
bfloat16 with FP32 arithmetic, minibatches with a
short tail and several slices, the fixed step, the per-epoch loss, the
sizes of the efficiency experiment (sampled), and the argument checks."""
import numpy as np
import pytest

import oracle as orc
import paper_1901_09266_amd as dode
from synth import make_dense_instance
from gpu_helpers import say, dev, rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def run(B, y, perms, chunk, eta, f64, optimizer=0, loss=True, q0=None):
    t = torch.float64 if f64 else torch.float32
    m, n = B.shape
    q = dev(np.zeros(n) if q0 is None else q0, t)
    A = torch.zeros(n, dtype=t, device="cuda")
    hist = dode.dense_spgd_run(dev(B, t), dev(y, t), q, A, dev(perms, torch.int32), chunk, eta,
                               optimizer=optimizer, loss_hist=loss)
    torch.cuda.synchronize()
    return q.cpu().numpy(), A.cpu().numpy(), hist


@pytest.mark.parametrize("f64", [True, False])
@pytest.mark.parametrize("m,n,chunk", [(100, 64, 100), (173, 61, 40), (300, 257, 77), (50, 7, 8),
                                        (1, 1, 1), (3, 1, 2), (1, 5, 4), (260, 12, 300)])
def test_matches_oracle(f64, m, n, chunk):
    B, y, _, perms = make_dense_instance(n, m=m, epochs=4, seed=31)
    y = y - 0.3 * y.mean()          # active bounds
    say("dense", f64, m, n, chunk)
    q, A, hist = run(B, y, perms, chunk, 0.05, f64)
    Bo = B if f64 else B.astype(np.float32).astype(np.float64)
    yo = y if f64 else y.astype(np.float32).astype(np.float64)
    qo, Ao, ho = orc.dense_spgd(Bo, yo, perms, chunk, 0.05)
    if f64:
        assert rel(q, qo) <= 1e-12 and rel(A, Ao) <= 1e-12
        np.testing.assert_allclose(hist, ho, rtol=1e-12)
    else:
        # FP32 dot products of length n and row sums of length chunk: a few
        # 1e-7 per step, through 4 epochs of Adagrad steps of size ~eta
        assert rel(q, qo) <= 2e-4 and rel(A, Ao) <= 2e-4
        np.testing.assert_allclose(hist, ho, rtol=2e-4)


def run_bf16(B, y, perms, chunk, eta, loss=True):
    """B rounded to bfloat16 on the host (the oracle gets the same values)."""
    Bh = torch.as_tensor(np.ascontiguousarray(B), dtype=torch.float32).to(torch.bfloat16)
    m, n = B.shape
    q = torch.zeros(n, dtype=torch.float32, device="cuda")
    A = torch.zeros(n, dtype=torch.float32, device="cuda")
    hist = dode.dense_spgd_run(Bh.cuda(), dev(y, torch.float32), q, A, dev(perms, torch.int32),
                               chunk, eta, loss_hist=loss)
    torch.cuda.synchronize()
    return q.cpu().numpy(), A.cpu().numpy(), hist, Bh.to(torch.float64).numpy()


@pytest.mark.parametrize("m,n,chunk", [(100, 64, 100), (173, 61, 40), (300, 257, 77), (50, 7, 8),
                                        (1, 1, 1), (260, 16, 300), (129, 24, 128)])
def test_bf16_matrix_matches_oracle(m, n, chunk):
    """B stored as bfloat16, FP32 arithmetic: equals the oracle run on the
    bf16-rounded B to FP32 rounding (the 16-byte path for n % 8 == 0, the
    scalar path otherwise)."""
    B, y, _, perms = make_dense_instance(n, m=m, epochs=4, seed=35)
    y = y - 0.3 * y.mean()
    say("dense bf16", m, n, chunk)
    q, A, hist, Bo = run_bf16(B, y, perms, chunk, 0.05)
    qo, Ao, ho = orc.dense_spgd(Bo, y.astype(np.float32).astype(np.float64), perms, chunk, 0.05)
    assert rel(q, qo) <= 2e-4 and rel(A, Ao) <= 2e-4
    np.testing.assert_allclose(hist, ho, rtol=2e-4)


def test_bf16_matrix_paper_size_sampled():
    """n = 6000 square with B in bfloat16, 3 epochs of one 8192-row
    minibatch: losses and a sample of q against the oracle on the same B."""
    n = 6000
    B, y, _, perms = make_dense_instance(n, epochs=3, seed=36)
    say("dense bf16 6000")
    q, _, hist, Bo = run_bf16(B, y, perms, 8192, 1e-3)
    qo, _, ho = orc.dense_spgd(Bo, y.astype(np.float32).astype(np.float64), perms, 8192, 1e-3)
    np.testing.assert_allclose(hist, ho, rtol=1e-4)
    idx = np.random.default_rng(1).choice(n, 200, replace=False)
    np.testing.assert_allclose(q[idx], qo[idx], rtol=1e-4, atol=1e-7)


def test_fixed_step_fp64():
    B, y, _, perms = make_dense_instance(33, m=90, epochs=5, seed=32)
    eta = 1.0 / np.linalg.eigvalsh(B.T @ B)[-1]
    say("dense fixed step")
    q, _, hist = run(B, y - 1.0, perms, 32, eta, True, optimizer=1)
    qo, _, ho = orc.dense_spgd(B, y - 1.0, perms, 32, eta, optimizer=1)
    assert rel(q, qo) <= 1e-12
    np.testing.assert_allclose(hist, ho, rtol=1e-12)


def test_paper_sizes_sampled():
    """n = 6000 square, one minibatch of all rows per epoch (chunk 8192 of
    Algorithm 1): after 3 epochs in FP32 the loss history and a sample of q
    match the oracle run on the same FP32-rounded data."""
    n = 6000
    B, y, _, perms = make_dense_instance(n, epochs=3, seed=33)
    B32 = B.astype(np.float32)
    say("dense 6000")
    q, _, hist = run(B32, y, perms, 8192, 1e-3, False)
    qo, _, ho = orc.dense_spgd(B32.astype(np.float64), y.astype(np.float32).astype(np.float64),
                               perms, 8192, 1e-3)
    np.testing.assert_allclose(hist, ho, rtol=1e-4)
    idx = np.random.default_rng(0).choice(n, 200, replace=False)
    np.testing.assert_allclose(q[idx], qo[idx], rtol=1e-4, atol=1e-7)


def test_zero_epochs_and_checks():
    B, y, _, perms = make_dense_instance(16, m=20, epochs=1, seed=34)
    t = torch.float64
    q = torch.ones(16, dtype=t, device="cuda")
    A = torch.zeros(16, dtype=t, device="cuda")
    say("dense checks")
    dode.dense_spgd_run(dev(B, t), dev(y, t), q, A, torch.zeros((0, 20), dtype=torch.int32,
                                                                device="cuda"), 8, 0.1)
    assert torch.all(q == 1)
    bad = perms.copy()
    bad[0, 3] = bad[0, 4]
    with pytest.raises(dode.DodeError, match="permutation"):
        dode.dense_spgd_run(dev(B, t), dev(y, t), q, A, dev(bad, torch.int32), 8, 0.1)
    with pytest.raises(dode.DodeError, match="chunk"):
        dode.dense_spgd_run(dev(B, t), dev(y, t), q, A, dev(perms, torch.int32), 0, 0.1)
    with pytest.raises(dode.DodeError, match="eta"):
        dode.dense_spgd_run(dev(B, t), dev(y, t), q, A, dev(perms, torch.int32), 8, -1.0)
