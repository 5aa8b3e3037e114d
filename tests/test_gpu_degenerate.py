"""GPU: degenerate inputs of the SPGD path (Algorithm 1) through the C ABI.

- calls on zero days are no-ops;
- zero epochs leave the plan's state as loaded;
- a cluster with no days next to clusters with days;
- one minibatch per epoch (b >= H*L rows: the whole day is the minibatch);
- a day whose observations are all zero keeps q = 0 exactly (r = 0, g = 0);
- a single-interval day (H = T = 1, one lag).

Bars as in the parity tests: FP64 1e-9 on the loss history, reduced precision
1e-3 per day against the oracle run on the same rounded values.
"""
import numpy as np
import pytest

import oracle as orc
import paper_1901_09266_amd as dode
from synth import make_instance, make_perms, chunk_h_blocks
from gpu_helpers import say, make_dar, dev, dequantized_values

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def values(inst, storage):
    return inst.W if storage == "f64" else dequantized_values(inst, storage)


def state_dtype(storage):
    return torch.float64 if storage == "f64" else torch.float32


def run_plan(inst, storage, E, perms, batch_rows, Q0=None, n_run=None):
    """Plan of E epochs; runs n_run of them (all by default)."""
    dt = state_dtype(storage)
    dar = make_dar(inst, storage)
    p = dode.make_params(epochs=E, batch_rows=batch_rows, eta=5.0)
    plan = dode.spgd_plan_create(dar, inst.day_cluster, p, perm=perms, stream=0)
    if Q0 is None:
        Q0 = torch.zeros((inst.D, inst.T, inst.P), dtype=dt, device="cuda")
    dode.spgd_plan_load(plan, dev(inst.x, dt), Q0)
    n_run = E if n_run is None else n_run
    loss = torch.zeros((n_run, inst.D), dtype=torch.float64, device="cuda")
    dode.spgd_run(plan, 0, n_run, loss=loss)
    Q = torch.empty_like(Q0)
    A = torch.empty_like(Q0)
    dode.spgd_plan_store(plan, Q, A)
    torch.cuda.synchronize()
    return Q.cpu().numpy(), A.cpu().numpy(), loss.cpu().numpy().T, dode.spgd_plan_info(plan)


@pytest.mark.parametrize("storage", ["f64", "bf16"])
def test_zero_day_calls_are_noops(storage):
    inst = make_instance(P=6, L=9, T=8, K=3, sizes=(2,), inc=0.4, pattern="bernoulli",
                         x_dtype="f64", seed=201)
    say("zero-day calls", storage)
    dt = state_dtype(storage)
    dar = make_dar(inst, storage)
    Q = torch.zeros((0, inst.T, inst.P), dtype=dt, device="cuda")
    X = torch.zeros((0, inst.H, inst.L), dtype=dt, device="cuda")
    G = torch.zeros((0, inst.T, inst.P), dtype=dt, device="cuda")
    loss = torch.zeros((0,), dtype=torch.float64, device="cuda")
    dode.dode_apply(dar, 0, Q, X)
    dode.dode_loss(dar, 0, Q, X, loss)
    dode.dode_loss_noalloc(dar, 0, Q, X, loss)
    dode.dode_grad(dar, 0, Q, X, G)
    dode.dode_metrics(dar, 0, Q, X, loss, loss.clone(), loss.clone())
    dode.spgd_step(dar, 0, np.array([0, 3], dtype=np.int32), X, Q, G,
                   dode.make_params(epochs=1, batch_rows=2 * inst.L))
    torch.cuda.synchronize()


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_zero_epochs_leave_the_state(storage):
    inst = make_instance(P=20, L=40, T=24, K=4, sizes=(7, 5), inc=0.2, pattern="corridor",
                         x_dtype="f32", seed=202)
    say("zero epochs", storage)
    rng = np.random.default_rng(5)
    q0 = rng.uniform(0, 10, (inst.D, inst.T, inst.P)).astype(np.float32)
    Q0 = dev(q0, torch.float32)
    perms = make_perms(203, 3, inst.C, inst.H)
    Q, A, _, _ = run_plan(inst, storage, 3, perms, 5 * inst.L, Q0=Q0, n_run=0)
    assert np.array_equal(Q, q0)
    assert not A.any()


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16", "fp8"])
def test_cluster_without_days(storage):
    """Three clusters, the middle one without days: the plan covers the others
    and matches the oracle on the same permutations."""
    inst = make_instance(P=30, L=60, T=24, K=4, sizes=(35, 0, 20), inc=0.15, pattern="corridor",
                         demand="gamma", noise="mult5",
                         x_dtype="f64" if storage == "f64" else "f32", seed=204)
    say("cluster without days", storage, inst.D)
    assert inst.C == 3 and not (inst.day_cluster == 1).any()
    E = 8
    perms = make_perms(205, E, inst.C, inst.H)
    batch_rows = 4 * inst.L
    bh = chunk_h_blocks(inst.L, inst.H, batch_rows)
    x64 = inst.x.astype(np.float64)
    Qo, _, ho = orc.spgd(inst, x64, perms, E, bh, optimizer=0, eta=5.0, W=values(inst, storage))
    Q, _, hg, info = run_plan(inst, storage, E, perms, batch_rows)
    if storage in ("bf16", "fp8"):
        assert info["day_tile"] > 0, "the matrix-core kernels should run here"
    tol = 1e-9 if storage == "f64" else 1e-3
    assert np.max(np.abs(hg - ho) / ho) <= tol


@pytest.mark.parametrize("storage", ["f64", "bf16"])
def test_one_minibatch_per_epoch(storage):
    """b >= H*L rows: every epoch is one full-batch step of Algorithm 1 (the
    permutation only reorders the intervals of the one minibatch)."""
    inst = make_instance(P=24, L=50, T=20, K=5, sizes=(40,), inc=0.15, pattern="corridor",
                         demand="gamma", noise="mult5",
                         x_dtype="f64" if storage == "f64" else "f32", seed=206)
    say("one minibatch per epoch", storage)
    E = 6
    perms = make_perms(207, E, inst.C, inst.H)
    batch_rows = 10 * inst.H * inst.L
    bh = chunk_h_blocks(inst.L, inst.H, batch_rows)
    assert bh == inst.H
    x64 = inst.x.astype(np.float64)
    Qo, _, ho = orc.spgd(inst, x64, perms, E, bh, optimizer=0, eta=5.0, W=values(inst, storage))
    Q, _, hg, info = run_plan(inst, storage, E, perms, batch_rows)
    assert info["minibatch_intervals"] == inst.H and info["n_minibatches"] == 1
    tol = 1e-9 if storage == "f64" else 1e-3
    assert np.max(np.abs(hg - ho) / ho) <= tol


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_zero_observations_keep_zero_demand(storage):
    """A day with x = 0 everywhere: from q = 0 the residual and the gradient are
    zero, the Adagrad step is 0 / (0 + eps) = 0, so q and A stay exactly 0 while
    the other days move."""
    inst = make_instance(P=20, L=40, T=24, K=4, sizes=(33,), inc=0.2, pattern="corridor",
                         demand="gamma", noise="mult5", x_dtype="f32", seed=208)
    say("zero observations", storage)
    inst.x[5] = 0.0
    perms = make_perms(209, 4, inst.C, inst.H)
    Q, A, _, _ = run_plan(inst, storage, 4, perms, 4 * inst.L)
    assert not Q[5].any() and not A[5].any()
    assert Q[4].any() and Q[6].any()


@pytest.mark.parametrize("storage", ["f64", "bf16"])
def test_single_interval_day(storage):
    """H = T = 1 with one lag: the day is one block, one minibatch, one
    departure interval."""
    inst = make_instance(P=16, L=30, T=1, K=1, sizes=(20,), inc=0.3, pattern="bernoulli",
                         demand="gamma", noise="mult5",
                         x_dtype="f64" if storage == "f64" else "f32", seed=210)
    say("single interval", storage)
    E = 10
    perms = make_perms(211, E, inst.C, inst.H)
    x64 = inst.x.astype(np.float64)
    Qo, _, ho = orc.spgd(inst, x64, perms, E, 1, optimizer=0, eta=5.0, W=values(inst, storage))
    _, _, hg, _ = run_plan(inst, storage, E, perms, inst.L)
    tol = 1e-9 if storage == "f64" else 1e-3
    assert np.max(np.abs(hg - ho) / ho) <= tol
