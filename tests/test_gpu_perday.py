"""Per-day assignment ratios (every day its own rho, the paper's literal
setup): one cluster per day through the same C ABI, against the FP64 oracle,
in every storage type, with several minibatches, the plan/graph path and the
one-call solve."""
import numpy as np
import pytest

import oracle as orc
import paper_1901_09266_amd as dode
from synth import make_instance, make_perms, chunk_h_blocks
from gpu_helpers import say, make_dar, dev, rel, dequantized_values

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def per_day_instance(seed=90):
    return make_instance(P=24, L=60, T=36, K=5, sizes=(1,) * 7, inc=0.15, pattern="corridor",
                         demand="gamma", noise="mult5", x_dtype="f32", seed=seed)


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16", "fp8"])
def test_per_day_solve_matches_oracle(storage):
    inst = per_day_instance()
    assert inst.C == inst.D == 7 and len({w.tobytes() for w in inst.W}) == 7
    say("per-day solve", storage)
    E, batch_rows, eta = 20, 9 * inst.L, 5.0
    perms = make_perms(91, E, inst.C, inst.H)
    bh = chunk_h_blocks(inst.L, inst.H, batch_rows)
    Wq = dequantized_values(inst, storage) if storage in ("bf16", "fp8") else None
    if storage == "f32":
        Wq = [w.astype(np.float32).astype(np.float64) for w in inst.W]
    x64 = inst.x.astype(np.float64)
    Qo, Ao, ho = orc.spgd(inst, x64, perms, E, bh, optimizer=0, eta=eta, W=Wq)
    dt = torch.float64 if storage == "f64" else torch.float32
    dar = make_dar(inst, storage)
    Qd = torch.zeros((inst.D, inst.T, inst.P), dtype=dt, device="cuda")
    Ad = torch.zeros_like(Qd)
    p = dode.make_params(epochs=E, batch_rows=batch_rows, eta=eta, optimizer=0)
    hg = dode.spgd_solve(dar, inst.day_cluster, dev(x64, dt), Qd, Ad, p, perm=perms, loss_hist=True)
    torch.cuda.synchronize()
    tol = 1e-10 if storage == "f64" else 1e-3
    assert np.max(np.abs(hg - ho) / ho) <= tol
    if storage == "f64":
        assert rel(Qd.cpu().numpy(), Qo) <= 1e-8


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_per_day_plan_matches_solve(storage):
    """The plan (day groups of one day each, graph replay) gives the one-call
    solve's bits."""
    inst = per_day_instance(seed=92)
    say("per-day plan", storage)
    E, batch_rows, eta = 6, 7 * inst.L, 5.0
    perms = make_perms(93, E, inst.C, inst.H)
    dar = make_dar(inst, storage)
    X = dev(inst.x, torch.float32)
    p = dode.make_params(epochs=E, batch_rows=batch_rows, eta=eta, optimizer=0, day_tile=16)
    Q1 = torch.zeros((inst.D, inst.T, inst.P), dtype=torch.float32, device="cuda")
    A1 = torch.zeros_like(Q1)
    dode.spgd_solve(dar, inst.day_cluster, X, Q1, A1, p, perm=perms)
    plan = dode.spgd_plan_create(dar, inst.day_cluster, p, perm=perms, stream=0)
    Q2 = torch.zeros_like(Q1)
    A2 = torch.zeros_like(Q1)
    dode.spgd_plan_load(plan, X, Q2, A2, stream=0)
    dode.spgd_run(plan, 0, E, stream=0)
    dode.spgd_plan_store(plan, Q2, A2, stream=0)
    torch.cuda.synchronize()
    assert torch.equal(Q1, Q2) and torch.equal(A1, A2)


@pytest.mark.parametrize("storage", ["bf16", "fp8"])
def test_fastest_path_for_one_day_clusters(storage):
    """kernel_path 0 takes the sparse kernels when no cluster has more than 2
    days: the plan reports no day tile and gives kernel_path 1's bits."""
    inst = per_day_instance(seed=94)
    say("path choice", storage)
    E = 5
    perms = make_perms(95, E, inst.C, inst.H)
    dar = make_dar(inst, storage)
    X = dev(inst.x, torch.float32)
    outs = []
    for path in (0, 1):
        p = dode.make_params(epochs=E, batch_rows=7 * inst.L, eta=5.0, kernel_path=path)
        plan = dode.spgd_plan_create(dar, inst.day_cluster, p, perm=perms, stream=0)
        assert dode.spgd_plan_info(plan)["day_tile"] == 0
        Q = torch.zeros((inst.D, inst.T, inst.P), dtype=torch.float32, device="cuda")
        dode.spgd_plan_load(plan, X, Q)
        dode.spgd_run(plan, 0, E)
        dode.spgd_plan_store(plan, Q)
        torch.cuda.synchronize()
        outs.append(Q.cpu().numpy())
    np.testing.assert_array_equal(outs[0], outs[1])
