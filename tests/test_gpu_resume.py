"""Checkpoint and resume: the solver state is (Q, the Adagrad accumulator A,
the epoch index, the permutations).  Stopping after E1 epochs, storing the
state to host memory, building a new plan, loading it and running the
remaining epochs gives the uninterrupted run's bits, in every storage type."""
import numpy as np
import pytest

import paper_1901_09266_amd as dode
from synth import make_instance, make_perms
from gpu_helpers import say, make_dar, dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16", "fp8"])
def test_resume_matches_uninterrupted(storage):
    inst = make_instance(P=30, L=60, T=48, K=5, sizes=(20, 13, 4), inc=0.15, pattern="corridor",
                         demand="gamma", noise="mult5", seed=61)
    say("resume", storage)
    E, E1 = 10, 4
    perms = make_perms(62, E, inst.C, inst.H)
    dt = torch.float64 if storage == "f64" else torch.float32
    dar = make_dar(inst, storage)
    X = dev(inst.x, dt)
    shape = (inst.D, inst.T, inst.P)
    p = dode.make_params(epochs=E, batch_rows=9 * inst.L, eta=5.0)

    def fresh_plan():
        return dode.spgd_plan_create(dar, inst.day_cluster, p, perm=perms, stream=0)

    # uninterrupted
    plan = fresh_plan()
    dode.spgd_plan_load(plan, X, torch.zeros(shape, dtype=dt, device="cuda"))
    dode.spgd_run(plan, 0, E)
    Qa, Aa = torch.empty(shape, dtype=dt, device="cuda"), torch.empty(shape, dtype=dt, device="cuda")
    dode.spgd_plan_store(plan, Qa, Aa)
    torch.cuda.synchronize()
    del plan
    # E1 epochs, checkpoint to host, new plan, resume at epoch E1
    plan = fresh_plan()
    dode.spgd_plan_load(plan, X, torch.zeros(shape, dtype=dt, device="cuda"))
    dode.spgd_run(plan, 0, E1)
    Qc, Ac = torch.empty(shape, dtype=dt, device="cuda"), torch.empty(shape, dtype=dt, device="cuda")
    dode.spgd_plan_store(plan, Qc, Ac)
    torch.cuda.synchronize()
    ckpt = (Qc.cpu().numpy().copy(), Ac.cpu().numpy().copy())
    del plan, Qc, Ac
    plan = fresh_plan()
    dode.spgd_plan_load(plan, X, dev(ckpt[0], dt), dev(ckpt[1], dt))
    dode.spgd_run(plan, E1, E - E1)
    Qb, Ab = torch.empty(shape, dtype=dt, device="cuda"), torch.empty(shape, dtype=dt, device="cuda")
    dode.spgd_plan_store(plan, Qb, Ab)
    torch.cuda.synchronize()
    assert torch.equal(Qa, Qb) and torch.equal(Aa, Ab)
    assert float(Qa.abs().sum()) > 0
