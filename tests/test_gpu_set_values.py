"""dar_set_values: values written into a handle built from other values give
what a handle built from them directly gives, for the sparse kernels
(dode_apply on the sliced copies) and for the matrix-core tiles (an SPGD
plan), in every storage type."""
import numpy as np
import pytest

import paper_1901_09266_amd as dode
from synth import make_instance, make_perms
from gpu_helpers import say, dev, rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16", "fp8"])
def test_set_values_equals_create(storage):
    inst = make_instance(P=30, L=60, T=24, K=4, sizes=(20,), inc=0.15, pattern="corridor",
                         demand="gamma", noise="mult5", seed=81)
    # new values exactly representable in FP32, so host (FP64) and device
    # (FP32) conversions to the storage type see the same number
    W1 = (inst.W[0] * 0.7 + 0.01).astype(np.float32).astype(np.float64)
    dt = torch.float64 if storage == "f64" else torch.float32
    say("set values", storage)
    a = dode.dar_create(inst.P, inst.L, inst.T, inst.H, inst.K, inst.row_ptr, inst.col_idx,
                        [inst.W[0]], storage=storage, stream=0)
    dode.dar_set_values(a, 0, dev(W1, dt))
    b = dode.dar_create(inst.P, inst.L, inst.T, inst.H, inst.K, inst.row_ptr, inst.col_idx,
                        [W1], storage=storage, stream=0)
    Q = dev(inst.qstar, dt)
    Xa = torch.empty((inst.D, inst.H, inst.L), dtype=dt, device="cuda")
    Xb = torch.empty_like(Xa)
    dode.dode_apply(a, 0, Q, Xa)
    dode.dode_apply(b, 0, Q, Xb)
    # SPGD through plans (matrix-core tiles for BF16/FP8)
    E = 4
    perms = make_perms(82, E, inst.C, inst.H)
    X = dev(inst.x, dt)
    outs = []
    for dar in (a, b):
        p = dode.make_params(epochs=E, batch_rows=6 * inst.L, eta=5.0)
        plan = dode.spgd_plan_create(dar, inst.day_cluster, p, perm=perms, stream=0)
        Qp = torch.zeros((inst.D, inst.T, inst.P), dtype=dt, device="cuda")
        dode.spgd_plan_load(plan, X, Qp)
        dode.spgd_run(plan, 0, E)
        dode.spgd_plan_store(plan, Qp)
        outs.append(Qp)
    torch.cuda.synchronize()
    if storage == "fp8":
        # the device requantisation divides in FP32, the host in FP64: a code
        # can land on the other side of a rounding tie (one E4M3 step)
        assert rel(Xa.cpu().numpy(), Xb.cpu().numpy()) <= 2e-2
        assert rel(outs[0].cpu().numpy(), outs[1].cpu().numpy()) <= 2e-2
    else:
        assert torch.equal(Xa, Xb)
        assert torch.equal(outs[0], outs[1])
