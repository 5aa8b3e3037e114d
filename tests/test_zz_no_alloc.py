"""dode_loss_noalloc (the allocation-free variant of dode_loss) against
dode_loss through the C ABI: the same bits on two calls in a row, the second
with fewer days (the shared scratch keeps the first call's partials), for
FP64, FP32 and BF16 values; the FP64 losses also against the oracle; calls past
the 4 MiB scratch are argument errors raised before any launch."""
import numpy as np
import pytest

import oracle as orc
import paper_1901_09266_amd as dode
from synth import make_instance
from gpu_helpers import say, make_dar, dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
def test_loss_noalloc_equals_loss(storage):
    inst = make_instance(P=30, L=60, T=48, K=5, sizes=(40, 9), inc=0.15, pattern="corridor",
                         demand="gamma", noise="mult5", x_dtype="f64", seed=71)
    say("loss_noalloc", storage)
    dt = torch.float64 if storage == "f64" else torch.float32
    dar = make_dar(inst, storage)
    rng = np.random.default_rng(72)
    Q = rng.uniform(0, 30, (inst.D, inst.T, inst.P))
    for c, n in ((0, 40), (0, 13), (1, 9), (1, 2)):
        days = inst.days_of(c)[:n]
        Qd, Xd = dev(Q[days], dt), dev(inst.x[days], dt)
        a = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
        b = torch.full((n,), -2.0, dtype=torch.float64, device="cuda")
        dode.dode_loss(dar, c, Qd, Xd, a)
        dode.dode_loss_noalloc(dar, c, Qd, Xd, b)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(b.cpu().numpy(), a.cpu().numpy())
        if storage == "f64":
            lo = np.array([orc.loss(inst, inst.W[c], Q[d], inst.x[d]) for d in days])
            np.testing.assert_allclose(b.cpu().numpy(), lo, rtol=1e-12)


def test_loss_noalloc_rejects_calls_past_its_scratch():
    inst = make_instance(P=3, L=4, T=288, K=2, sizes=(1822,), inc=0.6, pattern="bernoulli",
                         demand="uniform50", noise="add1", x_dtype="f64", seed=73)
    say("loss_noalloc limit")
    dar = make_dar(inst, "f32")
    Q = torch.zeros((inst.D, inst.T, inst.P), dtype=torch.float32, device="cuda")
    X = dev(inst.x, torch.float32)
    # 1820 days x 288 rows x 8 bytes fit in 4 MiB; 1821 do not
    ok = torch.empty(1820, dtype=torch.float64, device="cuda")
    dode.dode_loss_noalloc(dar, 0, Q[:1820], X[:1820], ok)
    ref = torch.empty(1820, dtype=torch.float64, device="cuda")
    dode.dode_loss(dar, 0, Q[:1820], X[:1820], ref)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(ok.cpu().numpy(), ref.cpu().numpy())
    bad = torch.empty(1821, dtype=torch.float64, device="cuda")
    with pytest.raises(dode.DodeError, match="DODE_ERR_ARG.*scratch"):
        dode.dode_loss_noalloc(dar, 0, Q[:1821], X[:1821], bad)
