"""GPU parity at the full shapes of the benchmark workloads.

- 150 OD x 500 links x 288 intervals, K = 6, 1095 days in 8 clusters
  (400 ... 15), bf16 values, 3 epochs of the grouped plan (minibatches of
  16 intervals), checked day by day against the oracle on the first and last
  day of every cluster, run on the same bf16-rounded values.
- 400 OD x 1500 links x 288 intervals, K = 6 (minibatches of 5 intervals),
  clusters of 36, 5 and 2 days, FP8 values with two full-batch refinement
  steps per epoch on the corrected values, 3 epochs, against the oracle
  running the same composition on sampled days; with the chunked adjoint
  and with the schedule timed by the benchmark (64-day waves, order 1).
- The full config-5 workload: 1095 days in 12 clusters (300 ... 10), FP8
  with two refinement steps, 2 epochs in the launch configuration the
  benchmark times (64-day waves, order-1 adjoint, two day slabs), checked on
  the first and last day of three clusters (the largest, a middle one and
  the smallest).
The config-3 plan runs the schedule the benchmark times there (32-day
waves, chunked adjoint, two day slabs).

Bars: per-day loss after every epoch within 1e-4 relative (the FP32
arithmetic of the kernels against FP64 on the same values), the demand
within 2e-3 of each entry (floor 1e-3 of the largest entry).
"""
import functools

import numpy as np
import pytest

import oracle as orc
import paper_1901_09266_amd as dode
from synth import make_config, make_instance, make_perms, chunk_h_blocks
from gpu_helpers import say, make_dar, dev, rel_elem, dequantized_values, fp8_values

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def run_plan(inst, storage, E, perms, refine=0, adj_order=1, day_tile=32, slabs=1):
    dar = make_dar(inst, storage, correction=refine > 0)
    p = dode.make_params(epochs=E, batch_rows=8192, eta=5.0, refine_steps=refine,
                         adj_order=adj_order, day_tile=day_tile, slabs=slabs)
    plan = dode.spgd_plan_create(dar, inst.day_cluster, p, perm=perms, stream=0)
    Q0 = torch.zeros((inst.D, inst.T, inst.P), dtype=torch.float32, device="cuda")
    dode.spgd_plan_load(plan, dev(inst.x, torch.float32), Q0)
    info = dode.spgd_plan_info(plan)
    loss = torch.zeros((E, inst.D), dtype=torch.float64, device="cuda")
    dode.spgd_run(plan, 0, E, loss=loss)
    Q = torch.empty_like(Q0)
    dode.spgd_plan_store(plan, Q)
    torch.cuda.synchronize()
    return Q.cpu().numpy().astype(np.float64), loss.cpu().numpy().T, info


def test_config3_full_shape_bf16_plan():
    inst = make_config(3)
    say("config-3 shape bf16 plan, 1095 days, 3 epochs")
    E = 3
    perms = make_perms(inst.seed + 1, E, inst.C, inst.H)
    bh = chunk_h_blocks(inst.L, inst.H, 8192)
    Qg, hg, info = run_plan(inst, "bf16", E, perms, adj_order=2, day_tile=32, slabs=2)
    assert info["day_tile"] == 32 and info["minibatch_intervals"] == bh == 16
    sample = np.concatenate([[d[0], d[-1]] for d in (inst.days_of(c) for c in range(inst.C))])
    Wq = dequantized_values(inst, "bf16")
    x64 = inst.x.astype(np.float64)
    Qo, _, ho = orc.spgd(inst, x64, perms, E, bh, days=sample, optimizer=0, eta=5.0, W=Wq)
    assert np.max(np.abs(hg[sample] - ho) / ho) <= 1e-4
    assert rel_elem(Qg[sample], Qo) <= 2e-3


@functools.lru_cache(maxsize=1)
def config5_shape():
    return make_instance(P=400, L=1500, T=288, K=6, sizes=(36, 5, 2), inc=0.08,
                         pattern="corridor", demand="gamma", noise="mult5", x_dtype="f32",
                         seed=1901)


# (day tile, adjoint order): the chunked adjoint, and the schedule the tuner
# picks for the config-5 benchmark (64-day waves, OD-tile-major adjoint)
@pytest.mark.parametrize("day_tile,adj_order", [(32, 2), (64, 1)])
def test_config5_shape_fp8_refinement_plan(day_tile, adj_order):
    inst = config5_shape()
    say("config-5 shape fp8 + 2 refinement steps, 43 days, 3 epochs", day_tile, adj_order)
    E, R = 3, 2
    perms = make_perms(1902, E, inst.C, inst.H)
    bh = chunk_h_blocks(inst.L, inst.H, 8192)
    Qg, hg, info = run_plan(inst, "fp8", E, perms, refine=R, adj_order=adj_order,
                            day_tile=day_tile)
    assert info["minibatch_intervals"] == bh == 5 and info["day_tile"] == day_tile
    sample = np.array([0, 35, 36, 40, 42])
    Wq = dequantized_values(inst, "fp8")
    Wr = dequantized_values(inst, "fp8corr")
    x64 = inst.x.astype(np.float64)
    ident = np.tile(np.arange(inst.H, dtype=np.int32), (1, inst.C, 1))
    Q = A = None
    hist = []
    for e in range(E):
        Q, A, _ = orc.spgd(inst, x64, perms[e:e + 1], 1, bh, days=sample, q0=Q, A0=A, W=Wq,
                           record_loss=False)
        for _ in range(R):
            Q, A, _ = orc.spgd(inst, x64, ident, 1, inst.H, days=sample, q0=Q, A0=A, W=Wr,
                               record_loss=False)
        hist.append(orc.metrics(inst, x64, Q, days=sample, W=Wq)[0])
    ho = np.stack(hist, axis=1)
    assert np.max(np.abs(hg[sample] - ho) / ho) <= 1e-4
    assert rel_elem(Qg[sample], Q) <= 2e-3


def oracle_fp8_refine(inst, x64, perms, E, R, bh, sample, Wq, Wr):
    """The oracle's composition of the FP8 form with refinement: each epoch the
    minibatches of Algorithm 1 on the FP8 values, then R full-batch steps on the
    corrected values; the per-day loss after each epoch on the FP8 values."""
    ident = np.tile(np.arange(inst.H, dtype=np.int32), (1, inst.C, 1))
    Q = A = None
    hist = []
    for e in range(E):
        Q, A, _ = orc.spgd(inst, x64, perms[e:e + 1], 1, bh, days=sample, q0=Q, A0=A, W=Wq,
                           record_loss=False)
        for _ in range(R):
            Q, A, _ = orc.spgd(inst, x64, ident, 1, inst.H, days=sample, q0=Q, A0=A, W=Wr,
                               record_loss=False)
        hist.append(orc.metrics(inst, x64, Q, days=sample, W=Wq)[0])
    return Q, np.stack(hist, axis=1)


@pytest.mark.timeout(900)
def test_config5_full_size_fp8_refinement_plan():
    inst = make_config(5)
    say("config-5 full size fp8 + 2 refinement steps, 1095 days, 2 epochs, 64,1,2")
    E, R = 2, 2
    perms = make_perms(inst.seed + 1, E, inst.C, inst.H)
    bh = chunk_h_blocks(inst.L, inst.H, 8192)
    Qg, hg, info = run_plan(inst, "fp8", E, perms, refine=R, adj_order=1, day_tile=64, slabs=2)
    assert info["minibatch_intervals"] == bh == 5 and info["day_tile"] == 64
    assert inst.D == 1095 and inst.C == 12
    say("config-5 full size: GPU plan done, oracle on sampled days")
    clusters = [0, inst.C // 2, inst.C - 1]
    sample = np.concatenate([[inst.days_of(c)[0], inst.days_of(c)[-1]] for c in clusters])
    # the values of the sampled clusters only (the oracle reads no other)
    Wq, Wr = [np.zeros(1)] * inst.C, [np.zeros(1)] * inst.C
    for c in clusters:
        Wq[c], Wr[c] = fp8_values(inst.W[c], inst.col_idx)
        say("config-5 full size: values of cluster", c)
    # the oracle converts the sampled days' rows to FP64 (exactly, from FP32)
    Q, ho = oracle_fp8_refine(inst, inst.x, perms, E, R, bh, sample, Wq, Wr)
    assert np.max(np.abs(hg[sample] - ho) / ho) <= 1e-4
    assert rel_elem(Qg[sample], Q) <= 2e-3
