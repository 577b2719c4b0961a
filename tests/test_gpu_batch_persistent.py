"""GPU parity of the persistent batched form (the whole task list of many
products in one launch: tickets, per-instance stage counters, bounded waits)
against the phase form of the same batch (bitwise: same tasks, same plans)
and against the CPU oracle (integer inputs, exact)."""
import numpy as np
import pytest

import mf_inputs as mi
from oracle import matmul as om

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
mf = pytest.importorskip("paper_2312_12732_amd.mf", reason="libmf.so not built")

SIZES = mi.batch_sizes(24, 30) + [100, 300, 513, 64, 1, 1024]


def algos_for(sizes):
    w = mf.mf_algo_builtin("winograd")
    s = mf.mf_algo_builtin("strassen")
    s69 = mf.mf_algo_builtin("strassen1969")
    choices = [(None, 0), (w, 1), (w, 2), (s, 1), (s69, 1), (w, 3)]
    pick = [choices[i % len(choices)] for i in range(len(sizes))]
    return [a for a, _ in pick], [d for _, d in pick]


def run(batch, dA, dB):
    dC = [torch.full_like(a, float("nan")) for a in dA]
    mf.mf_batch_run(batch, dA, dB, dC)
    torch.cuda.synchronize()
    return dC


@pytest.mark.parametrize("code,tdt", [(mf.MF_F64, torch.float64), (mf.MF_F32, torch.float32)])
def test_persistent_equals_phase_form_and_oracle(code, tdt):
    print(f"persistent batch, dtype code {code}, {len(SIZES)} instances", flush=True)
    algos, depths = algos_for(SIZES)
    cut = [0] * len(SIZES)
    pers = mf.mf_batch_create(SIZES, algos, depths, cut, code, form=mf.MF_BATCH_PERSISTENT)
    phase = mf.mf_batch_create(SIZES, algos, depths, cut, code)
    Ai = [mi.int_uniform(n, 1300 + i) for i, n in enumerate(SIZES)]
    Bi = [mi.int_uniform(n, 1400 + i) for i, n in enumerate(SIZES)]
    dA = [torch.from_numpy(a.astype(np.float64)).to("cuda:0", tdt) for a in Ai]
    dB = [torch.from_numpy(b.astype(np.float64)).to("cuda:0", tdt) for b in Bi]
    got = run(pers, dA, dB)
    assert not pers.aborted()
    want = run(phase, dA, dB)
    for A, B, g, w in zip(Ai, Bi, got, want):
        assert torch.equal(g, w)
        assert np.array_equal(g.cpu().numpy().astype(np.float64), om.classical_mm(A, B).astype(np.float64))
    # uniform inputs, two runs in a row: bitwise equal to the phase form each time
    for rep in range(2):
        dA = [torch.from_numpy(mi.uniform(n, 1500 + 50 * rep + i)).to("cuda:0", tdt) for i, n in enumerate(SIZES)]
        dB = [torch.from_numpy(mi.uniform(n, 1600 + 50 * rep + i)).to("cuda:0", tdt) for i, n in enumerate(SIZES)]
        got = run(pers, dA, dB)
        assert not pers.aborted()
        want = run(phase, dA, dB)
        assert all(torch.equal(g, w) for g, w in zip(got, want))


def test_persistent_matches_standalone_classical():
    sizes = [256, 640, 1024]
    b = mf.mf_batch_create(sizes, [None] * 3, [0] * 3, [0] * 3, mf.MF_F64, form=mf.MF_BATCH_PERSISTENT)
    dA = [torch.from_numpy(mi.uniform(n, 1 + i)).cuda() for i, n in enumerate(sizes)]
    dB = [torch.from_numpy(mi.uniform(n, 11 + i)).cuda() for i, n in enumerate(sizes)]
    got = run(b, dA, dB)
    assert not b.aborted()
    for A, B, C in zip(dA, dB, got):
        ref = torch.empty_like(A)
        mf.mf_classical_mm(A, B, ref)
        torch.cuda.synchronize()
        assert torch.equal(C, ref)
