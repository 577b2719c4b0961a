"""GPU checks of the batched-form autotuner: it measures every candidate a
size admits, skips depths the level rule would not take, and its choices
drive a batch whose results are exact on integer inputs."""
import numpy as np
import pytest

import mf_inputs as mi

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
mf = pytest.importorskip("paper_2312_12732_amd.mf", reason="libmf.so not built")


def test_tuner_candidates_and_choice():
    s = mf.mf_algo_builtin("winograd")
    sizes = [128, 200, 512]
    choices, ms = mf.mf_autotune_batch(sizes, mf.MF_F64, [s], 2, work_flops=2e9, max_copies=64, reps=2)
    # 128: no level is taken (the leaf would fall below the tile), both depths skipped
    assert ms[0][0] > 0 and ms[0][1] == -1 and ms[0][2] == -1 and choices[0] == (None, 0)
    # 200: one level (200 -> 100 padded to the tile), depth 2 skipped
    assert ms[1][1] > 0 and ms[1][2] == -1
    # 512: both depths are real plans
    assert all(x > 0 for x in ms[2])
    # the fastest candidate, unless it beats the classical GEMM by less than 5%
    for (al, d), row in zip(choices, ms):
        best = min(x for x in row if x > 0)
        if d == 0:
            assert row[0] == best or best > 0.95 * row[0]
        else:
            assert row[d] == best and best <= 0.95 * row[0]


def test_tuned_batch_is_exact():
    s = mf.mf_algo_builtin("winograd")
    sizes = [256, 640, 128, 1024, 384]
    choices, _ = mf.mf_autotune_batch(sorted(set(sizes)), mf.MF_F32, [s], 3, work_flops=4e9, max_copies=32, reps=1)
    pick = dict(zip(sorted(set(sizes)), choices))
    b = mf.mf_batch_create(sizes, [pick[n][0] for n in sizes], [pick[n][1] for n in sizes], [0] * len(sizes),
                           mf.MF_F32)
    As = [mi.int_uniform(n, 70 + i).astype(np.float32) for i, n in enumerate(sizes)]
    Bs = [mi.int_uniform(n, 80 + i).astype(np.float32) for i, n in enumerate(sizes)]
    dA = [torch.from_numpy(a).cuda() for a in As]
    dB = [torch.from_numpy(b_).cuda() for b_ in Bs]
    dC = [torch.full_like(a, float("nan")) for a in dA]
    mf.mf_batch_run(b, dA, dB, dC)
    torch.cuda.synchronize()
    assert not b.aborted()
    for A, B, C in zip(As, Bs, dC):
        assert np.array_equal(C.cpu().numpy().astype(np.float64), A.astype(np.float64) @ B.astype(np.float64))
