"""GPU parity of the batched form on its benchmark workload: sizes
n = 64 round(exp(U(ln 128, ln 2048)) / 64) drawn with seed 30, FP64 and FP32
batches, every instance checked against the CPU oracle.  Plans cycle through
the classical GEMM, the paper's Strassen, Strassen-Winograd at depth 1 and 2
and <4,4,4;49> (Winograd composed with itself), so every eligible algorithm
runs inside one batch; a second test drives a batch from the autotuner with
Strassen and <4,4,4;49> among its candidates."""
import numpy as np
import pytest

import mf_inputs as mi
from oracle import matmul as om

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
mf = pytest.importorskip("paper_2312_12732_amd.mf", reason="libmf.so not built")

COUNT = 64


def config4_sizes():
    """The first COUNT sizes of the 512-instance draw, with its largest size
    (2048) in place of the last one so that the top of the range is covered."""
    full = mi.batch_sizes(512, 30)
    sizes = full[:COUNT]
    sizes[-1] = max(full)
    assert max(sizes) == 2048 and min(sizes) >= 128 and all(n % 64 == 0 for n in sizes)
    return sizes


def cycled_plans():
    wino = mf.mf_algo_builtin("winograd")
    stras = mf.mf_algo_builtin("strassen")
    c444 = mf.mf_algo_compose(wino, wino)
    return [(None, 0), (stras, 1), (wino, 1), (wino, 2), (c444, 1)]


def run_batch(sizes, algos, depths, code, tdt, seed0):
    b = mf.mf_batch_create(sizes, algos, depths, [0] * len(sizes), code)
    dA, dB, dC = [], [], []
    for i, n in enumerate(sizes):
        A = torch.empty(n, n, dtype=tdt, device="cuda:0")
        B = torch.empty(n, n, dtype=tdt, device="cuda:0")
        mf.mf_fill_uniform(A, 2 * (seed0 + i))
        mf.mf_fill_uniform(B, 2 * (seed0 + i) + 1)
        dA.append(A)
        dB.append(B)
        dC.append(torch.full_like(A, float("nan")))
    mf.mf_batch_run(b, dA, dB, dC)
    torch.cuda.synchronize()
    assert not b.aborted()
    return b, dA, dB, dC


def assert_exact(C_dev, A, B, i):
    """C equals the integer product A B, entry for entry."""
    assert np.array_equal(C_dev.cpu().numpy(), om.classical_mm(A, B).astype(np.float64)), f"instance {i}"


def host_operands(n, i, seed0, npdt):
    A = mi.counter_uniform(n * n, 2 * (seed0 + i), npdt).astype(np.float64).reshape(n, n)
    B = mi.counter_uniform(n * n, 2 * (seed0 + i) + 1, npdt).astype(np.float64).reshape(n, n)
    return A, B


@pytest.mark.parametrize("name", ["f64", "f32"])
def test_config4_every_instance_against_oracle(name):
    code, tdt, npdt, tol = {"f64": (mf.MF_F64, torch.float64, np.float64, 1e-11),
                            "f32": (mf.MF_F32, torch.float32, np.float32, 2e-5)}[name]
    sizes = config4_sizes()
    plans = cycled_plans()
    algos = [plans[i % len(plans)][0] for i in range(len(sizes))]
    depths = [plans[i % len(plans)][1] for i in range(len(sizes))]
    print(f"config4 {name}: {len(sizes)} instances, sizes {min(sizes)}..{max(sizes)}", flush=True)
    _, _, _, dC = run_batch(sizes, algos, depths, code, tdt, 31)
    worst = 0.0
    for i, n in enumerate(sizes):
        A, B = host_operands(n, i, 31, npdt)
        rows = np.sort(np.random.default_rng(i).choice(n, size=min(n, 48), replace=False))
        got = dC[i][torch.from_numpy(rows).cuda()].cpu().numpy().astype(np.float64)
        assert np.isfinite(got).all(), f"instance {i} (n={n}) has non-finite entries"
        err = om.rel_fro_error(got, om.rows_reference(A, B, rows))
        worst = max(worst, err)
        assert err < tol, f"instance {i} n={n} depth {depths[i]}: rel err {err:.3e}"
    print(f"config4 {name}: worst sampled rel err {worst:.3e}", flush=True)


def sampled_block_operands(n, i, seed0, npdt, k=48):
    """Rows `rows` of A and columns `cols` of B of instance i (the same
    counter-generated values the device fills), drawn without the rest of
    either matrix."""
    g = np.random.default_rng(10_000 + i)
    rows = np.sort(g.choice(n, size=min(n, k), replace=False))
    cols = np.sort(g.choice(n, size=min(n, k), replace=False))
    j = np.arange(n, dtype=np.uint64)
    a_idx = rows.astype(np.uint64)[:, None] * np.uint64(n) + j[None, :]
    b_idx = j[:, None] * np.uint64(n) + cols.astype(np.uint64)[None, :]
    A_rows = mi.counter_uniform_at(a_idx, 2 * (seed0 + i), npdt).astype(np.float64)
    B_cols = mi.counter_uniform_at(b_idx, 2 * (seed0 + i) + 1, npdt).astype(np.float64)
    return rows, cols, A_rows, B_cols


@pytest.mark.parametrize("name,form", [("f64", "phases"), ("f32", "phases"), ("f64", "persistent")])
def test_config4_all_512_instances_sampled_blocks(name, form):
    """All 512 instances of the batched workload, plans cycling through every
    eligible algorithm: a 48 x 48 block of every C (random rows and columns)
    against the oracle product of the same rows of A and columns of B."""
    code, tdt, npdt, tol = {"f64": (mf.MF_F64, torch.float64, np.float64, 1e-11),
                            "f32": (mf.MF_F32, torch.float32, np.float32, 2e-5)}[name]
    sizes = mi.batch_sizes(512, 30)
    if form == "phases":
        plans = cycled_plans()
        kw = {}
    else:  # the combinations the persistent kernel takes
        wino = mf.mf_algo_builtin("winograd")
        plans = [(None, 0), (mf.mf_algo_builtin("strassen"), 1), (wino, 1), (wino, 2)]
        kw = {"form": mf.MF_BATCH_PERSISTENT}
    algos = [plans[i % len(plans)][0] for i in range(len(sizes))]
    depths = [plans[i % len(plans)][1] for i in range(len(sizes))]
    print(f"config4 all 512 {name} {form}", flush=True)
    b = mf.mf_batch_create(sizes, algos, depths, [0] * len(sizes), code, **kw)
    dA, dB, dC = [], [], []
    for i, n in enumerate(sizes):
        A = torch.empty(n, n, dtype=tdt, device="cuda:0")
        B = torch.empty(n, n, dtype=tdt, device="cuda:0")
        mf.mf_fill_uniform(A, 2 * (31 + i))
        mf.mf_fill_uniform(B, 2 * (31 + i) + 1)
        dA.append(A)
        dB.append(B)
        dC.append(torch.full_like(A, float("nan")))
    mf.mf_batch_run(b, dA, dB, dC)
    torch.cuda.synchronize()
    assert not b.aborted()
    worst = 0.0
    for i, n in enumerate(sizes):
        rows, cols, A_rows, B_cols = sampled_block_operands(n, i, 31, npdt)
        blk = dC[i][torch.from_numpy(rows).cuda()][:, torch.from_numpy(cols).cuda()]
        got = blk.cpu().numpy().astype(np.float64)
        assert np.isfinite(got).all(), f"instance {i} (n={n}) has non-finite entries"
        err = om.rel_fro_error(got, om.rows_reference(A_rows, B_cols, np.arange(len(rows))))
        worst = max(worst, err)
        assert err < tol, f"instance {i} n={n} depth {depths[i]}: rel err {err:.3e}"
    print(f"config4 all 512 {name} {form}: worst sampled rel err {worst:.3e}", flush=True)


def test_config4_fp64_integer_exact():
    """Integer-valued FP64 operands: every instance equals the exact product."""
    sizes = config4_sizes()
    plans = cycled_plans()
    algos = [plans[(i + 2) % len(plans)][0] for i in range(len(sizes))]
    depths = [plans[(i + 2) % len(plans)][1] for i in range(len(sizes))]
    b = mf.mf_batch_create(sizes, algos, depths, [0] * len(sizes), mf.MF_F64)
    As = [mi.int_uniform(n, 3000 + i) for i, n in enumerate(sizes)]
    Bs = [mi.int_uniform(n, 4000 + i) for i, n in enumerate(sizes)]
    dA = [torch.from_numpy(a.astype(np.float64)).cuda() for a in As]
    dB = [torch.from_numpy(x.astype(np.float64)).cuda() for x in Bs]
    dC = [torch.full_like(a, float("nan")) for a in dA]
    mf.mf_batch_run(b, dA, dB, dC)
    torch.cuda.synchronize()
    for i, (A, B) in enumerate(zip(As, Bs)):
        assert_exact(dC[i], A, B, i)


def test_tuner_with_strassen_and_444_candidates_drives_exact_batch():
    """The tuner measures the paper's Strassen, Strassen-Winograd and
    <4,4,4;49> at every depth a size admits; the batch it picks is exact."""
    stras = mf.mf_algo_builtin("strassen")
    wino = mf.mf_algo_builtin("winograd")
    c444 = mf.mf_algo_compose(wino, wino)
    sizes = [128, 640, 1024, 2048]
    choices, ms = mf.mf_autotune_batch(sizes, mf.MF_F64, [stras, wino, c444], 2, work_flops=4e10,
                                       max_copies=64, reps=1)
    # candidates: classical, strassen d1 d2, winograd d1 d2, <4,4,4;49> d1 d2
    assert all(len(row) == 7 for row in ms)
    assert ms[0][1:] == [-1] * 6  # 128: no level is taken
    for row in ms[2:]:  # 1024 and 2048: every algorithm runs at depth 1
        assert row[0] > 0 and row[1] > 0 and row[3] > 0 and row[5] > 0
    pick = dict(zip(sizes, choices))
    run_sizes = [2048, 128, 1024, 640, 2048]
    b = mf.mf_batch_create(run_sizes, [pick[n][0] for n in run_sizes], [pick[n][1] for n in run_sizes],
                           [0] * len(run_sizes), mf.MF_F64)
    As = [mi.int_uniform(n, 5000 + i) for i, n in enumerate(run_sizes)]
    Bs = [mi.int_uniform(n, 6000 + i) for i, n in enumerate(run_sizes)]
    dA = [torch.from_numpy(a.astype(np.float64)).cuda() for a in As]
    dB = [torch.from_numpy(x.astype(np.float64)).cuda() for x in Bs]
    dC = [torch.full_like(a, float("nan")) for a in dA]
    mf.mf_batch_run(b, dA, dB, dC)
    torch.cuda.synchronize()
    for i, (A, B) in enumerate(zip(As, Bs)):
        assert_exact(dC[i], A, B, i)


def test_batch_runs_on_two_streams_in_a_row():
    """One batch plan run back to back on two streams with different operands:
    the second run's instance table must not reach the device before the first
    run's kernels have read theirs."""
    wino = mf.mf_algo_builtin("winograd")
    sizes = [1024, 512, 768]
    b = mf.mf_batch_create(sizes, [wino] * 3, [2, 1, 1], [0] * 3, mf.MF_F64)
    ops = []
    for r in range(2):
        As = [mi.int_uniform(n, 7000 + 10 * r + i) for i, n in enumerate(sizes)]
        Bs = [mi.int_uniform(n, 7500 + 10 * r + i) for i, n in enumerate(sizes)]
        dA = [torch.from_numpy(a.astype(np.float64)).cuda() for a in As]
        dB = [torch.from_numpy(x.astype(np.float64)).cuda() for x in Bs]
        dC = [torch.full_like(a, float("nan")) for a in dA]
        ops.append((As, Bs, dA, dB, dC))
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    mf.mf_batch_run(b, *ops[0][2:], stream=s1)
    mf.mf_batch_run(b, *ops[1][2:], stream=s2)
    torch.cuda.synchronize()
    for As, Bs, _, _, dC in ops:
        for A, B, C in zip(As, Bs, dC):
            assert np.array_equal(C.cpu().numpy(), om.classical_mm(A, B).astype(np.float64))


def test_config4_persistent_form_equals_phase_form():
    """The same 64-instance batch in one persistent launch (plans cycling
    through classical, Strassen d1 and Winograd d1/d2: the combinations the
    persistent kernel takes) gives bitwise the phase form's results, and
    integer inputs give the exact product."""
    sizes = config4_sizes()
    wino = mf.mf_algo_builtin("winograd")
    stras = mf.mf_algo_builtin("strassen")
    plans = [(None, 0), (stras, 1), (wino, 1), (wino, 2)]
    algos = [plans[i % len(plans)][0] for i in range(len(sizes))]
    depths = [plans[i % len(plans)][1] for i in range(len(sizes))]
    cut = [0] * len(sizes)
    for code, tdt in ((mf.MF_F64, torch.float64), (mf.MF_F32, torch.float32)):
        print(f"config4 persistent, dtype code {code}", flush=True)
        pers = mf.mf_batch_create(sizes, algos, depths, cut, code, form=mf.MF_BATCH_PERSISTENT)
        phase = mf.mf_batch_create(sizes, algos, depths, cut, code)
        As = [mi.int_uniform(n, 8000 + i) for i, n in enumerate(sizes)]
        Bs = [mi.int_uniform(n, 8500 + i) for i, n in enumerate(sizes)]
        dA = [torch.from_numpy(a.astype(np.float64)).to("cuda:0", tdt) for a in As]
        dB = [torch.from_numpy(x.astype(np.float64)).to("cuda:0", tdt) for x in Bs]
        got = [torch.full_like(a, float("nan")) for a in dA]
        want = [torch.full_like(a, float("nan")) for a in dA]
        mf.mf_batch_run(pers, dA, dB, got)
        mf.mf_batch_run(phase, dA, dB, want)
        torch.cuda.synchronize()
        assert not pers.aborted()
        for i, (A, B) in enumerate(zip(As, Bs)):
            assert torch.equal(got[i], want[i]), f"instance {i}"
            assert_exact(got[i].double(), A, B, i)
