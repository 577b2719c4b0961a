"""Host-side checks of the batched form's task graph.

The library exports the task list (type, instance, wait counter, wait value,
done counter) in launch order.  These tests check, on the CPU, that the order
is topological with exact counts, and replay the device protocol - workers
take tickets in order, wait until a counter reaches its value, then increment
their own counter - under random interleavings and worker counts: every run
must finish (no deadlock) and every task must start after its dependencies.
A planted mistake (a wait value one too high) must be detected."""
import numpy as np
import pytest

import mf_inputs as mi

mf = pytest.importorskip("paper_2312_12732_amd.mf", reason="libmf.so not built")


def make_batch(seed=30, count=24, dtype=None):
    sizes = mi.batch_sizes(count, seed)
    algos, depths = [], []
    s = mf.mf_algo_builtin("winograd")
    s2 = mf.mf_algo_compose(s, s)
    for i, n in enumerate(sizes):
        kind = i % 4
        if kind == 0:
            algos.append(None)
            depths.append(0)
        elif kind == 1:
            algos.append(s)
            depths.append(1)
        elif kind == 2:
            algos.append(s)
            depths.append(2)
        else:
            algos.append(s2)
            depths.append(1)
    return mf.mf_batch_create(sizes, algos, depths, [0] * count, dtype or mf.MF_F64), sizes


def check_topological(desc, nctr):
    produced = np.zeros(nctr, dtype=np.int64)
    for t, (typ, inst, wc, wv, dc) in enumerate(desc):
        assert typ in (0, 1)
        assert 0 <= dc < nctr
        if wc >= 0:
            # every task it waits for comes earlier, and exactly wv of them exist overall
            assert produced[wc] == wv, (t, wc, produced[wc], wv)
        produced[dc] += 1
    return produced


def replay(desc, nctr, workers, rng):
    """Simulate workers taking tickets in order; returns completion order or
    raises on deadlock."""
    ctr = np.zeros(nctr, dtype=np.int64)
    ntasks = len(desc)
    ticket = 0
    running = []  # (task, started)
    done_order = []
    started_at = {}
    steps = 0
    while len(done_order) < ntasks:
        steps += 1
        assert steps < 100 * ntasks + 1000, "no progress: deadlock"
        # idle workers take tickets
        while len(running) < workers and ticket < ntasks:
            running.append([ticket, False])
            ticket += 1
        progressed = False
        order = rng.permutation(len(running))
        for k in order:
            t, started = running[k]
            typ, inst, wc, wv, dc = desc[t]
            if not started:
                if wc < 0 or ctr[wc] >= wv:
                    running[k][1] = True
                    started_at[t] = len(done_order)
                    progressed = True
            elif rng.random() < 0.5:
                ctr[dc] += 1
                done_order.append(t)
                running[k] = None
                progressed = True
        running = [r for r in running if r is not None]
        if not progressed and all(r[1] is False for r in running) and running:
            # every running worker is blocked: only possible on a deadlock
            blocked = [(r[0], desc[r[0]][2], ctr[desc[r[0]][2]], desc[r[0]][3]) for r in running]
            raise AssertionError(f"deadlock: {blocked[:4]}")
    return done_order


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_task_graph_is_topological(dtype):
    b, sizes = make_batch(dtype=mf.MF_F64 if dtype == "f64" else mf.MF_F32)
    ntasks, nctr, desc = b.tasks()
    assert ntasks == len(desc) > 0
    produced = check_topological(desc, nctr)
    # every instance has GEMM tasks and counters are all used
    assert set(desc[desc[:, 0] == 1][:, 1]) == set(range(len(sizes)))
    assert (produced > 0).all()


@pytest.mark.parametrize("workers", [1, 2, 7, 64])
@pytest.mark.parametrize("seed", [0, 1])
def test_replay_no_deadlock_and_order(workers, seed):
    b, _ = make_batch(seed=30 + seed, count=12)
    ntasks, nctr, desc = b.tasks()
    rng = np.random.default_rng(seed)
    order = replay(desc, nctr, workers, rng)
    assert sorted(order) == list(range(ntasks))


def test_planted_wrong_wait_value_is_caught():
    b, _ = make_batch(count=8)
    ntasks, nctr, desc = b.tasks()
    bad = desc.copy()
    k = int(np.flatnonzero(bad[:, 2] >= 0)[0])
    bad[k, 3] += 1
    with pytest.raises(AssertionError):
        check_topological(bad, nctr)
    with pytest.raises(AssertionError):
        replay(bad, nctr, 4, np.random.default_rng(0))


def test_batch_workspace_and_validation():
    b, sizes = make_batch(count=8)
    assert b.workspace_bytes() > 0
    with pytest.raises(mf.MFError):
        mf.mf_batch_create([128, 0], [None, None], [0, 0], [0, 0])
    with pytest.raises(mf.MFError):
        mf.mf_batch_create([256], [None], [1], [0])  # depth > 0 without an algorithm
    with pytest.raises(mf.MFError) as e:
        mf.mf_batch_create([256], [None], [0], [0], mf.MF_F32 | mf.MF_LEAF_BF16)
    assert e.value.status == mf.MF_ERR_UNSUPPORTED


def check_phases(desc, phases):
    """The phases partition the task list, each holds one task type, and every
    task's input stage is produced entirely by earlier phases (launch order
    on the stream is then enough: no waits inside a launch)."""
    assert len(phases) >= 1 and phases[0][0] == 0 and phases[-1][1] == len(desc)
    phase_of = np.empty(len(desc), dtype=np.int64)
    for p, (beg, end, gemm) in enumerate(phases):
        assert beg < end
        if p:
            assert beg == phases[p - 1][1]
        assert set(desc[beg:end, 0].tolist()) == {1 if gemm else 0}
        phase_of[beg:end] = p
    last_phase_of_ctr = {}
    for t, (typ, inst, wc, wv, dc) in enumerate(desc):
        last_phase_of_ctr[dc] = max(last_phase_of_ctr.get(dc, -1), phase_of[t])
    for t, (typ, inst, wc, wv, dc) in enumerate(desc):
        if wc >= 0:
            assert last_phase_of_ctr[wc] < phase_of[t], (t, wc)
    return phase_of


@pytest.mark.parametrize("seed", [30, 31, 32])
def test_phases_order_dependencies(seed):
    b, sizes = make_batch(seed=seed, count=24)
    nt, nctr, desc = b.tasks()
    phases = b.phases()
    check_phases(desc, phases)
    # exactly one GEMM phase, after every pre-addition phase and before every post-addition phase
    gemm = [p for p, ph in enumerate(phases) if ph[2] == 1]
    assert len(gemm) == 1


def test_phase_check_catches_a_misplaced_task():
    b, _ = make_batch(seed=33, count=12)
    nt, nctr, desc = b.tasks()
    phases = b.phases().copy()
    # plant: move the GEMM phase boundary one task earlier, so a pre-addition task is
    # taken as GEMM work (type mismatch) -- the check must reject it
    g = int(np.flatnonzero(phases[:, 2] == 1)[0])
    if g > 0:
        phases[g - 1, 1] -= 1
        phases[g, 0] -= 1
        with pytest.raises(AssertionError):
            check_phases(desc, phases)
    # plant: the last addition task (a post-addition chunk) waits on its own stage
    # counter, which tasks of its own phase produce -- the check must reject it
    bad = desc.copy()
    post = int(np.flatnonzero(bad[:, 0] == 0)[-1])
    bad[post, 2] = bad[post, 4]
    with pytest.raises(AssertionError):
        check_phases(bad, b.phases())


def test_classical_only_batch_is_one_gemm_phase():
    b = mf.mf_batch_create([256, 640, 1024], [None] * 3, [0] * 3, [0] * 3, mf.MF_F64)
    phases = b.phases()
    assert phases.tolist() == [[0, 4 + 25 + 64, 1]]
