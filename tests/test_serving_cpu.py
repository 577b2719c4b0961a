"""CPU checks of the serving runtime's admission controller (through the
library's host-only simulation) and of the counter-based operand generator's
host implementation."""
import numpy as np
import pytest

import mf_inputs as mi

mf = pytest.importorskip("paper_2312_12732_amd.mf", reason="libmf.so not built")


def random_load(seed, count=300):
    g = np.random.default_rng(seed)
    t = np.cumsum(g.exponential(1.0, count))
    service = g.uniform(0.5, 6.0, count)
    need = g.integers(1, 40, count) * (1 << 20)
    return t, service, need


def concurrency(t_admit, t_done):
    ev = sorted([(a, 1) for a in t_admit] + [(d, -1) for d in t_done], key=lambda x: (x[0], x[1]))
    cur = peak = 0
    for _, k in ev:
        cur += k
        peak = max(peak, cur)
    return peak


def budget_peak(t_admit, t_done, need):
    ev = sorted([(a, n) for a, n in zip(t_admit, need)] + [(d, -n) for d, n in zip(t_done, need)],
                key=lambda x: (x[0], x[1]))
    cur = peak = 0
    for _, k in ev:
        cur += k
        peak = max(peak, cur)
    return peak


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("slots,budget_mb", [(1, 64), (4, 64), (8, 100), (16, 1000)])
def test_fifo_admission_respects_budget_and_slots(seed, slots, budget_mb):
    t, service, need = random_load(seed)
    budget = budget_mb << 20
    ta, td, peak = mf.mf_admission_simulate(t, service, need, slots, budget)
    assert peak <= budget
    assert budget_peak(ta, td, need) <= budget
    assert concurrency(ta, td) <= slots
    assert (ta >= t).all()
    assert np.allclose(td, ta + service)
    assert (np.diff(ta) >= 0).all()  # strict FIFO: admission order = arrival order


def test_overtaking_mode():
    t, service, need = random_load(5)
    ta, td, peak = mf.mf_admission_simulate(t, service, need, 4, 64 << 20, allow_overtake=True)
    assert peak <= 64 << 20 and concurrency(ta, td) <= 4 and (ta >= t).all()
    fifo_wait = np.mean(mf.mf_admission_simulate(t, service, need, 4, 64 << 20)[0] - t)
    assert np.mean(ta - t) <= fifo_wait + 1e-9


def test_single_slot_is_serial():
    t, service, need = random_load(3, 50)
    ta, td, _ = mf.mf_admission_simulate(t, service, need, 1, 1 << 40)
    assert (ta[1:] >= td[:-1] - 1e-12).all()


def test_request_larger_than_budget_rejected():
    with pytest.raises(mf.MFError) as e:
        mf.mf_admission_simulate([0.0], [1.0], [100], 1, 99)
    assert e.value.status == mf.MF_ERR_NOMEM


def splitmix_reference(seed, i):
    """SplitMix64 output for counter state seed + (i + 1) * gamma, with explicit
    64-bit masking (a second, scalar implementation)."""
    M = (1 << 64) - 1
    z = (seed + (i + 1) * 0x9E3779B97F4A7C15) & M
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
    return z ^ (z >> 31)


def test_counter_generator_matches_published_splitmix():
    # First two outputs of SplitMix64 started from state 0 (published test values).
    assert splitmix_reference(0, 0) == 0xE220A8397B1DCDAF
    assert splitmix_reference(0, 1) == 0x6E789E6AA1B965F4
    v = mi.counter_uniform(1000, 12345)
    for i in (0, 1, 2, 500, 999):
        u = (splitmix_reference(12345, i) >> 11) * 2.0 ** -53
        assert v[i] == 2.0 * u - 1.0
    assert v.min() >= -1.0 and v.max() < 1.0
    f = mi.counter_uniform(1000, 12345, np.float32)
    assert np.array_equal(f, v.astype(np.float32))


def test_counter_generator_at_chosen_positions():
    """counter_uniform_at draws any subset of the stream: equal to the scalar
    SplitMix64 reference at large, unordered and repeated positions, and to
    the full stream's slice."""
    idx = np.array([5_000_000_123, 7, 0, 7, 2**33 + 1], dtype=np.uint64)
    v = mi.counter_uniform_at(idx, 99)
    for k, i in enumerate(idx.tolist()):
        assert v[k] == 2.0 * ((splitmix_reference(99, i) >> 11) * 2.0 ** -53) - 1.0
    full = mi.counter_uniform(3000, 4242, np.float32)
    rows = np.array([[2999, 0], [17, 1500]], dtype=np.uint64)
    got = mi.counter_uniform_at(rows, 4242, np.float32)
    assert got.shape == (2, 2) and got.dtype == np.float32
    assert np.array_equal(got, full[rows.astype(np.int64)])


def test_arena_fragmentation_blocks_fifo_head_until_space_coalesces():
    # budget 3 MiB: A (offset 0), B (1 MiB) and C (2 MiB) fill it.  When B ends at t=1
    # only its 1 MiB hole is free, so the 2 MiB request D waits; when A ends at t=5
    # its block coalesces with B's hole into 2 MiB at offset 0 and D is admitted
    mib = 1 << 20
    t = [0.0, 0.0, 0.0, 0.1]
    service = [5.0, 1.0, 9.0, 1.0]
    need = [mib, mib, mib, 2 * mib]
    ta, td, peak = mf.mf_admission_simulate(t, service, need, 4, 3 * mib)
    assert ta[:3].tolist() == [0.0, 0.0, 0.0]
    assert ta[3] == 5.0  # A's block (offset 0) and B's (offset 1 MiB) coalesce into 2 MiB
    assert peak == 3 * mib


def test_arena_first_fit_needs_contiguous_space():
    # budget 4 MiB: A(1) B(1) C(1) D(1) fill it; B and D end, leaving two 1 MiB holes
    # (2 MiB free, not contiguous); a 2 MiB request waits until C ends
    mib = 1 << 20
    t = [0.0, 0.0, 0.0, 0.0, 0.5]
    service = [10.0, 1.0, 3.0, 1.0, 1.0]
    need = [mib, mib, mib, mib, 2 * mib]
    ta, td, _ = mf.mf_admission_simulate(t, service, need, 8, 4 * mib)
    assert ta[4] == 3.0
