"""GPU checks of the serving runtime: requests of mixed sizes and dtypes
served concurrently give the same results as each request served alone
(bitwise: the plan is a pure function of (n, dtype) and the kernels are
deterministic), match the CPU oracle on independently generated operands,
and overlap on the device."""
import numpy as np
import pytest

import mf_inputs as mi
from oracle import matmul as om

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
mf = pytest.importorskip("paper_2312_12732_amd.mf", reason="libmf.so not built")

REQS = [(300, "f32", 1), (1000, "f64", 2), (128, "f32", 3), (2048, "f32", 4), (700, "f64", 5), (1536, "f64", 6),
        (256, "f32", 7), (1200, "f32", 8), (2500, "f64", 9), (64, "f64", 10)]
POLICY = dict(depth_min_n_f64=(512, 1500, 0, 0), depth_min_n_f32=(1024, 2000, 0, 0))


def code(dt):
    return mf.MF_F64 if dt == "f64" else mf.MF_F32


def tdtype(dt):
    return torch.float64 if dt == "f64" else torch.float32


def serve(reqs, slots):
    # pinned outputs first, so that the requests are submitted back to back
    outs = [torch.empty(n, n, dtype=tdtype(dt)).pin_memory() for n, dt, _ in reqs]
    srv = mf.Server(slots, 16 << 30, mf.mf_algo_builtin("winograd"), **POLICY)
    for (n, dt, seed), out in zip(reqs, outs):
        srv.submit(n, code(dt), seed, out)
    srv.drain()
    st = srv.stats()
    srv.close()
    return [o.numpy().astype(np.float64) for o in outs], st


def test_generator_matches_host():
    for dt, npdt in (("f64", np.float64), ("f32", np.float32)):
        t = torch.empty(12345, dtype=tdtype(dt), device="cuda:0")
        mf.mf_fill_uniform(t, 777)
        torch.cuda.synchronize()
        assert np.array_equal(t.cpu().numpy(), mi.counter_uniform(12345, 777, npdt))


def test_mix_equals_alone_and_oracle():
    mixed, st = serve(REQS, slots=4)
    for k, (n, dt, seed) in enumerate(REQS):
        alone, _ = serve([(n, dt, seed)], slots=1)
        assert np.array_equal(mixed[k], alone[0]), (n, dt)
        npdt = np.float64 if dt == "f64" else np.float32
        A = mi.counter_uniform(n * n, 2 * seed, npdt).astype(np.float64).reshape(n, n)
        B = mi.counter_uniform(n * n, 2 * seed + 1, npdt).astype(np.float64).reshape(n, n)
        err = om.rel_fro_error(mixed[k], om.classical_mm(A, B))
        assert err < (1e-11 if dt == "f64" else 2e-5), (n, dt, err)
    assert (st["t_admit"] >= st["t_arrive"]).all() and (st["t_done"] >= st["t_admit"]).all()
    assert set(st["depth"].tolist()) >= {0, 1, 2}


def block_operands(n, seed, npdt, k=48, pick=0):
    """Rows of A and columns of B of a request (its counter-generated
    operands: A from 2 seed, B from 2 seed + 1), drawn without the rest."""
    g = np.random.default_rng(20_000 + pick)
    rows = np.sort(g.choice(n, size=min(n, k), replace=False))
    cols = np.sort(g.choice(n, size=min(n, k), replace=False))
    j = np.arange(n, dtype=np.uint64)
    A_rows = mi.counter_uniform_at(rows.astype(np.uint64)[:, None] * np.uint64(n) + j[None, :], 2 * seed, npdt)
    B_cols = mi.counter_uniform_at(j[:, None] * np.uint64(n) + cols.astype(np.uint64)[None, :], 2 * seed + 1, npdt)
    return rows, cols, A_rows.astype(np.float64), B_cols.astype(np.float64)


def test_serving_workload_draw_mix_alone_and_oracle():
    """300 requests of the serving workload's own draw (n log-uniform in
    [256, 8192], 70% FP32, seed 40) with its depth policy, served 8 at a time:
    every request with n <= 2048 and a 5% sample of the larger ones equal,
    bit for bit, the same request served alone, and a 48 x 48 block of each
    (random rows and columns) matches the oracle."""
    reqs = mi.serving_requests(300, 40)
    policy = dict(depth_min_n_f64=(2048, 4096, 0, 0), depth_min_n_f32=(2048, 4096, 0, 0))
    g = np.random.default_rng(41)
    check = [k for k, (n, _) in enumerate(reqs) if n <= 2048 or g.random() < 0.05]
    assert len(check) > 150 and any(reqs[k][0] > 2048 for k in check)
    seed = [3000 + k for k in range(len(reqs))]
    outs = {k: torch.empty(reqs[k][0], reqs[k][0], dtype=tdtype(reqs[k][1])).pin_memory() for k in check}
    print(f"serving draw: {len(reqs)} requests, {len(check)} checked", flush=True)
    srv = mf.Server(8, 64 << 30, mf.mf_algo_builtin("winograd"), **policy)
    for k, (n, dt) in enumerate(reqs):
        srv.submit(n, code(dt), seed[k], outs.get(k))
    srv.drain()
    depth = srv.stats()["depth"]
    srv.close()
    assert set(depth.tolist()) >= {0, 1, 2}
    alone = mf.Server(1, 64 << 30, mf.mf_algo_builtin("winograd"), **policy)
    worst = {"f64": 0.0, "f32": 0.0}
    for k in check:
        n, dt = reqs[k]
        out = torch.empty(n, n, dtype=tdtype(dt)).pin_memory()
        alone.submit(n, code(dt), seed[k], out)
        alone.drain()
        assert torch.equal(out, outs[k]), (k, n, dt)
        npdt = np.float64 if dt == "f64" else np.float32
        rows, cols, A_rows, B_cols = block_operands(n, seed[k], npdt, pick=k)
        got = outs[k].numpy()[np.ix_(rows, cols)].astype(np.float64)
        err = om.rel_fro_error(got, om.rows_reference(A_rows, B_cols, np.arange(len(rows))))
        worst[dt] = max(worst[dt], err)
        assert err < (1e-11 if dt == "f64" else 2e-5), (k, n, dt, err)
    alone.close()
    print(f"serving draw: worst sampled rel err {worst}", flush=True)


def test_requests_overlap_on_the_device():
    """Requests on different slots run at the same time on the device: on the
    device's own timeline (events recorded on each slot's stream, measured
    from one origin event) two requests' intervals intersect."""
    reqs = [(2048, "f64", 21), (2048, "f64", 22), (1536, "f32", 23), (2048, "f32", 24)]
    _, st = serve(reqs, slots=4)
    d0, d1 = st["device_start_ms"], st["device_end_ms"]
    assert (d0 >= 0).all() and (d1 > d0).all(), (d0, d1)
    overlap = [(a, b) for a in range(len(reqs)) for b in range(a + 1, len(reqs)) if d0[a] < d1[b] and d0[b] < d1[a]]
    print(f"device intervals (ms): {list(zip(d0.round(3), d1.round(3)))}; overlapping pairs {overlap}", flush=True)
    assert overlap, (d0, d1)
    # with one slot the same requests run one after another
    _, st1 = serve(reqs, slots=1)
    e0, e1 = st1["device_start_ms"], st1["device_end_ms"]
    order = np.argsort(e0)
    assert (e0[order][1:] >= e1[order][:-1] - 1e-3).all(), (e0, e1)


def test_caller_operands_equal_standalone_product():
    """Requests on caller-owned device operands give bitwise the result of
    the standalone product with the same plan (depth from the server's policy)."""
    wino = mf.mf_algo_builtin("winograd")
    srv = mf.Server(4, 8 << 30, wino, **POLICY)
    cases = [(1600, torch.float64, 2), (2100, torch.float32, 2), (1000, torch.float64, 1), (300, torch.float64, 0)]
    ops = []
    for k, (n, tdt, depth) in enumerate(cases):
        A = torch.from_numpy(mi.uniform(n, 500 + k)).to("cuda:0", tdt)
        B = torch.from_numpy(mi.uniform(n, 600 + k)).to("cuda:0", tdt)
        C = torch.full_like(A, float("nan"))
        ops.append((A, B, C, depth))
    torch.cuda.synchronize()
    for A, B, C, _ in ops:
        srv.submit_operands(A, B, C)
    srv.drain()
    st = srv.stats()
    srv.close()
    for (A, B, C, depth), d in zip(ops, st["depth"]):
        assert d == depth
        ref = torch.empty_like(A)
        mf.mf_fastmm(wino, depth, 0, A, B, ref)
        torch.cuda.synchronize()
        assert torch.equal(C, ref)


def test_budget_limits_concurrency():
    # a budget that fits one 2048 fp64 request at a time serialises them
    srv = mf.Server(4, 1, None)
    need = srv.need_bytes(2048, mf.MF_F64)
    srv.close()
    srv = mf.Server(4, need, None)
    for s in range(3):
        srv.submit(2048, mf.MF_F64, 100 + s)
    srv.drain()
    st = srv.stats()
    srv.close()
    order = np.argsort(st["t_admit"])
    ta, td = st["t_admit"][order], st["t_done"][order]
    assert (ta[1:] >= td[:-1]).all()
    with pytest.raises(mf.MFError) as e:
        srv2 = mf.Server(2, need - 1, None)
        try:
            srv2.submit(2048, mf.MF_F64, 1)
        finally:
            srv2.close()
    assert e.value.status == mf.MF_ERR_NOMEM
