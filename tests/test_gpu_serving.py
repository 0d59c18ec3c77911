"""Serving: continuous batching through za_server_* (GPU).

A served request must give the same state, bit for bit, as the single
context path and as the same request served alone; admission must respect
the HBM budget; a failing request must not disturb the others."""
import numpy as np
import pytest

import oracle as orc
from paper_2603_26272_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_2603_26272_amd import za
    za.lib()
    return torch.device("cuda:0")


def ctx_solve(P, q0, steps, dev):
    from paper_2603_26272_amd.za import Context
    q = torch.from_numpy(np.ascontiguousarray(q0)).to(dev)
    with Context(P) as ctx:
        ctx.solve(q, 0.0, steps)
    torch.cuda.synchronize()
    return q.cpu().numpy()


def serve(reqs, budget=1 << 30, slots=64):
    """reqs: list of (P, q0, steps) -> list of (status, q)."""
    from paper_2603_26272_amd.za import Server
    out = [None] * len(reqs)
    with Server(budget, slots) as sv:
        ids = [sv.submit(P, q0, n) for P, q0, n in reqs]
        sv.drain()
        for i, (rid, (P, _, _)) in enumerate(zip(ids, reqs)):
            done, st, q, stats = sv.poll(rid, P)
            assert done
            out[i] = (st, q, stats)
    return out


def test_served_equals_single_context(dev):
    cases = [W.quadrants_2d(1, 160, 144), W.riemann_1d(2, 3000)]
    P32, q32 = W.quadrants_2d(3, 130, 70)
    cases.append((P32.fp32(), q32))
    P1, q1 = W.riemann_1d(4, 900)
    cases.append((P1.fp32(), q1))
    reqs = [(P, q0, 17) for P, q0 in cases]
    res = serve(reqs)
    for (P, q0, n), (st, q, stats) in zip(reqs, res):
        assert st == 0 and stats["steps"] == n
        ref = ctx_solve(P, q0, n, dev)
        assert np.array_equal(q, ref), (P.dim, P.precision, np.abs(q - ref).max())


@pytest.mark.parametrize("pinned_mb", ["0", "1"])
def test_pageable_staging_bitwise(dev, monkeypatch, pinned_mb):
    """Uploads and result downloads through pageable memory (no pinned
    staging pool, or one too small for most requests) give the same states
    as the pinned path."""
    reqs = [(r.problem, r.q0, min(r.steps, 40)) for r in
            W.serving_stream(200.0, n_requests=12, seed=5, max_1d=8192, max_2d=256)]
    pinned = serve(reqs, budget=2 << 30, slots=12)
    monkeypatch.setenv("ZA_SRV_PINNED_MB", pinned_mb)
    pageable = serve(reqs, budget=2 << 30, slots=12)
    for i, (a, b) in enumerate(zip(pinned, pageable)):
        assert a[0] == b[0] == 0
        assert np.array_equal(a[1], b[1]), i


def test_served_matches_oracle(dev):
    P, q0 = W.riemann_1d(7, 512)
    (st, q, _), = serve([(P, q0, 30)])
    ref, steps, t, ost = orc.solve(P, q0, 0.0, 30)
    tol = 1e-10 * (np.abs(ref) + np.abs(ref).max(axis=(1, 2), keepdims=True))
    assert st == 0 and np.all(np.abs(q - ref) <= tol)


def test_alone_versus_mix_bitwise(dev):
    reqs = [(r.problem, r.q0, min(r.steps, 60)) for r in
            W.serving_stream(200.0, n_requests=24, seed=11, max_1d=8192, max_2d=256)]
    mixed = serve(reqs, budget=2 << 30, slots=24)
    for i in range(0, 24, 3):
        alone = serve([reqs[i]])
        assert mixed[i][0] == alone[0][0] == 0
        assert np.array_equal(mixed[i][1], alone[0][1]), i


def test_admission_under_tight_budget(dev):
    from paper_2603_26272_amd import za
    reqs = [(*W.quadrants_2d(s, 256), 10) for s in range(6)]
    per = za.workspace_bytes(reqs[0][0])
    budget = int(2.5 * per)          # at most two requests resident at a time
    res = serve(reqs, budget=budget, slots=16)
    alone = serve([reqs[3]])
    assert all(r[0] == 0 for r in res)
    assert np.array_equal(res[3][1], alone[0][1])
    # admissions were staggered: some request waited for memory
    admits = sorted(r[2]["admit_ns"] - r[2]["arrival_ns"] for r in res)
    assert admits[-1] > admits[0]
    P, q0 = W.quadrants_2d(0, 1024)
    with za.Server(budget, 4) as sv:
        with pytest.raises(za.ZaError) as ei:
            sv.submit(P, q0, 5)
        assert ei.value.status == za.ZA_ERR_NOMEM


def test_failing_request_is_isolated(dev):
    from paper_2603_26272_amd.za import ZA_ERR_NONFINITE
    good = [(*W.riemann_1d(s, 1000), 25) for s in range(3)]
    Pb, qb = W.riemann_1d(9, 1000)
    qb = qb.copy()
    qb[0, 0, 500] = np.nan
    res = serve(good[:2] + [(Pb, qb, 25)] + good[2:])
    assert res[2][0] == ZA_ERR_NONFINITE and res[2][2]["steps"] == 0
    for i, j in ((0, 0), (1, 1), (3, 2)):
        assert res[i][0] == 0
        assert np.array_equal(res[i][1], serve([good[j]])[0][1])


def test_served_chunk_counts_bitwise(dev, monkeypatch):
    """FP64 requests use the looped x-sweep (segments of 64 nc - 1 cells; in
    1D it also leaves the wave speeds, one row per wavefront).
    ZA_SRV_XL_CHUNKS forces nc at admission (clamped to 1 .. 64); every
    choice gives the states of the single context path's one-shot sweep
    bitwise."""
    reqs = [(*W.riemann_1d(5, 5000), 12), (*W.quadrants_2d(6, 700, 90), 12), (*W.riemann_1d(8, 300), 12),
            (*W.quadrants_2d(9, 65, 130), 12)]
    monkeypatch.setenv("ZA_XL_CHUNKS", "0")
    ref = [ctx_solve(P, q0, n, dev) for P, q0, n in reqs]
    monkeypatch.delenv("ZA_XL_CHUNKS")
    for nc in (0, 1, 3, 7):
        monkeypatch.setenv("ZA_SRV_XL_CHUNKS", str(nc))
        res = serve(reqs)
        for i, (st, q, stats) in enumerate(res):
            assert st == 0 and stats["steps"] == 12, (nc, i, st)
            assert np.array_equal(q, ref[i]), (nc, i)
    monkeypatch.delenv("ZA_SRV_XL_CHUNKS")


def test_requests_finish_mid_burst_bitwise(dev):
    """Requests with very different step counts share bursts of up to eight
    RK3 steps; each stops on the device at its own count (and later bursts
    skip it), so every result equals the single context's run of exactly
    that many steps."""
    steps = (1, 2, 3, 9, 17, 40)
    cases = [W.riemann_1d(20 + i, 700 + 50 * i) for i in range(3)] + \
            [W.quadrants_2d(30 + i, 96 + 8 * i, 80) for i in range(3)]
    reqs = [(P, q0, n) for (P, q0), n in zip(cases, steps)]
    res = serve(reqs)
    for (P, q0, n), (st, q, stats) in zip(reqs, res):
        assert st == 0 and stats["steps"] == n, (n, st, stats["steps"])
        assert np.array_equal(q, ctx_solve(P, q0, n, dev)), n


def test_injected_launch_failure_ends_requests_without_hang(dev, monkeypatch):
    """A launch failure (injected on the host: ZA_SRV_FAIL_BURST=1 makes the
    first burst report a launch error, no kernel is touched) ends every
    request of the failing class with ZA_ERR_DEVICE and releases it, so
    drain returns instead of waiting forever; requests admitted afterwards
    run normally, and a new server is unaffected."""
    from paper_2603_26272_amd import za
    monkeypatch.setenv("ZA_SRV_FAIL_BURST", "1")
    reqs = [(*W.riemann_1d(40 + s, 800), 12) for s in range(4)]
    statuses = []
    with za.Server(1 << 30, 16) as sv:
        monkeypatch.delenv("ZA_SRV_FAIL_BURST")
        ids = [sv.submit(P, q0, n) for P, q0, n in reqs]
        with pytest.raises(za.ZaError) as ei:
            sv.drain()
        assert ei.value.status == za.ZA_ERR_DEVICE
        for rid, (P, q0, n) in zip(ids, reqs):
            done, st, q, stats = sv.poll(rid, P)
            assert done
            statuses.append(st)
            if st == 0:
                assert np.array_equal(q, ctx_solve(P, q0, n, dev))
    assert za.ZA_ERR_DEVICE in statuses
    assert all(s in (0, za.ZA_ERR_DEVICE) for s in statuses)
    res = serve(reqs[:2])
    assert all(r[0] == 0 for r in res)


@pytest.mark.parametrize("which", ["upload", "download"])
def test_injected_transfer_failure_ends_one_request(dev, monkeypatch, which):
    """A failed copy (injected on the host: ZA_SRV_FAIL_XFER=k makes the
    transfer thread's k-th copy report an error without copying) ends that
    one request with ZA_ERR_DEVICE; the others finish normally, drain returns
    (reporting the error) and a new server is unaffected.  Requests are
    submitted one by one after the previous finished, so copy 1 is the first
    upload and copy 4 the second download."""
    from paper_2603_26272_amd import za
    monkeypatch.setenv("ZA_SRV_FAIL_XFER", "1" if which == "upload" else "4")
    reqs = [(*W.riemann_1d(60 + s, 700), 9) for s in range(3)]
    statuses = []
    with za.Server(1 << 30, 8) as sv:
        monkeypatch.delenv("ZA_SRV_FAIL_XFER")
        ids = []
        for P, q0, n in reqs:
            ids.append(sv.submit(P, q0, n))
            try:
                sv.drain()
            except za.ZaError as e:
                assert e.status == za.ZA_ERR_DEVICE
        for rid, (P, q0, n) in zip(ids, reqs):
            done, st, q, stats = sv.poll(rid, P)
            assert done
            statuses.append(st)
            if st == 0:
                assert np.array_equal(q, ctx_solve(P, q0, n, dev))
    bad = 0 if which == "upload" else 1
    assert statuses[bad] == za.ZA_ERR_DEVICE
    assert all(s == 0 for i, s in enumerate(statuses) if i != bad), statuses
    res = serve(reqs[:2])
    assert all(r[0] == 0 for r in res)

