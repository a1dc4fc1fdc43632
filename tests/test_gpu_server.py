"""GPU checks of the serving entry points (phiks_server_*).

A served request is one phiks_apply; whatever else runs beside it (the other requests
of its lane, ticked together, and the other lanes), its output must be bitwise the
output of phiks_plan (tolerance relative, vnorms = NULL) + phiks_apply for that request
alone, in its precision (FP64, FP32 or BF16x3 mu-mode products)."""
import threading

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu
ph = pytest.importorskip("paper_2210_07667_amd")
TOL = 2.0 ** -53
GiB = 1 << 30


@pytest.fixture(autouse=True)
def _need_gpu():
    if ph.device_count() < 1:
        pytest.skip("no GPU")


def small_sessions():
    """Sessions of several shapes (odd sizes too), operators and phi orders."""
    S = workloads.Session
    return [
        S("fd2_24x24", [24, 24], [workloads.fd2_dirichlet(24)] * 2, 1e-3, 2),
        S("adr_40x33", [40, 33], [workloads.adr_1d(40, 0.5, 1.0, -1.0), workloads.adr_1d(33, 0.5, 0.5, -1.0)], 2e-3, 3),
        S("bruss_16^3", [16, 16, 16], [0.02 * workloads.fd2_neumann(16) - 4 / 3 * np.eye(16)] * 3, 5e-3, 1),
        S("fd2_32x24x20", [32, 24, 20], [workloads.fd2_dirichlet(m) for m in (32, 24, 20)], 1e-3, 3),
        S("cheb_50", [50], [workloads.cheb_d2_dirichlet(50)], 1e-4, 2),
        S("adr_64x64", [64, 64], [workloads.adr_1d(64, 0.5, b, -1.0) for b in (1.0, 0.5)], 1e-3, 3),
    ]


def reference(sess, v, ns=1, precision=0):
    plan = ph.phiks_plan(sess.A, sess.tau, sess.p, ns, TOL, "same_vector", precision=precision)
    out = ph.apply_arrays(plan, ph.DeviceArray.from_numpy(v))
    ph.synchronize()
    plan.close()
    return out.to_numpy()


def run_requests(server, sessions, picks, seed, ns_of=lambda k: 1, prec_of=lambda k: 0):
    rng = np.random.default_rng(seed)
    ops = {}
    reqs = []
    for k, si in enumerate(picks):
        sess = sessions[si]
        ns = ns_of(k)
        prec = prec_of(k)
        v = rng.standard_normal(sess.N)
        dv = ph.DeviceArray.from_numpy(v)
        out = ph.DeviceArray(ns * (sess.p + 1) * sess.N)
        if si not in ops:
            ops[si] = server.register(sess.A)
        t = server.submit(ops[si], sess.tau, sess.p, ns, TOL, dv.ptr, out.ptr, precision=prec)
        reqs.append((si, ns, prec, v, dv, out, t))
    lat = [server.wait(r[-1]) for r in reqs]
    return reqs, lat


def test_served_results_equal_single_calls():
    sessions = small_sessions()
    server = ph.Server(hbm_budget=4 * GiB, workspace_bytes=1 * GiB, max_active=16, lanes=2)
    rng = np.random.default_rng(0)
    picks = rng.integers(len(sessions), size=40).tolist()
    # two-scale requests (another step count) and FP32 / BF16x3 requests in the mix
    ns_of = lambda k: 2 if k % 7 == 3 else 1
    prec_of = lambda k: (ph.PHIKS_FP32 if k % 5 == 1 else ph.PHIKS_BF16X3 if k % 5 == 2 else ph.PHIKS_FP64)
    reqs, lat = run_requests(server, sessions, picks, 1, ns_of=ns_of, prec_of=prec_of)
    for si, ns, prec, v, _, out, _ in reqs:
        ref = reference(sessions[si], v, ns, prec)
        assert np.array_equal(out.to_numpy(), ref), (sessions[si].name, prec)
    st = server.stats()
    print(f"[server] stats {st}, latency p50 {np.median(lat) * 1e3:.2f} ms max {max(lat) * 1e3:.2f} ms")
    keys = {(picks[k], ns_of(k), prec_of(k)) for k in range(len(picks))}
    assert st["completed"] == len(picks)
    assert st["cache_misses"] == len(keys)
    assert st["cache_hits"] == len(picks) - len(keys)
    server.close()


def test_eviction_under_a_small_budget():
    sessions = small_sessions()
    # 1 MB left for plans beside the 60 MB arena: fewer than the five sessions need
    server = ph.Server(hbm_budget=61 << 20, workspace_bytes=60 << 20, max_active=4, lanes=1)
    picks = [0, 1, 3, 5, 0, 1, 3, 5, 2, 2]
    reqs, _ = run_requests(server, sessions, picks, 2)
    for si, ns, prec, v, _, out, _ in reqs:
        assert np.array_equal(out.to_numpy(), reference(sessions[si], v, ns)), sessions[si].name
    st = server.stats()
    print(f"[server small budget] stats {st}")
    assert st["evictions"] > 0
    server.close()


def test_submit_errors():
    server = ph.Server(hbm_budget=1 * GiB, workspace_bytes=8 << 20, max_active=4)
    sess = small_sessions()[0]
    dv = ph.DeviceArray(sess.N)
    out = ph.DeviceArray(3 * sess.N)
    op = server.register(sess.A)
    with pytest.raises(ph.PhiksError) as e:
        server.submit(op, -1.0, sess.p, 1, TOL, dv.ptr, out.ptr)
    assert e.value.status == ph.PHIKS_EINVAL
    with pytest.raises(ph.PhiksError) as e:
        server.submit(op + 100, sess.tau, sess.p, 1, TOL, dv.ptr, out.ptr)
    assert e.value.status == ph.PHIKS_EINVAL
    with pytest.raises(ph.PhiksError) as e:
        server.submit(op, sess.tau, sess.p, 1, TOL, dv.ptr, out.ptr, precision=7)
    assert e.value.status == ph.PHIKS_EINVAL
    bad = [workloads.fd2_dirichlet(24), np.full((24, 24), np.nan)]
    with pytest.raises(ph.PhiksError) as e:
        server.register(bad)
    assert e.value.status == ph.PHIKS_ENONFINITE
    big = workloads.Session("big", [128, 128, 64], [workloads.fd2_dirichlet(m) for m in (128, 128, 64)], 1e-3, 4)
    dvb = ph.DeviceArray(big.N)
    outb = ph.DeviceArray(5 * big.N)
    with pytest.raises(ph.PhiksError) as e:
        server.submit(server.register(big.A), big.tau, big.p, 1, TOL, dvb.ptr, outb.ptr)
    assert e.value.status == ph.PHIKS_EWORKSPACE
    server.close()


def test_concurrent_submitters():
    sessions = small_sessions()
    server = ph.Server(hbm_budget=4 * GiB, workspace_bytes=1 * GiB, max_active=8)
    results = {}

    def client(cid):
        picks = [(cid + k) % len(sessions) for k in range(12)]
        results[cid] = run_requests(server, sessions, picks, 10 + cid)

    th = [threading.Thread(target=client, args=(c,)) for c in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for cid, (reqs, _) in results.items():
        for si, ns, prec, v, _, out, _ in reqs:
            assert np.array_equal(out.to_numpy(), reference(sessions[si], v, ns)), (cid, sessions[si].name)
    assert server.stats()["completed"] == 24
    server.close()


def test_request_joins_running_lane_and_finishes_first():
    """Continuous batching inside a lane: four long 2D 1024^2 requests (p = 4, s = 11:
    55 Tucker operators, ~110 ticks) start; a short request of the same lane (p = 1 at
    a small step, s = 2: 7 Tucker operators, ~15 ticks) submitted while they run joins
    the lane's schedule at the next tick and completes before all of them, bitwise
    equal to its single call."""
    lng = workloads.Session("adr_1024", [1024, 1024],
                            [workloads.adr_1d(1024, 0.5, b, -1.0) for b in (1.0, 0.5)], 4e-3, 4)
    sht = workloads.Session("adr_1024_short", [1024, 1024], lng.A, 1e-7, 1)
    server = ph.Server(hbm_budget=8 * GiB, workspace_bytes=2 * GiB, max_active=8, lanes=3)
    assert ph.server_lane(lng.N, 3) == ph.server_lane(sht.N, 3)
    rng = np.random.default_rng(5)
    op = server.register(lng.A)
    # warm the plan cache (plans of both requests), so the timed requests only run steps
    for sess in (lng, sht):
        v = ph.DeviceArray.from_numpy(rng.standard_normal(sess.N))
        o = ph.DeviceArray((sess.p + 1) * sess.N)
        server.wait(server.submit(op, sess.tau, sess.p, 1, TOL, v.ptr, o.ptr))
    # every buffer first (allocations and copies would otherwise space the submissions)
    longs = []
    for k in range(4):
        v = rng.standard_normal(lng.N)
        longs.append([v, ph.DeviceArray.from_numpy(v), ph.DeviceArray((lng.p + 1) * lng.N), None])
    vs = rng.standard_normal(sht.N)
    dvs, os_ = ph.DeviceArray.from_numpy(vs), ph.DeviceArray((sht.p + 1) * sht.N)
    ph.synchronize()
    for x in longs:
        x[3] = server.submit(op, lng.tau, lng.p, 1, TOL, x[1].ptr, x[2].ptr)
    import time
    time.sleep(0.002)   # the long requests are on the GPU
    t_sub = ph.server_clock()
    ts = server.submit(op, sht.tau, sht.p, 1, TOL, dvs.ptr, os_.ptr)
    lat_s, done_s = server.wait_times(ts)
    done_l = [server.wait_times(t)[1] for (_, _, _, t) in longs]
    print(f"[server join] short done {(done_s - t_sub) * 1e3:.2f} ms after submission; "
          f"long requests done at {[round((d - t_sub) * 1e3, 2) for d in done_l]} ms")
    assert all(done_s < d for d in done_l)
    assert all(d > t_sub for d in done_l)       # they were still running at submission
    assert np.array_equal(os_.to_numpy(), reference(sht, vs))
    for v, _, o, _ in longs:
        assert np.array_equal(o.to_numpy(), reference(lng, v))
    server.close()


def test_lanes_overlap_small_requests_pass_large_ones():
    """A 3D 160^3 request (lane 2) and 2D 256^2 requests (lane 0) submitted after it: the
    small requests complete while the large one is still running."""
    big = workloads.Session("adr_160^3", [160, 160, 160],
                            [workloads.adr_1d(160, 0.5, b, -1.0) for b in (1.0, 0.5, 0.25)], 2e-3, 4)
    small = workloads.Session("fd2_256^2", [256, 256], [workloads.fd2_dirichlet(256)] * 2, 1e-4, 2)
    server = ph.Server(hbm_budget=16 * GiB, workspace_bytes=4 * GiB, max_active=8, lanes=3)
    assert ph.server_lane(big.N, 3) != ph.server_lane(small.N, 3)
    rng = np.random.default_rng(6)
    ob, osm = server.register(big.A), server.register(small.A)
    for sess, op in ((big, ob), (small, osm)):
        v = ph.DeviceArray.from_numpy(rng.standard_normal(sess.N))
        o = ph.DeviceArray((sess.p + 1) * sess.N)
        server.wait(server.submit(op, sess.tau, sess.p, 1, TOL, v.ptr, o.ptr))
    vb = rng.standard_normal(big.N)
    dvb, obuf = ph.DeviceArray.from_numpy(vb), ph.DeviceArray((big.p + 1) * big.N)
    smalls = []
    for k in range(4):
        v = rng.standard_normal(small.N)
        smalls.append([v, ph.DeviceArray.from_numpy(v), ph.DeviceArray((small.p + 1) * small.N), None])
    ph.synchronize()
    tb = server.submit(ob, big.tau, big.p, 1, TOL, dvb.ptr, obuf.ptr)
    for x in smalls:
        x[3] = server.submit(osm, small.tau, small.p, 1, TOL, x[1].ptr, x[2].ptr)
    done_s = [server.wait_times(t)[1] for (_, _, _, t) in smalls]
    done_b = server.wait_times(tb)[1]
    print(f"[server lanes] small requests done {[round((d - done_b) * 1e3, 2) for d in done_s]} ms "
          "relative to the large one")
    assert max(done_s) < done_b
    for v, _, o, _ in smalls:
        assert np.array_equal(o.to_numpy(), reference(small, v))
    assert np.array_equal(obuf.to_numpy(), reference(big, vb))
    server.close()


def test_request_deadlines():
    """Deadlines (one running request at a time): B, queued behind a long request A
    with a 0.1 ms timeout, completes with PHIKS_ETIMEDOUT without running (its output
    untouched); C, whose timeout (1 ms) is far below its run time, is stopped at a step
    boundary with PHIKS_ETIMEDOUT; A and a later request D without a deadline complete
    bitwise equal to their single calls."""
    lng = workloads.Session("adr_1024", [1024, 1024],
                            [workloads.adr_1d(1024, 0.5, b, -1.0) for b in (1.0, 0.5)], 4e-3, 4)
    server = ph.Server(hbm_budget=8 * GiB, workspace_bytes=2 * GiB, max_active=1, lanes=1)
    rng = np.random.default_rng(9)
    op = server.register(lng.A)
    v0 = ph.DeviceArray.from_numpy(rng.standard_normal(lng.N))
    o0 = ph.DeviceArray((lng.p + 1) * lng.N)
    server.wait(server.submit(op, lng.tau, lng.p, 1, TOL, v0.ptr, o0.ptr))   # plan cached
    vals = [rng.standard_normal(lng.N) for _ in range(4)]
    dv = [ph.DeviceArray.from_numpy(x) for x in vals]
    outs = [ph.DeviceArray.from_numpy(np.full((lng.p + 1) * lng.N, np.nan)) for _ in range(4)]
    ph.synchronize()
    print("[server deadlines] A + B queued behind it", flush=True)
    ta = server.submit(op, lng.tau, lng.p, 1, TOL, dv[0].ptr, outs[0].ptr)
    tb = server.submit(op, lng.tau, lng.p, 1, TOL, dv[1].ptr, outs[1].ptr, timeout=1e-4)
    with pytest.raises(ph.PhiksError) as e:
        server.wait(tb)
    assert e.value.status == ph.PHIKS_ETIMEDOUT
    server.wait(ta)
    assert np.isnan(outs[1].to_numpy()).all()          # B never ran
    print("[server deadlines] C stopped while running", flush=True)
    tc = server.submit(op, lng.tau, lng.p, 1, TOL, dv[2].ptr, outs[2].ptr, timeout=1e-3)
    with pytest.raises(ph.PhiksError) as e:
        server.wait(tc)
    assert e.value.status == ph.PHIKS_ETIMEDOUT
    print("[server deadlines] D", flush=True)
    td = server.submit(op, lng.tau, lng.p, 1, TOL, dv[3].ptr, outs[3].ptr, timeout=60.0)
    server.wait(td)
    for k in (0, 3):
        assert np.array_equal(outs[k].to_numpy(), reference(lng, vals[k]))
    assert server.stats()["timed_out"] == 2
    with pytest.raises(ph.PhiksError) as e:
        server.submit(op, lng.tau, lng.p, 1, TOL, dv[3].ptr, outs[3].ptr, timeout=-1.0)
    assert e.value.status == ph.PHIKS_EINVAL
    server.close()
