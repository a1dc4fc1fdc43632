"""GPU checks of the serving entry points (phiks_server_*).

A served request is one phiks_apply; whatever group the server runs it in, its output
must be bitwise the output of phiks_plan (tolerance relative, vnorms = NULL) +
phiks_apply for that request alone."""
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


def reference(sess, v, ns=1):
    plan = ph.phiks_plan(sess.A, sess.tau, sess.p, ns, TOL, "same_vector")
    out = ph.apply_arrays(plan, ph.DeviceArray.from_numpy(v))
    ph.synchronize()
    plan.close()
    return out.to_numpy()


def run_requests(server, sessions, picks, seed, ns_of=lambda k: 1):
    rng = np.random.default_rng(seed)
    ops = {}
    reqs = []
    for k, si in enumerate(picks):
        sess = sessions[si]
        ns = ns_of(k)
        v = rng.standard_normal(sess.N)
        dv = ph.DeviceArray.from_numpy(v)
        out = ph.DeviceArray(ns * (sess.p + 1) * sess.N)
        if si not in ops:
            ops[si] = server.register(sess.A)
        t = server.submit(ops[si], sess.tau, sess.p, ns, TOL, dv.ptr, out.ptr)
        reqs.append((si, ns, v, dv, out, t))
    lat = [server.wait(t) for (_, _, _, _, _, t) in reqs]
    return reqs, lat


def test_served_results_equal_single_calls():
    sessions = small_sessions()
    server = ph.Server(hbm_budget=4 * GiB, workspace_bytes=1 * GiB, max_group=16)
    rng = np.random.default_rng(0)
    picks = rng.integers(len(sessions), size=40).tolist()
    # a few two-scale requests: they form groups of their own (n_scales differs)
    reqs, lat = run_requests(server, sessions, picks, 1, ns_of=lambda k: 2 if k % 7 == 3 else 1)
    for si, ns, v, _, out, _ in reqs:
        ref = reference(sessions[si], v, ns)
        assert np.array_equal(out.to_numpy(), ref), sessions[si].name
    st = server.stats()
    print(f"[server] stats {st}, latency p50 {np.median(lat) * 1e3:.2f} ms max {max(lat) * 1e3:.2f} ms")
    keys = {(picks[k], 2 if k % 7 == 3 else 1) for k in range(len(picks))}
    assert st["completed"] == len(picks)
    assert st["cache_misses"] == len(keys)
    assert st["cache_hits"] == len(picks) - len(keys)
    server.close()


def test_eviction_under_a_small_budget():
    sessions = small_sessions()
    # 1 MB left for plans beside the 60 MB arena: fewer than the five sessions need
    server = ph.Server(hbm_budget=61 << 20, workspace_bytes=60 << 20, max_group=4)
    picks = [0, 1, 3, 5, 0, 1, 3, 5, 2, 2]
    reqs, _ = run_requests(server, sessions, picks, 2)
    for si, ns, v, _, out, _ in reqs:
        assert np.array_equal(out.to_numpy(), reference(sessions[si], v, ns)), sessions[si].name
    st = server.stats()
    print(f"[server small budget] stats {st}")
    assert st["evictions"] > 0
    server.close()


def test_submit_errors():
    server = ph.Server(hbm_budget=1 * GiB, workspace_bytes=8 << 20, max_group=4)
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
    server = ph.Server(hbm_budget=4 * GiB, workspace_bytes=1 * GiB, max_group=8)
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
        for si, ns, v, _, out, _ in reqs:
            assert np.array_equal(out.to_numpy(), reference(sessions[si], v, ns)), (cid, sessions[si].name)
    assert server.stats()["completed"] == 24
    server.close()
