"""phiks_apply_noalloc (fixed per-device scratch, no workspace argument, no device
allocation) against phiks_apply on the same plan and vector: two calls in a row,
the second with a smaller problem, each output compared bitwise (both entry points
run the same kernels on the same operands), and the first also against the FP64
oracle with the same (s, q) at the FP64 bar of 1e-12.  A plan whose workspace
exceeds the fixed scratch is refused before any device work."""
import numpy as np
import pytest

import workloads
from oracle import phiks as ophiks

pytestmark = pytest.mark.gpu
ph = pytest.importorskip("paper_2210_07667_amd")


@pytest.fixture(autouse=True)
def _need_gpu():
    if ph.device_count() < 1:
        pytest.skip("no GPU")


def adr_ops(n):
    betas = (1.0, 0.5, 0.25)
    return [workloads.adr_1d(k, 0.5, betas[i], -1.0) for i, k in enumerate(n)]


def one_call(n, tau, p, ns, seed, check_oracle):
    A = adr_ops(n)
    v = workloads.randn_vec(n, seed)
    print(f"[noalloc] n={n} tau={tau} p={p} ns={ns}", flush=True)
    plan = ph.phiks_plan(A, tau, p, ns, 2.0 ** -53, "same_vector")
    assert plan.workspace_size() <= ph.NOALLOC_SCRATCH_BYTES
    dv = ph.DeviceArray.from_numpy(v)
    ref = ph.apply_arrays(plan, dv)
    out = ph.DeviceArray.from_numpy(np.full(ns * (p + 1) * v.size, np.nan))
    ph.phiks_apply_noalloc(plan, dv.ptr, out.ptr)
    ph.synchronize()
    info = plan.info()
    plan.close()
    got, want = out.to_numpy(), ref.to_numpy()
    assert np.array_equal(got, want), float(np.nanmax(np.abs(got - want)))
    if check_oracle:
        o = ophiks.phi_same_vector(A, tau, v, p, ns, info["s"], info["q"])
        got = got.reshape(ns, p + 1, -1)
        for j in range(ns):
            for ell in range(p + 1):
                err = np.abs(got[j, ell] - o[j, ell]).max() / np.abs(o[j, ell]).max()
                assert err < 1e-12, (j, ell, err)


def test_noalloc_matches_apply_two_calls():
    one_call([40, 33, 20], 1e-3, 4, 2, 71, True)
    one_call([12, 10, 9], 2e-2, 3, 1, 72, False)     # smaller: reuses the same scratch


def test_noalloc_refuses_oversized_plan():
    n = [128, 128, 128]
    plan = ph.phiks_plan(adr_ops(n), 1e-3, 4, 1, 2.0 ** -53, "same_vector")
    assert plan.workspace_size() > ph.NOALLOC_SCRATCH_BYTES
    dv = ph.DeviceArray(128 ** 3)
    out = ph.DeviceArray(5 * 128 ** 3)
    with pytest.raises(ph.PhiksError) as e:
        ph.phiks_apply_noalloc(plan, dv.ptr, out.ptr)
    assert e.value.status == ph.PHIKS_EWORKSPACE
    plan.close()
