"""GPU checks of the mixed-precision path (mu-mode products in FP32 MFMA; small
exponentials, quadrature sums, squaring recurrence and outputs in FP64) against the
FP64 oracle run with the same plan (s, q).

The paper fixes no precision for this variant, so the bar is a stated one: relative
infinity-norm difference <= 2e-5 per output (each FP32 product carries ~n 2^-24
relative error; a call chains ~35 Tucker operators and s squaring steps).  The
measured errors are printed."""
import numpy as np
import pytest

import workloads
from oracle import phiks as ophiks

pytestmark = pytest.mark.gpu
ph = pytest.importorskip("paper_2210_07667_amd")
TOL_FP32 = 2e-5


@pytest.fixture(autouse=True)
def _need_gpu():
    if ph.device_count() < 1:
        pytest.skip("no GPU")


def relerr(got, ref):
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


def ops(n, betas=(1.0, 0.5, 0.25, 0.125)):
    return [workloads.adr_1d(k, 0.5, betas[i], -1.0) for i, k in enumerate(n)]


@pytest.mark.parametrize("n,tau,p,ns", [([40, 33, 20], 1e-3, 4, 2), ([64, 64, 64], 1e-3, 4, 1),
                                        ([33, 17], 5e-3, 3, 2), ([7], 0.3, 2, 1)])
def test_fp32_apply_vs_oracle(n, tau, p, ns):
    A = ops(n)
    v = workloads.randn_vec(n, 31)
    plan = ph.phiks_plan(A, tau, p, ns, 2.0 ** -53, "same_vector", precision=ph.PHIKS_FP32)
    out = ph.apply_arrays(plan, ph.DeviceArray.from_numpy(v))
    ph.synchronize()
    info = plan.info()
    plan.close()
    got = out.to_numpy().reshape(ns, p + 1, -1)
    ref = ophiks.phi_same_vector(A, tau, v, p, ns, info["s"], info["q"])
    errs = [[relerr(got[j, l], ref[j, l]) for l in range(p + 1)] for j in range(ns)]
    print(f"[fp32 apply] n={n} plan={info} rel errors={np.array(errs).round(9).tolist()}")
    assert max(max(e) for e in errs) < TOL_FP32


def test_fp32_combine_vs_oracle():
    w = workloads.config_allen_cahn_3d(tau=1e-2)
    plan = ph.phiks_plan(w.A, w.tau, w.p, w.n_scales, w.tol, "lincomb", precision=ph.PHIKS_FP32)
    out = ph.combine_arrays(plan, [ph.DeviceArray.from_numpy(x) for x in w.vs])
    ph.synchronize()
    info = plan.info()
    plan.close()
    got = out.to_numpy().reshape(w.n_scales, -1)
    ref = ophiks.phi_lincomb(w.A, w.tau, w.vs, w.p, w.n_scales, info["s"], info["q"])
    errs = [relerr(got[j], ref[j]) for j in range(w.n_scales)]
    print(f"[fp32 combine] allen-cahn 64^3 plan={info} rel errors={errs}")
    assert max(errs) < TOL_FP32


def test_fp32_adr_256_against_fp64_path():
    """Full 256^3 workload: FP32 path against the FP64 path (itself checked against the
    oracle in test_gpu_parity.py)."""
    w = workloads.config_adr_3d()
    v = ph.DeviceArray.from_numpy(w.v)
    outs = {}
    for prec in (ph.PHIKS_FP64, ph.PHIKS_FP32):
        plan = ph.phiks_plan(w.A, w.tau, w.p, w.n_scales, w.tol, w.task, precision=prec)
        outs[prec] = ph.apply_arrays(plan, v).to_numpy().reshape(w.p + 1, -1)
        plan.close()
    errs = [relerr(outs[ph.PHIKS_FP32][l], outs[ph.PHIKS_FP64][l]) for l in range(w.p + 1)]
    print(f"[fp32 apply] adr 256^3 rel errors vs fp64 = {errs}")
    assert max(errs) < TOL_FP32
