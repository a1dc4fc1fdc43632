"""GPU checks of the mixed-precision paths (mu-mode products in FP32 MFMA, or in BF16x3:
three BF16 MFMA products per FP32 product; small exponentials, quadrature sums, squaring
recurrence and outputs in FP64) against the FP64 oracle run with the same plan (s, q).

The paper fixes no precision for these variants, so the bar is a stated one, the
relative infinity-norm difference per output, derived from the arithmetic:
  FP32    <= 2e-6: a mu-mode product rounds its FP32 operands and its output once each
          (u = 2^-24 = 6.0e-8 relative), ~3u per product, so ~3du = 5.4e-7 per Tucker
          operator at d = 3.  The squaring recurrence passes the error of earlier levels
          on with coefficients of norm <= 1 for these dissipative operators, which at
          most about doubles it: ~1.1e-6; bar 2e-6.  (Measured <= 6e-7.)
  BF16x3  <= 1e-4: each term a*b of a contraction is formed to within 3 * 2^-16 of
          |a b| (the dropped lo*lo term and the two split remainders); these are
          rounding errors of either sign, so a contraction over K = n_mu >= 64 terms
          carries ~3 * 2^-16 / sqrt(K) <= 5.7e-6, ~1.7e-5 per Tucker operator at d = 3,
          ~3.4e-5 after the recurrence as above; bar 1e-4.  (Measured <= 1.3e-5.)
The measured errors are printed."""
import functools

import numpy as np
import pytest

import workloads
from oracle import phiks as ophiks

pytestmark = pytest.mark.gpu
ph = pytest.importorskip("paper_2210_07667_amd")
TOL = {"fp32": 2e-6, "bf16x3": 1e-4}
PREC = {"fp32": ph.PHIKS_FP32, "bf16x3": ph.PHIKS_BF16X3}


@pytest.fixture(autouse=True)
def _need_gpu():
    if ph.device_count() < 1:
        pytest.skip("no GPU")


def relerr(got, ref):
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


def ops(n, betas=(1.0, 0.5, 0.25, 0.125)):
    return [workloads.adr_1d(k, 0.5, betas[i], -1.0) for i, k in enumerate(n)]


# the two larger shapes reach every BF16x3 tile (128x128, 128x64, 64x128, 64x64) with
# ragged M, N and K tails, and (K = 97) the path without 16-byte loads; the small
# ones fall back to the FP32 kernel for products too small to fill the GPU
APPLY_CASES = [([40, 33, 20], 1e-3, 4, 2), ([64, 64, 64], 1e-3, 4, 1), ([33, 17], 5e-3, 3, 2),
               ([7], 0.3, 2, 1), ([160, 144, 100], 1e-3, 4, 1), ([150, 97, 130], 2e-3, 3, 2),
               # modes > 1 on the direct-to-LDS FP32 / BF16x3 kernels with tiles overhanging
               # M and N (160 = 128 + 32, 96 = 64 + 32; 224 = 128 + 96, 72 = 64 + 8)
               ([96, 160, 128], 1e-3, 3, 1), ([72, 224, 160], 1e-3, 2, 1),
               # d = 2 BF16x3 pair chain (node phase: the last mode reads pair words on
               # 128 x 64 tiles, M = 352 = 2*128 + 96, N = 520 = 8*64 + 8); FP32 first mode
               # with an FP64 A on the direct-to-LDS kernel, M = 7200 = 56*128 + 32
               ([520, 352], 1e-3, 4, 1), ([96, 72, 100], 1e-3, 3, 1),
               # squaring launches on the direct-to-LDS kernels with a ragged N (third mode:
               # N = 7200 = 112*64 + 32; the pre-step slices clamp their last columns)
               ([100, 72, 128], 1e-3, 3, 1),
               # K tails of 12 on the FP32 direct-to-LDS kernel (K = 60 with an FP64 A,
               # K = 300 with an n-contiguous B) and a skinny squaring product on 64 x 64
               # tiles (third mode: M = K = 28, N = 18000)
               ([60, 300, 28], 1e-3, 3, 1)]


@functools.lru_cache(maxsize=None)
def oracle_apply(case, s, q):
    n, tau, p, ns = APPLY_CASES[case]
    A = ops(n)
    v = workloads.randn_vec(n, 31)
    return ophiks.phi_same_vector(A, tau, v, p, ns, s, q)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("case", range(len(APPLY_CASES)))
def test_mixed_apply_vs_oracle(case, prec):
    n, tau, p, ns = APPLY_CASES[case]
    A = ops(n)
    v = workloads.randn_vec(n, 31)
    print(f"[{prec} apply] n={n} tau={tau} p={p} ns={ns}", flush=True)
    plan = ph.phiks_plan(A, tau, p, ns, 2.0 ** -53, "same_vector", precision=PREC[prec])
    out = ph.apply_arrays(plan, ph.DeviceArray.from_numpy(v))
    ph.synchronize()
    info = plan.info()
    plan.close()
    got = out.to_numpy().reshape(ns, p + 1, -1)
    ref = oracle_apply(case, info["s"], info["q"])
    errs = [[relerr(got[j, l], ref[j, l]) for l in range(p + 1)] for j in range(ns)]
    print(f"[{prec} apply] n={n} plan={info} rel errors={np.array(errs).round(9).tolist()}")
    assert max(max(e) for e in errs) < TOL[prec]


COMBINE_CASES = [("allen-cahn 64^3", None), ("adr 160x144x100", [160, 144, 100])]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("case", range(len(COMBINE_CASES)))
def test_mixed_combine_vs_oracle(case, prec):
    name, n = COMBINE_CASES[case]
    if n is None:
        w = workloads.config_allen_cahn_3d(tau=1e-2)
        A, tau, vs, p, ns, tol = w.A, w.tau, w.vs, w.p, w.n_scales, w.tol
    else:
        A, tau, p, ns = ops(n), 1e-3, 3, 2
        vs = [workloads.randn_vec(n, 40 + k) for k in range(p + 1)]
        tol = 2.0 ** -53
    print(f"[{prec} combine] {name}", flush=True)
    plan = ph.phiks_plan(A, tau, p, ns, tol, "lincomb", precision=PREC[prec])
    out = ph.combine_arrays(plan, [ph.DeviceArray.from_numpy(x) for x in vs])
    ph.synchronize()
    info = plan.info()
    plan.close()
    got = out.to_numpy().reshape(ns, -1)
    ref = ophiks.phi_lincomb(A, tau, vs, p, ns, info["s"], info["q"])
    errs = [relerr(got[j], ref[j]) for j in range(ns)]
    print(f"[{prec} combine] {name} plan={info} rel errors={errs}")
    assert max(errs) < TOL[prec]


def test_mixed_adr_256_against_fp64_path():
    """Full 256^3 workload: both mixed paths against the FP64 path (itself checked
    against the oracle in test_gpu_parity.py)."""
    w = workloads.config_adr_3d()
    v = ph.DeviceArray.from_numpy(w.v)
    outs = {}
    for prec in (ph.PHIKS_FP64, ph.PHIKS_FP32, ph.PHIKS_BF16X3):
        plan = ph.phiks_plan(w.A, w.tau, w.p, w.n_scales, w.tol, w.task, precision=prec)
        outs[prec] = ph.apply_arrays(plan, v).to_numpy().reshape(w.p + 1, -1)
        plan.close()
    for name in ("fp32", "bf16x3"):
        errs = [relerr(outs[PREC[name]][l], outs[ph.PHIKS_FP64][l]) for l in range(w.p + 1)]
        print(f"[{name} apply] adr 256^3 rel errors vs fp64 = {errs}")
        assert max(errs) < TOL[name]
