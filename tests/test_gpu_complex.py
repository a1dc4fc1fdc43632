"""GPU parity of complex plans (phiks_plan_complex): complex A_mu and tau, vectors of
complex values as interleaved float64, against the FP64 oracle (complex arithmetic)
with the same (s, q), and against the brute-force augmented-matrix exponential.

Bars: 1e-12 relative against the oracle (as the real FP64 path).  Against the brute
force on the validation operators of Section 4.1 the paper reports relative
differences of at most 4.7e-13 for single phi-functions and 2.6e-12 for linear
combinations (its Fig. 1, phiks against an independent method); those are the bars
there."""
import numpy as np
import pytest

import workloads
from oracle import brute, phiks as ophiks

pytestmark = pytest.mark.gpu
ph = pytest.importorskip("paper_2210_07667_amd")
TOL = 1e-12


@pytest.fixture(autouse=True)
def _need_gpu():
    if ph.device_count() < 1:
        pytest.skip("no GPU")


def relerr(got, ref):
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


def apply_complex(A, tau, v, p, ns, vnorm=True):
    plan = ph.phiks_plan_complex(A, tau, p, ns, 2.0 ** -53, "same_vector",
                                 [np.linalg.norm(v)] if vnorm else None)
    out = ph.apply_arrays(plan, ph.DeviceArray.from_numpy(v))
    ph.synchronize()
    info = plan.info()
    plan.close()
    return out.to_complex().reshape(ns, p + 1, -1), info


def dense_complex(n, seed):
    rng = np.random.default_rng(seed)
    return [(rng.standard_normal((k, k)) + 1j * rng.standard_normal((k, k))) / np.sqrt(k) for k in n]


CASES = [
    ("validation d=3 n=20", lambda: workloads.validation_table1(3, 20), 1.0, 5, 2),
    ("validation d=6 n=8", lambda: workloads.validation_table1(6, 8), 1.0, 5, 2),
    ("dense d=2 [12,9] complex tau", lambda: (dense_complex([12, 9], 1),
                                              workloads.randn_vec([12, 9], 2) + 1j * workloads.randn_vec([12, 9], 3)),
     0.7 + 0.4j, 3, 2),
    ("dense d=3 [10,7,5]", lambda: (dense_complex([10, 7, 5], 4),
                                    workloads.randn_vec([10, 7, 5], 5) + 1j * workloads.randn_vec([10, 7, 5], 6)),
     0.3 - 0.2j, 4, 1),
]


@pytest.mark.parametrize("case", range(len(CASES)), ids=[c[0] for c in CASES])
def test_complex_apply_vs_oracle(case):
    name, make, tau, p, ns = CASES[case]
    A, v = make()
    print(f"[complex apply] {name}", flush=True)
    got, info = apply_complex(A, tau, v, p, ns)
    ref = ophiks.phi_same_vector(A, tau, v, p, ns, info["s"], info["q"])
    errs = [relerr(got[j, l], ref[j, l]) for j in range(ns) for l in range(p + 1)]
    print(f"[complex apply] {name} plan={info} max rel err {max(errs):.2e}")
    assert max(errs) < TOL


def test_complex_combine_vs_oracle():
    A, v = workloads.validation_table1(3, 16)
    rng = np.random.default_rng(7)
    vs = [v] + [rng.standard_normal(v.size) + 1j * rng.standard_normal(v.size) for _ in range(3)]
    plan = ph.phiks_plan_complex(A, 1.0, 3, 2, 2.0 ** -53, "lincomb",
                                 [np.linalg.norm(x) for x in vs])
    out = ph.combine_arrays(plan, [ph.DeviceArray.from_numpy(x) for x in vs])
    ph.synchronize()
    info = plan.info()
    plan.close()
    got = out.to_complex().reshape(2, -1)
    ref = ophiks.phi_lincomb(A, 1.0, vs, 3, 2, info["s"], info["q"])
    errs = [relerr(got[j], ref[j]) for j in range(2)]
    print(f"[complex combine] plan={info} rel errs {errs}")
    assert max(errs) < TOL


def test_validation_accuracy_against_brute_force():
    """Section 4.1 operators (d = 2, n = 16, N = 256): single phi-functions within 4.7e-13
    and the linear combination within 2.6e-12 of the augmented-matrix exponential."""
    A, v = workloads.validation_table1(2, 16)
    p = 5
    got, info = apply_complex(A, 1.0, v, p, 1)
    ref = brute.phi_actions_dense(A, 1.0, v, p)
    errs = [relerr(got[0, l], ref[l]) for l in range(p + 1)]
    print(f"[complex vs brute force] phi_0..phi_5 rel errs {np.round(errs, 16).tolist()}")
    assert max(errs) < 4.7e-13
    vs = [v] * (p + 1)
    plan = ph.phiks_plan_complex(A, 1.0, p, 1, 2.0 ** -53, "lincomb", [np.linalg.norm(v)] * (p + 1))
    out = ph.combine_arrays(plan, [ph.DeviceArray.from_numpy(x) for x in vs])
    ph.synchronize()
    plan.close()
    refc = brute.augmented(A, 1.0, vs)
    e = relerr(out.to_complex(), refc)
    print(f"[complex combination vs brute force] rel err {e:.2e}")
    assert e < 2.6e-12


def test_complex_rejects_bad_input():
    A, v = workloads.validation_table1(2, 6)
    with pytest.raises(ph.PhiksError) as e:
        ph.phiks_plan_complex(A, 0.0, 2, 1, 1e-10)
    assert e.value.status == ph.PHIKS_EINVAL
    bad = [A[0].copy(), A[1].copy()]
    bad[1][2, 3] = complex(np.nan, 0.0)
    with pytest.raises(ph.PhiksError) as e:
        ph.phiks_plan_complex(bad, 1.0, 2, 1, 1e-10)
    assert e.value.status == ph.PHIKS_ENONFINITE
