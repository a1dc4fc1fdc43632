"""GPU exponential integrators (paper_2210_07667_amd.integrators) on the ADR problem of
Section 4.2: the errors the paper prints (tests/golden/adr_integrators.json) and the
oracle integrators (pinned to the same values in test_oracle_integrators.py).  Also
the device vector ops they use, against NumPy."""
import json
import os

import numpy as np
import pytest

import workloads
from oracle import integrators as oi

pytestmark = pytest.mark.gpu
ph = pytest.importorskip("paper_2210_07667_amd")
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "adr_integrators.json")))


@pytest.fixture(autouse=True)
def _need_gpu():
    if ph.device_count() < 1:
        pytest.skip("no GPU")


def rel_inf(u, ex):
    return float(np.abs(u - ex).max() / np.abs(ex).max())


def test_vector_ops_match_numpy():
    rng = np.random.default_rng(0)
    n = 1001
    x, y = rng.standard_normal(n), rng.standard_normal(n)
    dx, dy, do = ph.DeviceArray.from_numpy(x), ph.DeviceArray.from_numpy(y), ph.DeviceArray(n)
    cases = [(ph.PHIKS_VOP_AXPBY, 0.5, -2.0, True, 0.5 * x - 2.0 * y),
             (ph.PHIKS_VOP_AXPBY, 3.0, 0.0, False, 3.0 * x),
             (ph.PHIKS_VOP_RATIONAL, -1.5, 0.7, True, -1.5 / (1 + (0.7 * x) ** 2) + y),
             (ph.PHIKS_VOP_RATIONAL, 1.0, 1.0, False, 1 / (1 + x * x)),
             (ph.PHIKS_VOP_CUBIC, 2.0, 0.25, True, 2.0 * (x - x ** 3) + 0.25 * y)]
    for op, a, b, use_y, ref in cases:
        ph.vector_op(op, n, a, dx.ptr, b, dy.ptr if use_y else None, do.ptr)
        np.testing.assert_allclose(do.to_numpy(), ref, rtol=1e-14, atol=1e-14)
    # out aliasing an input
    ph.vector_op(ph.PHIKS_VOP_AXPBY, n, 2.0, dx.ptr, 1.0, dy.ptr, dy.ptr)
    np.testing.assert_allclose(dy.to_numpy(), 2.0 * x + y, rtol=1e-14)
    with pytest.raises(ph.PhiksError):
        ph.vector_op(7, n, 1.0, dx.ptr, 1.0, None, do.ptr)


@pytest.fixture(scope="module")
def adr():
    return workloads.adr_integration_problem(20)


def test_exp_euler_on_gpu(adr):
    from paper_2210_07667_amd import integrators as gi
    g = gi.ADRNonlinearity(adr.u0, adr.w)
    u = gi.exp_euler(adr.A, adr.u0, g, 0.1, 300).to_numpy()
    err = rel_inf(u, adr.exact(0.1))
    ref = oi.exp_euler(adr.A, adr.u0, oi.adr_nonlinearity(adr), 0.1, 300)
    d = rel_inf(u, ref)
    print(f"[gpu expEuler 300] error {err!r} (paper phiks {GOLD['exp_euler']['phiks'][0]!r}); vs oracle {d:.2e}")
    assert abs(err / GOLD["exp_euler"]["phiks"][0] - 1) < 1e-6
    assert abs(err / GOLD["exp_euler"]["kiops"][0] - 1) < 1e-6
    assert d < 1e-11


def test_etd2rk_on_gpu(adr):
    from paper_2210_07667_amd import integrators as gi
    g = gi.ADRNonlinearity(adr.u0, adr.w)
    u = gi.etd2rk(adr.A, adr.u0, g, 0.1, 200).to_numpy()
    err = rel_inf(u, adr.exact(0.1))
    ref = oi.etd2rk(adr.A, adr.u0, oi.adr_nonlinearity(adr), 0.1, 200)
    d = rel_inf(u, ref)
    print(f"[gpu ETD2RK 200] error {err!r} (paper kiops {GOLD['etd2rk']['kiops'][0]!r}); vs oracle {d:.2e}")
    for method in ("kiops", "bamphi", "phipm_simul_iom"):
        assert abs(err / GOLD["etd2rk"][method][0] - 1) < 1e-5, method
    assert d < 1e-11


def test_allen_cahn_exp_euler_matches_oracle():
    """The Allen-Cahn model (K = eps Lap, g = u - u^3) on 24^3: a few exponential Euler
    steps on the GPU against the oracle integrator."""
    from paper_2210_07667_amd import integrators as gi
    w = workloads.config_allen_cahn_3d(n=24, tau=1e-2)
    u0 = w.vs[0]
    u = gi.exp_euler(w.A, u0, gi.AllenCahnNonlinearity(u0.size), 0.05, 5).to_numpy()
    ref = oi.exp_euler(w.A, u0, lambda t, x: x - x ** 3, 0.05, 5)
    d = rel_inf(u, ref)
    print(f"[gpu Allen-Cahn expEuler] vs oracle {d:.2e}")
    assert d < 1e-12


@pytest.mark.parametrize("scheme,steps", [("exprk3s3", 10), ("exprk4s6", 5)])
def test_higher_order_schemes_on_gpu_match_oracle(adr, scheme, steps):
    from paper_2210_07667_amd import integrators as gi
    g = gi.ADRNonlinearity(adr.u0, adr.w)
    u = getattr(gi, scheme)(adr.A, adr.u0, g, 0.1, steps).to_numpy()
    ref = getattr(oi, scheme)(adr.A, adr.u0, oi.adr_nonlinearity(adr), 0.1, steps)
    d = rel_inf(u, ref)
    err = rel_inf(u, adr.exact(0.1))
    print(f"[gpu {scheme} {steps} steps] error {err:.3e}; vs oracle {d:.2e}")
    assert d < 1e-11


@pytest.mark.parametrize("smart", [True, False])
def test_exprk4s5_brusselator_matches_oracle(smart):
    """The five-stage fourth-order scheme (eq. expRK4s5; smart: the five lines of eq.
    expRK4s5_smart) on the two-species Brusselator system (block-diagonal K, 12^3 grid per
    species, Neumann FD2), GPU driver against the oracle driver of the same form."""
    from paper_2210_07667_amd import integrators as gi
    pr = workloads.brusselator_problem(n=12, d=3)
    g_gpu = gi.BrusselatorNonlinearity(pr.a, pr.b, pr.N)
    g_cpu = oi.brusselator_nonlinearity(pr.a, pr.b, pr.N)
    u = gi.exprk4s5(pr.blocks, pr.w0, g_gpu, 0.5, 3, smart=smart).to_numpy()
    ref = oi.exprk4s5(pr.blocks, pr.w0, g_cpu, 0.5, 3, smart=smart)
    d = rel_inf(u, ref)
    print(f"[gpu expRK4s5 brusselator smart={smart}] vs oracle {d:.2e}")
    assert d < 1e-11


def test_exprk4s5_adr_matches_oracle_and_converges(adr):
    """One block (the ADR problem of Section 4.2): GPU against the oracle, and the GPU
    errors against the exact solution fall at fourth order."""
    from paper_2210_07667_amd import integrators as gi
    g = gi.ADRNonlinearity(adr.u0, adr.w)
    e = []
    for steps in (5, 10):
        u = gi.exprk4s5([adr.A], adr.u0, g, 0.1, steps).to_numpy()
        e.append(rel_inf(u, adr.exact(0.1)))
        if steps == 5:
            ref = oi.exprk4s5([adr.A], adr.u0, oi.adr_nonlinearity(adr), 0.1, 5, smart=True)
            assert rel_inf(u, ref) < 1e-11
    rate = np.log2(e[0] / e[1])
    print(f"[gpu expRK4s5 adr] errors {e} observed order {rate:.2f}")
    assert abs(rate - 4) < 0.3


def test_brusselator_vector_ops_match_numpy():
    rng = np.random.default_rng(3)
    n = 777
    x, y = rng.standard_normal(n), rng.standard_normal(n)
    dx, dy, do = ph.DeviceArray.from_numpy(x), ph.DeviceArray.from_numpy(y), ph.DeviceArray(n)
    ph.vector_op(ph.PHIKS_VOP_BRUSS_U, n, 1.5, dx.ptr, 0.0, dy.ptr, do.ptr)
    np.testing.assert_allclose(do.to_numpy(), 1.5 + x * x * y, rtol=1e-14, atol=1e-14)
    ph.vector_op(ph.PHIKS_VOP_BRUSS_V, n, 3.0, dx.ptr, 0.0, dy.ptr, do.ptr)
    np.testing.assert_allclose(do.to_numpy(), 3.0 * x - x * x * y, rtol=1e-14, atol=1e-14)
