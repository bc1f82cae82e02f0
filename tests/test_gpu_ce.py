"""GPU parity of the Chapman-Enskog viscosity path: transport cross-section
and viscosity against hard-sphere closed forms and against the FP64 oracle
for the Jager form."""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_21244_amd import _lib
    _lib.load()
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def api(dev):
    from paper_2602_21244_amd import api as A
    return A


def test_hard_sphere_closed_forms(dev, api):
    say("CE hard sphere")
    d = 3.0
    pot = api.potential_hs(d)
    E = torch.tensor([50.0, 500.0, 5e4], dtype=torch.float64, device=dev)
    Q = api.transport_q2(E, 4e-10, pot, n_panels=64, n_gl=8).cpu().numpy()
    np.testing.assert_allclose(Q, 2.0 / 3.0 * math.pi * (d * 1e-10) ** 2, rtol=1e-12)
    T = torch.tensor([300.0, 3000.0], dtype=torch.float64, device=dev)
    om, mu = api.viscosity_ce(T, W.AR_MASS, 4e-10, pot, n_panels=64, n_gl=8, n_lag=8)
    np.testing.assert_allclose(om.cpu().numpy(), math.pi * (d * 1e-10) ** 2, rtol=1e-12)
    want = 5.0 / 16.0 * np.sqrt(math.pi * W.AR_MASS * W.KB * T.cpu().numpy()) / (math.pi * (d * 1e-10) ** 2)
    np.testing.assert_allclose(mu.cpu().numpy(), want, rtol=1e-12)
    om_p, _ = api.viscosity_ce(T, W.AR_MASS, 4e-10, pot, n_panels=64, n_gl=8, n_lag=8,
                               mode=api.L.CE_AS_PRINTED)
    np.testing.assert_allclose(om_p.cpu().numpy(), Q[0], rtol=1e-12)


def test_jager_cross_section_and_viscosity_match_oracle(orc, dev, api):
    say("CE Jager")
    pot = api.potential_jager(W.JAGER_PLACEHOLDER)
    P = orc.potential_jager(W.JAGER_PLACEHOLDER)
    b_cut = 2.5e-9
    E = np.array([20.0, 150.0, 1000.0, 3e4])
    Qg = api.transport_q2(torch.as_tensor(E, device=dev), b_cut, pot, n_panels=256,
                          n_gl=8).cpu().numpy()
    Qo = orc.transport_q2(P, E, b_cut, n_panels=256, n_gl=8)
    say("  Q2 rel err", np.abs(Qg - Qo) / Qo)
    np.testing.assert_allclose(Qg, Qo, rtol=1e-6)
    T = np.array([1500.0, 3000.0, 6000.0])
    om, mu = api.viscosity_ce(torch.as_tensor(T, device=dev), W.AR_MASS, b_cut, pot,
                              n_panels=256, n_gl=8, n_lag=16)
    oo = orc.collision_integral(P, T, b_cut, n_lag=16, n_panels=256, n_gl=8)
    mo = orc.viscosity_ce(oo, T, W.AR_MASS)
    say("  mu (Pa s)", mu.cpu().numpy(), "oracle", mo)
    np.testing.assert_allclose(om.cpu().numpy(), oo, rtol=1e-6)
    np.testing.assert_allclose(mu.cpu().numpy(), mo, rtol=1e-6)
