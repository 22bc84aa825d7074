"""Pins of the oracle's one-axis (flux-decay) machine with IEEE type-1 exciter.

Each pin compares the oracle with a fact that does not come from its own
equations: the single-machine infinite-bus closed forms (d-axis current,
electrical power, the voltage divider for the terminal voltage, the loaded
transient time constant T'd = T'do (X'd + Xe)/(Xd + Xe)), the exciter's
characteristic polynomial read off the IEEE type-1 block diagram, the
equilibrium, and the limit in which the model reduces to the (separately
pinned) classical model.
"""
import numpy as np
import pytest

import oracle
import workloads

XD, XDP, TDO, KA, TA, KE, TE, KF, TF = range(9)


def jacobian(sc, y0, h=1e-6):
    P = len(sc["dist"]["gen"])
    z = np.zeros(P)
    J = np.zeros((len(y0), len(y0)))
    for k in range(len(y0)):
        hk = h * max(1.0, abs(y0[k]))
        yp = y0.copy(); yp[k] += hk
        ym = y0.copy(); ym[k] -= hk
        J[:, k] = (oracle.rhs(sc, yp, z) - oracle.rhs(sc, ym, z)) / (2 * hk)
    return J


SMIB_CASES = [dict(), dict(Xe=0.2, Xd=2.0, Xdp=0.25, delta0=0.3, E=1.2),
              dict(Xe=0.7, Xd=1.2, Xdp=0.4, delta0=1.0, E=0.95, KA=15.0, TA=0.02)]


@pytest.mark.parametrize("kw", SMIB_CASES)
def test_smib_operating_point_closed_form(kw):
    """Efd0, VR0, RF0 and Vref from the SMIB closed forms: Id0 =
    (E'q - V cos d)/X, Efd0 = E'q + (Xd - X'd) Id0, Vt = |(Xe E~' + X'd V)/X|."""
    sc = workloads.smib_fluxdecay(**kw)
    q = sc["model_params"][0]
    X = q[XDP] + kw.get("Xe", 0.4)
    E, d0, V = sc["E"][0], sc["delta0"][0], sc["V_inf"]
    y0, vref = oracle.initial_state(sc)
    Id0 = (E - V * np.cos(d0)) / X
    efd0 = E + (q[XD] - q[XDP]) * Id0
    Vt0 = abs((kw.get("Xe", 0.4) * E * np.exp(1j * d0) + q[XDP] * V) / X)
    np.testing.assert_allclose(y0[:6], [d0, 0.0, E, efd0, q[KE] * efd0, q[KF] / q[TF] * efd0],
                               rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(vref[0], Vt0 + q[KE] * efd0 / q[KA], rtol=1e-13)


@pytest.mark.parametrize("kw", SMIB_CASES)
def test_smib_network_sensitivities(kw):
    """Finite-difference derivatives of the oracle's right-hand side against
    the SMIB closed forms Pe = E'q V sin d / X, Id = (E'q - V cos d)/X and the
    divider Vt; the E'q row gives the loaded time constant T'd."""
    sc = workloads.smib_fluxdecay(**kw)
    q = sc["model_params"][0]
    Xe = kw.get("Xe", 0.4)
    X = q[XDP] + Xe
    V, H = sc["V_inf"], sc["H"][0]
    y0, _ = oracle.initial_state(sc)
    J = jacobian(sc, y0)
    d, eq = y0[0], y0[2]
    # E'q row: d/dE'q = -1/T'd, d/d delta = -(Xd - X'd) dId/d delta / T'do
    Tdp = q[TDO] * (q[XDP] + Xe) / (q[XD] + Xe)
    np.testing.assert_allclose(J[2, 2], -1.0 / Tdp, rtol=1e-8)
    np.testing.assert_allclose(J[2, 0], -(q[XD] - q[XDP]) * V * np.sin(d) / X / q[TDO], rtol=1e-7)
    np.testing.assert_allclose(J[2, 3], 1.0 / q[TDO], rtol=1e-8)
    # speed row: dPe/d delta and dPe/dE'q from Pe = E'q V sin d / X
    np.testing.assert_allclose(J[1, 0], -eq * V * np.cos(d) / X / (2 * H), rtol=1e-7)
    np.testing.assert_allclose(J[1, 2], -V * np.sin(d) / X / (2 * H), rtol=1e-7)
    # regulator row: -KA/TA dVt/dx with Vt from the voltage divider
    def vt(dd, ee):
        return abs((Xe * ee * np.exp(1j * dd) + q[XDP] * V) / X)
    h = 1e-6
    dvt_dd = (vt(d + h, eq) - vt(d - h, eq)) / (2 * h)
    dvt_de = (vt(d, eq + h) - vt(d, eq - h)) / (2 * h)
    np.testing.assert_allclose(J[4, 0], -q[KA] / q[TA] * dvt_dd, rtol=1e-6)
    np.testing.assert_allclose(J[4, 2], -q[KA] / q[TA] * dvt_de, rtol=1e-6)


@pytest.mark.parametrize("kw", SMIB_CASES + [dict(KA=200.0, KF=0.02, TF=0.3, TE=0.1, KE=0.5)])
def test_exciter_characteristic_polynomial(kw):
    """The (Efd, VR, RF) block of the Jacobian has the roots of
    (KE + s TE)(1 + s TA)(1 + s TF) + KA KF s, the closed-loop polynomial of
    the type-1 block diagram."""
    sc = workloads.smib_fluxdecay(**kw)
    q = sc["model_params"][0]
    y0, _ = oracle.initial_state(sc)
    J = jacobian(sc, y0)
    blk = J[np.ix_([3, 4, 5], [3, 4, 5])]
    ev = np.sort_complex(np.linalg.eigvals(blk))
    poly = np.polymul(np.polymul([q[TE], q[KE]], [q[TA], 1.0]), [q[TF], 1.0])
    poly = np.polyadd(poly, [q[KA] * q[KF], 0.0])
    roots = np.sort_complex(np.roots(poly))
    np.testing.assert_allclose(ev, roots, rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("n", [1, 10, 50])
def test_equilibrium(n):
    """At the operating point every derivative vanishes; with sigma = 0 the
    statistics are constant with zero variance."""
    sc = (workloads.smib_fluxdecay() if n == 1 else
          workloads.fluxdecay(n_gen=n, n_dist=min(5, n - 1), N=8, K=10, T=0.5, dt=0.01))
    y0, _ = oracle.initial_state(sc)
    f = oracle.rhs(sc, y0, np.zeros(len(sc["dist"]["gen"])))
    assert np.abs(f).max() <= 1e-12
    sc0 = dict(sc, dist=dict(sc["dist"], sigma=np.zeros(len(sc["dist"]["gen"]))), N=8)
    o = oracle.run(sc0)
    assert np.abs(o["var"]).max() <= 1e-24
    assert np.abs(o["mean"] - y0).max() <= 1e-11


def test_classical_limit():
    """With T'do and TE huge and KA = 0, E'q stays at E and the machine angles,
    speeds and disturbances follow the classical model on the same noise."""
    sc = workloads.fluxdecay(n_gen=12, n_dist=4, N=16, K=20, T=1.0, dt=0.01)
    sc["model_params"][:, TDO] = 1e13
    sc["model_params"][:, TE] = 1e13
    sc["model_params"][:, KA] = 0.0
    fd = oracle.run(sc, want_traj=True)["traj"]
    cl = oracle.run(dict(sc, model="classical", model_params=None), want_traj=True)["traj"]
    n, P = 12, 4
    np.testing.assert_allclose(fd[:, :, :2 * n], cl[:, :, :2 * n], rtol=0, atol=1e-9)
    np.testing.assert_allclose(fd[:, :, 6 * n:], cl[:, :, 2 * n:], rtol=0, atol=1e-15)
    assert np.abs(fd[:, :, 2 * n:3 * n] - sc["E"]).max() <= 1e-9


def test_fluxdecay_rejects_bad_parameters():
    sc = workloads.smib_fluxdecay()
    bad = sc["model_params"].copy(); bad[0, TDO] = 0.0
    with pytest.raises(RuntimeError):
        oracle.run(dict(sc, model_params=bad))
    with pytest.raises(RuntimeError):
        oracle.run(dict(sc, integrator="trap"))
