"""Pins of the oracle's network events (the paper's case study trips a
generator at t = 1 s and evaluates the RMS frequency deviation, Sec. V-B):
from the event step on, the reduced admittance is the post-event one, and a
tripped machine loses its mechanical power and injections.

  * A line switch on the single machine against an infinite bus (X -> X2 at
    t_e), without damping or noise: the swing energy
    W = H w_b dw^2 - Pm delta - (E V / X2) cos(delta) is constant after the
    event, and the state is the operating point before it.
  * A small line switch with damping: the deviation from the new equilibrium
    follows the linearised closed form x(t) = x0 e^{-a t}(cos w_d t +
    (a / w_d) sin w_d t).
  * A generator trip on a lossy network: the post-event right-hand side at
    random states against the textbook real form on the network reduced by a
    plain numpy full-network solve without the tripped machine; the tripped
    machine only decays, d dw/dt = -D dw / 2H.
"""
import math

import numpy as np
import pytest

import oracle
import workloads

WB = 2 * math.pi * 60.0


def smib_switch(X1=0.5, X2=0.7, D=0.0, sigma=0.0, t_e=1.0, T=6.0, dt=0.001, **kw):
    sc = workloads.smib(N=2, K=4, T=T, dt=dt, sigma=sigma, D=D, X=X1, **kw)
    y2 = 1.0 / (1j * X2)
    sc["event"] = dict(t=t_e, Y=np.array([[y2]]), Yinf=np.array([-y2]))
    return sc


def test_smib_line_switch_conserves_swing_energy():
    sc = smib_switch()
    r = oracle.run(sc, zeta=np.zeros((4, 2)), want_traj=True)
    tr = r["traj"][0]
    d0 = r["delta0"][0]
    s_e = int(round(1.0 / sc["dt"]))
    # before the event: the operating point (Pe = Pm for X1)
    assert np.max(np.abs(tr[:s_e + 1, 0] - d0)) < 1e-12
    assert np.max(np.abs(tr[:s_e + 1, 1])) < 1e-12
    H, Pm, E = 3.5, 0.8, 1.1
    pmax2 = E * 1.0 / 0.7
    W = H * WB * tr[s_e:, 1] ** 2 - Pm * tr[s_e:, 0] - pmax2 * np.cos(tr[s_e:, 0])
    scale = Pm * abs(d0) + pmax2
    assert np.max(np.abs(W - W[0])) <= 1e-9 * scale, np.max(np.abs(W - W[0]))
    # it swings: the angle moves well away from the old operating point
    assert tr[s_e:, 0].max() - d0 > 0.1


def test_smib_small_line_switch_matches_linear_closed_form():
    eps = 1e-3
    X1, D = 0.5, 2.0
    X2 = X1 * (1 + eps)
    sc = smib_switch(X1=X1, X2=X2, D=D, T=5.0, dt=0.001)
    r = oracle.run(sc, zeta=np.zeros((4, 2)), want_traj=True)
    tr = r["traj"][0]
    H, Pm, E = 3.5, 0.8, 1.1
    d0 = math.asin(Pm * X1 / E)
    d1 = math.asin(Pm * X2 / E)
    Ks = E / X2 * math.cos(d1)
    a = D / (4 * H)
    wn2 = WB * Ks / (2 * H)
    wd = math.sqrt(wn2 - a * a)
    s_e = 1000
    t = (np.arange(tr.shape[0] - s_e)) * sc["dt"]
    x0 = d0 - d1
    lin = x0 * np.exp(-a * t) * (np.cos(wd * t) + a / wd * np.sin(wd * t))
    err = np.max(np.abs(tr[s_e:, 0] - d1 - lin))
    assert err <= 5 * eps * abs(x0), (err, abs(x0))


def _reduced_numpy(net):
    """Y_red = Y_AA - Y_AB Y_BB^-1 Y_BA of the full network (generator internal
    nodes kept, buses eliminated), by a plain dense solve."""
    nb, ng = net["n_bus"], net["n_gen"]
    Y = np.zeros((ng + nb, ng + nb), dtype=complex)
    for f, t, rr, x in zip(net["br_from"], net["br_to"], net["br_r"], net["br_x"]):
        y = 1 / (rr + 1j * x)
        Y[ng + f, ng + f] += y; Y[ng + t, ng + t] += y
        Y[ng + f, ng + t] -= y; Y[ng + t, ng + f] -= y
    for b in range(nb):
        Y[ng + b, ng + b] += net["load_g"][b] + 1j * net["load_b"][b]
    for g, (b, xd) in enumerate(zip(net["gen_bus"], net["gen_xdp"])):
        y = 1 / (1j * xd)
        Y[g, g] += y; Y[ng + b, ng + b] += y
        Y[g, ng + b] -= y; Y[ng + b, g] -= y
    return Y[:ng, :ng] - Y[:ng, ng:] @ np.linalg.solve(Y[ng:, ng:], Y[ng:, :ng])


@pytest.mark.parametrize("g", [0, 2])
def test_generator_trip_post_event_rhs(g):
    sc = workloads.multimachine(n_gen=4, n_dist=3, N=4, K=5, T=0.5, dt=0.005, net_seed=44, seed=1)
    sc["event"] = dict(t=0.1, tripped=g)
    n = sc["n_gen"]
    net = sc["net"]
    keep = [k for k in range(n) if k != g]
    Ysmall = _reduced_numpy(dict(net, n_gen=n - 1, gen_bus=np.asarray(net["gen_bus"])[keep],
                                 gen_xdp=np.asarray(net["gen_xdp"])[keep]))
    Yp = oracle.post_event_admittance(sc)
    np.testing.assert_allclose(Yp[np.ix_(keep, keep)], Ysmall, rtol=1e-11, atol=1e-11)
    assert np.all(Yp[g, :] == 0) and np.all(Yp[:, g] == 0)
    # Pm of the pre-event operating point (the oracle's, pinned elsewhere)
    Pm = oracle.run(sc, zeta=np.zeros((15, 4)))["Pm"]
    d = sc["dist"]
    rng = np.random.default_rng(g)
    E, H, D = sc["E"], sc["H"], sc["D"]
    for _ in range(6):
        delta = sc["delta0"] + rng.uniform(-0.5, 0.5, n)
        dw = rng.uniform(-0.01, 0.01, n)
        xi = rng.uniform(-0.2, 0.2, 3)
        w = rng.normal(size=3)
        y = np.concatenate([delta, dw, xi])
        got = oracle.rhs_post(sc, y, w)
        ref = np.zeros_like(y)
        ref[:n] = WB * dw
        for i in range(n):
            if i == g:
                ref[n + i] = -D[i] * dw[i] / (2 * H[i])
                continue
            pe = sum(E[i] * E[k] * (Yp[i, k].real * math.cos(delta[i] - delta[k]) +
                                    Yp[i, k].imag * math.sin(delta[i] - delta[k])) for k in range(n))
            inj = sum(xi[p] for p in range(3) if d["gen"][p] == i)
            ref[n + i] = (Pm[i] + inj - pe - D[i] * dw[i]) / (2 * H[i])
        ref[2 * n:] = -d["theta"] * xi + d["sigma"] * w
        np.testing.assert_allclose(got, ref, rtol=1e-11, atol=1e-12)


def test_event_run_equals_plain_run_before_the_event():
    sc = workloads.config2(N=8, K=20, T=0.5)
    ev = dict(sc, event=dict(t=0.25, tripped=3))
    a = oracle.run(sc, want_traj=True)["traj"]
    b = oracle.run(ev, want_traj=True)["traj"]
    s_e = 50
    assert np.array_equal(a[:, :s_e + 1], b[:, :s_e + 1])
    assert np.max(np.abs(a[:, -1] - b[:, -1])) > 1e-3


def test_event_rejections():
    sc = workloads.config2(N=4, K=5, T=0.5)
    for t in (0.5, 0.6, 0.1234):  # at or beyond T, not a whole number of steps
        with pytest.raises(RuntimeError):
            oracle.run(dict(sc, event=dict(t=t, tripped=1)))
    with pytest.raises(RuntimeError):
        oracle.run(dict(sc, event=dict(t=0.25, tripped=10, Y=np.zeros((10, 10)))))
