"""Seeded synthetic workloads (inputs only).

This module is shared by the tests, the benchmark, the product binding's callers
and the oracle's callers.  It draws scenario descriptions from a seed and holds
none of the method's arithmetic: no network reduction, no equilibrium, no
sampling design, no integration.  Operating-point quantities that depend on the
method (the reduced admittance, Pm of the multimachine systems, delta0 of the
infinite-bus system) are left for each side to compute.

The synthetic networks stand in for the IEEE 39-bus system of the paper's case
study (Sec. V-A): they have its shape (39 buses, 10 generators, 46 branches, one
large-inertia equivalent machine) and nothing else of it.

Scenario dict keys (consumed by both ``oracle.run`` and the product binding):
  n_gen, f0, H, D, E [n], delta0 [n] or None, Pm [n] or None,
  Y (complex [n, n]) or None, net (network dict) when Y is None,
  infinite_bus, V_inf, Yinf (complex [n]),
  dist = {gen [P] int, theta [P], sigma [P], xi0 [P] or None, and optionally
          proc [P] (general Ito processes: dicts with kind 'ou' | 'gauss' |
          'beta' | 'gamma' | 'laplace' (Table I rows, with a, b, theta) |
          'poly' (mu and sg, three polynomial coefficients each, eq. 11), and
          gain, ref: the process enters its machine's power as gain (xi - ref))},
  calculus ('ito' | 'stratonovich'),
  T, dt, K, N, seed, basis ('paper'|'eigen'), sampler ('lhs'|'srs'),
  integrator ('rk4'|'trap'), ddof, and optionally model ('classical' |
  'fluxdecay') with model_params [n, 9] (Xd, X'd, T'do, KA, TA, KE, TE, KF, TF).
Network dict keys: n_bus, n_gen, br_from, br_to, br_r, br_x, br_b, load_g,
  load_b, gen_bus, gen_xdp.
"""
from __future__ import annotations

import numpy as np


def smib(N=1000, K=40, T=10.0, dt=0.01, seed=1, theta=0.5, sigma=0.05, H=3.5, D=2.0,
         Pm=0.8, E=1.1, X=0.5, basis="paper", sampler="lhs", integrator="rk4"):
    """Single machine against an infinite bus (1.0 at angle 0) through X.

    The classical model with one OU disturbance on Pm.  The defaults are the
    1000-sample, K=40, 1000-step parity workload.  delta0 is left for the
    method to solve (Pe(delta0) = Pm).
    """
    y = 1.0 / (1j * X)
    return dict(
        n_gen=1, f0=60.0, H=np.array([H]), D=np.array([D]), E=np.array([E]),
        delta0=None, Pm=np.array([Pm]), Y=np.array([[y]]), net=None,
        infinite_bus=True, V_inf=1.0, Yinf=np.array([-y]),
        dist=dict(gen=np.array([0], dtype=np.int32), theta=np.array([theta]),
                  sigma=np.array([sigma]), xi0=None),
        T=T, dt=dt, K=K, N=N, seed=seed, basis=basis, sampler=sampler,
        integrator=integrator, ddof=1)


def network(n_gen: int, seed: int, n_bus: int | None = None, n_branch: int | None = None):
    """Random connected network with generator internal nodes.

    Recipe: a random spanning tree over the buses plus random extra edges up to
    n_branch; X ~ U[0.01, 0.1] pu, R = 0.1 X, no line charging; generators on
    n_gen distinct random buses with X'd ~ U[0.02, 0.1]; constant-impedance
    loads P_L ~ U[0.5, 5], Q_L = 0.3 P_L (shunt g = P_L, b = -Q_L at 1 pu) on
    every non-generator bus.  Defaults follow the 39-bus shape: n_bus =
    round(3.9 n_gen), n_branch = round(1.18 n_bus).
    """
    rng = np.random.default_rng(seed)
    if n_bus is None:
        n_bus = max(int(round(3.9 * n_gen)), n_gen + 1)
    if n_branch is None:
        n_branch = max(int(round(1.18 * n_bus)), n_bus - 1)
    order = rng.permutation(n_bus)
    edges = set()
    br = []
    for k in range(1, n_bus):
        a = int(order[k]); b = int(order[rng.integers(0, k)])
        key = (min(a, b), max(a, b))
        edges.add(key)
        br.append(key)
    max_edges = n_bus * (n_bus - 1) // 2
    while len(br) < min(n_branch, max_edges):
        a, b = (int(v) for v in rng.integers(0, n_bus, size=2))
        if a == b:
            continue
        key = (min(a, b), max(a, b))
        if key in edges:
            continue
        edges.add(key)
        br.append(key)
    br = np.array(br, dtype=np.int32)
    x = rng.uniform(0.01, 0.1, size=len(br))
    gen_bus = rng.choice(n_bus, size=n_gen, replace=False).astype(np.int32)
    xdp = rng.uniform(0.02, 0.1, size=n_gen)
    PL = rng.uniform(0.5, 5.0, size=n_bus)
    is_gen = np.zeros(n_bus, dtype=bool)
    is_gen[gen_bus] = True
    PL[is_gen] = 0.0
    return dict(n_bus=n_bus, n_gen=n_gen, br_from=br[:, 0].copy(), br_to=br[:, 1].copy(),
                br_r=0.1 * x, br_x=x, br_b=np.zeros(len(br)), load_g=PL, load_b=-0.3 * PL,
                gen_bus=gen_bus, gen_xdp=xdp)


def multimachine(n_gen=10, n_dist=3, N=10_000, K=100, T=20.0, dt=0.005, net_seed=39, seed=2,
                 n_bus=None, n_branch=None, basis="paper", sampler="lhs", integrator="rk4"):
    """Classical multimachine system on a seeded synthetic network.

    H ~ U[3, 10] s with the last machine an H = 500 s equivalent, D = 2 pu,
    E ~ U[1.0, 1.1], delta0 ~ U[-0.25, 0.25] (0 for the equivalent);
    Pm is left to the method (equilibrium: Pm := Pe(delta0)).  n_dist OU
    disturbances at distinct non-equivalent machines, theta ~ U[0.2, 1] 1/s,
    sigma ~ U[0.02, 0.1] pu.  Defaults: the 10-machine, 39-bus, N = 1e4,
    K = 100, 4000-step workload.
    """
    net = network(n_gen, net_seed, n_bus, n_branch)
    rng = np.random.default_rng(net_seed + 1_000_003)
    H = rng.uniform(3.0, 10.0, size=n_gen)
    H[-1] = 500.0
    E = rng.uniform(1.0, 1.1, size=n_gen)
    d0 = rng.uniform(-0.25, 0.25, size=n_gen)
    d0[-1] = 0.0
    cand = np.arange(n_gen - 1) if n_gen > 1 else np.arange(1)
    n_dist_eff = min(n_dist, len(cand))
    gen = np.sort(rng.choice(cand, size=n_dist_eff, replace=False)).astype(np.int32)
    if n_dist > n_dist_eff:  # more processes than machines: reuse machines
        extra = rng.choice(cand, size=n_dist - n_dist_eff, replace=True).astype(np.int32)
        gen = np.concatenate([gen, extra])
    theta = rng.uniform(0.2, 1.0, size=n_dist)
    sigma = rng.uniform(0.02, 0.1, size=n_dist)
    return dict(
        n_gen=n_gen, f0=60.0, H=H, D=np.full(n_gen, 2.0), E=E, delta0=d0, Pm=None,
        Y=None, net=net, infinite_bus=False, V_inf=1.0, Yinf=None,
        dist=dict(gen=gen, theta=theta, sigma=sigma, xi0=None),
        T=T, dt=dt, K=K, N=N, seed=seed, basis=basis, sampler=sampler,
        integrator=integrator, ddof=1)


def fluxdecay(n_gen=200, n_dist=10, N=50_000, K=100, T=30.0, dt=0.005, net_seed=200, seed=6,
              n_bus=None, n_branch=None, basis="paper", sampler="lhs"):
    """One-axis (flux-decay) machines with IEEE type-1 exciters on a seeded
    synthetic network: the large requests of the served workload (200
    machines, 10 OU disturbances, T = 30 s, N = 5e4, K = 100 by default).

    Machine data as ``multimachine`` (E is E'q at t = 0) plus, per machine,
    X'd from the network, Xd = X'd * U[4, 8], T'do ~ U[4, 8] s, KA ~ U[10, 25],
    TA ~ U[0.02, 0.1] s, KE = 1, TE ~ U[0.3, 0.8] s, KF ~ U[0.08, 0.15],
    TF ~ U[0.5, 1.5] s (gains chosen so that the linearised systems are stable).
    The method sets Efd, VR, RF and Vref at equilibrium.
    """
    sc = multimachine(n_gen=n_gen, n_dist=n_dist, N=N, K=K, T=T, dt=dt, net_seed=net_seed,
                      seed=seed, n_bus=n_bus, n_branch=n_branch, basis=basis, sampler=sampler)
    rng = np.random.default_rng(net_seed + 2_000_029)
    xdp = sc["net"]["gen_xdp"]
    mp = np.zeros((n_gen, 9))
    mp[:, 0] = xdp * rng.uniform(4.0, 8.0, size=n_gen)
    mp[:, 1] = xdp
    mp[:, 2] = rng.uniform(4.0, 8.0, size=n_gen)
    mp[:, 3] = rng.uniform(10.0, 25.0, size=n_gen)
    mp[:, 4] = rng.uniform(0.02, 0.1, size=n_gen)
    mp[:, 5] = 1.0
    mp[:, 6] = rng.uniform(0.3, 0.8, size=n_gen)
    mp[:, 7] = rng.uniform(0.08, 0.15, size=n_gen)
    mp[:, 8] = rng.uniform(0.5, 1.5, size=n_gen)
    sc.update(model="fluxdecay", model_params=mp)
    return sc


def smib_fluxdecay(Xe=0.4, Xd=1.6, Xdp=0.3, Tdo=6.0, KA=30.0, TA=0.05, KE=1.0, TE=0.5,
                   KF=0.05, TF=1.0, H=3.5, D=2.0, E=1.1, delta0=0.6, V_inf=1.0, **kw):
    """One flux-decay machine behind X'd against an infinite bus through Xe
    (reduced to the internal node), one OU disturbance on Pm."""
    X = Xdp + Xe
    y = 1.0 / (1j * X)
    d = dict(N=64, K=20, T=1.0, dt=0.01, seed=1, theta=0.5, sigma=0.05)
    d.update(kw)
    return dict(
        n_gen=1, f0=60.0, H=np.array([H]), D=np.array([D]), E=np.array([E]),
        delta0=np.array([delta0]), Pm=None, Y=np.array([[y]]), net=None,
        infinite_bus=True, V_inf=V_inf, Yinf=np.array([-y]),
        dist=dict(gen=np.array([0], dtype=np.int32), theta=np.array([d["theta"]]),
                  sigma=np.array([d["sigma"]]), xi0=None),
        T=d["T"], dt=d["dt"], K=d["K"], N=d["N"], seed=d["seed"], basis="paper",
        sampler="lhs", integrator="rk4", ddof=1, model="fluxdecay",
        model_params=np.array([[Xd, Xdp, Tdo, KA, TA, KE, TE, KF, TF]]))


# The polynomial Ito model of the per-unit wind power identified in the
# paper's case study (eq. 11): drift and diffusion coefficients of 1, P, P^2.
WIND_MU = (0.0535, -0.0899, 0.0349)
WIND_SIGMA = (-0.410, 0.919, -0.505)


def with_processes(sc: dict, specs, calculus: str = "ito", xi0=None) -> dict:
    """A copy of scenario ``sc`` whose P disturbances are the general Ito
    processes ``specs`` (one dict per process, module docstring), with the
    initial values ``xi0`` (default: zero)."""
    d = dict(sc["dist"])
    P = len(d["gen"])
    assert len(specs) == P
    d["proc"] = [dict(s) for s in specs]
    if xi0 is not None:
        d["xi0"] = np.asarray(xi0, dtype=np.float64).reshape(P)
    out = dict(sc, dist=d, calculus=calculus)
    return out


def wind_smib(N=1000, K=100, T=60.0, dt=0.01, seed=11, gain=1.0, P0=0.9, **kw):
    """The single machine driven by the wind model of eq. 11: the wind power
    P_t starts at P0 and enters the machine as gain (P_t - P0), so that t = 0
    is the operating point."""
    sc = smib(N=N, K=K, T=T, dt=dt, seed=seed, **kw)
    spec = dict(kind="poly", mu=WIND_MU, sg=WIND_SIGMA, gain=gain, ref=P0)
    return with_processes(sc, [spec], xi0=[P0])


def wind_trip(N=1000, K=6, T=60.0, dt=0.01, seed=21, gain=10.0, P0=0.9, tripped=3, t_trip=1.0,
              **kw):
    """The case-study shape of the paper (Sec. V-B) on the 10-machine
    synthetic system: one wind process of eq. 11 (per unit of the farm's
    rating) entering a machine as gain (P_t - P0), and a generator trip at
    t_trip; the response is the RMS of the centre-of-inertia frequency
    deviation over [0, T] (rrf_weights: H_i / sum H on the speed deviations).
    KLE order K = 6 as in the paper's comparison."""
    sc = multimachine(n_dist=1, N=N, K=K, T=T, dt=dt, seed=seed, **kw)
    spec = dict(kind="poly", mu=WIND_MU, sg=WIND_SIGMA, gain=gain, ref=P0)
    sc = with_processes(sc, [spec], xi0=[P0])
    sc["event"] = dict(t=t_trip, tripped=tripped)
    return sc


def coi_frequency_weights(sc: dict):
    """rrf_weights of the centre-of-inertia frequency deviation: H_i / sum H
    on the speed deviations, zero elsewhere."""
    n = int(sc["n_gen"])
    P = len(sc["dist"]["gen"])
    w = np.zeros(2 * n + P)
    H = np.asarray(sc["H"], dtype=np.float64)
    w[n:2 * n] = H / H.sum()
    return w


def config1(**kw):
    """SMIB, N=1000, K=40, T=10 s, dt=0.01 s (1000 RK4 steps), seed 1."""
    return smib(**kw)


def config2(**kw):
    """10 machines on a 39-bus synthetic network, P=3, K=100, T=20, dt=0.005, N=1e4."""
    d = dict(n_gen=10, n_dist=3, N=10_000, K=100, T=20.0, dt=0.005, net_seed=39, seed=2)
    d.update(kw)
    return multimachine(**d)


def config2_general(**kw):
    """The 10-machine system with Table I's Beta and Gamma rows and the wind
    model of eq. 11 in place of its three OU processes (each starting at its
    reference, so t = 0 is the operating point)."""
    sc = config2(**kw)
    specs = [dict(kind="beta", a=6.0, b=9.0, theta=0.5, gain=2.0, ref=0.4),
             dict(kind="gamma", a=4.0, b=20.0, theta=1.0, gain=3.0, ref=0.2),
             dict(kind="poly", mu=WIND_MU, sg=WIND_SIGMA, gain=5.0, ref=0.85)]
    return with_processes(sc, specs, xi0=[0.4, 0.2, 0.85])


def config3(**kw):
    """The 10-machine system with N = 1e5 (mixed-precision workload), seed 3."""
    d = dict(N=100_000, seed=3)
    d.update(kw)
    return config2(**d)


def uneven_batch(n_scen=64, seed=4, dt=0.005, n_range=(3, 50), p_range=(1, 6),
                 T_range=(5.0, 30.0), K_range=(40, 150), N_range=(500, 20_000)):
    """Scenario set for the batched form: n, P, T uniform; K and N log-uniform."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(n_scen):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        P = int(rng.integers(p_range[0], p_range[1] + 1))
        T = float(np.round(rng.uniform(*T_range) / dt) * dt)
        K = int(np.round(np.exp(rng.uniform(np.log(K_range[0]), np.log(K_range[1])))))
        N = int(np.round(np.exp(rng.uniform(np.log(N_range[0]), np.log(N_range[1])))))
        out.append(multimachine(n_gen=n, n_dist=P, N=N, K=K, T=T, dt=dt,
                                net_seed=int(seed * 100_000 + 17 * s + 1), seed=int(seed * 1000 + s)))
    return out
