"""Pins of the oracle's general Ito disturbances (eq. 4 with state-dependent
drift and diffusion; the rows of Table I; the wind model of eq. 11), CPU only.

The process does not feed back from the machines, so its column of the
outputs is the disturbance alone.  What fixes the expected values:

  * For a drift that is linear in xi (every row of Table I) and a squared
    diffusion g(xi) = g0 + g1 xi + g2 xi^2, Ito's formula closes the first two
    moments:  m1' = -theta (m1 - m),  m2' = 2 E[xi mu] + E[g]  -- a linear ODE
    solved here by a matrix exponential (scipy).  The oracle's KLE paths with
    the Ito correction must reproduce these within sampling error; without it
    (Stratonovich) the Gamma row's mean moves to a/b + 1/(2b), the Ito mean
    of the corrected drift -- the calculus question settled numerically.
  * The Laplace row's stationary variance is 2 b^2 (its density's variance).
  * The Gaussian row is an OU process around a: with the same rate, the
    diffusion sqrt(2 theta b) and the injection taken relative to a, the run
    equals the OU run to rounding.
  * The wind model (eq. 11) against a plain numpy Euler-Maruyama simulation
    of eq. 5 (independent code, many more samples), mean and variance.
  * The traditional Monte Carlo basis (one normal per step at the midpoint
    stages) carries its own noise-induced drift, (3/8) sigma sigma'; with that
    correction its Gamma mean follows the Ito closed form too.
"""
import numpy as np
import pytest
from scipy.linalg import expm

import oracle
import workloads

XI = 2  # output column of the process in a single-machine scenario (delta, dw, xi)


def moments(theta, m, g, x0, ts):
    """(mean, variance) at times ts of d xi = -theta (xi - m) dt + sqrt(g(xi)) dW
    (Ito), g = g0 + g1 xi + g2 xi^2, from the closed moment equations."""
    g0, g1, g2 = g
    A = np.array([[-theta, 0.0, theta * m],
                  [2.0 * theta * m + g1, -2.0 * theta + g2, g0],
                  [0.0, 0.0, 0.0]])
    out = []
    for t in ts:
        v = expm(A * t) @ np.array([x0, x0 * x0, 1.0])
        out.append((v[0], v[1] - v[0] ** 2))
    return np.array(out)


def process_run(spec, x0, T=3.0, dt=0.005, K=150, N=4000, calculus="ito", basis="paper",
                sampler="lhs", seed=5):
    sc = workloads.smib(N=N, K=K, T=T, dt=dt, seed=seed, basis=basis, sampler=sampler)
    sc = workloads.with_processes(sc, [dict(spec, gain=0.0)], calculus=calculus, xi0=[x0])
    r = oracle.run(sc)
    return r["mean"][:, XI], r["var"][:, XI]


def test_gamma_row_ito_moments_and_stratonovich_shift():
    a, b, th, x0, dt = 4.0, 2.0, 1.0, 1.0, 0.005
    spec = dict(kind="gamma", a=a, b=b, theta=th)
    ts = np.array([1.0, 2.0, 3.0])
    idx = np.round(ts / dt).astype(int)
    ref = moments(th, a / b, (0.0, 2.0 * th / b, 0.0), x0, ts)
    mean, var = process_run(spec, x0)
    # sampling: std of xi below 1, N = 4000 LHS samples
    assert np.max(np.abs(mean[idx] - ref[:, 0])) < 0.015
    assert np.max(np.abs(var[idx] / ref[:, 1] - 1.0)) < 0.08
    # the KLE ODE as written converges to the Stratonovich solution, whose Ito
    # drift is mu + sigma sigma'/2 = -theta (xi - (a/b + 1/(2b)))
    ms = a / b + 1.0 / (2.0 * b)
    mean_s, _ = process_run(spec, x0, calculus="stratonovich")
    ref_s = ms + (x0 - ms) * np.exp(-th * ts)
    assert np.max(np.abs(mean_s[idx] - ref_s)) < 0.015
    assert np.min(np.abs(mean_s[idx] - ref[:, 0])) > 0.1  # the two calculi differ


def test_beta_row_ito_moments():
    a, b, th, x0, dt, T = 2.0, 3.0, 0.5, 0.1, 0.005, 4.0
    c = 2.0 * th / (a + b)
    ts = np.array([2.0, 4.0])
    idx = np.round(ts / dt).astype(int)
    ref = moments(th, a / (a + b), (0.0, c, -c), x0, ts)
    mean, var = process_run(dict(kind="beta", a=a, b=b, theta=th), x0, T=T)
    assert np.max(np.abs(mean[idx] - ref[:, 0])) < 0.004
    assert np.max(np.abs(var[idx] / ref[:, 1] - 1.0)) < 0.05
    # the stationary Beta(a, b) variance is approached
    assert abs(ref[-1, 1] - a * b / ((a + b) ** 2 * (a + b + 1))) < 0.01


def test_laplace_row_stationary_variance():
    a, b, th = 0.5, 0.2, 2.0
    mean, var = process_run(dict(kind="laplace", a=a, b=b, theta=th), a, T=3.0)
    assert abs(mean[-1] - a) < 0.01          # symmetric about a: the mean stays
    assert abs(var[-1] / (2 * b * b) - 1.0) < 0.06
    # without the correction the diffusion's kink pushes mass outwards
    _, var_s = process_run(dict(kind="laplace", a=a, b=b, theta=th), a, T=3.0,
                           calculus="stratonovich")
    assert var_s[-1] / (2 * b * b) > 1.2


def test_gaussian_row_is_ou_about_its_mean():
    a, b, th, x0 = 0.7, 0.004, 0.5, 0.03
    base = workloads.smib(N=64, K=40, T=4.0, dt=0.01)
    ou = workloads.with_processes(base, [dict(kind="ou")], xi0=[x0])
    ou["dist"]["theta"] = np.array([th])
    ou["dist"]["sigma"] = np.array([np.sqrt(2 * th * b)])
    ga = workloads.with_processes(base, [dict(kind="gauss", a=a, b=b, theta=th, ref=a)],
                                  xi0=[a + x0])
    r0 = oracle.run(ou, want_traj=True)["traj"]
    r1 = oracle.run(ga, want_traj=True)["traj"]
    assert np.max(np.abs((r1[..., XI] - a) - r0[..., XI])) < 1e-13
    assert np.max(np.abs(r1[..., :XI] - r0[..., :XI])) < 1e-11
    # and the machine sees the process (the run is not the undisturbed one)
    assert np.max(np.abs(r0[..., 1])) > 1e-4


def _euler_maruyama_wind(N, T, h, x0, seed):
    """Eq. 5 for eq. 11, in numpy: x <- x + h mu(x) + sigma(x) sqrt(h) z."""
    rng = np.random.default_rng(seed)
    m0, m1, m2 = workloads.WIND_MU
    s0, s1, s2 = workloads.WIND_SIGMA
    x = np.full(N, x0)
    for _ in range(int(round(T / h))):
        z = rng.standard_normal(N)
        x = x + h * (m0 + m1 * x + m2 * x * x) + (s0 + s1 * x + s2 * x * x) * np.sqrt(h) * z
    return x


def test_wind_model_against_euler_maruyama():
    T, x0 = 20.0, 0.85
    em = _euler_maruyama_wind(200_000, T, 0.005, x0, seed=3)
    sc = workloads.wind_smib(N=4000, K=60, T=T, dt=0.02, P0=x0, gain=0.0)
    r = oracle.run(sc)
    m, v = r["mean"][-1, XI], r["var"][-1, XI]
    se_m = np.sqrt(em.var() / 200_000) + np.sqrt(v / 4000)
    assert abs(m - em.mean()) < 4 * se_m + 2e-4
    assert abs(v / em.var() - 1.0) < 0.06
    # the process moved: its variance at T is far above the start's zero
    assert v > 1e-4


def test_em_basis_carries_its_own_correction():
    """The one-hot (traditional Monte Carlo) basis with the 3/8 correction:
    the Gamma row's mean follows the Ito closed form (the smooth-basis 1/2
    would leave a bias of about -0.054 at t = 2)."""
    a, b, th, x0, dt, T = 4.0, 2.0, 1.0, 1.0, 0.004, 2.0
    S = int(round(T / dt))
    mean, _ = process_run(dict(kind="gamma", a=a, b=b, theta=th), x0, T=T, dt=dt, K=S,
                          N=4000, basis="em")
    ref = moments(th, a / b, (0.0, 2.0 * th / b, 0.0), x0, [1.0, 2.0])[:, 0]
    assert np.max(np.abs(mean[[S // 2, S]] - ref)) < 0.025


def test_process_injection_gain_and_reference():
    """gain (xi - ref) enters the machine's power balance: with the process
    held at ref the machine stays at its operating point; a unit step of xi
    accelerates the rotor by gain / 2H."""
    base = workloads.smib(N=2, K=4, T=1.0, dt=0.01)
    sc = workloads.with_processes(base, [dict(kind="gauss", a=0.5, b=0.0, theta=0.0,
                                              gain=3.0, ref=0.5)], xi0=[0.5])
    tr = oracle.run(sc, zeta=np.zeros((4, 2)), want_traj=True)["traj"][0]
    assert np.max(np.abs(tr[:, 1])) < 1e-14 and np.max(np.abs(tr[:, XI] - 0.5)) < 1e-15
    d0 = tr[0, 0]
    y = np.array([d0, 0.0, 1.5])
    dy = oracle.rhs(sc, y, np.zeros(1))
    assert abs(dy[1] - 3.0 * 1.0 / (2 * 3.5)) < 1e-12


def test_rejections():
    base = workloads.smib(N=4, K=4, T=0.2, dt=0.01)
    g = dict(kind="gamma", a=2.0, b=1.0, theta=1.0)
    for sc in (workloads.with_processes(dict(base, integrator="trap"), [g]),
               workloads.with_processes(base, [dict(g, a=-1.0)]),
               workloads.with_processes(base, [dict(kind="beta", a=1.0, b=0.0, theta=1.0)]),
               workloads.with_processes(base, [dict(g, kind=9)]),
               dict(workloads.with_processes(base, [g]), calculus=7)):
        with pytest.raises(RuntimeError):
            oracle.run(sc)
    sm = workloads.with_processes(base, [g])
    sm["dist"]["sigma_mat"] = np.eye(1)
    with pytest.raises(RuntimeError):
        oracle.run(sm)
