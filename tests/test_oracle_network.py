"""Pins of the oracle's multimachine network coupling (eqs. 1-2 instantiated as
the swing equations on the Kron-reduced network, and the one-axis machine with
its IEEE type-1 exciter) away from the operating point, with losses.

The oracle forms the electrical power in complex form, Pe_i = Re(E~_i conj(I_i))
with I = Y E~.  The checks here use the textbook real forms instead:
  Pe_i = sum_k E_i E_k (G_ik cos d_ik + B_ik sin d_ik) + E_i V (Gi_i cos d_i + Bi_i sin d_i),
its partial derivatives, and the dq stator equations of the one-axis machine
(Vd = X'd Iq, Vq = E'q - X'd Id, Pe = E'q Iq).  The dynamic check linearises the
10-machine workload with that Jacobian and solves the linear system's response
to every KLE basis function exactly by the matrix exponential (scipy), which the
oracle's small-amplitude unit responses must reproduce.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sl

import oracle
import workloads

WB = 2 * math.pi * 60.0


def lossy_system(n, seed, inf=False, P=2):
    """Random lossy, non-symmetric reduced admittance (conductances of the
    order of the susceptances' tenth), explicit delta0 and Pm (not an
    equilibrium: the checks below evaluate the right-hand side anywhere)."""
    rng = np.random.default_rng(seed)
    G = rng.uniform(-0.6, 0.6, (n, n)) + np.diag(rng.uniform(0.5, 2.0, n))
    B = rng.uniform(2.0, 8.0, (n, n)) - np.diag(rng.uniform(15.0, 30.0, n))
    Y = G + 1j * B
    gen = rng.choice(n, size=P, replace=True).astype(np.int32)
    sc = dict(n_gen=n, f0=60.0, H=rng.uniform(3, 10, n), D=rng.uniform(0.5, 3, n),
              E=rng.uniform(1.0, 1.15, n), delta0=rng.uniform(-0.4, 0.4, n),
              Pm=rng.uniform(0.2, 3.0, n), Y=Y, net=None, infinite_bus=inf, V_inf=1.03,
              Yinf=(rng.uniform(0.1, 0.5, n) - 1j * rng.uniform(2, 6, n)) if inf else None,
              dist=dict(gen=gen, theta=rng.uniform(0.2, 1.0, P), sigma=rng.uniform(0.02, 0.1, P),
                        xi0=None),
              T=1.0, dt=0.01, K=2, N=2, seed=0, basis="paper", sampler="lhs",
              integrator="rk4", ddof=1)
    return sc


def pe_textbook(sc, delta):
    n = sc["n_gen"]
    Y = np.asarray(sc["Y"])
    G, B, E = Y.real, Y.imag, sc["E"]
    pe = np.zeros(n)
    for i in range(n):
        for k in range(n):
            dik = delta[i] - delta[k]
            pe[i] += E[i] * E[k] * (G[i, k] * math.cos(dik) + B[i, k] * math.sin(dik))
        if sc["infinite_bus"]:
            gi, bi = sc["Yinf"][i].real, sc["Yinf"][i].imag
            pe[i] += E[i] * sc["V_inf"] * (gi * math.cos(delta[i]) + bi * math.sin(delta[i]))
    return pe


def dpe_textbook(sc, delta):
    """d Pe_i / d delta_k of the real form above."""
    n = sc["n_gen"]
    Y = np.asarray(sc["Y"])
    G, B, E = Y.real, Y.imag, sc["E"]
    J = np.zeros((n, n))
    for i in range(n):
        for k in range(n):
            if k == i:
                continue
            dik = delta[i] - delta[k]
            J[i, k] = E[i] * E[k] * (G[i, k] * math.sin(dik) - B[i, k] * math.cos(dik))
            J[i, i] += E[i] * E[k] * (-G[i, k] * math.sin(dik) + B[i, k] * math.cos(dik))
        if sc["infinite_bus"]:
            gi, bi = sc["Yinf"][i].real, sc["Yinf"][i].imag
            J[i, i] += E[i] * sc["V_inf"] * (-gi * math.sin(delta[i]) + bi * math.cos(delta[i]))
    return J


def swing_rhs_textbook(sc, y, w):
    n, d = sc["n_gen"], sc["dist"]
    P = len(d["gen"])
    delta, dw, xi = y[:n], y[n:2 * n], y[2 * n:]
    pe = pe_textbook(sc, delta)
    acc = sc["Pm"] - pe - sc["D"] * dw
    for p in range(P):
        acc[d["gen"][p]] += xi[p]
    return np.concatenate([WB * dw, acc / (2 * sc["H"]), -d["theta"] * xi + d["sigma"] * w])


def random_state(sc, rng):
    n, P = sc["n_gen"], len(sc["dist"]["gen"])
    return np.concatenate([sc["delta0"] + rng.uniform(-1.0, 1.0, n), rng.uniform(-0.01, 0.01, n),
                           rng.uniform(-0.2, 0.2, P)])


def test_two_machine_lossy_closed_form():
    """n = 2, no infinite bus: Pe_1 = G11 E1^2 + E1 E2 (G12 cos d12 + B12 sin d12)
    read off the oracle's right-hand side (Pm - Pe = 2H dw' at dw = 0, xi = 0)."""
    sc = lossy_system(2, 7)
    Y = sc["Y"]
    E = sc["E"]
    rng = np.random.default_rng(1)
    for _ in range(20):
        d = rng.uniform(-3, 3, 2)
        y = np.concatenate([d, np.zeros(2), np.zeros(2)])
        dy = oracle.rhs(sc, y, np.zeros(2))
        pe = sc["Pm"] - 2 * sc["H"] * dy[2:4]
        d12 = d[0] - d[1]
        pe1 = Y[0, 0].real * E[0] ** 2 + E[0] * E[1] * (Y[0, 1].real * math.cos(d12) +
                                                        Y[0, 1].imag * math.sin(d12))
        pe2 = Y[1, 1].real * E[1] ** 2 + E[1] * E[0] * (Y[1, 0].real * math.cos(-d12) +
                                                        Y[1, 0].imag * math.sin(-d12))
        assert abs(pe[0] - pe1) <= 1e-12 * (1 + abs(pe1))
        assert abs(pe[1] - pe2) <= 1e-12 * (1 + abs(pe2))


@pytest.mark.parametrize("n,inf", [(3, False), (3, True), (10, False), (10, True)])
def test_swing_rhs_matches_real_form(n, inf):
    """Every component of the right-hand side at random states far from the
    operating point (angles moved by up to 1 rad, speed deviations, disturbance
    values and white-noise inputs), lossy non-symmetric Y, with and without an
    infinite bus."""
    sc = lossy_system(n, 100 + n, inf=inf, P=3)
    rng = np.random.default_rng(n)
    for _ in range(10):
        y = random_state(sc, rng)
        w = rng.normal(size=3)
        got = oracle.rhs(sc, y, w)
        ref = swing_rhs_textbook(sc, y, w)
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("n,inf", [(3, True), (10, False)])
def test_swing_jacobian_matches_real_form_and_differences(n, inf):
    sc = lossy_system(n, 200 + n, inf=inf, P=3)
    rng = np.random.default_rng(5)
    P = 3
    ny = 2 * n + P
    for _ in range(5):
        y = random_state(sc, rng)
        J = oracle.rhs_jac(sc, y)
        ref = np.zeros((ny, ny))
        ref[:n, n:2 * n] = WB * np.eye(n)
        ref[n:2 * n, :n] = -dpe_textbook(sc, y[:n]) / (2 * sc["H"])[:, None]
        ref[n:2 * n, n:2 * n] = np.diag(-sc["D"] / (2 * sc["H"]))
        for p, g in enumerate(sc["dist"]["gen"]):
            ref[n + g, 2 * n + p] += 1.0 / (2 * sc["H"][g])
            ref[2 * n + p, 2 * n + p] = -sc["dist"]["theta"][p]
        np.testing.assert_allclose(J, ref, rtol=1e-12, atol=1e-12)
        # and central differences of the oracle's own right-hand side
        h = 1e-6
        fd = np.zeros((ny, ny))
        for k in range(ny):
            e = np.zeros(ny); e[k] = h
            fd[:, k] = (oracle.rhs(sc, y + e, np.zeros(P)) - oracle.rhs(sc, y - e, np.zeros(P))) / (2 * h)
        np.testing.assert_allclose(J, fd, rtol=0, atol=1e-6 * np.abs(J).max())


def test_multimachine_equilibrium_solve_uses_the_coupling():
    """delta0 solved by the oracle's Newton iteration (infinite-bus systems):
    the textbook real form vanishes there for a lossy 3-machine system."""
    sc = lossy_system(3, 31, inf=True, P=1)
    # Pm from the textbook form at a known angle vector; the oracle must find it
    target = np.array([0.3, -0.1, 0.2])
    sc["Pm"] = pe_textbook(sc, target)
    sc["delta0"] = None
    r = oracle.run(dict(sc, N=2, K=1, T=0.02, dt=0.01), zeta=np.zeros((1, 2)))
    np.testing.assert_allclose(r["delta0"], target, rtol=0, atol=1e-10)


# ---------------------------------------------------------------------------
# One-axis machines with IEEE type-1 exciters: dq stator equations
# ---------------------------------------------------------------------------
def fd_rhs_textbook(sc, y, w, vref):
    n, d = sc["n_gen"], sc["dist"]
    P = len(d["gen"])
    Y = np.asarray(sc["Y"])
    G, B = Y.real, Y.imag
    q = sc["model_params"]
    Xd, Xdp, Tdo, KA, TA, KE, TE, KF, TF = (q[:, c] for c in range(9))
    delta, dw, eq, efd, vr, rf = (y[k * n:(k + 1) * n] for k in range(6))
    xi = y[6 * n:]
    Iq = np.zeros(n); Id = np.zeros(n)
    for i in range(n):
        re = im = 0.0
        for k in range(n):
            phi = delta[k] - delta[i]
            re += eq[k] * (G[i, k] * math.cos(phi) - B[i, k] * math.sin(phi))
            im += eq[k] * (G[i, k] * math.sin(phi) + B[i, k] * math.cos(phi))
        if sc["infinite_bus"]:
            gi, bi = sc["Yinf"][i].real, sc["Yinf"][i].imag
            re += sc["V_inf"] * (gi * math.cos(delta[i]) + bi * math.sin(delta[i]))
            im += sc["V_inf"] * (bi * math.cos(delta[i]) - gi * math.sin(delta[i]))
        Iq[i], Id[i] = re, -im
    pe = eq * Iq
    vt = np.hypot(Xdp * Iq, eq - Xdp * Id)
    acc = sc["Pm"] - pe - sc["D"] * dw
    for p in range(P):
        acc[d["gen"][p]] += xi[p]
    return np.concatenate([
        WB * dw, acc / (2 * sc["H"]),
        (-eq - (Xd - Xdp) * Id + efd) / Tdo,
        (-KE * efd + vr) / TE,
        (-vr + KA * rf - KA * KF / TF * efd + KA * (vref - vt)) / TA,
        (-rf + KF / TF * efd) / TF,
        -d["theta"] * xi + d["sigma"] * w])


@pytest.mark.parametrize("n,inf", [(3, True), (8, False)])
def test_fluxdecay_rhs_matches_dq_equations(n, inf):
    sc = lossy_system(n, 300 + n, inf=inf, P=2)
    rng = np.random.default_rng(9)
    mp = np.zeros((n, 9))
    mp[:, 1] = rng.uniform(0.03, 0.1, n)
    mp[:, 0] = mp[:, 1] * rng.uniform(4, 8, n)
    mp[:, 2] = rng.uniform(4, 8, n)
    mp[:, 3] = rng.uniform(10, 25, n)
    mp[:, 4] = rng.uniform(0.02, 0.1, n)
    mp[:, 5] = 1.0
    mp[:, 6] = rng.uniform(0.3, 0.8, n)
    mp[:, 7] = rng.uniform(0.08, 0.15, n)
    mp[:, 8] = rng.uniform(0.5, 1.5, n)
    sc.update(model="fluxdecay", model_params=mp)
    y0, vref = oracle.initial_state(sc)
    for _ in range(8):
        y = y0 + np.concatenate([rng.uniform(-0.8, 0.8, n), rng.uniform(-0.01, 0.01, n),
                                 rng.uniform(-0.2, 0.2, n), rng.uniform(-0.5, 0.5, n),
                                 rng.uniform(-0.5, 0.5, n), rng.uniform(-0.1, 0.1, n),
                                 rng.uniform(-0.2, 0.2, 2)])
        w = rng.normal(size=2)
        got = oracle.rhs(sc, y, w)
        ref = fd_rhs_textbook(sc, y, w, vref)
        np.testing.assert_allclose(got, ref, rtol=1e-11, atol=1e-11)


# ---------------------------------------------------------------------------
# Dynamics of the 10-machine workload: small-amplitude KLE unit responses
# against the exact response of its linearisation
# ---------------------------------------------------------------------------
def _linear_system(sc, Y):
    n, d = sc["n_gen"], sc["dist"]
    P = len(d["gen"])
    s = dict(sc, Y=Y, infinite_bus=False)
    J = dpe_textbook(s, sc["delta0"])
    ny = 2 * n + P
    A = np.zeros((ny, ny))
    A[:n, n:2 * n] = WB * np.eye(n)
    A[n:2 * n, :n] = -J / (2 * sc["H"])[:, None]
    A[n:2 * n, n:2 * n] = np.diag(-sc["D"] / (2 * sc["H"]))
    for p, g in enumerate(d["gen"]):
        A[n + g, 2 * n + p] += 1.0 / (2 * sc["H"][g])
        A[2 * n + p, 2 * n + p] = -d["theta"][p]
    return A


def _cosine_response(A, b, a, amp, times):
    """x' = A x + b amp cos(a t), x(0) = 0, at the given times, by the matrix
    exponential of the system augmented with the rotation (cos, sin)."""
    ny = A.shape[0]
    Mx = np.zeros((ny + 2, ny + 2))
    Mx[:ny, :ny] = A
    Mx[:ny, ny] = amp * b
    Mx[ny, ny + 1] = -a
    Mx[ny + 1, ny] = a
    z0 = np.zeros(ny + 2); z0[ny] = 1.0
    return np.array([(sl.expm(Mx * t) @ z0)[:ny] for t in times])


def test_ten_machine_kle_unit_responses_match_linearisation():
    K = 100
    sc = workloads.config2(K=K)
    n, P = sc["n_gen"], 3
    T = sc["T"]
    Y = oracle.kron(sc["net"])  # pinned against a full-network solve elsewhere
    A = _linear_system(sc, Y)
    ev = np.linalg.eigvals(A)
    assert np.abs(ev).max() * sc["dt"] < 0.15  # RK4 resolves every mode
    # the conductances matter in this system: the lossless Jacobian differs
    assert np.abs(Y.real).max() > 0.05 * np.abs(Y.imag).max()
    M = P * K
    eps = 1e-5
    Z = np.concatenate([eps * np.eye(M), -eps * np.eye(M)], axis=1)
    tr = oracle.run(dict(sc, N=2 * M), zeta=Z, want_traj=True)["traj"]
    r = (tr[:M] - tr[M:]) / (2 * eps)  # [M][S+1][V] responses to zeta = e_m
    times = np.array([2.0, 10.0, 20.0])
    idx = np.round(times / sc["dt"]).astype(int)
    lin = np.zeros((M, len(times), 2 * n + P))
    for p in range(P):
        b = np.zeros(2 * n + P); b[2 * n + p] = sc["dist"]["sigma"][p]
        for j in range(K):
            a = j * math.pi / T
            amp = math.sqrt(1 / T) if j == 0 else math.sqrt(2 / T)
            lin[p * K + j] = _cosine_response(A, b, a, amp, times)
    for v in range(2 * n + P):
        scale = np.abs(lin[..., v]).max()
        np.testing.assert_allclose(r[:, idx, v], lin[..., v], rtol=0, atol=2e-4 * scale,
                                   err_msg=f"output {v}")
    # K-truncated variance of every output at t = T (the quantity Alg. 1 estimates)
    var_o = np.sum(r[:, -1, :] ** 2, axis=0)
    var_l = np.sum(lin[:, -1, :] ** 2, axis=0)
    np.testing.assert_allclose(var_o, var_l, rtol=5e-4)
