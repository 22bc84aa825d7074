"""Pins of the FP64 oracle against what the paper and mathematics fix.

Nothing here compares the oracle with itself: every check is against a library
routine run at test time (numpy's Philox, scipy's ndtri/ndtr/expm/solve_ivp),
a closed form, an invariant, or brute force on tiny inputs.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.integrate as si
import scipy.linalg as sl
import scipy.special as sp

import oracle
import workloads


# --------------------------------------------------------------------------
# Philox-4x64-10 (counter-based generator, Salmon et al. SC'11)
# --------------------------------------------------------------------------
def np_philox_block(key, ctr):
    """First block numpy's Philox-4x64-10 yields for counter ``ctr``.

    numpy adds one (with carry across the four words) to the 256-bit counter
    before it produces a block, so it is seeded with ctr - 1.
    """
    c = sum(int(w) << (64 * k) for k, w in enumerate(ctr))
    kk = int(key[0]) | (int(key[1]) << 64)
    bg = np.random.Philox(key=kk, counter=(c - 1) % 2**256)
    return bg.random_raw(4)


def test_philox_matches_numpy():
    rng = np.random.default_rng(0)
    for _ in range(50):
        key = [int(v) for v in rng.integers(0, 2**63, size=2, dtype=np.int64)]
        ctr = [int(v) for v in rng.integers(0, 2**63, size=4, dtype=np.int64)]
        ref = np_philox_block(key, ctr)
        got = oracle.philox(ctr, key)
        assert np.array_equal(ref, got), (key, ctr)
    # counters whose low word is zero exercise numpy's carry
    for ctr in ([0, 0, 0, 1], [0, 5, 0, 2], [0, 0, 9, 3]):
        assert np.array_equal(np_philox_block([3, 4], ctr), oracle.philox(ctr, [3, 4]))


def test_u01_strictly_inside_unit_interval():
    lo = oracle.u01(0)
    hi = oracle.u01(2**64 - 1)
    assert lo == 0.5 * 2.0**-52
    assert hi == 1.0 - 0.5 * 2.0**-52
    assert 0.0 < lo < hi < 1.0


# --------------------------------------------------------------------------
# Inverse normal CDF (AS 241, PPND16)
# --------------------------------------------------------------------------
def test_ppnd16_vs_scipy_ndtri():
    p = np.concatenate([np.logspace(-12, -1, 400), np.linspace(0.01, 0.99, 999),
                        1.0 - np.logspace(-12, -1, 400)])
    got = oracle.ppnd16(p)
    ref = sp.ndtri(p)
    err = np.abs(got - ref) / np.maximum(np.abs(ref), 1e-3)
    assert err.max() <= 2e-15, err.max()
    # round trip through the CDF
    assert np.max(np.abs(sp.ndtr(got) - p) / np.minimum(p, 1 - p)) < 1e-12


def test_ppnd16_symmetry_and_ends():
    p = np.array([0.5, 0.25, 0.125, 2.0**-20, 2.0**-40])
    a = oracle.ppnd16(p)
    b = oracle.ppnd16(1.0 - p)
    assert a[0] == 0.0
    np.testing.assert_allclose(a, -b, rtol=1e-15, atol=0)
    assert oracle.ppnd16([0.0])[0] == -np.inf and oracle.ppnd16([1.0])[0] == np.inf


# --------------------------------------------------------------------------
# LHS (Sec. IV-B): one sample per stratum per coordinate
# --------------------------------------------------------------------------
@pytest.mark.parametrize("N", list(range(1, 40)) + [63, 64, 65, 100, 1000, 4097])
def test_strata_rows_are_permutations(N):
    st, z = oracle.lhs(seed=7, M=5, N=N)
    for row in st:
        assert np.array_equal(np.sort(row), np.arange(N))
    # zeta lies in its stratum of the CDF
    lo = sp.ndtri(st / N)
    hi = sp.ndtri((st + 1) / N)
    assert np.all(z >= lo - 1e-12 * (1 + np.abs(lo)))
    assert np.all(z <= hi + 1e-12 * (1 + np.abs(hi)))


def test_lhs_element_from_its_definition():
    """zeta = ndtri((s + U)/N) with U from numpy's Philox at (i, n, 0, JITTER=2)."""
    seed, M, N = 11, 4, 50
    st, z = oracle.lhs(seed, M, N)
    for i in range(M):
        for n in range(N):
            x = int(np_philox_block([seed, 0], [i, n, 0, 2])[0])
            U = ((x >> 12) + 0.5) * 2.0**-52
            p = (st[i, n] + U) / N
            assert abs(z[i, n] - sp.ndtri(p)) <= 2e-15 * max(1.0, abs(z[i, n]))


def test_srs_element_from_its_definition():
    seed, M, N = 5, 3, 20
    st, z = oracle.lhs(seed, M, N, sampler=1)
    assert np.all(st == -1)
    for i in range(M):
        for n in range(N):
            x = int(np_philox_block([seed, 0], [i, n, 0, 3])[0])
            U = ((x >> 12) + 0.5) * 2.0**-52
            assert abs(z[i, n] - sp.ndtri(U)) <= 2e-15 * max(1.0, abs(z[i, n]))


def test_strata_permutations_are_uniform():
    """All 24 permutations of 4 strata appear with equal frequency (chi-square)."""
    M = 24000
    st, _ = oracle.lhs(seed=3, M=M, N=4)
    perms = {p: k for k, p in enumerate(itertools.permutations(range(4)))}
    counts = np.zeros(24)
    for row in st:
        counts[perms[tuple(int(v) for v in row)]] += 1
    exp = M / 24
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert chi2 < 60.0, chi2  # 23 dof: p ~ 4e-5


@pytest.mark.parametrize("N,M", [(16, 20000), (100, 6000), (1000, 3000)])
def test_strata_permutations_are_uniform_beyond_one_bit(N, M):
    """The permutation of larger rows (N = 16: a 4-bit Feistel network;
    N = 100, 1000: cycle-walked on 8 and 10 bits): over M rows, the stratum
    of each sample is uniform over [0, N) (chi-square on the N x N position
    counts), the strata of samples 0 and 1 are a uniform pair of distinct
    values, and successive differences are uniform.  A round function that
    mixes too little leaves structure in one of these."""
    st, _ = oracle.lhs(seed=17, M=M, N=N)
    # position: counts[i][v] = rows whose sample i has stratum v
    counts = np.zeros((N, N))
    for i in range(N):
        counts[i] += np.bincount(st[:, i], minlength=N)
    exp = M / N
    chi2 = ((counts - exp) ** 2 / exp).sum()
    dof = (N - 1) ** 2
    assert abs(chi2 - dof) < 6.0 * np.sqrt(2.0 * dof), (chi2, dof)
    # pairs of samples 0 and 1 (N (N - 1) cells; for N = 1000 the pair
    # space is too large for M rows: the low decimal digits of each instead)
    a, b = st[:, 0].astype(np.int64), st[:, 1].astype(np.int64)
    assert np.all(a != b)
    if N <= 100:
        idx = a * N + b
        pc = np.bincount(idx, minlength=N * N).reshape(N, N)
        cells = pc[~np.eye(N, dtype=bool)]
        e = M / (N * (N - 1))
        chi = ((cells - e) ** 2 / e).sum()
        dof = N * (N - 1) - 1
    else:
        pc = np.bincount((a % 10) * 10 + (b % 10), minlength=100)
        e = M / 100.0
        chi = ((pc - e) ** 2 / e).sum()  # near-uniform: distinct values barely bias the digits
        dof = 99
    assert abs(chi - dof) < 6.0 * np.sqrt(2.0 * dof), (chi, dof)
    # successive differences (mod N), over all positions
    d = np.diff(st.astype(np.int64), axis=1) % N
    dc = np.bincount(d.ravel(), minlength=N)[1:]  # 0 never occurs
    e = d.size / (N - 1)
    chi = ((dc - e) ** 2 / e).sum()
    assert abs(chi - (N - 2)) < 6.0 * np.sqrt(2.0 * (N - 2)), chi


def test_lhs_row_means_are_small():
    N = 1000
    _, z = oracle.lhs(seed=1, M=40, N=N)
    assert np.abs(z.mean(axis=1)).max() <= 5.0 / N
    # the SRS design does not have this property
    _, zs = oracle.lhs(seed=1, M=40, N=N, sampler=1)
    assert np.abs(zs.mean(axis=1)).max() > 5.0 / N


def test_lhs_subset_columns_match_full_design():
    st, z = oracle.lhs(seed=9, M=6, N=300)
    sel = np.array([0, 7, 299, 150])
    st2, z2 = oracle.lhs(seed=9, M=6, N=300, sel=sel)
    assert np.array_equal(st[:, sel], st2)
    assert np.array_equal(z[:, sel], z2)


# --------------------------------------------------------------------------
# KLE basis (Sec. IV-A, eq. 7)
# --------------------------------------------------------------------------
def _trap_weights(C, h):
    w = np.full(C, h)
    w[0] = w[-1] = h / 2
    return w


@pytest.mark.parametrize("kind", [0, 1])
def test_basis_orthonormal(kind):
    """The trapezoid rule on the grid is exact for these cosine products."""
    T, S, K = 10.0, 500, 60
    Phi = oracle.basis(kind, K, S, T)
    w = _trap_weights(2 * S + 1, T / (2 * S))
    G = (Phi * w) @ Phi.T
    assert np.max(np.abs(G - np.eye(K))) < 1e-13


def _var_wk(kind, K, t, T):
    """Var W_K(t) = sum_j (int_0^t m_j)^2, written from the integrals."""
    if kind == 0:
        v = t * t / T
        for j in range(1, K):
            v += (2.0 / T) * (T / (j * math.pi) * math.sin(j * math.pi * t / T)) ** 2
        return v
    v = 0.0
    for j in range(K):
        a = (j + 0.5) * math.pi / T
        v += (2.0 / T) * (math.sin(a * t) / a) ** 2
    return v


@pytest.mark.parametrize("kind,K,t,expect", [
    (0, 6, 5.0, 4.832639), (0, 40, 5.0, 4.974675), (0, 100, 5.0, 4.989868),
    (0, 1000, 5.0, 4.998987), (0, 6, 10.0, 10.0), (0, 40, 10.0, 10.0),
    (1, 6, 10.0, 9.663037), (1, 40, 10.0, 9.949342), (1, 100, 10.0, 9.979736),
    (1, 6, 5.0, 4.831519), (1, 40, 5.0, 4.974671),
])
def test_var_wk_closed_form(kind, K, t, expect):
    """KLE identity (eq. 6): Var W_K(t) -> t, from the basis by quadrature."""
    T = 10.0
    S = 2000
    Phi = oracle.basis(kind, K, S, T)
    h = T / (2 * S)
    c = int(round(t / h))
    # cumulative integral of each basis row by Simpson's rule on [0, t]
    ints = si.simpson(Phi[:, :c + 1], dx=h, axis=1)
    v = float(np.sum(ints ** 2))
    assert abs(v - expect) < 2e-6 * max(1.0, expect), (v, expect)
    assert abs(_var_wk(kind, K, t, T) - expect) < 1e-6 * max(1.0, expect)


def test_var_wk_converges_to_t():
    for t in [1.0, 2.5, 7.0]:
        errs = [abs(_var_wk(0, K, t, 10.0) - t) for K in (10, 100, 1000)]
        assert errs[0] > errs[1] > errs[2]
        # the omitted tail is at most sum_{j>=K} 2T/(j pi)^2 ~ 2T/(pi^2 K)
        assert errs[2] < 2 * 10.0 / (math.pi ** 2 * 999)


def test_eigen_basis_is_the_wiener_kle():
    """Nystrom on min(s,t): lambda_k = T^2/((k-1/2)^2 pi^2), e_k = sqrt(2/T) sin.

    The eigen basis rows are the time derivatives of sqrt(lambda_k) e_k(t).
    """
    T, n = 10.0, 2000
    h = T / n
    t = (np.arange(n) + 0.5) * h
    Kmat = np.minimum.outer(t, t) * h
    lam, vec = np.linalg.eigh(Kmat)
    lam = lam[::-1][:5]
    vec = vec[:, ::-1][:, :5]
    k = np.arange(1, 6)
    lam_ref = T ** 2 / ((k - 0.5) ** 2 * np.pi ** 2)
    assert np.max(np.abs(lam - lam_ref) / lam_ref) < 1e-4
    S = 1000
    Phi = oracle.basis(1, 5, S, T)
    tt = np.linspace(0, T, 2 * S + 1)
    cum = si.cumulative_trapezoid(Phi, tt, axis=1, initial=0.0)
    for j in range(5):
        e = vec[:, j] / np.sqrt(h)  # unit L2 norm on [0,T]
        e_interp = np.interp(tt, t, e)
        sgn = np.sign(np.dot(cum[j], e_interp))
        mid = slice(10, -10)
        ratio = cum[j][mid] * sgn
        np.testing.assert_allclose(ratio, np.sqrt(lam[j]) * e_interp[mid] * 1.0,
                                   rtol=0, atol=3e-3 * np.sqrt(lam[j]))


# --------------------------------------------------------------------------
# Kron reduction of the network equations (eqs. 1-2)
# --------------------------------------------------------------------------
def test_kron_two_machine_series_closed_form():
    xl, x1, x2 = 0.3, 0.2, 0.1
    net = dict(n_bus=2, n_gen=2, br_from=[0], br_to=[1], br_r=[0.0], br_x=[xl], br_b=None,
               load_g=None, load_b=None, gen_bus=[0, 1], gen_xdp=[x1, x2])
    Y = oracle.kron(net)
    y = 1.0 / (1j * (x1 + xl + x2))
    np.testing.assert_allclose(Y, y * np.array([[1, -1], [-1, 1]]), rtol=1e-14, atol=1e-14)


def _ybus_full(net):
    nb, ng = net["n_bus"], net["n_gen"]
    Y = np.zeros((ng + nb, ng + nb), dtype=complex)
    for f, t, r, x in zip(net["br_from"], net["br_to"], net["br_r"], net["br_x"]):
        y = 1 / (r + 1j * x)
        Y[ng + f, ng + f] += y; Y[ng + t, ng + t] += y
        Y[ng + f, ng + t] -= y; Y[ng + t, ng + f] -= y
    for b in range(nb):
        Y[ng + b, ng + b] += net["load_g"][b] + 1j * net["load_b"][b]
    for g, (b, xd) in enumerate(zip(net["gen_bus"], net["gen_xdp"])):
        y = 1 / (1j * xd)
        Y[g, g] += y; Y[ng + b, ng + b] += y
        Y[g, ng + b] -= y; Y[ng + b, g] -= y
    return Y


def test_kron_matches_full_network_solve():
    net = workloads.network(10, seed=39)
    Y = oracle.kron(net)
    assert np.max(np.abs(Y - Y.T)) < 1e-12 * np.max(np.abs(Y))
    Yf = _ybus_full(net)
    ng = net["n_gen"]
    rng = np.random.default_rng(0)
    for _ in range(5):
        E = rng.normal(size=ng) + 1j * rng.normal(size=ng)
        # zero injection at buses: V_B = -Y_BB^{-1} Y_BA E
        VB = -np.linalg.solve(Yf[ng:, ng:], Yf[ng:, :ng] @ E)
        I_full = Yf[:ng, :ng] @ E + Yf[:ng, ng:] @ VB
        np.testing.assert_allclose(Y @ E, I_full, rtol=1e-11, atol=1e-11)


# --------------------------------------------------------------------------
# OU disturbance through the truncated KLE (eqs. 4, 8, 9)
# --------------------------------------------------------------------------
def _ou_kle_response(theta, sigma, j, t, T, kind=0):
    """sigma * int_0^t exp(-theta (t - s)) m_j(s) ds in closed form."""
    if kind == 0:
        if j == 0:
            return sigma * math.sqrt(1 / T) * (1 - math.exp(-theta * t)) / theta
        a = j * math.pi / T
    else:
        a = (j + 0.5) * math.pi / T
    amp = math.sqrt(2 / T)
    # int_0^t e^{-theta(t-s)} cos(a s) ds
    val = (theta * math.cos(a * t) + a * math.sin(a * t) - theta * math.exp(-theta * t)) / (theta ** 2 + a ** 2)
    return sigma * amp * val


def _unit_runs(sc, K):
    """Responses to zeta = e_j, j = 0..K-1, and to zeta = 0 (last column)."""
    Z = np.concatenate([np.eye(K), np.zeros((K, 1))], axis=1)
    sc = dict(sc, K=K, N=K + 1)
    return oracle.run(sc, zeta=Z, want_traj=True)["traj"]


@pytest.mark.parametrize("K,expect", [(40, 2.4998173e-3)])
def test_ou_truncated_variance(K, expect):
    sc = workloads.smib()
    tr = _unit_runs(sc, K)
    S = tr.shape[1] - 1
    xi = tr[:K, :, 2] - tr[K, :, 2]
    var_k = np.sum(xi ** 2, axis=0)
    # closed-form integral of each mode, every 100 steps
    for s in range(0, S + 1, 100):
        t = s * sc["dt"]
        ref = sum(_ou_kle_response(0.5, 0.05, j, t, sc["T"]) ** 2 for j in range(K))
        assert abs(var_k[s] - ref) <= 1e-8 * max(ref, 1e-6), (s, var_k[s], ref)
    assert abs(var_k[-1] - expect) < 1e-9
    # and the untruncated OU value as K grows
    exact = 0.05 ** 2 / (2 * 0.5) * (1 - math.exp(-2 * 0.5 * 10.0))
    assert abs(exact - 2.4998865e-3) < 1e-10
    assert abs(var_k[-1] - exact) / exact < 1e-4


def test_ou_monte_carlo_mean_and_variance():
    sc = workloads.smib(N=1000)
    r = oracle.run(sc)
    t = np.arange(r["mean"].shape[0]) * sc["dt"]
    var_ou = 0.05 ** 2 / 1.0 * (1 - np.exp(-t))
    # LHS: the mean of xi is tiny; the variance is within MC error (~4%, use 4 sigma)
    assert np.max(np.abs(r["mean"][:, 2])) < 5e-4
    sl_ = slice(200, None)
    rel = np.abs(r["var"][sl_, 2] - var_ou[sl_]) / var_ou[sl_]
    assert rel.max() < 0.16, rel.max()


# --------------------------------------------------------------------------
# The swing equations: SMIB linearisation (Lyapunov / Van Loan) and KLE modes
# --------------------------------------------------------------------------
SMIB = dict(H=3.5, D=2.0, E=1.1, X=0.5, Pm=0.8, theta=0.5, sigma=0.05)


def _smib_linear():
    p = SMIB
    wb = 2 * math.pi * 60
    d0 = math.asin(p["Pm"] * p["X"] / p["E"])
    Ks = p["E"] / p["X"] * math.cos(d0)
    A = np.array([[0, wb, 0], [-Ks / (2 * p["H"]), -p["D"] / (2 * p["H"]), 1 / (2 * p["H"])],
                  [0, 0, -p["theta"]]])
    B = np.array([0.0, 0.0, p["sigma"]])
    return d0, Ks, A, B


def test_smib_operating_point():
    d0, Ks, A, B = _smib_linear()
    r = oracle.run(workloads.smib(N=2, K=1, T=0.02, dt=0.01), zeta=np.zeros((1, 2)))
    assert abs(r["delta0"][0] - 0.372168533960326) < 1e-14
    assert abs(d0 - 0.372168533960326) < 1e-14
    assert abs(Ks - 2.04939015319192) < 1e-12
    ev = np.linalg.eigvals(A)
    assert np.any(np.abs(ev - (-0.1428571 + 10.5048222j)) < 1e-6)


def _van_loan(A, B, t):
    n = A.shape[0]
    Mb = np.block([[-A, np.outer(B, B)], [np.zeros((n, n)), A.T]]) * t
    F = sl.expm(Mb)
    return F[n:, n:].T @ F[:n, n:]


@pytest.mark.parametrize("t,vd,vw", [(1, 6.904862e-4, 1.907367e-7), (2, 9.289488e-4, None),
                                     (5, 1.3707133e-3, None), (10, 1.5717392e-3, 7.594685e-7)])
def test_van_loan_reference_values(t, vd, vw):
    _, _, A, B = _smib_linear()
    Sg = _van_loan(A, B, t)
    assert abs(Sg[0, 0] - vd) / vd < 1e-6
    if vw:
        assert abs(Sg[1, 1] - vw) / vw < 1e-6


def _linear_mode_response(A, B, K, T, times, kind=0):
    """Response of the linearised SMIB to sigma*m_j(t) (scipy, tight tolerance)."""
    out = np.zeros((K, len(times), 3))
    for j in range(K):
        if kind == 0:
            f = (lambda s: math.sqrt(1 / T)) if j == 0 else \
                (lambda s, j=j: math.sqrt(2 / T) * math.cos(j * math.pi * s / T))
        def rhs(s, x, f=f):
            return A @ x + B * f(s)
        sol = si.solve_ivp(rhs, (0, T), np.zeros(3), t_eval=times, rtol=1e-11, atol=1e-14,
                           method="DOP853")
        out[j] = sol.y.T
    return out


def test_smib_kle_modes_match_linearised_system():
    """Nonlinear SMIB at small amplitude: central differences in zeta_j give the
    linear mode responses; their squares sum to the K-truncated variance."""
    K = 40
    eps = 1e-4
    sc = workloads.smib(K=K)
    Z = np.concatenate([eps * np.eye(K), -eps * np.eye(K)], axis=1)
    tr = oracle.run(dict(sc, N=2 * K), zeta=Z, want_traj=True)["traj"]
    r = (tr[:K] - tr[K:]) / (2 * eps)  # [K][S+1][V]
    _, _, A, B = _smib_linear()
    times = np.array([1.0, 5.0, 10.0])
    idx = (times / sc["dt"]).round().astype(int)
    lin = _linear_mode_response(A, B, K, sc["T"], times)
    # RK4 at dt = 0.01 is O((w dt)^4) accurate: ~1e-3 relative on the fastest
    # modes (forcing up to 12 rad/s beside the 10.5 rad/s swing mode)
    for v in range(3):
        scale = np.abs(lin[..., v]).max()
        np.testing.assert_allclose(r[:, idx, v], lin[..., v], rtol=0, atol=1e-3 * scale)
    var_d = np.sum(r[:, -1, 0] ** 2)
    var_w = np.sum(r[:, -1, 1] ** 2)
    assert abs(var_d - 1.5696544e-3) / 1.5696544e-3 < 2e-5
    assert abs(var_w - 7.352999e-7) / 7.352999e-7 < 2e-5
    # truncation bias relative to the Van Loan value (K = 40: -0.13% on delta)
    vl = _van_loan(A, B, 10.0)
    assert -2.0e-3 < (var_d - vl[0, 0]) / vl[0, 0] < -1.0e-3


def test_smib_large_k_reaches_van_loan():
    K = 160
    eps = 1e-4
    sc = workloads.smib(K=K)
    Z = np.concatenate([eps * np.eye(K), -eps * np.eye(K)], axis=1)
    tr = oracle.run(dict(sc, N=2 * K), zeta=Z, want_traj=True)["traj"]
    r = (tr[:K] - tr[K:]) / (2 * eps)
    _, _, A, B = _smib_linear()
    for s, t in [(500, 5.0), (1000, 10.0)]:
        vl = _van_loan(A, B, t)
        assert abs(np.sum(r[:, s, 0] ** 2) - vl[0, 0]) / vl[0, 0] < 3e-4
        assert abs(np.sum(r[:, s, 1] ** 2) - vl[1, 1]) / vl[1, 1] < 3e-3


def test_rk4_fourth_order():
    """Halving dt on a forced deterministic response cuts the error ~16x."""
    K = 8
    zeta = np.zeros((K, 1)); zeta[5, 0] = 2.0
    sols = {}
    for dt in [0.02, 0.01, 0.005, 0.00125]:
        sc = workloads.smib(K=K, T=4.0, dt=dt, N=1)
        tr = oracle.run(sc, zeta=zeta, want_traj=True)["traj"][0]
        sols[dt] = tr[-1]
    ref = sols[0.00125]
    e1 = np.abs(sols[0.02][:2] - ref[:2]).max()
    e2 = np.abs(sols[0.01][:2] - ref[:2]).max()
    e3 = np.abs(sols[0.005][:2] - ref[:2]).max()
    p1, p2 = np.log2(e1 / e2), np.log2(e2 / e3)
    assert 3.7 < p1 < 4.5 and 3.7 < p2 < 4.3, (p1, p2)


def test_trapezoid_second_order_and_consistent():
    K = 8
    zeta = np.zeros((K, 1)); zeta[3, 0] = 1.5
    ref = oracle.run(workloads.smib(K=K, T=4.0, dt=0.0025, N=1), zeta=zeta, want_traj=True)["traj"][0][-1]
    errs = []
    for dt in [0.01, 0.005]:
        sc = workloads.smib(K=K, T=4.0, dt=dt, N=1, integrator="trap")
        tr = oracle.run(sc, zeta=zeta, want_traj=True)["traj"][0]
        errs.append(np.abs(tr[-1][:2] - ref[:2]).max())
    p = np.log2(errs[0] / errs[1])
    assert 1.8 < p < 2.3, errs


def test_small_noise_limit_matches_linear_variance():
    """Monte Carlo of the nonlinear SMIB with sigma -> eps*sigma: Var/eps^2 is
    the K-truncated linear value up to Monte Carlo error (LHS, N=1000)."""
    eps = 1e-3
    sc = workloads.smib(sigma=0.05 * eps)
    r = oracle.run(sc)
    v = r["var"][-1, 0] / eps ** 2
    assert abs(v - 1.5696544e-3) / 1.5696544e-3 < 0.16


# --------------------------------------------------------------------------
# Multimachine system: equilibrium, stability, statistics
# --------------------------------------------------------------------------
def test_equilibrium_residual_and_zero_noise():
    sc = workloads.config2(N=4, T=1.0)
    r0 = oracle.run(dict(sc, dist=dict(sc["dist"], sigma=np.zeros(3))))
    n = sc["n_gen"]
    assert np.max(r0["var"]) == 0.0
    assert np.max(np.abs(r0["mean"][:, :n] - sc["delta0"])) < 1e-12
    assert np.max(np.abs(r0["mean"][:, n:2 * n])) < 1e-12
    y0 = np.concatenate([sc["delta0"], np.zeros(n), np.zeros(3)])
    dy = oracle.rhs(sc, y0, np.zeros(3))
    assert np.max(np.abs(dy)) < 1e-12


def test_equilibrium_power_from_kron_network():
    """Pm := Pe(delta0) with Pe = Re(E~ conj(Y E~)) computed here from the
    reduced admittance (the reduction itself is pinned above)."""
    sc = workloads.config2(N=2, T=0.01)
    Y = oracle.kron(sc["net"])
    Et = sc["E"] * np.exp(1j * sc["delta0"])
    Pe = np.real(Et * np.conj(Y @ Et))
    r = oracle.run(sc, zeta=np.zeros((300, 2)))
    np.testing.assert_allclose(r["Pm"], Pe, rtol=1e-13)


def test_multimachine_workload_is_small_signal_stable():
    for sc in [workloads.config2()]:
        n = sc["n_gen"]
        Y = oracle.kron(sc["net"])
        E, d = sc["E"], sc["delta0"]
        Et = E * np.exp(1j * d)
        Icur = Y @ Et
        J = np.zeros((n, n))
        for i in range(n):
            for k in range(n):
                J[i, k] = np.real(Et[i] * np.conj(Y[i, k] * 1j * Et[k]))
            J[i, i] += np.real(1j * Et[i] * np.conj(Icur[i]))
        wb = 2 * np.pi * 60
        M2 = 2 * sc["H"]
        A = np.block([[np.zeros((n, n)), wb * np.eye(n)],
                      [-J / M2[:, None], -np.diag(sc["D"] / M2)]])
        ev = np.linalg.eigvals(A)
        nz = ev[np.abs(ev) > 1e-8]
        assert np.max(nz.real) < 0, np.max(nz.real)


def test_statistics_match_numpy():
    sc = workloads.config2(N=37, T=0.5)
    r = oracle.run(sc, want_traj=True)
    tr = r["traj"]
    np.testing.assert_allclose(r["mean"], tr.mean(axis=0), rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(r["var"], tr.var(axis=0, ddof=1), rtol=1e-12, atol=1e-30)
    r0 = oracle.run(dict(sc, ddof=0))
    np.testing.assert_allclose(r0["var"], tr.var(axis=0, ddof=0), rtol=1e-12, atol=1e-30)


def test_subset_run_uses_the_same_design():
    sc = workloads.config2(N=50, T=0.25)
    full = oracle.run(sc, want_traj=True)["traj"]
    sel = np.array([3, 17, 49])
    sub = oracle.run(sc, sel=sel, want_traj=True)["traj"]
    assert np.array_equal(full[sel], sub)


# ---- traditional Monte Carlo (eq. 5) as the one-hot "EM" basis ----

def test_em_basis_rows_are_one_hot():
    S, T = 50, 0.5
    Phi = oracle.basis(2, S, S, T)
    nz = np.argwhere(Phi != 0.0)
    assert nz.shape == (S, 2)
    assert np.array_equal(nz[:, 1], 2 * np.arange(S) + 1)  # the midpoint stage of each step
    assert np.allclose(Phi[nz[:, 0], nz[:, 1]], 1.5 / np.sqrt(T / S), rtol=0, atol=1e-15)


def test_em_unit_impulse_gives_the_eq5_increment():
    """One unit normal in step j: RK4 on d xi = -theta xi dt + sigma w dt with
    the midpoint-stage forcing 1.5/sqrt(h) (zero at the step ends) gives, by
    RK4 applied to the linear equation, xi(t_{j+1}) = sigma sqrt(h) (1 -
    theta h / 2 + theta^2 h^2 / 8): the EM increment sigma sqrt(h) of eq. 5 up
    to O(theta h), and 0 before step j."""
    h, S, theta, sigma, j = 0.01, 40, 0.5, 0.05, 7
    sc = workloads.smib(N=2, K=S, T=S * h, dt=h, theta=theta, sigma=sigma, basis="em")
    z = np.zeros((S, 1)); z[j, 0] = 1.0
    r = oracle.run(sc, zeta=z, sel=np.array([0]), want_traj=True)
    xi = r["traj"][0, :, 2]
    assert np.all(xi[: j + 1] == 0.0)
    th = theta * h
    expect = sigma * np.sqrt(h) * (1.0 - th / 2.0 + th * th / 8.0)
    assert abs(xi[j + 1] - expect) <= 1e-15 * abs(expect) + 1e-18
    # after the impulse the free decay is the RK4 amplification per step
    a = 1.0 - th + th ** 2 / 2 - th ** 3 / 6 + th ** 4 / 24
    assert abs(xi[j + 2] - a * xi[j + 1]) <= 1e-15


def test_em_paths_have_the_scheme_variance():
    """SRS normals through the EM basis: the sample variance of xi(T) over
    N = 4000 paths agrees, within four standard errors, with the variance of
    the scheme xi_{s+1} = a xi_s + b zeta_s (a, b as above), which itself is
    within O(theta h) of the OU closed form sigma^2/(2 theta)(1 - e^{-2 theta T})."""
    h, S, theta, sigma, N = 0.01, 200, 0.5, 0.05, 4000
    sc = workloads.smib(N=N, K=S, T=S * h, dt=h, theta=theta, sigma=sigma, basis="em",
                        sampler="srs", seed=11)
    r = oracle.run(sc)
    v = r["var"][S, 2]
    th = theta * h
    a = 1.0 - th + th ** 2 / 2 - th ** 3 / 6 + th ** 4 / 24
    b = sigma * np.sqrt(h) * (1.0 - th / 2.0 + th * th / 8.0)
    v_scheme = b * b * (1.0 - a ** (2 * S)) / (1.0 - a * a)
    v_ou = sigma ** 2 / (2 * theta) * (1.0 - np.exp(-2 * theta * S * h))
    assert abs(v_scheme - v_ou) <= 0.01 * v_ou
    se = v_scheme * np.sqrt(2.0 / (N - 1))
    assert abs(v - v_scheme) <= 4.0 * se, (v, v_scheme, se)
    assert abs(r["mean"][S, 2]) <= 4.0 * np.sqrt(v_scheme / N)


# --- correlation-reducing LHS permutation (Sec. IV-B, LHS Step 2) -----------


def test_decorrelate_rows_keep_their_values_and_strata():
    # Each row is only rearranged: the same values, one per stratum, and the
    # reported rank of an entry is the stratum its value lies in.
    M, N = 6, 64
    st, z = oracle.lhs(3, M, N, 0)
    z2, r = oracle.lhs_decorrelate(z)
    assert np.array_equal(np.sort(z2, axis=1), np.sort(z, axis=1))
    assert np.array_equal(np.sort(r, axis=1), np.tile(np.arange(N, dtype=np.int32), (M, 1)))
    assert np.array_equal(np.floor(sp.ndtr(z2) * N).astype(np.int32), r)
    assert not np.array_equal(z2, z)


def test_decorrelate_hand_worked_two_by_four():
    # Rows x1 = (-3, -1, 1, 3), x2 = (-1, -3, 3, 1): covariance 20/3, 4, 20/3,
    # so the second score is proportional to x2 - 0.6 x1 = (0.8, -2.4, 2.4,
    # -0.8), of ranks (2, 0, 3, 1); x2 takes its sorted values (-3, -1, 1, 3)
    # in that order, (1, -3, 3, -1), orthogonal to x1.  The first score is x1
    # scaled, so x1 stays.
    x = np.array([[-3.0, -1.0, 1.0, 3.0], [-1.0, -3.0, 3.0, 1.0]])
    z2, r = oracle.lhs_decorrelate(x)
    assert np.array_equal(z2, np.array([[-3.0, -1.0, 1.0, 3.0], [1.0, -3.0, 3.0, -1.0]]))
    assert np.array_equal(r, np.array([[0, 1, 2, 3], [2, 0, 3, 1]]))
    assert float(z2[0] @ z2[1]) == 0.0


@pytest.mark.parametrize("M,N", [(10, 500), (30, 1000)])
def test_decorrelate_reduces_correlation(M, N):
    # A random pairing leaves off-diagonal correlations of about 1/sqrt(N);
    # ranks matched to whitened scores leave a small fraction of that.
    off = ~np.eye(M, dtype=bool)
    for seed in range(4):
        _, z = oracle.lhs(100 + seed, M, N, 0)
        z2, _ = oracle.lhs_decorrelate(z)
        before = np.sqrt((np.corrcoef(z)[off] ** 2).mean())
        after = np.sqrt((np.corrcoef(z2)[off] ** 2).mean())
        assert before > 0.5 / math.sqrt(N)
        assert after < 0.1 / math.sqrt(N)


def test_decorrelate_single_row_unchanged():
    st, z = oracle.lhs(9, 1, 40, 0)
    z2, r = oracle.lhs_decorrelate(z)
    assert np.array_equal(z2, z)
    assert np.array_equal(r, st)


def test_decorrelate_invariant_under_affine_row_maps():
    # Scaling a row by a positive factor and shifting it changes neither the
    # ranks of any score row nor, hence, the rearrangement.
    M, N = 5, 80
    _, z = oracle.lhs(21, M, N, 0)
    a = np.array([1.0, 3.5, 0.25, 2.0, 1.0])[:, None]
    b = np.array([0.0, -2.0, 5.0, 0.0, 1.0])[:, None]
    _, r = oracle.lhs_decorrelate(z)
    _, rs = oracle.lhs_decorrelate(a * z + b)
    assert np.array_equal(r, rs)


def test_decorrelate_ranks_match_independent_whitening():
    # The same rearrangement from numpy's Cholesky, a triangular solve and a
    # stable argsort.
    M, N = 8, 120
    _, z = oracle.lhs(5, M, N, 0)
    Lc = np.linalg.cholesky(np.cov(z))
    sc = sl.solve_triangular(Lc, z - z.mean(axis=1, keepdims=True), lower=True)
    ranks = np.empty((M, N), dtype=np.int32)
    for i in range(M):
        ranks[i, np.argsort(sc[i], kind="stable")] = np.arange(N)
    z2, r = oracle.lhs_decorrelate(z)
    assert np.array_equal(r, ranks)
    assert np.array_equal(z2, np.take_along_axis(np.sort(z, axis=1), ranks, axis=1))


def test_decorrelate_rejects_degenerate_designs():
    _, z = oracle.lhs(1, 4, 4, 0)
    with pytest.raises(ValueError):
        oracle.lhs_decorrelate(z)  # N <= M: covariance singular
    _, z = oracle.lhs(1, 3, 30, 0)
    dup = np.vstack([z, z[:1]])
    with pytest.raises(ValueError):
        oracle.lhs_decorrelate(dup)  # a repeated row
    bad = z.copy()
    bad[1, 7] = np.nan
    with pytest.raises(ValueError):
        oracle.lhs_decorrelate(bad)


def test_lhs_decor_sampler_subset_matches_full_design():
    st, z = oracle.lhs(8, 5, 70, 2)
    sel = np.array([69, 0, 33, 12])
    st_s, z_s = oracle.lhs(8, 5, 70, 2, sel=sel)
    assert np.array_equal(z_s, z[:, sel]) and np.array_equal(st_s, st[:, sel])
    _, z0 = oracle.lhs(8, 5, 70, 0)
    z2, r = oracle.lhs_decorrelate(z0)
    assert np.array_equal(z, z2) and np.array_equal(st, r)


# --- correlated disturbances: a diffusion matrix (Sec. III, eq. 4) ----------

_SMAT = np.array([[0.09, 0.0, 0.03], [0.05, 0.07, 0.0], [-0.02, 0.04, 0.06]])


def test_diffusion_matrix_unit_responses_closed_form():
    # A unit coefficient on mode j of noise q drives process p through
    # sigma_pq: xi_p(t) = sigma_pq int_0^t exp(-theta_p (t-s)) m_j(s) ds.
    K = 3
    sc = workloads.config2(N=2, T=0.5)
    sc["dist"] = dict(sc["dist"], sigma_mat=_SMAT)
    n, P = sc["n_gen"], 3
    M = P * K
    Z = np.concatenate([np.eye(M), np.zeros((M, 1))], axis=1)
    tr = oracle.run(dict(sc, K=K, N=M + 1), zeta=Z, want_traj=True)["traj"]
    theta = sc["dist"]["theta"]
    S = tr.shape[1] - 1
    for q in range(P):
        for j in range(K):
            col = q * K + j
            for p in range(P):
                xi = tr[col, :, 2 * n + p] - tr[M, :, 2 * n + p]
                for s in range(0, S + 1, 20):
                    t = s * sc["dt"]
                    ref = _ou_kle_response(theta[p], _SMAT[p, q], j, t, sc["T"])
                    # RK4 at dt = 5 ms against the exact integral: (a dt)^4 for
                    # the fastest mode, a = 2 pi / T, is about 2e-5
                    assert abs(xi[s] - ref) <= 1e-6 * max(abs(ref), 1e-6), (q, j, p, s)


def test_diagonal_diffusion_matrix_equals_sigma_vector():
    sc = workloads.config2(N=40, T=0.3, K=8)
    a = oracle.run(sc)
    sc2 = dict(sc, dist=dict(sc["dist"], sigma_mat=np.diag(sc["dist"]["sigma"])))
    b = oracle.run(sc2)
    assert np.array_equal(a["mean"], b["mean"]) and np.array_equal(a["var"], b["var"])


def test_diffusion_matrix_cross_covariance():
    # Sample covariance of xi_p, xi_q at t = T against (S S^T)-weighted sums of
    # the truncated-KLE mode responses, within 5 standard errors.
    K, N = 10, 4000
    sc = workloads.config2(N=N, T=0.5, K=K)
    sc["dist"] = dict(sc["dist"], sigma_mat=_SMAT)
    n, P = sc["n_gen"], 3
    sel = np.arange(N)
    tr = oracle.run(sc, sel=sel, want_traj=True)["traj"]
    xi = tr[:, -1, 2 * n:2 * n + P]
    theta = sc["dist"]["theta"]
    T = sc["T"]
    R = np.array([[_ou_kle_response(theta[p], 1.0, j, T, T) for j in range(K)] for p in range(P)])
    ref = (_SMAT @ _SMAT.T) * (R @ R.T)
    cov = np.cov(xi.T)
    for p in range(P):
        for q in range(P):
            se = math.sqrt((ref[p, p] * ref[q, q] + ref[p, q] ** 2) / N)
            assert abs(cov[p, q] - ref[p, q]) <= 5 * se, (p, q, cov[p, q], ref[p, q])
    assert abs(np.corrcoef(xi.T)[1, 0]) > 0.2  # the matrix does correlate them


# --- scalar RRF: RMS over the horizon (eq. 3; Sec. V-B) ---------------------


def test_rrf_rms_constant_and_sine():
    S, V, dt = 400, 3, 0.05
    t = np.arange(S + 1) * dt
    T = S * dt
    tr = np.zeros((3, S + 1, V))
    tr[0, :, 1] = 0.7                                  # constant: RMS = |w c|
    tr[1, :, 1] = np.sin(2 * np.pi * 3 * t / T)        # whole periods: RMS = 1/sqrt(2)
    tr[2, :, 0] = 2.0
    tr[2, :, 2] = -1.0                                 # w . y = 2 w0 - w2
    w = np.array([0.5, 2.0, 1.0])
    r = oracle.rrf_rms(tr, w, dt)
    assert abs(r[0] - 1.4) < 1e-14
    assert abs(r[1] - 2.0 / math.sqrt(2.0)) < 1e-12
    assert abs(r[2] - 0.0) < 1e-15


def test_rrf_rms_scaling_and_coi_frame():
    rng = np.random.default_rng(3)
    n, S, V, dt = 5, 120, 4, 0.01
    tr = rng.normal(size=(n, S + 1, V))
    w = np.array([0.2, 0.3, 0.5, 0.0])
    r = oracle.rrf_rms(tr, w, dt)
    assert np.allclose(oracle.rrf_rms(-3.0 * tr, w, dt), 3.0 * r, rtol=1e-14)
    # centre-of-inertia deviation: weights e_i - H/sum H remove a common mode
    H = np.array([2.0, 3.0, 5.0])
    wc = np.append(np.eye(3)[1] - H / H.sum(), 0.0)
    common = tr.copy()
    common[:, :, :3] = tr[:, :, :1]                    # every machine the same
    assert np.all(oracle.rrf_rms(common, wc, dt) < 1e-14)
    # trapezoid rule written out for one trajectory
    u = tr[2] @ w
    ref = math.sqrt(((u[0] ** 2 + u[-1] ** 2) / 2 + (u[1:-1] ** 2).sum()) * dt / (S * dt))
    assert abs(r[2] - ref) < 1e-14
