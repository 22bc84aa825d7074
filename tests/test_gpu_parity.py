"""GPU path (through the C ABI) against the FP64 oracle on the same seeded inputs.

Tolerances (per output variable v, normalised by max_s |oracle| of v, since
the variance at t = 0 is exactly zero):
  strata / indices      bit-exact
  zeta (FP64)           1e-15 relative (AS 241 evaluated in a different order)
  basis, KLE paths FP64 1e-13 of the row scale (MFMA accumulation order)
  trajectories, FP64    1e-10
  mean / var, FP64      1e-10
  mean / var, FP32 and BF16x3   1e-4 (mean relative to max(|mean|, std))
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(fmc):
    return fmc.Context(0)


def _np(t):
    return t.detach().cpu().numpy()


def mean_err(a, mean_ref, var_ref):
    """Error of an estimated mean relative to the variable's scale
    max_s max(|mean|, std): the LHS mean of a zero-mean disturbance is O(1/N),
    so |mean| alone is no scale for it."""
    a = np.asarray(a, dtype=np.float64)
    num = np.abs(a - mean_ref).max(axis=0)
    den = np.maximum(np.abs(mean_ref).max(axis=0), np.sqrt(np.abs(var_ref)).max(axis=0))
    den = np.where(den == 0, 1.0, den)
    return float((num / den).max())


def rel_err(a, b):
    """max over variables of max_s |a-b| / max_s |b| (arrays [..., S+1, V])."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    num = np.abs(a - b).reshape(-1, a.shape[-1]).max(axis=0)
    den = np.abs(b).reshape(-1, b.shape[-1]).max(axis=0)
    den = np.where(den == 0, 1.0, den)
    return float((num / den).max())


# ----------------------------------------------------------------- LHS
@pytest.mark.parametrize("M,N", [(1, 1), (3, 2), (5, 63), (4, 64), (7, 65), (40, 1000),
                                 (2, 10007), (300, 257)])
@pytest.mark.parametrize("sampler", [0, 1])
def test_lhs_bit_exact(ctx, M, N, sampler):
    st, z = ctx.lhs(seed=1234 + N, M=M, N=N, sampler=sampler)
    ost, oz = oracle.lhs(1234 + N, M, N, sampler=sampler)
    assert np.array_equal(_np(st), ost)
    zz = _np(z)
    assert np.all(np.abs(zz - oz) <= 1e-15 * np.maximum(1.0, np.abs(oz)))


def test_lhs_large_sampled(ctx):
    """The N = 1e5, M = 300 design of the mixed-precision workload: sampled columns."""
    M, N = 300, 100_000
    st, z = ctx.lhs(seed=3, M=M, N=N)
    sel = np.array([0, 1, 777, 50_000, 99_998, 99_999])
    ost, oz = oracle.lhs(3, M, N, sel=sel)
    assert np.array_equal(_np(st[:, sel]), ost)
    assert np.all(np.abs(_np(z[:, sel]) - oz) <= 1e-15 * np.maximum(1.0, np.abs(oz)))
    # every row is a permutation of the strata (property at full size)
    sts = np.sort(_np(st[:8]), axis=1)
    assert np.array_equal(sts, np.tile(np.arange(N, dtype=np.int32), (8, 1)))


# --------------------------------------------------------------- basis
@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("K,S,T", [(1, 1, 1.0), (40, 1000, 10.0), (100, 4000, 20.0), (7, 13, 0.65)])
def test_basis(ctx, kind, K, S, T):
    phi = _np(ctx.basis(kind, K, S, T))
    ref = oracle.basis(kind, K, S, T)
    assert np.max(np.abs(phi - ref)) <= 1e-15 * np.sqrt(2.0 / T) * 4


@pytest.mark.parametrize("S,T", [(1, 0.01), (50, 0.5), (400, 4.0)])
def test_em_basis(ctx, S, T):
    """The one-hot basis of the traditional Monte Carlo baseline (eq. 5)."""
    phi = _np(ctx.basis(2, S, S, T))
    ref = oracle.basis(2, S, S, T)
    assert np.array_equal(phi != 0, ref != 0)
    assert np.max(np.abs(phi - ref)) <= 1e-15 * np.abs(ref).max()


# ------------------------------------------------------------ KLE paths
@pytest.mark.parametrize("P,K,N,S", [(1, 40, 1000, 100), (3, 100, 777, 60), (2, 5, 65, 9),
                                     (1, 1, 1, 1), (2, 150, 2049, 130), (1, 32, 256, 16),
                                     (1, 7, 100, 20), (3, 12, 130, 40)])
@pytest.mark.parametrize("prec,tol", [("f64", 1e-13), ("f32", 2e-7), ("bf16x3", 4e-5)])
def test_kle_paths(ctx, P, K, N, S, prec, tol):
    T = 0.01 * S
    _, z = ctx.lhs(seed=5, M=P * K, N=N)
    phi = ctx.basis(0, K, S, T)
    C = 2 * S + 1
    c0 = 3 if C > 5 else 0
    Cc = C - c0
    w = _np(ctx.kle_paths(z, phi, P, K, Cc, c0=c0, precision=prec)).astype(np.float64)
    ref = oracle.kle_paths(_np(z), _np(phi), P, K, c0, Cc)
    scale = np.sqrt(np.sum(_np(phi)[:, c0:c0 + Cc, None] ** 2, axis=0)).max() * np.abs(_np(z)).max()
    assert np.max(np.abs(w - ref)) <= tol * scale


@pytest.mark.parametrize("prec,tol", [("f64", 1e-13), ("f32", 2e-7)])
def test_kle_paths_wide_offsets(ctx, prec, tol):
    """More than 2^27 paths: a lane's byte offsets inside a k-step of four
    rows no longer fit 32 bits, and the contraction takes 64-bit offsets.
    Sampled columns (the first, the last, and some across the range) against
    the oracle on the same columns."""
    import torch
    P, K, S = 1, 6, 3
    N = (1 << 27) + 1000
    g = torch.Generator(device="cuda").manual_seed(7)
    z = torch.randn(P * K, N, dtype=torch.float64, device="cuda", generator=g)
    phi = ctx.basis(0, K, S, 0.03)
    C = 2 * S + 1
    w = ctx.kle_paths(z, phi, P, K, C, precision=prec)
    sel = np.unique(np.concatenate([[0, 1, N // 2, N - 2, N - 1],
                                    np.random.default_rng(3).integers(0, N, 200)]))
    idx = torch.as_tensor(sel, device="cuda")
    got = _np(w[:, :, idx]).astype(np.float64)
    zs = _np(z[:, idx])
    del w, z
    ref = oracle.kle_paths(zs, _np(phi), P, K, 0, C)
    scale = np.sqrt(np.sum(_np(phi)[:, :C, None] ** 2, axis=0)).max() * np.abs(zs).max()
    assert np.max(np.abs(got - ref)) <= tol * scale


# --------------------------------------------------------------- Kron
@pytest.mark.parametrize("n_gen,seed", [(10, 39), (3, 7), (50, 11), (1, 2), (200, 200)])
def test_kron(ctx, n_gen, seed):
    """Small networks reduce in LDS on one workgroup, large ones (50 and 200
    machines: 195 and 780 buses) by node elimination over many workgroups."""
    net = workloads.network(n_gen, seed)
    Y = ctx.kron_reduce(net)
    ref = oracle.kron(net)
    assert np.max(np.abs(Y - ref)) <= 1e-12 * np.max(np.abs(ref))


# --------------------------------------------------------- whole method
def _traj_check(ctx, sc, sel, prec="f64", tol=1e-10, **kw):
    r = ctx.run(sc, precision=prec, traj_idx=sel, **kw)
    o = oracle.run(sc, sel=sel, want_traj=True)
    e = rel_err(_np(r["traj"]), o["traj"])
    assert e <= tol, e
    return r


def test_smib_fp64_parity(ctx):
    sc = workloads.config1()
    sel = np.array([0, 1, 500, 998, 999])
    r = _traj_check(ctx, sc, sel)
    o = oracle.run(sc)
    assert rel_err(_np(r["mean"]), o["mean"]) <= 1e-10
    assert rel_err(_np(r["var"]), o["var"]) <= 1e-10
    assert r["report"]["n_nonfinite"] == 0


def test_multimachine_fp64_parity_reduced(ctx):
    sc = workloads.config2(N=1000, T=2.0)
    sel = np.array([0, 63, 64, 999])
    r = _traj_check(ctx, sc, sel)
    o = oracle.run(sc)
    assert rel_err(_np(r["mean"]), o["mean"]) <= 1e-10
    assert rel_err(_np(r["var"]), o["var"]) <= 1e-10


def test_multimachine_fp64_full_size_sampled(ctx):
    """N = 1e4, K = 100, S = 4000 in the benchmarked launch configuration:
    sampled trajectories against the oracle run on those samples only."""
    sc = workloads.config2()
    sel = np.array([0, 4321, 9983, 9999])
    r = _traj_check(ctx, sc, sel)
    m, v = _np(r["mean"]), _np(r["var"])
    assert np.all(np.isfinite(m)) and np.all(np.isfinite(v)) and np.all(v >= 0)
    assert np.all(v[0] == 0)


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
def test_reduced_precision_statistics(ctx, prec):
    for sc in [workloads.config1(), workloads.config2(N=1000, T=2.0)]:
        r = ctx.run(sc, precision=prec)
        o = oracle.run(sc)
        em = mean_err(_np(r["mean"]), o["mean"], o["var"])
        ev = rel_err(_np(r["var"]), o["var"])
        print(f"{prec}: mean err {em:.3e}, var err {ev:.3e}")
        assert em <= 1e-4 and ev <= 1e-4, (prec, em, ev)


def test_unit_vector_design_matches_oracle(ctx):
    """zeta supplied by the caller (unit vectors): the deterministic KLE modes."""
    import torch
    K = 40
    sc = workloads.smib(K=K, N=K + 1)
    Z = np.concatenate([np.eye(K), np.zeros((K, 1))], axis=1)
    zt = torch.tensor(Z, dtype=torch.float64, device="cuda")
    sel = np.arange(K + 1)
    r = ctx.run(sc, traj_idx=sel, zeta_in=zt)
    o = oracle.run(sc, zeta=Z, want_traj=True)
    assert rel_err(_np(r["traj"]), o["traj"]) <= 1e-10


def test_time_chunks_do_not_change_results(ctx):
    sc = workloads.config2(N=300, T=1.0)
    a = ctx.run(sc, time_chunk=7)
    b = ctx.run(sc, time_chunk=200)
    c = ctx.run(sc)
    for k in ("mean", "var"):
        assert np.array_equal(_np(a[k]), _np(b[k]))
        assert np.array_equal(_np(a[k]), _np(c[k]))


def test_repeat_runs_bit_identical(ctx):
    sc = workloads.config2(N=500, T=0.5)
    a = ctx.run(sc, precision="f32")
    b = ctx.run(sc, precision="f32")
    assert np.array_equal(_np(a["var"]), _np(b["var"]))


@pytest.mark.parametrize("vid", [7, 8, 9, 10, 15, 16, 17, 18, 19, 20, 21, 22, 23, 24, 25, 26, 27, 28, 29, 30, 31, 32, 33])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_variants_agree(ctx, vid, prec):
    """Every integrator variant (padded lane variants, lanes-per-trajectory
    groups) reproduces the oracle on a ragged sample count, trajectories
    included."""
    sc = workloads.config2(N=333, T=0.5)
    sel = np.array([0, 5, 17, 331, 332])
    o = oracle.run(sc, want_traj=True)
    r = ctx.run(sc, variant=vid, precision=prec, traj_idx=sel)
    tol = 1e-10 if prec == "f64" else 1e-4
    assert rel_err(_np(r["traj"]), o["traj"][sel]) <= (tol if prec == "f64" else 2e-3)
    assert rel_err(_np(r["var"]), o["var"]) <= tol
    assert mean_err(_np(r["mean"]), o["mean"], o["var"]) <= tol


def test_invalid_arguments(ctx, fmc):
    sc = workloads.config1(N=10, T=0.1)
    for bad in [dict(dt=0.0), dict(dt=0.003), dict(N=1), dict(K=0), dict(ddof=10)]:
        with pytest.raises(fmc.FmcError) as e:
            ctx.run(dict(sc, **bad))
        assert e.value.code == fmc.EINVAL
    with pytest.raises(fmc.FmcError):
        ctx.run(dict(sc, dist=dict(sc["dist"], theta=np.array([-1.0]))))
    with pytest.raises(fmc.FmcError):
        ctx.run(dict(sc, H=np.array([0.0])))


def test_nonfinite_paths_are_counted(ctx, fmc):
    """A deliberately unstable scenario (tiny inertia: RK4 at dt = 0.01 blows up)."""
    sc = workloads.smib(N=100, T=1.0, H=1e-5, sigma=5.0)
    r = ctx.run(sc, allow_nonfinite=True)
    assert r["rc"] == fmc.ENONFINITE
    assert r["report"]["n_nonfinite"] > 0
    assert r["report"]["first_nonfinite"] >= 0


@pytest.mark.parametrize("sampler", ["srs", "lhs"])
def test_em_baseline_fp64_parity(ctx, sampler):
    """Traditional Monte Carlo (eq. 5 increments through the one-hot basis,
    K = S) on the 10-machine system: FP64 trajectories and statistics against
    the oracle; FP32 statistics to the reduced-precision bound."""
    sc = workloads.config2(N=300, T=0.4)
    sc = dict(sc, basis="em", K=80, sampler=sampler)
    sel = np.array([0, 150, 299])
    r = _traj_check(ctx, sc, sel)
    o = oracle.run(sc)
    assert rel_err(_np(r["mean"]), o["mean"]) <= 1e-10
    assert rel_err(_np(r["var"]), o["var"]) <= 1e-10
    r32 = ctx.run(sc, precision="f32")
    assert mean_err(_np(r32["mean"]), o["mean"], o["var"]) <= 1e-4
    assert rel_err(_np(r32["var"]), o["var"]) <= 1e-4


def test_em_basis_needs_k_equal_s(ctx, fmc):
    sc = dict(workloads.config2(N=100, T=0.4), basis="em", K=40)
    with pytest.raises(fmc.FmcError) as e:
        ctx.run(sc, precision="f64")
    assert e.value.code == fmc.EINVAL
