"""Scalar RRF (eq. 3): RMS over the horizon of a linear combination of the
outputs, here the system (centre-of-inertia) frequency deviation of Sec. V-B,
on the GPU through the C ABI against the FP64 oracle.  Bar: 1e-13 relative on
given trajectories (one reduction order against another), 1e-9 on the
trajectories of a whole FP64 run (which agree to 1e-10)."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(fmc):
    return fmc.Context(0)


@pytest.mark.parametrize("n,S,V", [(1, 1, 1), (5, 120, 4), (3, 1000, 23), (300, 257, 7),
                                   (2, 700, 61), (2, 9, 300), (2, 5, 2048)])
def test_rrf_given_trajectories(ctx, n, S, V):
    rng = np.random.default_rng(n + S)
    tr = rng.normal(size=(n, S + 1, V))
    w = rng.normal(size=V)
    td = ctx.torch.tensor(tr, dtype=ctx.torch.float64, device=ctx.device)
    got = ctx.rrf_rms(td, w, 0.01).cpu().numpy()
    ref = oracle.rrf_rms(tr, w, 0.01)
    assert np.all(np.abs(got - ref) <= 1e-13 * np.abs(ref))


def test_rrf_empty(ctx):
    td = ctx.torch.zeros((0, 11, 3), dtype=ctx.torch.float64, device=ctx.device)
    assert ctx.rrf_rms(td, np.ones(3), 0.1).numel() == 0


def test_rrf_of_the_method_coi_frequency(ctx):
    """Every sample's trajectory from fmc_run, then the RMS of the inertia-
    weighted frequency deviation; its mean and variance over the samples."""
    N = 64
    sc = workloads.config2(N=N, T=0.4, K=10)
    n = sc["n_gen"]
    V = 2 * n + len(sc["dist"]["gen"])
    H = np.asarray(sc["H"], dtype=np.float64)
    w = np.zeros(V)
    w[n:2 * n] = H / H.sum()
    r = ctx.run(sc, precision="f64", traj_idx=np.arange(N))
    got = ctx.rrf_rms(r["traj"], w, sc["dt"]).cpu().numpy()
    o = oracle.run(sc, sel=np.arange(N), want_traj=True)
    ref = oracle.rrf_rms(o["traj"], w, sc["dt"])
    assert np.all(np.abs(got - ref) <= 1e-9 * np.abs(ref).max())
    assert abs(got.mean() - ref.mean()) <= 1e-9 * ref.mean()
    assert abs(got.var(ddof=1) - ref.var(ddof=1)) <= 1e-8 * ref.var(ddof=1)


def test_rrf_rejections(ctx, fmc):
    t = ctx.torch
    td = t.zeros((2, 1, 3), dtype=t.float64, device=ctx.device)  # S = 0
    with pytest.raises(fmc.FmcError) as e:
        ctx.rrf_rms(td, np.ones(3), 0.1)
    assert e.value.code == fmc.EINVAL
    td = t.zeros((2, 5, 3), dtype=t.float64, device=ctx.device)
    with pytest.raises(fmc.FmcError) as e:
        ctx.rrf_rms(td, np.ones(3), 0.0)
    assert e.value.code == fmc.EINVAL


# ------------------------------------------------ RRF fused into the integrator
def _coi_weights(sc):
    n, P = sc["n_gen"], len(sc["dist"]["gen"])
    w = np.zeros(2 * n + P)
    H = np.asarray(sc["H"], dtype=np.float64)
    w[n:2 * n] = H / H.sum()
    return w


FUSED = [("10gen_f64", lambda: workloads.config2(N=300, K=20, T=1.0), "f64", -1),
         ("10gen_f64_lane", lambda: workloads.config2(N=70, K=20, T=0.5), "f64", 7),
         ("10gen_trip_f64", lambda: dict(workloads.config2(N=130, K=20, T=1.0),
                                         event=dict(t=0.5, tripped=2)), "f64", -1),
         ("smib_trap", lambda: workloads.smib(N=65, K=20, T=1.0, integrator="trap"), "f64", -1),
         ("10gen_f32", lambda: workloads.config2(N=300, K=20, T=1.0), "f32", -1),
         ("10gen_bf16x3", lambda: workloads.config2(N=300, K=20, T=1.0), "bf16x3", -1)]


@pytest.mark.parametrize("name,make,prec,variant", FUSED, ids=[c[0] for c in FUSED])
def test_fused_rrf_against_oracle(ctx, name, make, prec, variant):
    """The RRF accumulated in the integrator's epilogue (no trajectories
    stored) against the oracle's RMS of its own trajectories of every sample:
    1e-10 relative in FP64, 1e-4 in the reduced-precision forms; the samples'
    mean and variance of the RRF likewise."""
    sc = make()
    w = _coi_weights(sc) if sc["n_gen"] > 1 else np.array([0.0, 1.0, 0.0])
    r = ctx.run(sc, precision=prec, rrf_weights=w, variant=variant)
    o = oracle.run(sc, want_traj=True)
    ref = oracle.rrf_rms(o["traj"], w, sc["dt"])
    got = r["rrf"].cpu().numpy()
    tol = 1e-10 if prec == "f64" else 1e-4
    assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref))
    assert abs(got.mean() - ref.mean()) <= tol * abs(ref.mean())
    assert abs(got.var(ddof=1) - ref.var(ddof=1)) <= 2 * tol * ref.var(ddof=1)


def test_fused_rrf_time_chunks_and_stored_trajectories(ctx):
    sc = workloads.config2(N=200, K=20, T=1.0)
    w = _coi_weights(sc)
    a = ctx.run(sc, precision="f64", rrf_weights=w, traj_idx=np.arange(sc["N"]))
    b = ctx.run(sc, precision="f64", rrf_weights=w, time_chunk=13)
    assert np.array_equal(a["rrf"].cpu().numpy(), b["rrf"].cpu().numpy())
    # the same quantity from the stored trajectories (fmc_rrf_rms)
    c = ctx.rrf_rms(a["traj"], w, sc["dt"]).cpu().numpy()
    np.testing.assert_allclose(a["rrf"].cpu().numpy(), c, rtol=1e-13, atol=0)


def test_fused_rrf_rejections(ctx, fmc):
    fd = workloads.fluxdecay(n_gen=12, n_dist=3, N=20, K=10, T=0.2, net_seed=312)
    with pytest.raises(fmc.FmcError) as e:
        ctx.run(fd, precision="f32", rrf_weights=np.ones(6 * 12 + 3))
    assert e.value.code == fmc.EINVAL
