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
