"""Correlation-reducing LHS permutation (Sec. IV-B, LHS Step 2) on the GPU,
through the C ABI, against the FP64 oracle.

Bar: the ranks (strata) are integers decided in FP64 on both sides and must
agree bit for bit; the rearranged values are the input's own values, so they
agree bit for bit when both sides start from the same design, and to the
LHS's 1e-15 when each side draws its own design.  Statistics of a whole run
with the reduced design: 1e-10 in FP64, 1e-4 in FP32.
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


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    num = np.abs(a - b).reshape(-1, a.shape[-1]).max(axis=0)
    den = np.abs(b).reshape(-1, b.shape[-1]).max(axis=0)
    den = np.where(den == 0, 1.0, den)
    return float((num / den).max())


# M, N: one row, N = M + 1, ragged rank tiles (257, 1000), several covariance
# tiles (M = 40, 300), and the 10-machine workload's design (M = 300, N = 1e4)
SHAPES = [(1, 2), (3, 4), (5, 63), (12, 257), (40, 1000), (300, 1024), (300, 10_000)]


@pytest.mark.parametrize("M,N", SHAPES)
def test_decorrelate_same_input_bit_exact(ctx, M, N):
    _, oz = oracle.lhs(77 + N, M, N, 0)
    z = ctx.torch.tensor(oz, dtype=ctx.torch.float64, device=ctx.device)
    st = ctx.lhs_decorrelate(z)
    ez, er = oracle.lhs_decorrelate(oz)
    assert np.array_equal(_np(st), er)
    assert np.array_equal(_np(z), ez)


@pytest.mark.parametrize("M,N", SHAPES)
def test_lhs_decor_sampler_against_oracle(ctx, M, N):
    st, z = ctx.lhs(seed=5 + M, M=M, N=N, sampler="lhs_decor")
    ost, oz = oracle.lhs(5 + M, M, N, 2)
    assert np.array_equal(_np(st), ost)
    zz = _np(z)
    assert np.all(np.abs(zz - oz) <= 1e-15 * np.maximum(1.0, np.abs(oz)))


def test_decorrelate_general_design(ctx):
    """Not an LHS design: simple random sampling with affine rows and a
    strongly correlated pair; ranks are of the values themselves."""
    M, N = 9, 700
    _, x = oracle.lhs(11, M, N, 1)
    x = x * np.linspace(0.5, 3.0, M)[:, None] + np.arange(M)[:, None]
    x[4] = 0.8 * x[3] + 0.2 * x[4]
    z = ctx.torch.tensor(x, dtype=ctx.torch.float64, device=ctx.device)
    st = ctx.lhs_decorrelate(z)
    ez, er = oracle.lhs_decorrelate(x)
    assert np.array_equal(_np(st), er)
    assert np.array_equal(_np(z), ez)
    assert abs(np.corrcoef(ez)[3, 4]) < 0.05 < abs(np.corrcoef(x)[3, 4])


def test_decorrelate_without_strata(ctx):
    _, oz = oracle.lhs(3, 6, 90, 0)
    z = ctx.torch.tensor(oz, dtype=ctx.torch.float64, device=ctx.device)
    assert ctx.lhs_decorrelate(z, want_strata=False) is None
    assert np.array_equal(_np(z), oracle.lhs_decorrelate(oz)[0])


def test_decorrelate_rejections(ctx, fmc):
    t = ctx.torch
    for M, N in [(4, 4), (5, 3), (1025, 2000)]:
        z = t.zeros((M, N), dtype=t.float64, device=ctx.device)
        with pytest.raises(fmc.FmcError) as e:
            ctx.lhs_decorrelate(z)
        assert e.value.code == fmc.EINVAL
    # a repeated row: covariance singular, the design is left as it was
    _, x = oracle.lhs(1, 3, 30, 0)
    x = np.vstack([x, x[:1]])
    z = t.tensor(x, dtype=t.float64, device=ctx.device)
    with pytest.raises(fmc.FmcError) as e:
        ctx.lhs_decorrelate(z)
    assert e.value.code == fmc.EINVAL
    assert np.array_equal(_np(z), x)
    # a non-finite value: likewise
    x2 = x[:3].copy()
    x2[1, 4] = np.inf
    z = t.tensor(x2, dtype=t.float64, device=ctx.device)
    with pytest.raises(fmc.FmcError) as e:
        ctx.lhs_decorrelate(z)
    assert e.value.code == fmc.EINVAL
    assert np.array_equal(_np(z), x2)
    # the sampler form needs M < N as well
    with pytest.raises(fmc.FmcError) as e:
        ctx.lhs(seed=1, M=50, N=50, sampler="lhs_decor")
    assert e.value.code == fmc.EINVAL


def test_run_with_decorrelated_design(ctx):
    """The whole method with the reduced design: FP64 statistics and sampled
    trajectories against the oracle, the design returned bit-exact in its
    strata; FP32 statistics to the reduced-precision bound."""
    sc = dict(workloads.config2(N=300, T=0.4), K=20, sampler="lhs_decor")
    sel = np.array([0, 137, 299])
    r = ctx.run(sc, precision="f64", traj_idx=sel, want_design=True)
    o = oracle.run(sc, sel=sel, want_traj=True)
    assert _rel(_np(r["traj"]), o["traj"]) <= 1e-10
    full = oracle.run(sc)
    assert _rel(_np(r["mean"]), full["mean"]) <= 1e-10
    assert _rel(_np(r["var"]), full["var"]) <= 1e-10
    ost, oz = oracle.lhs(sc["seed"], 3 * 20, 300, 2)
    assert np.array_equal(_np(r["strata"]), ost)
    r32 = ctx.run(sc, precision="f32")
    assert _rel(_np(r32["var"]), full["var"]) <= 1e-4


def test_run_decor_rejections(ctx, fmc):
    sc = dict(workloads.config2(N=100, T=0.4), K=40, sampler="lhs_decor")  # M = 120 >= N
    with pytest.raises(fmc.FmcError) as e:
        ctx.run(sc, precision="f64")
    assert e.value.code == fmc.EINVAL
    sc = dict(workloads.config2(N=300, T=0.4), K=20, sampler="lhs_decor")
    with pytest.raises(fmc.FmcError) as e:
        ctx.run_batch([sc], precision="f32")
    assert e.value.code == fmc.EINVAL
    with pytest.raises(fmc.FmcError) as e:
        ctx.submit(sc, precision="f32")
    assert e.value.code == fmc.EINVAL
