"""Correlated disturbances (a diffusion matrix, eq. 4 with the full sigma of
Sec. III) on the GPU, through the C ABI, against the FP64 oracle.

The GPU mixes the design's coefficients through the matrix before the path
contraction (the paths are linear in them); the oracle mixes the white-noise
values inside its right-hand side.  Bar: 1e-10 in FP64 (trajectories and
statistics), 1e-4 in FP32.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

SMAT = np.array([[0.09, 0.0, 0.03], [0.05, 0.07, 0.0], [-0.02, 0.04, 0.06]])


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


def _mixed(**kw):
    sc = workloads.config2(**kw)
    sc["dist"] = dict(sc["dist"], sigma_mat=SMAT)
    return sc


@pytest.mark.parametrize("N,K,sampler", [(300, 20, "lhs"), (257, 7, "srs"), (200, 20, "lhs_decor")])
def test_diffusion_matrix_fp64_parity(ctx, N, K, sampler):
    sc = _mixed(N=N, T=0.4, K=K)
    sc["sampler"] = sampler
    sel = np.array([0, N // 2, N - 1])
    r = ctx.run(sc, precision="f64", traj_idx=sel)
    o = oracle.run(sc, sel=sel, want_traj=True)
    assert _rel(_np(r["traj"]), o["traj"]) <= 1e-10
    full = oracle.run(sc)
    assert _rel(_np(r["mean"]), full["mean"]) <= 1e-10
    assert _rel(_np(r["var"]), full["var"]) <= 1e-10


def test_diffusion_matrix_reduced_precision(ctx):
    sc = _mixed(N=400, T=0.4, K=20)
    full = oracle.run(sc)
    for prec in ("f32", "bf16x3"):
        r = ctx.run(sc, precision=prec)
        assert _rel(_np(r["var"]), full["var"]) <= 1e-4, prec


def test_diagonal_matrix_matches_sigma_vector(ctx):
    sc = workloads.config2(N=300, T=0.4, K=20)
    a = ctx.run(sc, precision="f64")
    sc2 = dict(sc, dist=dict(sc["dist"], sigma_mat=np.diag(sc["dist"]["sigma"])))
    b = ctx.run(sc2, precision="f64")
    assert _rel(_np(b["mean"]), _np(a["mean"])) <= 1e-12
    assert _rel(_np(b["var"]), _np(a["var"])) <= 1e-12


def test_diffusion_matrix_given_design(ctx):
    """zeta_in holds the coefficients of the independent noises; they are
    mixed the same way."""
    sc = _mixed(N=150, T=0.3, K=10)
    _, z = oracle.lhs(41, 30, 150, 1)
    zd = ctx.torch.tensor(z, dtype=ctx.torch.float64, device=ctx.device)
    r = ctx.run(sc, precision="f64", zeta_in=zd)
    o = oracle.run(sc, zeta=z)
    assert _rel(_np(r["var"]), o["var"]) <= 1e-10


def test_diffusion_matrix_rejections(ctx, fmc):
    sc = _mixed(N=100, T=0.3, K=10)
    bad = dict(sc, dist=dict(sc["dist"], sigma_mat=np.where(SMAT == 0.0, np.nan, SMAT)))
    with pytest.raises(fmc.FmcError) as e:
        ctx.run(bad, precision="f64")
    assert e.value.code == fmc.EINVAL
    with pytest.raises(fmc.FmcError) as e:
        ctx.run_batch([sc], precision="f32")
    assert e.value.code == fmc.EINVAL
    with pytest.raises(fmc.FmcError) as e:
        ctx.submit(sc, precision="f32")
    assert e.value.code == fmc.EINVAL
