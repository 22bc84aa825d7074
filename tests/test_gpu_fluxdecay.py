"""Flux-decay machines with IEEE type-1 exciters on the GPU (FP32 integration
with the network current on the matrix cores, FP64 setup and statistics)
against the FP64 oracle.

Tolerances as for the classical reduced-precision path: statistics 1e-4
(mean relative to max(|mean|, std), variance relative to max |var|, per
output variable); sampled FP32 trajectories 2e-3 of each variable's range.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


def mean_err(a, m, v):
    num = np.abs(a - m).max(axis=0)
    den = np.maximum(np.abs(m).max(axis=0), np.sqrt(np.abs(v)).max(axis=0))
    return float((num / np.where(den == 0, 1, den)).max())


def var_err(a, b):
    num = np.abs(a - b).max(axis=0)
    den = np.abs(b).max(axis=0)
    return float((num / np.where(den == 0, 1, den)).max())


def traj_err(a, b):
    # per variable: error relative to the variable's excursion over the run
    d = b - b[:, :1, :]
    num = np.abs(a - b).reshape(-1, a.shape[-1]).max(axis=0)
    den = np.maximum(np.abs(d).reshape(-1, a.shape[-1]).max(axis=0), 1e-6)
    return float((num / den).max())


@pytest.fixture(scope="module")
def ctx(fmc):
    return fmc.Context(0)


# (n, P, N, K, T): one and several 16-machine blocks, odd block counts,
# ragged trajectory tiles
CASES = [(1, 1, 40, 20, 1.0), (12, 3, 37, 30, 0.5), (37, 6, 50, 25, 0.4), (70, 10, 33, 20, 0.3)]


def scenario(n, P, N, K, T, seed=0):
    if n == 1:
        return workloads.smib_fluxdecay(N=N, K=K, T=T, dt=0.005, seed=3)
    return workloads.fluxdecay(n_gen=n, n_dist=P, N=N, K=K, T=T, dt=0.005, net_seed=300 + n,
                               seed=5 + seed)


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("prec,variant", [("f32", -1), ("bf16x3", -1), ("bf16x3", 1)])
def test_fluxdecay_matches_oracle(ctx, case, prec, variant):
    """FP32 network product (default) and, asked for with variant 1, the
    BF16 x3 network product, on short horizons."""
    sc = scenario(*case)
    N = sc["N"]
    sel = np.array([0, N // 2, N - 1])
    r = ctx.run(sc, precision=prec, traj_idx=sel, variant=variant)
    o = oracle.run(sc, want_traj=True)
    assert r["report"]["n_nonfinite"] == 0
    assert r["report"]["variant_id"] == (1 if variant == 1 else 0)
    em = mean_err(_np(r["mean"]), o["mean"], o["var"])
    ev = var_err(_np(r["var"]), o["var"])
    et = traj_err(_np(r["traj"]), o["traj"][sel])
    assert em <= 1e-4 and ev <= 1e-4 and et <= 2e-3, (case, em, ev, et)


def test_fluxdecay_chunks_and_row0(ctx):
    """Time chunks (state kept between them) do not change the result, and
    the first row is the operating point with zero variance."""
    sc = scenario(37, 6, 50, 25, 0.4)
    a = ctx.run(sc, precision="f32")
    b = ctx.run(sc, precision="f32", time_chunk=7)
    assert np.array_equal(_np(a["var"]), _np(b["var"]))
    assert np.array_equal(_np(a["mean"]), _np(b["mean"]))
    y0, _ = oracle.initial_state(sc)
    np.testing.assert_allclose(_np(a["mean"])[0], y0, rtol=0, atol=1e-12)
    assert np.all(_np(a["var"])[0] == 0)


def test_fluxdecay_200_machines(ctx):
    """The large-request shape (200 machines, 10 processes) on a short
    horizon: statistics against the oracle on all samples."""
    sc = workloads.fluxdecay(N=40, K=20, T=0.25, dt=0.005)
    r = ctx.run(sc, precision="f32", traj_idx=np.array([3, 39]))
    o = oracle.run(sc, want_traj=True)
    em = mean_err(_np(r["mean"]), o["mean"], o["var"])
    ev = var_err(_np(r["var"]), o["var"])
    et = traj_err(_np(r["traj"]), o["traj"][[3, 39]])
    assert em <= 1e-4 and ev <= 1e-4 and et <= 2e-3, (em, ev, et)


def test_fluxdecay_rejections(ctx, fmc):
    sc = scenario(12, 3, 37, 30, 0.5)
    with pytest.raises(fmc.FmcError) as e:
        ctx.run(sc, precision="f64")
    assert e.value.code == fmc.EINVAL
    bad = sc["model_params"].copy(); bad[0, 2] = -1.0
    with pytest.raises(fmc.FmcError) as e:
        ctx.run(dict(sc, model_params=bad), precision="f32")
    assert e.value.code == fmc.EINVAL
    with pytest.raises(fmc.FmcError) as e:  # 5 processes > 4 per wave for n <= 32
        ctx.run(scenario(12, 5, 37, 30, 0.5), precision="f32")
    assert e.value.code == fmc.EINVAL
    for prec, v in (("f32", 1), ("bf16x3", 2)):  # the BF16 product needs FMC_BF16X3
        with pytest.raises(fmc.FmcError) as e:
            ctx.run(sc, precision=prec, variant=v)
        assert e.value.code == fmc.EINVAL


def test_fluxdecay_long_horizon(ctx):
    """30 s (6000 steps) of 37 machines at N = 256 in FP32, mean and variance
    within the reduced-precision bound 1e-4 of the oracle for every output.
    The common rotor angle of a system without an infinite bus is a neutral
    mode that drifts by radians over such a horizon; the integrator keeps it
    in an FP64 offset per trajectory, so that FP32 rounding does not fall on
    the relative angles (before that, V_R of one machine reached 2.6e-4)."""
    sc = workloads.fluxdecay(n_gen=37, n_dist=6, N=256, K=50, T=30.0, dt=0.005, net_seed=337,
                             seed=5)
    r = ctx.run(sc, precision="f32")
    o = oracle.run(sc)
    em = mean_err(_np(r["mean"]), o["mean"], o["var"])
    ev = var_err(_np(r["var"]), o["var"])
    print(f"flux-decay 37 machines, 30 s, FP32: mean {em:.2e}, variance {ev:.2e}", flush=True)
    assert em <= 1e-4 and ev <= 1e-4, (em, ev)
