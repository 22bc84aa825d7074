"""General Ito disturbances on the GPU (eq. 4 with state-dependent drift and
diffusion: Table I's rows and the wind model of eq. 11), through the C ABI,
against the FP64 oracle.

Bars as for the OU paths: FP64 trajectories and mean/var within 1e-10 of
each output's scale, FP32 and BF16 x3 mean/var within 1e-4.
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


def rel_err(a, b):
    num = np.abs(a - b).reshape(-1, a.shape[-1]).max(axis=0)
    den = np.abs(b).reshape(-1, b.shape[-1]).max(axis=0)
    return float((num / np.where(den == 0, 1, den)).max())


def mean_err(a, m, v):
    num = np.abs(a - m).max(axis=0)
    den = np.maximum(np.abs(m).max(axis=0), np.sqrt(np.abs(v)).max(axis=0))
    return float((num / np.where(den == 0, 1, den)).max())


def smib_proc(spec, x0, N=200, K=40, T=2.0, dt=0.01, calculus="ito", basis="paper"):
    sc = workloads.smib(N=N, K=K, T=T, dt=dt, basis=basis)
    return workloads.with_processes(sc, [spec], calculus=calculus, xi0=[x0])


# every row of Table I, eq. 11, and the calculus and basis choices
SMIB_CASES = [
    ("gauss", lambda: smib_proc(dict(kind="gauss", a=0.2, b=0.01, theta=0.8, gain=1.0, ref=0.2), 0.25)),
    ("beta", lambda: smib_proc(dict(kind="beta", a=6.0, b=9.0, theta=0.5, gain=0.5, ref=0.4), 0.4)),
    ("gamma", lambda: smib_proc(dict(kind="gamma", a=4.0, b=20.0, theta=1.0, gain=1.0, ref=0.2), 0.2)),
    ("gamma_strat", lambda: smib_proc(dict(kind="gamma", a=4.0, b=20.0, theta=1.0, ref=0.2), 0.2,
                                      calculus="stratonovich")),
    ("laplace", lambda: smib_proc(dict(kind="laplace", a=0.1, b=0.05, theta=2.0, ref=0.1), 0.1)),
    ("wind", lambda: workloads.wind_smib(N=150, K=40, T=4.0, dt=0.01, gain=2.0)),
    ("gamma_em", lambda: smib_proc(dict(kind="gamma", a=4.0, b=20.0, theta=1.0, ref=0.2), 0.2,
                                   K=100, T=1.0, dt=0.01, basis="em")),
    ("ou_kind", lambda: smib_proc(dict(kind="ou", gain=0.7, ref=0.01), 0.01)),
]


@pytest.mark.parametrize("name,make", SMIB_CASES, ids=[c[0] for c in SMIB_CASES])
def test_smib_processes_fp64(ctx, name, make):
    sc = make()
    N = sc["N"]
    sel = np.array([0, N // 3, N - 1])
    r = ctx.run(sc, precision="f64", traj_idx=sel)
    o = oracle.run(sc, want_traj=True)
    assert rel_err(_np(r["traj"]), o["traj"][sel]) <= 1e-10
    assert mean_err(_np(r["mean"]), o["mean"], o["var"]) <= 1e-10
    assert rel_err(_np(r["var"]), o["var"]) <= 1e-10
    assert o["var"][-1, 2] > 0  # the process moved


def mixed_10gen(N=200, T=2.0, K=20, **kw):
    """The 10-machine system with a Beta, a Gamma and the wind process (each
    starting at its reference, so t = 0 is the operating point)."""
    return workloads.config2_general(N=N, K=K, T=T, **kw)


def test_multimachine_mixed_processes_fp64(ctx):
    sc = mixed_10gen(N=157)
    sel = np.array([0, 77, 156])
    w = np.zeros(2 * 10 + 3)
    w[10:20] = sc["H"] / np.sum(sc["H"])  # centre-of-inertia frequency deviation
    r = ctx.run(sc, precision="f64", traj_idx=sel, rrf_weights=w)
    o = oracle.run(sc, want_traj=True)
    assert rel_err(_np(r["traj"]), o["traj"][sel]) <= 1e-10
    assert mean_err(_np(r["mean"]), o["mean"], o["var"]) <= 1e-10
    assert rel_err(_np(r["var"]), o["var"]) <= 1e-10
    rr = oracle.rrf_rms(o["traj"], w, sc["dt"])
    assert np.max(np.abs(_np(r["rrf"]) - rr)) <= 1e-10 * np.max(np.abs(rr))


def test_processes_with_generator_trip(ctx):
    sc = mixed_10gen(N=100)
    sc["event"] = dict(t=1.0, tripped=3)
    r = ctx.run(sc, precision="f64")
    o = oracle.run(sc)
    assert mean_err(_np(r["mean"]), o["mean"], o["var"]) <= 1e-10
    assert rel_err(_np(r["var"]), o["var"]) <= 1e-10


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
def test_reduced_precision(ctx, prec):
    sc = mixed_10gen(N=300)
    r = ctx.run(sc, precision=prec)
    o = oracle.run(sc)
    assert mean_err(_np(r["mean"]), o["mean"], o["var"]) <= 1e-4
    assert rel_err(_np(r["var"]), o["var"]) <= 1e-4


def test_time_chunks_give_the_same_bits(ctx):
    sc = mixed_10gen(N=90, T=1.0)
    a = ctx.run(sc, precision="f64")
    b = ctx.run(sc, precision="f64", time_chunk=13)
    assert np.array_equal(_np(a["mean"]), _np(b["mean"]))
    assert np.array_equal(_np(a["var"]), _np(b["var"]))


# one trajectory per lane (7), ten lanes per trajectory in 1 and 4 waves (22,
# 24), two machines per lane (26), sixteen lanes (21) and 16-machine padding
# with eight process slots (30)
GEN_VARIANTS = [7, 22, 24, 26, 21, 30]


@pytest.mark.parametrize("vid", GEN_VARIANTS)
def test_every_variant_form_fp64(ctx, fmc, vid):
    """The general processes on every integrator form: the group kernels
    publish each process's injected power through the lane exchange."""
    sc = mixed_10gen(N=157, T=1.0)
    sel = np.array([0, 77, 156])
    r = ctx.run(sc, precision="f64", traj_idx=sel, variant=vid)
    o = oracle.run(sc, want_traj=True)
    assert rel_err(_np(r["traj"]), o["traj"][sel]) <= 1e-10
    assert mean_err(_np(r["mean"]), o["mean"], o["var"]) <= 1e-10
    assert rel_err(_np(r["var"]), o["var"]) <= 1e-10


@pytest.mark.parametrize("vid", [24, 26])
def test_group_forms_fp32(ctx, vid):
    sc = mixed_10gen(N=300)
    r = ctx.run(sc, precision="f32", variant=vid)
    o = oracle.run(sc)
    assert mean_err(_np(r["mean"]), o["mean"], o["var"]) <= 1e-4
    assert rel_err(_np(r["var"]), o["var"]) <= 1e-4


def test_autotune_for_general_processes(ctx, fmc):
    sc = mixed_10gen(N=64, T=0.5)
    vid = ctx.autotune(sc, precision="f64")
    r = ctx.run(sc, precision="f64", variant=vid)
    o = oracle.run(sc)
    assert mean_err(_np(r["mean"]), o["mean"], o["var"]) <= 1e-10
    assert rel_err(_np(r["var"]), o["var"]) <= 1e-10


def test_rejections(ctx, fmc):
    base = mixed_10gen(N=16, T=0.2)
    bad = [dict(base, integrator="trap"),
           workloads.with_processes(base, [dict(kind="gamma", a=-1.0, b=1.0, theta=1.0)] * 3),
           workloads.with_processes(base, [dict(kind=9)] * 3),
           dict(base, calculus=5)]
    sm = dict(base, dist=dict(base["dist"], sigma_mat=np.eye(3)))
    bad.append(sm)
    for sc in bad:
        with pytest.raises(fmc.FmcError) as e:
            ctx.run(sc, precision="f64")
        assert e.value.code == fmc.EINVAL
    with pytest.raises(fmc.FmcError) as e:
        ctx.run_batch([base], precision="f32")
    assert e.value.code == fmc.EINVAL
    with pytest.raises(fmc.FmcError) as e:
        ctx.submit(base, precision="f32")
    assert e.value.code == fmc.EINVAL
    fd = workloads.fluxdecay(n_gen=12, n_dist=3, N=20, K=10, T=0.5, net_seed=312)
    fdp = workloads.with_processes(fd, [dict(kind="gamma", a=4.0, b=2.0, theta=1.0)] * 3)
    with pytest.raises(fmc.FmcError) as e:
        ctx.run(fdp, precision="f32")
    assert e.value.code == fmc.EINVAL


@pytest.mark.parametrize("basis", ["paper", "em"])
def test_wind_trip_case_study_rrf(ctx, basis):
    """The case-study shape (eq. 11 wind process, generator trip at t = 1 s,
    RMS centre-of-inertia frequency deviation), shortened to 3 s, with the
    KLE basis (K = 6) and the traditional one-hot basis (K = S)."""
    sc = workloads.wind_trip(N=70, T=3.0, dt=0.01)
    if basis == "em":
        sc = dict(sc, basis="em", sampler="srs", K=300)
    w = workloads.coi_frequency_weights(sc)
    r = ctx.run(sc, precision="f64", rrf_weights=w, traj_idx=np.array([0, 69]))
    o = oracle.run(sc, want_traj=True)
    rr = oracle.rrf_rms(o["traj"], w, sc["dt"])
    assert np.max(np.abs(_np(r["rrf"]) - rr)) <= 1e-10 * np.max(np.abs(rr))
    assert rel_err(_np(r["traj"]), o["traj"][[0, 69]]) <= 1e-10
    assert mean_err(_np(r["mean"]), o["mean"], o["var"]) <= 1e-10
