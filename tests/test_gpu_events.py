"""Network events on the GPU (the case study's generator trip at t = 1 s and
a line switch of the single machine) against the oracle, through the C ABI.

Tolerances as for the event-free paths: FP64 trajectories and mean/var 1e-10
of each output's scale, FP32 and BF16 x3 mean/var 1e-4.
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


def smib_switch(integrator="rk4", N=100):
    sc = workloads.smib(N=N, K=40, T=3.0, dt=0.01, integrator=integrator)
    y2 = 1.0 / (1j * 0.65)
    sc["event"] = dict(t=1.0, Y=np.array([[y2]]), Yinf=np.array([-y2]))
    return sc


def trip(g=3, **kw):
    d = dict(N=200, K=20, T=2.0)
    d.update(kw)
    sc = workloads.config2(**d)
    sc["event"] = dict(t=1.0, tripped=g)
    return sc


CASES = [("smib_switch", lambda: smib_switch()),
         ("smib_switch_trap", lambda: smib_switch("trap")),
         ("trip_gen3", lambda: trip(3)),
         ("trip_gen0_ragged", lambda: trip(0, N=77)),
         ("trip_gen3_trap", lambda: trip(3, N=64, integrator="trap"))]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_event_fp64_matches_oracle(ctx, name, make):
    sc = make()
    N = sc["N"]
    sel = np.array([0, N // 2, N - 1])
    r = ctx.run(sc, precision="f64", traj_idx=sel)
    o = oracle.run(sc, want_traj=True)
    assert rel_err(_np(r["traj"]), o["traj"][sel]) <= 1e-10
    assert mean_err(_np(r["mean"]), o["mean"], o["var"]) <= 1e-10
    assert rel_err(_np(r["var"]), o["var"]) <= 1e-10
    # the event changes the run: compared with the same run without it
    plain = ctx.run({k: v for k, v in sc.items() if k != "event"}, precision="f64")
    s_e = int(round(sc["event"]["t"] / sc["dt"]))
    assert np.array_equal(_np(plain["mean"])[:s_e + 1], _np(r["mean"])[:s_e + 1])
    assert rel_err(_np(plain["mean"]), _np(r["mean"])) > 1e-6


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
def test_trip_reduced_precision(ctx, prec):
    sc = trip(3)
    r = ctx.run(sc, precision=prec)
    o = oracle.run(sc)
    assert mean_err(_np(r["mean"]), o["mean"], o["var"]) <= 1e-4
    assert rel_err(_np(r["var"]), o["var"]) <= 1e-4


def test_trip_chunks_and_explicit_admittance(ctx):
    sc = trip(5, N=100)
    a = ctx.run(sc, precision="f64")
    b = ctx.run(sc, precision="f64", time_chunk=7)  # the event falls inside a chunk of 7
    assert np.array_equal(_np(a["mean"]), _np(b["mean"]))
    assert np.array_equal(_np(a["var"]), _np(b["var"]))
    # the post-event admittance given explicitly (the oracle's reduction
    # without the tripped machine) instead of reduced by the library
    Yp = oracle.post_event_admittance(sc)
    c = ctx.run(dict(sc, event=dict(sc["event"], Y=Yp)), precision="f64")
    assert rel_err(_np(c["mean"]), _np(a["mean"])) <= 1e-11
    assert rel_err(_np(c["var"]), _np(a["var"])) <= 1e-11


def test_event_rejections(ctx, fmc):
    sc = trip(3, N=10, T=0.5)
    bad = [dict(t=0.5, tripped=3), dict(t=0.1234, tripped=3), dict(t=0.25, tripped=10),
           dict(t=0.25)]
    for ev in bad:
        with pytest.raises(fmc.FmcError) as e:
            ctx.run(dict(sc, event=ev), precision="f64")
        assert e.value.code == fmc.EINVAL, ev
    Y = np.ones((10, 10), dtype=complex)  # the tripped machine's row is not zero
    with pytest.raises(fmc.FmcError) as e:
        ctx.run(dict(sc, event=dict(t=0.25, tripped=3, Y=Y)), precision="f64")
    assert e.value.code == fmc.EINVAL
    ev = dict(sc, event=dict(t=0.25, tripped=3))
    with pytest.raises(fmc.FmcError) as e:
        ctx.run_batch([ev], precision="f32")
    assert e.value.code == fmc.EINVAL
    with pytest.raises(fmc.FmcError) as e:
        ctx.submit(ev, precision="f32")
    assert e.value.code == fmc.EINVAL
    fd = workloads.fluxdecay(n_gen=12, n_dist=3, N=20, K=10, T=0.5, net_seed=312)
    with pytest.raises(fmc.FmcError) as e:
        ctx.run(dict(fd, event=dict(t=0.25, tripped=1)), precision="f32")
    assert e.value.code == fmc.EINVAL
