"""The implicit trapezoidal integrator on the GPU (FP64, classical machines)
against the oracle's trapezoid (full Newton with a dense LU, the same
convergence test), through the C ABI.

Tolerances as for every FP64 path: trajectories and mean/var 1e-10 of each
output's scale.  The two Newton solves stop at |dz| <= 1e-13 (1 + |z|), so
their iterates agree far inside that.
"""
import ctypes as C

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


CASES = [
    ("smib", lambda: workloads.smib(N=100, K=40, T=2.0, dt=0.01, integrator="trap")),
    ("smib_ragged", lambda: workloads.smib(N=65, K=7, T=0.5, dt=0.01, integrator="trap")),
    ("10gen", lambda: workloads.config2(N=130, K=20, T=1.0, integrator="trap")),
    ("12gen_lossy", lambda: workloads.multimachine(n_gen=12, n_dist=5, N=70, K=15, T=0.6,
                                                    net_seed=12, seed=3, integrator="trap")),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_trapezoid_matches_oracle(ctx, name, make):
    sc = make()
    N = sc["N"]
    sel = np.array([0, N // 2, N - 1])
    r = ctx.run(sc, precision="f64", traj_idx=sel)
    o = oracle.run(sc, want_traj=True)
    assert rel_err(_np(r["traj"]), o["traj"][sel]) <= 1e-10
    assert mean_err(_np(r["mean"]), o["mean"], o["var"]) <= 1e-10
    assert rel_err(_np(r["var"]), o["var"]) <= 1e-10
    # and it is not the RK4 path: the two integrators differ at this step size
    rk = ctx.run(dict(sc, integrator="rk4"), precision="f64", traj_idx=sel)
    assert rel_err(_np(rk["traj"]), _np(r["traj"])) > 1e-9


def test_trapezoid_time_chunks_same_bits(ctx):
    sc = workloads.config2(N=100, K=20, T=0.5, integrator="trap")
    a = ctx.run(sc, precision="f64")
    b = ctx.run(sc, precision="f64", time_chunk=7)
    assert np.array_equal(_np(a["mean"]), _np(b["mean"]))
    assert np.array_equal(_np(a["var"]), _np(b["var"]))


def _oracle_rc(sc):
    pb, keep = oracle.problem(sc)
    S, V = oracle.steps(sc), oracle.n_out(sc)
    mean = np.zeros((S + 1, V)); var = np.zeros((S + 1, V))
    nf, nc = C.c_int64(0), C.c_int64(0)
    pm, d0 = np.zeros(pb.n_gen), np.zeros(pb.n_gen)
    rc = oracle.lib().orc_run(C.byref(pb), None, pb.N, None, mean.ctypes.data, var.ctypes.data,
                              None, C.addressof(nf), C.addressof(nc), pm.ctypes.data, d0.ctypes.data)
    return rc, nc.value


def test_trapezoid_reports_newton_failure(ctx, fmc):
    """A step far too long for the disturbance (dt = 0.25 s, sigma = 5 pu):
    the machine loses synchronism and Newton fails in both implementations;
    the outputs are still written (from the last iterates)."""
    sc = workloads.smib(N=16, K=8, T=5.0, dt=0.25, sigma=5.0, integrator="trap")
    rc, nc = _oracle_rc(sc)
    assert rc == -6 and nc == 16
    with pytest.raises(fmc.FmcError) as e:
        ctx.run(sc, precision="f64")
    assert e.value.code == fmc.ENOTCONV
    assert "16 sample paths" in str(e.value)


def test_trapezoid_rejections(ctx, fmc):
    sc = workloads.config2(N=10, K=5, T=0.1, integrator="trap")
    for prec in ("f32", "bf16x3"):
        with pytest.raises(fmc.FmcError) as e:
            ctx.run(sc, precision=prec)
        assert e.value.code == fmc.EINVAL
    big = workloads.multimachine(n_gen=17, n_dist=2, N=10, K=5, T=0.1, net_seed=17,
                                 integrator="trap")
    with pytest.raises(fmc.FmcError) as e:
        ctx.run(big, precision="f64")
    assert e.value.code == fmc.EINVAL
    with pytest.raises(fmc.FmcError) as e:
        ctx.run_batch([sc], precision="f32")
    assert e.value.code == fmc.EINVAL
