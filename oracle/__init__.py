"""Plain FP64 CPU oracle for the fast Monte Carlo (KLE + LHS) method.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
library never imports, links or calls it, and it shares no code with the GPU
path: the arithmetic lives in ``fmc_oracle.c`` (plain C, scalar loops, OpenMP
over samples only), this module only marshals arguments.

Parity unpinned: nothing.  Every function here is pinned by a CPU test against
a value fixed by mathematics or by a library routine (see tests/test_oracle_*.py);
the multimachine network coupling (electrical power, its Jacobian, the one-axis
machine's network quantities) is pinned away from the operating point, with
losses, against the textbook real and dq forms and against the exact response
of the linearised 10-machine system (tests/test_oracle_network.py).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fmc_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no GPU code, no shared sources)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fPIC",
               "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(C.Structure):
    _fields_ = [
        ("n_gen", C.c_int32), ("f0_hz", C.c_double),
        ("H", C.c_void_p), ("D", C.c_void_p), ("E", C.c_void_p),
        ("delta0", C.c_void_p), ("Pm", C.c_void_p),
        ("Y_re", C.c_void_p), ("Y_im", C.c_void_p),
        ("infinite_bus", C.c_int32), ("V_inf", C.c_double),
        ("Yinf_re", C.c_void_p), ("Yinf_im", C.c_void_p),
        ("n_proc", C.c_int32), ("dist_gen", C.c_void_p),
        ("theta", C.c_void_p), ("sigma", C.c_void_p), ("xi0", C.c_void_p),
        ("T", C.c_double), ("dt", C.c_double), ("K", C.c_int32), ("N", C.c_int64),
        ("seed", C.c_uint64),
        ("basis", C.c_int32), ("sampler", C.c_int32), ("integrator", C.c_int32),
        ("ddof", C.c_int32),
        ("model", C.c_int32), ("model_params", C.c_void_p),
        ("sigma_mat", C.c_void_p),
        ("t_event", C.c_double), ("tripped", C.c_int32),
        ("Yp_re", C.c_void_p), ("Yp_im", C.c_void_p),
        ("Yinfp_re", C.c_void_p), ("Yinfp_im", C.c_void_p),
        ("proc", C.c_void_p), ("calculus", C.c_int32),
    ]


class _Process(C.Structure):
    _fields_ = [("kind", C.c_int32), ("a", C.c_double), ("b", C.c_double),
                ("theta", C.c_double), ("mu", C.c_double * 3), ("sg", C.c_double * 3),
                ("gain", C.c_double), ("ref", C.c_double)]


_PROC_KIND = {"ou": 0, "gauss": 1, "beta": 2, "gamma": 3, "laplace": 4, "poly": 5}
_CALCULUS = {"ito": 0, "stratonovich": 1}


def _processes(specs):
    """ctypes array of process specs from a list of dicts: kind ('ou', the
    Table I rows 'gauss' / 'beta' / 'gamma' / 'laplace' with a, b, theta, or
    'poly' with mu and sg, three coefficients each), gain and ref of the
    injection gain (xi - ref)."""
    arr = (_Process * len(specs))()
    for q, d in zip(arr, specs):
        q.kind = _enum(d.get("kind", "ou"), _PROC_KIND)
        q.a, q.b, q.theta = float(d.get("a", 0.0)), float(d.get("b", 0.0)), float(d.get("theta", 0.0))
        for k, v in enumerate(d.get("mu", (0.0, 0.0, 0.0))):
            q.mu[k] = float(v)
        for k, v in enumerate(d.get("sg", (0.0, 0.0, 0.0))):
            q.sg[k] = float(v)
        q.gain, q.ref = float(d.get("gain", 1.0)), float(d.get("ref", 0.0))
    return arr


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)  # compiles when the library is missing or older than the source
        L = C.CDLL(_LIB)
        P = C.c_void_p
        L.orc_philox4x64_10.argtypes = [P, P, P]
        L.orc_u01.argtypes = [C.c_uint64]
        L.orc_u01.restype = C.c_double
        L.orc_lhs_stratum.argtypes = [C.c_uint64, C.c_int64, C.c_int64, C.c_int64]
        L.orc_lhs_stratum.restype = C.c_int64
        L.orc_ppnd16.argtypes = [C.c_double]
        L.orc_ppnd16.restype = C.c_double
        L.orc_lhs.argtypes = [C.c_uint64, C.c_int32, C.c_int64, C.c_int32, C.c_int64, P, P, P]
        L.orc_lhs_decorrelate.argtypes = [C.c_int32, C.c_int64, P, P]
        L.orc_rrf_rms.argtypes = [P, C.c_int64, C.c_int64, C.c_int32, P, C.c_double, P]
        L.orc_basis.argtypes = [C.c_int32, C.c_int32, C.c_int64, C.c_double, P]
        L.orc_kron.argtypes = [C.c_int32, C.c_int32, P, P, P, P, P, P, P, C.c_int32, P, P, P, P]
        L.orc_run.argtypes = [C.POINTER(_Problem), P, C.c_int64, P, P, P, P, P, P, P, P]
        L.orc_rhs.argtypes = [C.POINTER(_Problem), P, P, P]
        L.orc_initial_state.argtypes = [C.POINTER(_Problem), P, P]
        L.orc_rhs_jac.argtypes = [C.POINTER(_Problem), P, P]
        L.orc_rhs_post.argtypes = [C.POINTER(_Problem), P, P, P]
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.int32)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops over samples."""
    lib().orc_set_num_threads(int(n))


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    o = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(c.ctypes.data, k.ctypes.data, o.ctypes.data)
    return o


def u01(x: int) -> float:
    return float(lib().orc_u01(int(x)))


def stratum(seed: int, i: int, N: int, n: int) -> int:
    return int(lib().orc_lhs_stratum(seed, i, N, n))


def ppnd16(p):
    p = np.atleast_1d(np.asarray(p, dtype=np.float64))
    return np.array([lib().orc_ppnd16(float(x)) for x in p])


def lhs(seed: int, M: int, N: int, sampler: int = 0, sel=None):
    """Strata [M][n_sel] (int32, -1 for SRS) and zeta [M][n_sel] (FP64)."""
    s = None if sel is None else np.ascontiguousarray(sel, dtype=np.int64)
    n_sel = N if s is None else len(s)
    strata = np.zeros((M, n_sel), dtype=np.int32)
    zeta = np.zeros((M, n_sel), dtype=np.float64)
    rc = lib().orc_lhs(seed, M, N, sampler, n_sel, _p(s), strata.ctypes.data, zeta.ctypes.data)
    if rc != 0:
        raise ValueError(f"orc_lhs failed: {rc}")
    return strata, zeta


def lhs_decorrelate(zeta):
    """Correlation-reducing rearrangement of a design [M][N] (rows are the
    variables): returns the rearranged design and each entry's rank in its
    row (int32)."""
    z = np.array(zeta, dtype=np.float64, order="C", copy=True)
    M, N = z.shape
    ranks = np.zeros((M, N), dtype=np.int32)
    rc = lib().orc_lhs_decorrelate(M, N, z.ctypes.data, ranks.ctypes.data)
    if rc != 0:
        raise ValueError(f"orc_lhs_decorrelate failed: {rc}")
    return z, ranks


def rrf_rms(traj, w, dt: float):
    """RMS over the horizon of sum_v w_v y_v(t) for each trajectory [n][S+1][V]."""
    tr = np.ascontiguousarray(traj, dtype=np.float64)
    n, S1, V = tr.shape
    ww = np.ascontiguousarray(w, dtype=np.float64).reshape(V)
    out = np.zeros(n)
    rc = lib().orc_rrf_rms(tr.ctypes.data, n, S1 - 1, V, ww.ctypes.data, dt, out.ctypes.data)
    if rc != 0:
        raise ValueError(f"orc_rrf_rms failed: {rc}")
    return out


def basis(kind: int, K: int, S: int, T: float):
    Phi = np.zeros((K, 2 * S + 1), dtype=np.float64)
    rc = lib().orc_basis(kind, K, S, T, Phi.ctypes.data)
    if rc != 0:
        raise ValueError(f"orc_basis failed: {rc}")
    return Phi


def kron(net: dict):
    """Kron-reduced admittance (complex n_gen x n_gen) of a network dict."""
    ng = int(net["n_gen"])
    fr, to = _i32(net["br_from"]), _i32(net["br_to"])
    r, x = _f64(net["br_r"]), _f64(net["br_x"])
    b = _f64(net.get("br_b"))
    lg, lb = _f64(net.get("load_g")), _f64(net.get("load_b"))
    gb, xd = _i32(net["gen_bus"]), _f64(net["gen_xdp"])
    Yr = np.zeros((ng, ng)); Yi = np.zeros((ng, ng))
    rc = lib().orc_kron(int(net["n_bus"]), len(fr), _p(fr), _p(to), _p(r), _p(x), _p(b),
                        _p(lg), _p(lb), ng, _p(gb), _p(xd), Yr.ctypes.data, Yi.ctypes.data)
    if rc != 0:
        raise ValueError(f"orc_kron failed: {rc}")
    return Yr + 1j * Yi


_SAMPLER = {"lhs": 0, "srs": 1, "lhs_decor": 2}
_BASIS = {"paper": 0, "eigen": 1, "em": 2}
_INTEG = {"rk4": 0, "trap": 1}
_MODEL = {"classical": 0, "fluxdecay": 1}


def _enum(v, table):
    return table[v] if isinstance(v, str) else int(v)


class _Keep:
    """Holds the numpy arrays referenced by a _Problem."""


def post_event_admittance(sc: dict):
    """Reduced admittance after the scenario's event: the event's own Y, or,
    for a generator trip on a network scenario, the network reduced without
    the tripped generator's internal node, placed in the n x n matrix with a
    zero row and column for the tripped machine."""
    ev = sc["event"]
    n = int(sc["n_gen"])
    if ev.get("Y") is not None:
        return np.asarray(ev["Y"], dtype=np.complex128).reshape(n, n)
    g = int(ev.get("tripped", -1))
    if g < 0 or sc.get("net") is None:
        raise ValueError("an event needs its Y, or a tripped machine of a network scenario")
    net = sc["net"]
    keep = np.array([k for k in range(n) if k != g])
    small = kron(dict(net, n_gen=n - 1, gen_bus=np.asarray(net["gen_bus"])[keep],
                      gen_xdp=np.asarray(net["gen_xdp"])[keep]))
    Yp = np.zeros((n, n), dtype=np.complex128)
    Yp[np.ix_(keep, keep)] = small
    return Yp


def problem(sc: dict):
    """Build the C problem struct from a scenario dict (see workloads)."""
    keep = _Keep()
    n = int(sc["n_gen"])
    Y = sc.get("Y")
    if Y is None:
        Y = kron(sc["net"])
    Y = np.asarray(Y, dtype=np.complex128).reshape(n, n)
    keep.Yr, keep.Yi = _f64(Y.real), _f64(Y.imag)
    keep.H, keep.D, keep.E = _f64(sc["H"]), _f64(sc["D"]), _f64(sc["E"])
    keep.d0 = _f64(sc.get("delta0"))
    keep.Pm = _f64(sc.get("Pm"))
    inf = bool(sc.get("infinite_bus", False))
    if inf:
        Yinf = np.asarray(sc["Yinf"], dtype=np.complex128).reshape(n)
        keep.Yir, keep.Yii = _f64(Yinf.real), _f64(Yinf.imag)
    else:
        keep.Yir = keep.Yii = None
    d = sc["dist"]
    keep.dg = _i32(d["gen"])
    keep.th, keep.sg = _f64(d["theta"]), _f64(d["sigma"])
    keep.x0 = _f64(d.get("xi0"))
    keep.sm = _f64(np.asarray(d["sigma_mat"], dtype=np.float64).reshape(-1)) \
        if d.get("sigma_mat") is not None else None
    model = _enum(sc.get("model", 0), _MODEL)
    keep.mp = _f64(sc.get("model_params")) if model == 1 else None
    keep.proc = _processes(d["proc"]) if d.get("proc") is not None else None
    ev = sc.get("event")
    keep.Ypr = keep.Ypi = keep.Yipr = keep.Yipi = None
    if ev is not None:
        Yp = post_event_admittance(sc)
        keep.Ypr, keep.Ypi = _f64(Yp.real), _f64(Yp.imag)
        if ev.get("Yinf") is not None:
            Yip = np.asarray(ev["Yinf"], dtype=np.complex128).reshape(n)
            keep.Yipr, keep.Yipi = _f64(Yip.real), _f64(Yip.imag)
    pb = _Problem(
        n_gen=n, f0_hz=float(sc.get("f0", 60.0)),
        H=_p(keep.H), D=_p(keep.D), E=_p(keep.E), delta0=_p(keep.d0), Pm=_p(keep.Pm),
        Y_re=_p(keep.Yr), Y_im=_p(keep.Yi), infinite_bus=int(inf),
        V_inf=float(sc.get("V_inf", 1.0)), Yinf_re=_p(keep.Yir), Yinf_im=_p(keep.Yii),
        n_proc=len(keep.dg), dist_gen=_p(keep.dg), theta=_p(keep.th), sigma=_p(keep.sg),
        xi0=_p(keep.x0), T=float(sc["T"]), dt=float(sc["dt"]), K=int(sc["K"]),
        N=int(sc["N"]), seed=int(sc.get("seed", 0)),
        basis=_enum(sc.get("basis", 0), _BASIS), sampler=_enum(sc.get("sampler", 0), _SAMPLER),
        integrator=_enum(sc.get("integrator", 0), _INTEG), ddof=int(sc.get("ddof", 1)),
        model=model, model_params=_p(keep.mp), sigma_mat=_p(keep.sm),
        t_event=float(ev["t"]) if ev is not None else 0.0,
        tripped=int(ev.get("tripped", -1)) if ev is not None else -1,
        Yp_re=_p(keep.Ypr), Yp_im=_p(keep.Ypi), Yinfp_re=_p(keep.Yipr), Yinfp_im=_p(keep.Yipi),
        proc=C.addressof(keep.proc) if keep.proc is not None else None,
        calculus=_enum(sc.get("calculus", "ito"), _CALCULUS))
    return pb, keep


def n_out(sc: dict) -> int:
    """Output variables per time: 2n + P (classical) or 6n + P (flux decay)."""
    n = int(sc["n_gen"]); P = len(sc["dist"]["gen"])
    return (6 * n if _enum(sc.get("model", 0), _MODEL) == 1 else 2 * n) + P


def steps(sc: dict) -> int:
    return int(round(float(sc["T"]) / float(sc["dt"])))


def run(sc: dict, zeta=None, sel=None, want_traj=False, allow_nonfinite=False):
    """Run the method on a scenario.

    Returns dict(mean, var [(S+1), V], traj [n_sel, S+1, V] or None, Pm, delta0,
    nonfinite).  ``zeta`` ([M][n_sel]) replaces the LHS step; ``sel`` picks the
    samples of the N-sample design to run (statistics are over them).
    """
    pb, keep = problem(sc)
    n = pb.n_gen
    S = steps(sc)
    V = n_out(sc)
    s = None if sel is None else np.ascontiguousarray(sel, dtype=np.int64)
    n_sel = pb.N if s is None else len(s)
    z = None if zeta is None else np.ascontiguousarray(zeta, dtype=np.float64)
    if z is not None:
        assert z.shape == (pb.n_proc * pb.K, n_sel), z.shape
    mean = np.zeros((S + 1, V)); var = np.zeros((S + 1, V))
    traj = np.zeros((n_sel, S + 1, V)) if want_traj else None
    nf = C.c_int64(0); nc = C.c_int64(0)
    pm = np.zeros(n); d0 = np.zeros(n)
    rc = lib().orc_run(C.byref(pb), _p(z), n_sel, _p(s), mean.ctypes.data, var.ctypes.data,
                       _p(traj), C.addressof(nf), C.addressof(nc), pm.ctypes.data, d0.ctypes.data)
    if rc not in (0, -5) or (rc == -5 and not allow_nonfinite):
        raise RuntimeError(f"orc_run failed: {rc} (nonfinite={nf.value}, notconv={nc.value})")
    return dict(mean=mean, var=var, traj=traj, Pm=pm, delta0=d0, nonfinite=nf.value)


def rhs(sc: dict, y, w):
    pb, keep = problem(sc)
    y = _f64(y); w = _f64(w)
    dy = np.zeros_like(y)
    rc = lib().orc_rhs(C.byref(pb), y.ctypes.data, _p(w) if len(w) else None, dy.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"orc_rhs failed: {rc}")
    return dy


def rhs_post(sc: dict, y, w):
    """Right-hand side of the scenario's post-event model at state y."""
    pb, keep = problem(sc)
    y = _f64(y); w = _f64(w)
    dy = np.zeros_like(y)
    rc = lib().orc_rhs_post(C.byref(pb), y.ctypes.data, _p(w) if len(w) else None, dy.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"orc_rhs_post failed: {rc}")
    return dy


def rhs_jac(sc: dict, y):
    """Jacobian of the classical model's right-hand side at state y ([ny][ny])."""
    pb, keep = problem(sc)
    y = _f64(y)
    J = np.zeros((len(y), len(y)))
    rc = lib().orc_rhs_jac(C.byref(pb), y.ctypes.data, J.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"orc_rhs_jac failed: {rc}")
    return J


def initial_state(sc: dict):
    """Operating point (initial state [ny]) and exciter references Vref [n]
    (zeros for the classical model)."""
    pb, keep = problem(sc)
    y0 = np.zeros(n_out(sc)); vref = np.zeros(int(sc["n_gen"]))
    rc = lib().orc_initial_state(C.byref(pb), y0.ctypes.data, vref.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"orc_initial_state failed: {rc}")
    return y0, vref


def kle_paths(zeta, Phi, P: int, K: int, c0: int = 0, C_cols=None):
    """KLE white-noise surrogates (eqs. 8-9): w[c][p][n] = sum_j zeta[pK+j][n] Phi[j][c0+c].

    FP64 matrix products (numpy), one per process, nothing else.
    """
    zeta = np.asarray(zeta, dtype=np.float64)
    Phi = np.asarray(Phi, dtype=np.float64)
    if C_cols is None:
        C_cols = Phi.shape[1] - c0
    N = zeta.shape[1]
    w = np.zeros((C_cols, P, N))
    for p in range(P):
        w[:, p, :] = Phi[:K, c0:c0 + C_cols].T @ zeta[p * K:(p + 1) * K, :]
    return w
