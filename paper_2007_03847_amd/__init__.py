"""Python binding of libfmc (include/fmc.h): argument marshalling only.

Every step of the method runs in the library's gfx950 kernels; this module
converts scenario dicts (see ``workloads``) into the C structs, hands over
device pointers of torch tensors and the current HIP stream, and returns
torch tensors.  PyTorch supplies device memory and streams, nothing else.

The library is required: importing this package raises if ``libfmc.so`` has
not been built (``python -m paper_2007_03847_amd.build``).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfmc.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2007_03847_amd.build`")

# torch first: it brings up the HIP runtime and devices the process works
# with; loading the library before it leaves the library without a device.
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)

# ---------------------------------------------------------------- constants
OK, EINVAL, ENOMEM, EBUSY, EDEVICE, ENONFINITE, ENOTCONV, ECANCELLED, EAGAIN, ETIMEDOUT = \
    0, -1, -2, -3, -4, -5, -6, -7, -8, -9
F64, F32, BF16X3 = 0, 1, 2
BASIS = {"paper": 0, "eigen": 1, "em": 2}
SAMPLER = {"lhs": 0, "srs": 1, "lhs_decor": 2}
INTEGRATOR = {"rk4": 0, "trap": 1}
PRECISION = {"f64": F64, "f32": F32, "bf16x3": BF16X3}
CLASSICAL, FLUXDECAY_IEEET1 = 0, 1
MODEL = {"classical": CLASSICAL, "fluxdecay": FLUXDECAY_IEEET1}
FD_NPARAM = 9  # Xd, X'd, T'do, KA, TA, KE, TE, KF, TF
MEM_HOST, MEM_DEVICE = 0, 1
ABI_VERSION = 4

_P = C.c_void_p


class FmcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"fmc error {code}: {msg}")
        self.code = code


class Network(C.Structure):
    _fields_ = [("n_bus", C.c_int32), ("n_branch", C.c_int32), ("n_gen", C.c_int32),
                ("br_from", _P), ("br_to", _P), ("br_r", _P), ("br_x", _P), ("br_b", _P),
                ("load_g", _P), ("load_b", _P), ("gen_bus", _P), ("gen_xdp", _P)]


class Event(C.Structure):
    _fields_ = [("t", C.c_double), ("tripped", C.c_int32), ("Y_re", _P), ("Y_im", _P),
                ("Yinf_re", _P), ("Yinf_im", _P)]


class System(C.Structure):
    _fields_ = [("n_gen", C.c_int32), ("f0_hz", C.c_double),
                ("H", _P), ("D", _P), ("E", _P), ("delta0", _P), ("Pm", _P),
                ("Y_re", _P), ("Y_im", _P), ("net", C.POINTER(Network)),
                ("infinite_bus", C.c_int32), ("V_inf", C.c_double),
                ("Yinf_re", _P), ("Yinf_im", _P), ("model", C.c_int32), ("model_params", _P),
                ("event", C.POINTER(Event))]


class Process(C.Structure):
    _fields_ = [("kind", C.c_int32), ("a", C.c_double), ("b", C.c_double),
                ("theta", C.c_double), ("mu", C.c_double * 3), ("sg", C.c_double * 3),
                ("gain", C.c_double), ("ref", C.c_double)]


PROC_KIND = {"ou": 0, "gauss": 1, "beta": 2, "gamma": 3, "laplace": 4, "poly": 5}
CALCULUS = {"ito": 0, "stratonovich": 1}


class Disturbance(C.Structure):
    _fields_ = [("n_proc", C.c_int32), ("gen", _P), ("theta", _P), ("sigma", _P), ("xi0", _P),
                ("sigma_mat", _P), ("proc", C.POINTER(Process)), ("calculus", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("T", C.c_double), ("dt", C.c_double), ("K", C.c_int32), ("N", C.c_int64),
                ("seed", C.c_uint64), ("basis", C.c_int32), ("sampler", C.c_int32),
                ("integrator", C.c_int32), ("precision", C.c_int32), ("ddof", C.c_int32),
                ("variant", C.c_int32), ("time_chunk", C.c_int32), ("zeta_in", _P)]


class Report(C.Structure):
    _fields_ = [("t_total_s", C.c_double), ("t_lhs_s", C.c_double), ("t_gemm_s", C.c_double),
                ("t_integrate_s", C.c_double), ("t_stats_s", C.c_double),
                ("n_nonfinite", C.c_int64), ("first_nonfinite", C.c_int64),
                ("variant_id", C.c_int32), ("lanes_per_traj", C.c_int32), ("tile", C.c_int32),
                ("time_chunk", C.c_int32), ("hbm_peak_bytes", C.c_int64),
                ("queue_wait_s", C.c_double), ("latency_s", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Outputs(C.Structure):
    _fields_ = [("mean", _P), ("var", _P), ("n_traj", C.c_int32), ("traj_idx", _P),
                ("traj", _P), ("strata", _P), ("zeta", _P), ("mem_kind", C.c_int32),
                ("report", C.POINTER(Report)), ("rrf", _P), ("rrf_w", _P)]


class Scenario(C.Structure):
    _fields_ = [("sys", C.POINTER(System)), ("dist", C.POINTER(Disturbance)),
                ("par", C.POINTER(Params))]


_ctx_p = C.c_void_p
_sig = {
    "fmc_abi_version": ([], C.c_int),
    "fmc_last_error": ([], C.c_char_p),
    "fmc_context_create": ([C.c_int, C.c_size_t, _P, C.POINTER(_ctx_p)], C.c_int),
    "fmc_context_destroy": ([_ctx_p], C.c_int),
    "fmc_set_stream": ([_ctx_p, _P], C.c_int),
    "fmc_kron_reduce": ([_ctx_p, C.POINTER(Network), _P, _P], C.c_int),
    "fmc_lhs": ([_ctx_p, C.c_uint64, C.c_int32, C.c_int64, C.c_int32, _P, _P], C.c_int),
    "fmc_lhs_decorrelate": ([_ctx_p, C.c_int32, C.c_int64, _P, _P], C.c_int),
    "fmc_rrf_rms": ([_ctx_p, _P, C.c_int64, C.c_int64, C.c_int32, _P, C.c_double, _P], C.c_int),
    "fmc_rrf_rms_noalloc": ([_ctx_p, _P, C.c_int64, C.c_int64, C.c_int32, _P, C.c_double, _P],
                            C.c_int),
    "fmc_basis": ([_ctx_p, C.c_int32, C.c_int32, C.c_int64, C.c_double, _P], C.c_int),
    "fmc_kle_paths": ([_ctx_p, C.c_int32, C.c_int32, C.c_int32, C.c_int64, C.c_int64,
                       C.c_int64, _P, _P, C.c_int64, _P], C.c_int),
    "fmc_run": ([_ctx_p, C.POINTER(System), C.POINTER(Disturbance), C.POINTER(Params),
                 C.POINTER(Outputs)], C.c_int),
    "fmc_run_batch": ([_ctx_p, C.c_int32, C.POINTER(Scenario), C.POINTER(Outputs)], C.c_int),
    "fmc_submit": ([_ctx_p, C.POINTER(Scenario), C.POINTER(Outputs), C.POINTER(C.c_uint64)],
                   C.c_int),
    "fmc_poll": ([_ctx_p, C.c_uint64], C.c_int),
    "fmc_wait": ([_ctx_p, C.c_uint64, C.c_double], C.c_int),
    "fmc_cancel": ([_ctx_p, C.c_uint64], C.c_int),
    "fmc_footprint": ([C.POINTER(Scenario), C.POINTER(C.c_int64)], C.c_int),
    "fmc_autotune": ([_ctx_p, C.POINTER(Scenario), C.POINTER(C.c_int32)], C.c_int),
}
for _name, (_args, _res) in _sig.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res

EXPORTED = tuple(_sig)


def last_error() -> str:
    return _lib.fmc_last_error().decode()


def _check(rc, allow=()):
    if rc != OK and rc not in allow:
        raise FmcError(rc, last_error())
    return rc


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.int32)


def _ptr(a):
    return None if a is None else a.ctypes.data


def _dptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class _Keep(list):
    """Keeps the numpy arrays and ctypes objects a call points into alive."""


def _network(net, keep):
    arrs = dict(br_from=_i32(net["br_from"]), br_to=_i32(net["br_to"]), br_r=_f64(net["br_r"]),
                br_x=_f64(net["br_x"]), br_b=_f64(net.get("br_b")), load_g=_f64(net.get("load_g")),
                load_b=_f64(net.get("load_b")), gen_bus=_i32(net["gen_bus"]),
                gen_xdp=_f64(net["gen_xdp"]))
    keep.append(arrs)
    nw = Network(n_bus=int(net["n_bus"]), n_branch=len(arrs["br_from"]), n_gen=int(net["n_gen"]),
                 **{k: _ptr(v) for k, v in arrs.items()})
    keep.append(nw)
    return nw


def _enum(v, table):
    return table[v] if isinstance(v, str) else int(v)


def scenario_structs(sc: dict, precision="f64", variant=-1, time_chunk=0, zeta_in=None,
                     keep=None):
    """C structs (System, Disturbance, Params) for a scenario dict."""
    keep = _Keep() if keep is None else keep
    n = int(sc["n_gen"])
    a = dict(H=_f64(sc["H"]), D=_f64(sc["D"]), E=_f64(sc["E"]), delta0=_f64(sc.get("delta0")),
             Pm=_f64(sc.get("Pm")))
    Y = sc.get("Y")
    net_p = None
    if Y is not None:
        Y = np.asarray(Y, dtype=np.complex128).reshape(n, n)
        a["Y_re"], a["Y_im"] = _f64(Y.real), _f64(Y.imag)
    else:
        a["Y_re"] = a["Y_im"] = None
        net_p = C.pointer(_network(sc["net"], keep))
    inf = bool(sc.get("infinite_bus", False))
    if inf:
        Yinf = np.asarray(sc["Yinf"], dtype=np.complex128).reshape(n)
        a["Yinf_re"], a["Yinf_im"] = _f64(Yinf.real), _f64(Yinf.imag)
    else:
        a["Yinf_re"] = a["Yinf_im"] = None
    model = _enum(sc.get("model", 0), MODEL)
    mp = sc.get("model_params")
    a["model_params"] = (np.ascontiguousarray(mp, dtype=np.float64).reshape(n, -1)
                         if model == FLUXDECAY_IEEET1 and mp is not None else None)
    ev_p = None
    ev = sc.get("event")
    if ev is not None:
        e = {}
        if ev.get("Y") is not None:
            Ye = np.asarray(ev["Y"], dtype=np.complex128).reshape(n, n)
            e["Y_re"], e["Y_im"] = _f64(Ye.real), _f64(Ye.imag)
        if ev.get("Yinf") is not None:
            Yi = np.asarray(ev["Yinf"], dtype=np.complex128).reshape(n)
            e["Yinf_re"], e["Yinf_im"] = _f64(Yi.real), _f64(Yi.imag)
        keep.append(e)
        evs = Event(t=float(ev["t"]), tripped=int(ev.get("tripped", -1)),
                    **{k: _ptr(v) for k, v in e.items()})
        keep.append(evs)
        ev_p = C.pointer(evs)
    keep.append(a)
    sysd = System(n_gen=n, f0_hz=float(sc.get("f0", 60.0)), H=_ptr(a["H"]), D=_ptr(a["D"]),
                  E=_ptr(a["E"]), delta0=_ptr(a["delta0"]), Pm=_ptr(a["Pm"]),
                  Y_re=_ptr(a["Y_re"]), Y_im=_ptr(a["Y_im"]), net=net_p, infinite_bus=int(inf),
                  V_inf=float(sc.get("V_inf", 1.0)), Yinf_re=_ptr(a["Yinf_re"]),
                  Yinf_im=_ptr(a["Yinf_im"]), model=model, model_params=_ptr(a["model_params"]),
                  event=ev_p)
    d = sc["dist"]
    sm = d.get("sigma_mat")
    b = dict(gen=_i32(d["gen"]), theta=_f64(d["theta"]), sigma=_f64(d["sigma"]),
             xi0=_f64(d.get("xi0")),
             sigma_mat=None if sm is None else _f64(np.asarray(sm, dtype=np.float64).reshape(-1)))
    keep.append(b)
    procs = None
    if d.get("proc") is not None:
        procs = (Process * len(d["proc"]))()
        for q, spec in zip(procs, d["proc"]):
            q.kind = _enum(spec.get("kind", "ou"), PROC_KIND)
            q.a, q.b = float(spec.get("a", 0.0)), float(spec.get("b", 0.0))
            q.theta = float(spec.get("theta", 0.0))
            for j, v in enumerate(spec.get("mu", (0.0, 0.0, 0.0))):
                q.mu[j] = float(v)
            for j, v in enumerate(spec.get("sg", (0.0, 0.0, 0.0))):
                q.sg[j] = float(v)
            q.gain, q.ref = float(spec.get("gain", 1.0)), float(spec.get("ref", 0.0))
        keep.append(procs)
    dist = Disturbance(n_proc=len(b["gen"]), gen=_ptr(b["gen"]), theta=_ptr(b["theta"]),
                       sigma=_ptr(b["sigma"]), xi0=_ptr(b["xi0"]), sigma_mat=_ptr(b["sigma_mat"]),
                       proc=procs, calculus=_enum(sc.get("calculus", "ito"), CALCULUS))
    par = Params(T=float(sc["T"]), dt=float(sc["dt"]), K=int(sc["K"]), N=int(sc["N"]),
                 seed=int(sc.get("seed", 0)), basis=_enum(sc.get("basis", 0), BASIS),
                 sampler=_enum(sc.get("sampler", 0), SAMPLER),
                 integrator=_enum(sc.get("integrator", 0), INTEGRATOR),
                 precision=_enum(precision, PRECISION), ddof=int(sc.get("ddof", 1)),
                 variant=int(variant), time_chunk=int(time_chunk),
                 zeta_in=_dptr(zeta_in))
    keep.extend([sysd, dist, par])
    return sysd, dist, par, keep


def n_out(sc: dict) -> int:
    """Output variables per time: 2n + P (classical) or 6n + P (flux decay)."""
    n = int(sc["n_gen"]); P = len(sc["dist"]["gen"])
    return (6 * n if _enum(sc.get("model", 0), MODEL) == FLUXDECAY_IEEET1 else 2 * n) + P


def steps(sc: dict) -> int:
    """Output steps S = T/dt for sizing outputs (0 if dt is not positive; the
    library rejects such a scenario)."""
    dt = float(sc["dt"])
    if not dt > 0.0:
        return 0
    return max(int(round(float(sc["T"]) / dt)), 0)


class Context:
    """A library context on one device, bound to torch's current stream."""

    def __init__(self, device: int = 0, hbm_budget: int = 0, stream=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        self._h = _ctx_p()
        _check(_lib.fmc_context_create(device, hbm_budget, C.c_void_p(stream.cuda_stream),
                                       C.byref(self._h)))

    def close(self):
        if self._h:
            _lib.fmc_context_destroy(self._h)
            self._h = _ctx_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        self.stream = stream
        _check(_lib.fmc_set_stream(self._h, C.c_void_p(stream.cuda_stream)))

    # ---------------------------------------------------------- single steps
    def kron_reduce(self, net: dict):
        keep = _Keep()
        nw = _network(net, keep)
        ng = int(net["n_gen"])
        yr = np.zeros((ng, ng)); yi = np.zeros((ng, ng))
        _check(_lib.fmc_kron_reduce(self._h, C.byref(nw), yr.ctypes.data, yi.ctypes.data))
        return yr + 1j * yi

    def lhs(self, seed: int, M: int, N: int, sampler="lhs", want_strata=True):
        t = self.torch
        zeta = t.empty((M, N), dtype=t.float64, device=self.device)
        strata = t.empty((M, N), dtype=t.int32, device=self.device) if want_strata else None
        _check(_lib.fmc_lhs(self._h, seed, M, N, _enum(sampler, SAMPLER), _dptr(strata),
                            _dptr(zeta)))
        return strata, zeta

    def lhs_decorrelate(self, zeta, want_strata=True):
        """Correlation-reducing permutation of a device design [M][N] in place;
        returns the rank of each entry in its row (int32) if asked for."""
        t = self.torch
        assert zeta.dtype == t.float64 and zeta.is_contiguous() and zeta.dim() == 2
        assert zeta.device == t.device(self.device)
        M, N = zeta.shape
        strata = t.empty((M, N), dtype=t.int32, device=self.device) if want_strata else None
        _check(_lib.fmc_lhs_decorrelate(self._h, M, N, _dptr(zeta), _dptr(strata)))
        return strata

    def rrf_rms(self, traj, w, dt: float):
        """RMS over the horizon of sum_v w[v] y_v(t) for each trajectory of a
        device tensor [n][S+1][V] (FP64); returns a device tensor [n]."""
        t = self.torch
        assert traj.dtype == t.float64 and traj.is_contiguous() and traj.dim() == 3
        assert traj.device == t.device(self.device)
        n, S1, V = traj.shape
        ww = np.ascontiguousarray(w, dtype=np.float64).reshape(V)
        out = t.empty(n, dtype=t.float64, device=self.device)
        _check(_lib.fmc_rrf_rms(self._h, _dptr(traj), n, S1 - 1, V, ww.ctypes.data, float(dt),
                                _dptr(out)))
        return out

    def rrf_rms_noalloc(self, traj, w, dt: float, out):
        """rrf_rms through the allocation-free entry point: the caller passes
        the output tensor (device [n] FP64) as well."""
        t = self.torch
        assert traj.dtype == t.float64 and traj.is_contiguous() and traj.dim() == 3
        assert out.dtype == t.float64 and out.is_contiguous() and out.numel() >= traj.shape[0]
        n, S1, V = traj.shape
        ww = np.ascontiguousarray(w, dtype=np.float64).reshape(V)
        _check(_lib.fmc_rrf_rms_noalloc(self._h, _dptr(traj), n, S1 - 1, V, ww.ctypes.data,
                                        float(dt), _dptr(out)))
        return out

    def basis(self, kind, K: int, S: int, T: float):
        t = self.torch
        phi = t.empty((K, 2 * S + 1), dtype=t.float64, device=self.device)
        _check(_lib.fmc_basis(self._h, _enum(kind, BASIS), K, S, T, _dptr(phi)))
        return phi

    def kle_paths(self, zeta, phi, P: int, K: int, C_cols: int, c0: int = 0, precision="f64"):
        t = self.torch
        assert zeta.dtype == t.float64 and zeta.is_contiguous() and zeta.shape[0] == P * K
        assert phi.dtype == t.float64 and phi.is_contiguous() and phi.shape[0] >= K
        N = zeta.shape[1]
        prec = _enum(precision, PRECISION)
        dt = t.float64 if prec == F64 else t.float32
        w = t.empty((C_cols, P, N), dtype=dt, device=self.device)
        _check(_lib.fmc_kle_paths(self._h, prec, P, K, N, C_cols, c0, _dptr(zeta), _dptr(phi),
                                  phi.shape[1], _dptr(w)))
        return w

    def autotune(self, sc: dict, precision="f64") -> int:
        """Pick (and cache in the context) the fastest integrator variant."""
        sysd, dist, par, keep = scenario_structs(sc, precision)
        s = Scenario(C.pointer(sysd), C.pointer(dist), C.pointer(par))
        v = C.c_int32(-1)
        _check(_lib.fmc_autotune(self._h, C.byref(s), C.byref(v)))
        return int(v.value)

    # ------------------------------------------------------------ whole path
    def run(self, sc: dict, precision="f64", traj_idx=None, want_design=False, variant=-1,
            time_chunk=0, zeta_in=None, outputs=None, allow_nonfinite=False, rrf_weights=None):
        """Alg. 1 on the GPU.  Returns dict(mean, var[, traj, strata, zeta, rrf], report);
        rrf_weights ([V]) asks for the RRF of every sample accumulated while
        integrating (see fmc_outputs.rrf)."""
        t = self.torch
        n = int(sc["n_gen"]); P = len(sc["dist"]["gen"]); S = steps(sc)
        V = n_out(sc); M = P * int(sc["K"]); N = int(sc["N"])
        sysd, dist, par, keep = scenario_structs(sc, precision, variant, time_chunk, zeta_in)
        res = outputs or {}
        mean = res.get("mean"); var = res.get("var")
        if mean is None:
            mean = t.empty((S + 1, V), dtype=t.float64, device=self.device)
        if var is None:
            var = t.empty((S + 1, V), dtype=t.float64, device=self.device)
        traj = None
        idx = None
        if traj_idx is not None and len(traj_idx):
            idx = np.ascontiguousarray(traj_idx, dtype=np.int64)
            keep.append(idx)
            traj = t.empty((len(idx), S + 1, V), dtype=t.float64, device=self.device)
        strata = zeta = None
        if want_design:
            strata = t.empty((M, N), dtype=t.int32, device=self.device)
            zeta = t.empty((M, N), dtype=t.float64, device=self.device)
        rep = Report()
        rrf = rrf_w = None
        if rrf_weights is not None:
            rrf_w = np.ascontiguousarray(rrf_weights, dtype=np.float64).reshape(V)
            keep.append(rrf_w)
            rrf = t.empty(N, dtype=t.float64, device=self.device)
        out = Outputs(mean=_dptr(mean), var=_dptr(var), n_traj=0 if idx is None else len(idx),
                      traj_idx=_ptr(idx), traj=_dptr(traj), strata=_dptr(strata),
                      zeta=_dptr(zeta), mem_kind=MEM_DEVICE, report=C.pointer(rep),
                      rrf=_dptr(rrf), rrf_w=_ptr(rrf_w))
        rc = _lib.fmc_run(self._h, C.byref(sysd), C.byref(dist), C.byref(par), C.byref(out))
        _check(rc, allow=(ENONFINITE,) if allow_nonfinite else ())
        r = dict(mean=mean, var=var, report=rep.as_dict(), rc=rc)
        if traj is not None:
            r["traj"] = traj
        if rrf is not None:
            r["rrf"] = rrf
        if want_design:
            r["strata"] = strata
            r["zeta"] = zeta
        return r


def _outputs_for(ctx, sc, traj_idx, keep):
    t = ctx.torch
    n = int(sc["n_gen"]); P = len(sc["dist"]["gen"]); S = steps(sc)
    V = n_out(sc)
    mean = t.empty((S + 1, V), dtype=t.float64, device=ctx.device)
    var = t.empty((S + 1, V), dtype=t.float64, device=ctx.device)
    traj = None
    idx = None
    if traj_idx is not None and len(traj_idx):
        idx = np.ascontiguousarray(traj_idx, dtype=np.int64)
        keep.append(idx)
        traj = t.empty((len(idx), S + 1, V), dtype=t.float64, device=ctx.device)
    rep = Report()
    keep.append(rep)
    out = Outputs(mean=_dptr(mean), var=_dptr(var), n_traj=0 if idx is None else len(idx),
                  traj_idx=_ptr(idx), traj=_dptr(traj), strata=None, zeta=None,
                  mem_kind=MEM_DEVICE, report=C.pointer(rep))
    return out, dict(mean=mean, var=var, traj=traj, report=rep)


def _run_batch(ctx, scs, precision="f32", traj_idx=None, variant=-1, allow_nonfinite=False,
               time_chunk=0):
    keep = _Keep()
    n = len(scs)
    arr = (Scenario * n)()
    outs = (Outputs * n)()
    res = []
    for i, sc in enumerate(scs):
        v = variant[i] if isinstance(variant, (list, tuple)) else variant
        sysd, dist, par, _ = scenario_structs(sc, precision, v, time_chunk, keep=keep)
        arr[i] = Scenario(C.pointer(sysd), C.pointer(dist), C.pointer(par))
        ti = None if traj_idx is None else traj_idx[i]
        o, r = _outputs_for(ctx, sc, ti, keep)
        outs[i] = o
        res.append(r)
    rc = _lib.fmc_run_batch(ctx._h, n, arr, outs)
    _check(rc, allow=(ENONFINITE,) if allow_nonfinite else ())
    for r in res:
        rep = r.pop("report")
        r["report"] = rep.as_dict()
        r["rc"] = rc
        if r["traj"] is None:
            r.pop("traj")
    return res


Context.run_batch = lambda self, scs, precision="f32", traj_idx=None, variant=-1, \
    allow_nonfinite=False, time_chunk=0: _run_batch(self, scs, precision, traj_idx, variant,
                                                    allow_nonfinite, time_chunk)
Context.run_batch.__doc__ = """Batched form: a list of scenario dicts in one persistent launch.

Returns one dict(mean, var[, traj], report, rc) per scenario.  traj_idx, if
given, is a list (one entry per scenario, None allowed) of sample indices;
time_chunk > 0 sets the steps per tick (else 250); variant is one id for
every scenario or a list of ids (-1: tuned).  Variant ids 0-10 are the
lane variants, 11-13 the FP32 matrix-core variants for up to 32, 48, 64
machines and 14-16 their BF16 x3 forms (FMC_BF16X3 scenarios only), 17 and 18
the same pair for up to 16 machines."""


class Ticket:
    """A served request: its outputs (device tensors) stay referenced here
    until the library reports completion (poll or wait)."""

    def __init__(self, ctx, tid, mean, var, rep, keep):
        self.ctx, self.id, self.mean, self.var = ctx, tid, mean, var
        self._rep, self._keep = rep, keep
        self.rc = None

    def _final(self, rc, allow):
        self.rc = rc
        _check(rc, allow=allow)
        return dict(mean=self.mean, var=self.var, report=self._rep.as_dict(), rc=rc)

    def poll(self, allow_nonfinite=False):
        """None while the request runs, else its result dict."""
        rc = _lib.fmc_poll(self.ctx._h, self.id)
        if rc == EAGAIN:
            return None
        return self._final(rc, (ENONFINITE,) if allow_nonfinite else ())

    def wait(self, timeout=-1.0, allow_nonfinite=False):
        rc = _lib.fmc_wait(self.ctx._h, self.id, float(timeout))
        if rc == ETIMEDOUT:
            raise FmcError(rc, last_error())
        return self._final(rc, (ENONFINITE,) if allow_nonfinite else ())

    def cancel(self):
        _check(_lib.fmc_cancel(self.ctx._h, self.id))

    def __del__(self):
        # the library writes into this ticket's tensors until it completes:
        # a ticket dropped early is cancelled and waited for
        try:
            if self.rc is None and self.ctx._h:
                _lib.fmc_cancel(self.ctx._h, self.id)
                _lib.fmc_wait(self.ctx._h, self.id, -1.0)
        except Exception:
            pass


def _submit(ctx, sc, precision="f32", variant=-1, time_chunk=0):
    keep = _Keep()
    sysd, dist, par, _ = scenario_structs(sc, precision, variant, time_chunk, keep=keep)
    s = Scenario(C.pointer(sysd), C.pointer(dist), C.pointer(par))
    t = ctx.torch
    n = int(sc["n_gen"]); P = len(sc["dist"]["gen"]); S = steps(sc)
    V = n_out(sc)
    mean = t.empty((S + 1, V), dtype=t.float64, device=ctx.device)
    var = t.empty((S + 1, V), dtype=t.float64, device=ctx.device)
    # the server writes on its own stream: the tensors must exist before it runs
    t.cuda.current_stream(ctx.device).synchronize()
    rep = Report()
    out = Outputs(mean=_dptr(mean), var=_dptr(var), n_traj=0, traj_idx=None, traj=None,
                  strata=None, zeta=None, mem_kind=MEM_DEVICE, report=C.pointer(rep))
    keep.extend([s, out, rep])
    tid = C.c_uint64(0)
    _check(_lib.fmc_submit(ctx._h, C.byref(s), C.byref(out), C.byref(tid)))
    return Ticket(ctx, int(tid.value), mean, var, rep, keep)


Context.submit = lambda self, sc, precision="f32", variant=-1, time_chunk=0: \
    _submit(self, sc, precision, variant, time_chunk)
Context.submit.__doc__ = """Served form: admit one request (FmcError EBUSY / ENOMEM if it
does not fit now / ever) and return its Ticket (poll / wait / cancel)."""


def footprint(sc: dict, precision="f64", variant=-1) -> int:
    sysd, dist, par, keep = scenario_structs(sc, precision, variant)
    s = Scenario(C.pointer(sysd), C.pointer(dist), C.pointer(par))
    b = C.c_int64(0)
    _check(_lib.fmc_footprint(C.byref(s), C.byref(b)))
    return int(b.value)


_default_ctx = None


def context() -> Context:
    global _default_ctx
    if _default_ctx is None:
        _default_ctx = Context(0)
    return _default_ctx
