"""The C ABI library loads and exports every entry point include/fmc.h declares.

CPU-only: no compute call is made (there is no GPU here); only host-side
argument checks and the no-device error path run.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fmc.h")
LIB = os.path.join(ROOT, "paper_2007_03847_amd", "libfmc.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fmc_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ["fmc_context_create", "fmc_context_destroy", "fmc_kron_reduce", "fmc_lhs",
              "fmc_basis", "fmc_kle_paths", "fmc_run", "fmc_run_batch", "fmc_submit",
              "fmc_poll", "fmc_wait", "fmc_cancel", "fmc_last_error", "fmc_footprint"]:
        assert f in names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libfmc.so not built")
    return C.CDLL(LIB)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_exposes_every_symbol():
    import paper_2007_03847_amd as fmc
    assert set(declared_functions()) == set(fmc.EXPORTED)


def test_abi_version(lib):
    lib.fmc_abi_version.restype = C.c_int
    assert lib.fmc_abi_version() == 4


def test_footprint_and_validation_on_host():
    import paper_2007_03847_amd as fmc
    import workloads
    sc = workloads.config2()
    b64 = fmc.footprint(sc, "f64")
    b32 = fmc.footprint(sc, "f32")
    assert 0 < b32 < b64
    # zeta alone is M*N*8 bytes
    assert b64 > 300 * 10_000 * 8
    with pytest.raises(fmc.FmcError) as e:
        fmc.footprint(dict(sc, dt=0.0033))
    assert e.value.code == fmc.EINVAL
    with pytest.raises(fmc.FmcError):
        fmc.footprint(dict(sc, N=1))
    with pytest.raises(fmc.FmcError):
        fmc.footprint(dict(sc, dist=dict(sc["dist"], sigma=-np.ones(3))))
    with pytest.raises(fmc.FmcError):
        fmc.footprint(dict(sc, dist=dict(sc["dist"], gen=np.array([0, 1, 99], dtype=np.int32))))


def test_no_device_is_reported(lib):
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except Exception:
        pass
    h = C.c_void_p()
    lib.fmc_context_create.argtypes = [C.c_int, C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]
    rc = lib.fmc_context_create(0, 0, None, C.byref(h))
    assert rc == -4


def test_fluxdecay_validation_on_host():
    """Host-side checks of flux-decay scenarios (fmc_footprint validates
    without touching a device)."""
    import paper_2007_03847_amd as fmc
    import workloads
    sc = workloads.fluxdecay(n_gen=40, n_dist=6, N=100, K=20, T=0.1)
    b32 = fmc.footprint(sc, "f32")
    b16 = fmc.footprint(sc, "bf16x3")
    b16n = fmc.footprint(sc, "bf16x3", variant=1)  # BF16 x3 network product: its own Y copy
    assert b32 > 0 and b16 > 0 and b16n > b16
    for prec, v in (("f32", 1), ("bf16x3", 2), ("bf16x3", -2)):
        with pytest.raises(fmc.FmcError) as e:
            fmc.footprint(sc, prec, variant=v)
        assert e.value.code == fmc.EINVAL
    # the 196-bus reduction needs its (n_bus + n_gen)^2 complex work matrix
    W = sc["net"]["n_bus"] + sc["n_gen"]
    assert b32 > W * W * 16
    with pytest.raises(fmc.FmcError) as e:      # FP64 is not a flux-decay precision
        fmc.footprint(sc, "f64")
    assert e.value.code == fmc.EINVAL
    bad = sc["model_params"].copy(); bad[3, 4] = 0.0   # TA = 0
    with pytest.raises(fmc.FmcError) as e:
        fmc.footprint(dict(sc, model_params=bad), "f32")
    assert e.value.code == fmc.EINVAL
    bad = sc["model_params"].copy(); bad[0, 0] = float("nan")
    with pytest.raises(fmc.FmcError):
        fmc.footprint(dict(sc, model_params=bad), "f32")
    # 40 machines: 3 blocks of 16, 2 waves, at most 8 processes
    many = workloads.fluxdecay(n_gen=40, n_dist=9, N=100, K=20, T=0.1)
    with pytest.raises(fmc.FmcError) as e:
        fmc.footprint(many, "f32")
    assert e.value.code == fmc.EINVAL
    with pytest.raises(fmc.FmcError):
        fmc.footprint(dict(sc, model_params=None), "f32")


def test_served_footprint_grows_with_time_chunk_and_N():
    import paper_2007_03847_amd as fmc
    import workloads
    sc = workloads.config2(N=2000)
    a = fmc.footprint(sc, "f32")
    b = fmc.footprint(dict(sc, N=4000), "f32")
    assert b > a
    # zeta alone: M * N * 8 bytes
    assert a > 300 * 2000 * 8
