"""The C-ABI library: it loads, exports every function include/pisoc.h
declares, sizes workspaces and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

import paper_1404_0959_amd.pisoc as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions(name):
    src = open(os.path.join(ROOT, "include", name)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pisoc_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1404_0959_amd import build
    if not os.path.exists(P.LIB_PATH):
        build.build()
    return P.lib()


def test_exports_every_declared_function(lib):
    declared = header_functions("pisoc.h")
    assert declared, "no declarations parsed"
    missing = [f for f in declared if not hasattr(lib, f)]
    assert not missing, missing
    assert set(P.EXPORTED) <= set(declared)


def params(**kw):
    base = dict(gamma=1.4, C_=53.6, mu=1e-3, tau_p=(0.01,))
    base.update(kw)
    return P.make_params(kw.pop("n", 32), **base)


def test_workspace_sizes(lib):
    p = params()
    n32 = lib.pisoc_workspace_bytes(ctypes.byref(p))
    N = 32 ** 3
    # about 47 cell fields of FP64 plus small state
    assert 40 * 8 * N < n32 < 80 * 8 * N
    p2 = P.make_params(64, gamma=1.4, C_=53.6, mu=1e-3, tau_p=(0.01,))
    assert lib.pisoc_workspace_bytes(ctypes.byref(p2)) > 7 * n32
    pc = P.make_params(32, gamma=1.4, C_=53.6, mu=1e-3, tau_p=(0.01,), capture=True)
    assert lib.pisoc_workspace_bytes(ctypes.byref(pc)) >= n32 + 4 * 8 * N
    assert lib.pisoc_helm_workspace_bytes(32) >= 5 * 8 * N
    assert lib.pisoc_helm_workspace_bytes(3) == 0


@pytest.mark.parametrize("field,value", [
    ("n", 4), ("n", 2000), ("n_classes", 9), ("gamma", 1.0), ("C", 0.0), ("mu", -1.0),
    ("n_corr", 0), ("n_corr", 5), ("n_mom_sweeps", 0), ("n_dust_sweeps", 0), ("p_tol", 0.0),
    ("p_tol", 1.0), ("p_maxit", 0), ("precision", 7),
])
def test_invalid_params_rejected(lib, field, value):
    p = params()
    setattr(p, field, value)
    assert lib.pisoc_workspace_bytes(ctypes.byref(p)) == 0
    h = ctypes.c_void_p()
    st = lib.pisoc_init(ctypes.byref(p), None, 0, None, None, None, None, ctypes.byref(h))
    assert st == P.ERR_INVALID and not h.value


FOURIER = dict(R=1.0, cv=2.5, kappa=1e-3, T0=50.0)


@pytest.mark.parametrize("change", [
    dict(closure=2), dict(R_gas=0.0), dict(cv=-1.0), dict(kappa=-1e-3), dict(T0=0.0),
    dict(precision=P.FP32_REFINED, inner_tol=1e-6), dict(two_way=1),
])
def test_fourier_params_rejected(lib, change):
    """The Fourier closure's constants must be positive (kappa >= 0); it runs in
    FP64 without two-way coupling."""
    p = P.make_params(32, gamma=1.4, C_=53.6, mu=1e-3, tau_p=(0.01,), fourier=FOURIER)
    assert lib.pisoc_workspace_bytes(ctypes.byref(p)) > 0
    for k, v in change.items():
        setattr(p, k, v)
    assert lib.pisoc_workspace_bytes(ctypes.byref(p)) == 0


@pytest.mark.parametrize("change", [
    dict(time_scheme=2), dict(precision=P.FP32_REFINED, inner_tol=1e-6), dict(two_way=1),
    dict(closure=P.FOURIER, R_gas=1.0, cv=2.5, kappa=0.0, T0=1.0),
])
def test_bdf2_params_rejected(lib, change):
    """BDF2 runs in FP64 with the barotropic closure and one-way coupling."""
    p = P.make_params(32, gamma=1.4, C_=53.6, mu=1e-3, tau_p=(0.01,), bdf2=True)
    assert lib.pisoc_workspace_bytes(ctypes.byref(p)) > 0
    assert lib.pisoc_ens_workspace_bytes(ctypes.byref(p), 1) == 0
    for k, v in change.items():
        setattr(p, k, v)
    assert lib.pisoc_workspace_bytes(ctypes.byref(p)) == 0


@pytest.mark.parametrize("change", [
    dict(mom_tol=-1e-6), dict(mom_tol=1.0), dict(mom_maxit=0),
    dict(precision=P.FP32_REFINED, inner_tol=1e-6),
])
def test_mom_tol_params_rejected(lib, change):
    """The tolerance-solved momentum predictor: 0 < mom_tol < 1, mom_maxit >= 1,
    FP64, single grids."""
    p = P.make_params(32, gamma=1.4, C_=53.6, mu=1e-3, tau_p=(0.01,), mom_tol=1e-8)
    assert lib.pisoc_workspace_bytes(ctypes.byref(p)) > 0
    assert lib.pisoc_ens_workspace_bytes(ctypes.byref(p), 1) == 0
    for k, v in change.items():
        setattr(p, k, v)
    assert lib.pisoc_workspace_bytes(ctypes.byref(p)) == 0


def test_fourier_workspace_and_ensemble_rejection(lib):
    """The closure adds five FP64 cell fields; an ensemble member with it is
    rejected."""
    N = 32 ** 3
    pb = params()
    pf = P.make_params(32, gamma=1.4, C_=53.6, mu=1e-3, tau_p=(0.01,), fourier=FOURIER)
    assert lib.pisoc_workspace_bytes(ctypes.byref(pf)) >= \
        lib.pisoc_workspace_bytes(ctypes.byref(pb)) + 5 * 8 * N
    assert lib.pisoc_ens_workspace_bytes(ctypes.byref(pf), 1) == 0


def test_negative_tau_and_missing_dt_rejected(lib):
    p = params()
    p.tau_p[0] = -1.0
    assert lib.pisoc_workspace_bytes(ctypes.byref(p)) == 0
    p = params(cfl=0.0)
    assert lib.pisoc_workspace_bytes(ctypes.byref(p)) == 0
    p = params(cfl=0.0, dt_fixed=0.01)
    assert lib.pisoc_workspace_bytes(ctypes.byref(p)) > 0


def test_workspace_checked_before_gpu_work(lib):
    p = params()
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(256)
    # missing inputs
    assert lib.pisoc_init(ctypes.byref(p), dummy, 1 << 40, None, None, None, None,
                          ctypes.byref(h)) == P.ERR_INVALID
    # workspace too small / misaligned
    need = lib.pisoc_workspace_bytes(ctypes.byref(p))
    assert lib.pisoc_init(ctypes.byref(p), dummy, need - 1, dummy, dummy, dummy, None,
                          ctypes.byref(h)) == P.ERR_WORKSPACE
    assert lib.pisoc_init(ctypes.byref(p), ctypes.c_void_p(264), need, dummy, dummy, dummy, None,
                          ctypes.byref(h)) == P.ERR_WORKSPACE
    assert lib.pisoc_helm_solve(32, dummy, dummy, dummy, dummy, 1e-8, 10, None, 0, None,
                                None, None) == P.ERR_WORKSPACE
    assert lib.pisoc_helm_solve(32, dummy, dummy, dummy, dummy, 0.0, 10, dummy, 1 << 30, None,
                                None, None) == P.ERR_INVALID


def test_precond_solve_rejects_before_gpu_work(lib):
    """An unknown preconditioner is an invalid argument; a known one still
    checks its workspace first (no device is touched here)."""
    dummy = ctypes.c_void_p(256)
    assert lib.pisoc_helm_solve_precond(32, dummy, dummy, dummy, dummy, 1e-8, 10, 7, dummy,
                                        1 << 30, None, None, None) == P.ERR_INVALID
    for pc in (P.PRECOND_JACOBI, P.PRECOND_CHEB):
        assert lib.pisoc_helm_solve_precond(32, dummy, dummy, dummy, dummy, 1e-8, 10, pc, None,
                                            0, None, None, None) == P.ERR_WORKSPACE


def test_status_strings(lib):
    for st in (0, 1, 2, 3, -1, -2, -3, -4):
        assert lib.pisoc_status_string(st)
        assert lib.pisoc_status_string(st) != b"unknown status"


def test_noalloc_solve_rejects_before_gpu_work(lib):
    """Sizes beyond the static scratch's maximum, and bad arguments, are
    rejected before any GPU work (no device is touched here)."""
    dummy = ctypes.c_void_p(256)
    assert lib.pisoc_helm_solve_noalloc(P.HELM_NOALLOC_MAX_N + 16, dummy, dummy, dummy, dummy,
                                        1e-8, 10, None, None, None) == P.ERR_WORKSPACE
    assert lib.pisoc_helm_solve_noalloc(32, None, dummy, dummy, dummy, 1e-8, 10, None,
                                        None, None) == P.ERR_INVALID
    assert lib.pisoc_helm_solve_noalloc(32, dummy, dummy, dummy, dummy, 1e-8, 0, None,
                                        None, None) == P.ERR_INVALID


def test_stream_probe_rejects_before_gpu_work(lib):
    """The streaming probe checks its counts and pointers before any GPU work."""
    ins = (ctypes.c_void_p * 12)(*[256] * 12)
    outs = (ctypes.c_void_p * 8)(*[4096] * 8)
    for reads, writes, count, blocks in ((0, 1, 64, 0), (13, 1, 64, 0), (1, 0, 64, 0),
                                         (1, 9, 64, 0), (1, 1, 62, 0), (1, 1, -4, 0),
                                         (1, 1, 64, -1)):
        assert lib.pisoc_stream_probe(reads, writes, count, ins, outs, blocks,
                                      None) == P.ERR_INVALID
    assert lib.pisoc_stream_probe(1, 1, 64, None, outs, 0, None) == P.ERR_INVALID
    misaligned = (ctypes.c_void_p * 2)(256, 260)
    assert lib.pisoc_stream_probe(2, 1, 64, misaligned, outs, 0, None) == P.ERR_INVALID
    nulls = (ctypes.c_void_p * 2)(256, None)
    assert lib.pisoc_stream_probe(1, 2, 64, ins, nulls, 0, None) == P.ERR_INVALID
    # nothing to do: no launch, no device touched, the pointers not read
    assert lib.pisoc_stream_probe(1, 1, 0, ins, outs, 0, None) == P.OK
    assert lib.pisoc_stream_probe(1, 1, 0, None, None, 0, None) == P.OK


# C structs of the header and their ctypes mirrors in the binding
STRUCTS = {"pisoc_params": P.Params, "pisoc_step_info": P.StepInfo, "pisoc_stats": P.Stats,
           "pisoc_ens_class": P.EnsClass, "pisoc_kernel_stat": P.KernelStat}


def test_struct_layouts_match_header(tmp_path):
    """Every struct the binding passes across the ABI has the header's size
    and field offsets (compiled with the host C compiler)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "pisoc.h"', "int main(void) {"]
    for cname, py in STRUCTS.items():
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for field, _ in py._fields_:
            lines.append(f'printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n"):
        if line:
            cname, field, value = line.split()
            got[(cname, field)] = int(value)
    for cname, py in STRUCTS.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(py), cname
        for field, _ in py._fields_:
            assert got[(cname, field)] == getattr(py, field).offset, (cname, field)
