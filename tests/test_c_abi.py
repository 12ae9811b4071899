"""The C ABI from C: tests/c/guarded_solve.c includes only include/topoguard.h
(and the HIP runtime for allocation), links libtopoguard.so with gcc and runs
it.  On the CPU: grid facts against the oracle.  On the GPU: the guarded
floor policy from C on the default stream equals the Python binding's run on
torch's stream, bit for bit."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import ke as oke
from oracle import mesh
from paper_2607_26382_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "c", "guarded_solve.c")
LIBDIR = os.path.dirname(L.LIB_PATH)
ROCM = "/opt/rocm"


def _build(tmp_path):
    if shutil.which("gcc") is None or not os.path.exists(L.LIB_PATH):
        pytest.skip("gcc or the built library is missing")
    exe = str(tmp_path / "guarded_solve")
    cmd = ["gcc", "-std=c99", "-O1", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"), SRC,
           "-L", LIBDIR, "-ltopoguard", "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
           f"-Wl,-rpath,{LIBDIR}", f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}", "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe


def _run(exe, *args):
    out = subprocess.run([exe, *map(str, args)], check=True, capture_output=True, text=True, timeout=120).stdout
    kv, attempts = {}, []
    for line in out.splitlines():
        k, _, v = line.partition(" ")
        if k == "attempt":
            r, it, acc, eta = v.split()
            attempts.append((int(r), int(it), int(acc), float(eta)))
        else:
            kv[k] = float(v)
    return kv, attempts


def test_c_caller_host_facts(tmp_path):
    exe = _build(tmp_path)
    for dims in [(16, 8, 8), (5, 3, 2)]:
        kv, _ = _run(exe, "host", *dims)
        og = mesh.Grid(*dims)
        assert kv["n_elem"] == og.n_elem and kv["n_dof"] == og.n_dof and kv["n_free"] == og.n_free()
        assert kv["load_z"] == pytest.approx(-1.0, abs=1e-15)
        assert kv["ke_00"] == pytest.approx(oke.ke()[0, 0], rel=1e-15)


@pytest.mark.gpu
def test_c_caller_guarded_policy_equals_python(tmp_path):
    import torch

    from paper_2607_26382_amd import synth
    from paper_2607_26382_amd import topoguard as tg
    exe = _build(tmp_path)
    dims = (32, 16, 16)
    rho = synth.blobs(*dims, 1001)
    rfile = tmp_path / "rho.bin"
    rho.astype(np.float64).tofile(rfile)
    print(f"C caller: guarded policy on {dims}", flush=True)
    kv, attempts = _run(exe, "gpu", *dims, rfile)
    g = tg.Grid(*dims, max_restart=100, device="cuda")
    f = torch.tensor(g.edge_load(), device="cuda")
    u, out = g.select_floor(torch.tensor(rho, device="cuda"), f, tg.policy())
    assert int(kv["rung"]) == out["rung"] and int(kv["k0"]) == out["k0"]
    assert kv["r50"] == out["r50"] and kv["r100"] == out["r100"]
    assert [(a[0], a[1], a[2]) for a in attempts] == [(a["rung"], a["iterations"], int(a["accepted"]))
                                                      for a in out["attempts"]]
    assert [a[3] for a in attempts] == [a["true_eta"] for a in out["attempts"]]
    if out["rung"] >= 0:
        assert kv["true_eta"] == g.true_residual(f, u) and kv["true_eta"] <= 1e-6
        c = g.compliance_sensitivity(u, f=f, p=3.0, rho_min=out["floor"])["compliance"]
        assert kv["compliance"] == c
