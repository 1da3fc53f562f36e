"""A solve through the C ABI from a C program (tests/c_api/solve_bump.c,
no Python in the loop; MI355X only): it must succeed, come within 1e-3 of
the closed-form potential (the 32^3 discretisation error) and, given the
same node charge, return the same phi, bit for bit, as the Python binding's
solve of the same problem."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import mlc_inputs as mi
from paper_1702_08111_amd import mlc as gm

from gpu_common import context

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1702_08111_amd")


def test_c_program_solve(tmp_path):
    import torch
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    exe, src, out = tmp_path / "solve_bump", tmp_path / "f.bin", tmp_path / "phi.bin"
    fh = mi.bump_charge(32, mi.one_bump())
    fh.tofile(src)
    cmd = [cc, "-std=c99", "-O2", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "c_api", "solve_bump.c"), "-o", str(exe),
           "-L", PKG, "-l:libmlc.so", "-Wl,-rpath," + PKG, "-L", "/opt/rocm/lib", "-lamdhip64",
           "-Wl,-rpath,/opt/rocm/lib", "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe), str(src), str(out)], capture_output=True, text=True, timeout=120)
    print(r.stdout, flush=True)
    assert r.returncode == 0, r.stdout + r.stderr
    phi_c = np.fromfile(out, dtype=np.float64).reshape((33, 33, 33))
    f = torch.from_numpy(fh).cuda()
    plan = context().plan(gm.problem(32, 8, 3.0, 6.0, 4, 4, conv="fp64", Z=64))
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    phi = torch.empty_like(f)
    plan.solve(f, phi, ws)
    torch.cuda.synchronize()
    plan.close()
    assert np.array_equal(phi.cpu().numpy(), phi_c)
