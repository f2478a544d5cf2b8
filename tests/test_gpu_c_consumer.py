"""The library from plain C, without PyTorch: a C program (tests/c_consumer/
vmc_chain.c) allocates the workspace with hipMalloc and runs SR steps of the
N = 10 TFIM chain through the C ABI; its energies, CG iteration counts and final
parameters equal, bit for bit, those of the same steps through the Python layer."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_c_program_matches_python_layer(tmp_path):
    import torch
    assert torch.cuda.is_available()
    from paper_2112_10526_amd import _lib
    from paper_2112_10526_amd.nqs import VMCState
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    libdir = os.path.dirname(_lib.LIB_PATH)
    exe = tmp_path / "vmc_chain"
    r = subprocess.run([gcc, "-std=c99", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__",
                        "-I/opt/rocm/include", "-I", os.path.join(ROOT, "include"),
                        os.path.join(ROOT, "tests", "c_consumer", "vmc_chain.c"),
                        "-L", libdir, "-lnqs", "-L/opt/rocm/lib", "-lamdhip64",
                        f"-Wl,-rpath,{libdir}", "-Wl,-rpath,/opt/rocm/lib", "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    w = synth.WORKLOADS["tfim1d_n10"].replace(sigma=0.05)
    params = np.ascontiguousarray(w.params(), dtype=np.float64)
    pfile = tmp_path / "params.bin"
    params.tofile(pfile)
    steps = 3
    print("[case] C consumer, tfim1d_n10 fp64, 3 steps", flush=True)
    r = subprocess.run([str(exe), str(pfile), str(steps)], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    lines = r.stdout.split("\n")
    c_steps = [ln.split() for ln in lines[:steps]]
    c_params = np.array([float(x) for x in lines[steps:] if x.strip()])
    st = VMCState.from_workload(w, precision="fp64", params=params)
    for k in range(steps):
        rep = st.vmc_step(diag_shift=0.01, lr=0.02, tol=1e-10, maxiter=2000)
        assert float(c_steps[k][0]) == rep.energy["mean"], k
        assert int(c_steps[k][1]) == rep.sr.iterations, k
    np.testing.assert_array_equal(c_params, st.get_params())
    st.close()
