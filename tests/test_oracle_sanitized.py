"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (host
code, g++): every entry point runs on small inputs without a sanitizer report,
and gives the same results as the regular build that the tests load (integer
outputs bit for bit; floating-point ones to rounding, since the two builds use
different optimisation levels)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import synth
from oracle import core

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def sanitized_driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("asan") / "oracle_asan")
    cmd = [gxx, "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(ROOT, "oracle", "oracle.cpp"),
           os.path.join(ROOT, "tests", "oracle_sanitize_driver.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.fail(f"sanitizer build failed:\n{r.stderr}")
    return exe


def test_oracle_under_sanitizers(sanitized_driver, tmp_path, oracle_lib):
    N, M, n, C, S, K, seed = 12, 18, 40, 6, 3, 12, 11
    bonds = synth.chain_bonds(N)
    sub = synth.chain_sublattice(N)
    params = synth.rbm_params(N, M, 4, sigma=0.2)
    s = synth.random_configs(n, N, 5)
    ch = synth.random_configs(C, N, 6)
    chz = synth.sz0_configs(C, N, 7)
    d = tmp_path
    (d / "meta.txt").write_text(f"{N} {M} {n} {C} {S} {K} {bonds.shape[0]} {seed}\n")
    params.tofile(d / "params.bin")
    s.tofile(d / "s.bin")
    bonds.astype(np.int32).tofile(d / "bonds.bin")
    sub.tofile(d / "sub.bin")
    ch.tofile(d / "chains.bin")
    chz.tofile(d / "sz0chains.bin")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([sanitized_driver, str(d)], capture_output=True, text=True, env=env,
                       timeout=300)
    assert r.returncode == 0 and "ERROR" not in r.stderr and "runtime error" not in r.stderr, \
        r.stderr[-4000:]

    def out(name, dtype, shape):
        return np.fromfile(d / name, dtype=dtype).reshape(shape)

    ph = out("out_philox.bin", np.uint32, (16, 4))
    for k in range(16):
        ctr = [(k * 2654435761) & 0xFFFFFFFF, k, 3 * k, 1]
        np.testing.assert_array_equal(ph[k], core.philox(ctr, seed + k))
    np.testing.assert_array_equal(out("out_init.bin", np.int8, (C, N)),
                                  core.init_chains(N, C, seed, chain_offset=5))
    np.testing.assert_array_equal(out("out_init_sz0.bin", np.int8, (C, N)),
                                  core.init_chains(N, C, seed, chain_offset=5, total_sz_zero=True))
    rbm = core.Rbm(N, M, params)
    tfim = core.Hamiltonian.tfim(N, bonds, 1.0, 0.7)
    heis = core.Hamiltonian.heisenberg(N, bonds, 1.0, sub)
    for name, ref in (("out_logpsi.bin", core.log_psi(rbm, s)),
                      ("out_eloc_tfim.bin", core.local_energy(rbm, tfim, s)),
                      ("out_eloc_heis.bin", core.local_energy(rbm, heis, s)),
                      ("out_jacobian.bin", core.jacobian(rbm, s).ravel())):
        got = out(name, np.float64, ref.shape)
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)
    for rule in (0, 1):
        for mode in (0, 1):
            tag = f"{rule}{mode}"
            ref = core.sample(rbm, chz if rule else ch, S, K, seed, 7,
                              "local" if rule == 0 else "exchange", bonds, chain_offset=3,
                              mode="definition" if mode == 0 else "cached", log_accepts=True)
            assert ref.margins.min() > 1e-12
            np.testing.assert_array_equal(out(f"out_chains{tag}.bin", np.int8, (C, N)), ref.chains)
            np.testing.assert_array_equal(out(f"out_samples{tag}.bin", np.int8, (C, S, N)),
                                          ref.samples)
            np.testing.assert_array_equal(out(f"out_accepts{tag}.bin", np.uint8, (C, S * K)),
                                          ref.accepts)
            np.testing.assert_array_equal(out(f"out_nacc{tag}.bin", np.int64, (C,)),
                                          ref.n_accepted)
