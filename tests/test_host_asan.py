"""The library's host set-up arithmetic (fde_host.hpp: Grunwald and
second-order weights, symbol samples, the set-up FFT, the P_tri partition)
built with g++ under AddressSanitizer and UndefinedBehaviorSanitizer and
compared with the oracle (CPU only)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import grunwald, symbol

HERE = os.path.dirname(os.path.abspath(__file__))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.isdir(os.path.join(ROCM, "include", "hip")):
        pytest.skip("needs g++ and the HIP headers")
    exe = str(tmp_path_factory.mktemp("asan") / "host_check")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROCM, "include"),
           os.path.join(HERE, "host", "host_check.cpp"), "-o", exe, "-L" + os.path.join(ROCM, "lib"),
           "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]

    def run(text):
        env = dict(os.environ, ASAN_OPTIONS="abort_on_error=0:halt_on_error=1",
                   UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
        p = subprocess.run([exe], input=text, capture_output=True, text=True, env=env, timeout=120)
        assert p.returncode == 0 and "ERROR" not in p.stderr and "runtime error" not in p.stderr, p.stderr[-3000:]
        blocks, cur = [], []
        for line in p.stdout.splitlines():
            if line == "end":
                blocks.append(cur)
                cur = []
            else:
                cur.append([float(t) for t in line.split()])
        return [np.array(b) for b in blocks]
    return run


@pytest.mark.parametrize("alpha", [1.01, 1.3, 1.5, 1.77, 1.99])
def test_weights(driver, alpha):
    K = 4097
    g, w = driver(f"w {alpha} {K} 0\nw {alpha} {K} 1\n")
    np.testing.assert_allclose(g[:, 0], grunwald.grunwald(alpha, K + 1), rtol=1e-14, atol=0)
    np.testing.assert_allclose(w[:, 0], grunwald.wsgd(alpha, K + 1), rtol=1e-14, atol=1e-300)


@pytest.mark.parametrize("alpha", [1.1, 1.5, 1.9])
@pytest.mark.parametrize("n", [1, 7, 1000, 4095])
def test_symbol_samples(driver, alpha, n):
    s0, s1 = driver(f"s {alpha} {n} 0\ns {alpha} {n} 1\n")
    t = symbol.theta(n)
    for kind, got in (("shifted", s0), ("weighted", s1)):
        ref = symbol.F_symbol(alpha, t, kind)
        np.testing.assert_allclose(got[:, 0], ref, rtol=1e-12, atol=1e-14 * np.abs(ref).max())


@pytest.mark.parametrize("L", [1, 2, 8, 1024, 65536])
def test_setup_fft(driver, L):
    x = np.random.default_rng(L).uniform(-1, 1, (L, 2))
    text = f"f {L}\n" + "\n".join(f"{a:.17g} {b:.17g}" for a, b in x) + "\n"
    (y,) = driver(text)
    ref = np.fft.fft(x[:, 0] + 1j * x[:, 1])
    err = np.abs(y[:, 0] + 1j * y[:, 1] - ref).max()
    assert err <= 1e-15 * np.log2(max(L, 2)) * np.abs(ref).max() * 10


@pytest.mark.parametrize("n,pmax", [(2, 512), (3, 512), (1000, 512), (5000, 512), (7, 2)])
def test_tri_partition(driver, n, pmax):
    rng = np.random.default_rng(n)
    sub, sup = -rng.uniform(0, 1, n), -rng.uniform(0, 1, n)
    diag = 3.0 + rng.uniform(0, 1, n)
    text = f"t {n} {pmax}\n" + "\n".join(f"{a:.17g} {b:.17g} {c:.17g}" for a, b, c in zip(sub, diag, sup)) + "\n"
    (out,) = driver(text)
    p = int(out[0, 0])
    cs = out[1:, 0].astype(int)
    assert p == max(1, min(pmax, n // 2)) and len(cs) == p + 1
    assert cs[0] == 0 and cs[-1] == n and np.all(np.diff(cs) >= 2)
