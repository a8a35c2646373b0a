"""Pins for the oracle's control noise (Alg. 1 Step 1; Eq. 8)."""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

from oracle import philox as P

HERE = os.path.dirname(os.path.abspath(__file__))


def _rocrand_words(tmp_path, rows):
    """Run rocRAND's host-compiled Philox4x32-10 on (seed, ctr) rows."""
    gxx = shutil.which("g++")
    inc = "/opt/rocm/include"
    if gxx is None or not os.path.exists(os.path.join(inc, "rocrand", "rocrand_philox4x32_10.h")):
        pytest.skip("g++ or rocRAND headers unavailable")
    exe = str(tmp_path / "rr")
    subprocess.run([gxx, "-std=c++17", "-O1", "-I", inc, "-D__HIP_PLATFORM_AMD__",
                    os.path.join(HERE, "rocrand_philox_ref.cpp"), "-o", exe], check=True)
    text = "".join(f"{s:x} {c[0]:x} {c[1]:x} {c[2]:x} {c[3]:x}\n" for s, c in rows)
    out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
    return np.array([[int(t, 16) for t in line.split()] for line in out.strip().splitlines()],
                    dtype=np.uint64)


def test_philox_matches_rocrand_host_engine(tmp_path):
    rng = np.random.Generator(np.random.PCG64(11))
    rows = []
    for _ in range(300):
        seed = int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2))
        ctr = [int(v) for v in rng.integers(0, 2**32, size=4, dtype=np.uint64)]
        rows.append((seed, ctr))
    # structured counters used by the controller: (k, s, pid, tag)
    for k in (0, 1, 99):
        for s in (0, 1, 16383):
            rows.append((((2002 << 32) + 5), [k, s, 3, 0]))
    rows.append((0, [0, 0, 0, 0]))
    rows.append((2**64 - 1, [2**32 - 1] * 4))
    ref = _rocrand_words(tmp_path, rows)
    ours = np.stack([P.philox4x32_10(np.array(c, dtype=np.uint64), P.seed_key(s)) for s, c in rows])
    np.testing.assert_array_equal(ours.astype(np.uint64), ref)


def test_philox_vectorised_equals_scalar_calls():
    ctr = np.array([[k, s, 2, 0] for k in range(3) for s in range(5)], dtype=np.uint64)
    key = P.seed_key(123456789012345)
    vec = P.philox4x32_10(ctr, key)
    for i in range(ctr.shape[0]):
        np.testing.assert_array_equal(vec[i], P.philox4x32_10(ctr[i], key))


def test_uniforms_exact_in_binary32_and_open_interval():
    rng = np.random.Generator(np.random.PCG64(0))
    words = np.concatenate([np.array([0, 511, 512, 2**32 - 1, 2**31, 2**31 - 1], dtype=np.uint64),
                            rng.integers(0, 2**32, size=100_000, dtype=np.uint64)])
    u = P.uniform_open(words)
    assert np.all(u > 0.0) and np.all(u < 1.0)
    np.testing.assert_array_equal(u.astype(np.float32).astype(np.float64), u)
    assert u[0] == 2.0**-24 and u[3] == 1.0 - 2.0**-24
    assert u[1] == u[0] and u[2] == 3 * 2.0**-24


def test_box_muller_special_values():
    u1 = np.array([0.25, np.exp(-0.5)])
    z0, z1 = P.box_muller(u1, np.zeros(2))
    np.testing.assert_allclose(z0, np.sqrt(-2 * np.log(u1)), rtol=1e-15)
    np.testing.assert_allclose(z1, 0.0, atol=1e-15)
    z0, z1 = P.box_muller(u1, np.full(2, 0.25))
    np.testing.assert_allclose(z1, np.sqrt(-2 * np.log(u1)), rtol=1e-15)
    np.testing.assert_allclose(z0, 0.0, atol=1e-15)


def test_normals_are_standard_normal():
    n = 1 << 19
    z0, z1 = P.standard_normals(7, np.arange(n), seed=(2000 << 32) + 3)
    for z in (z0, z1):
        assert abs(z.mean()) < 6.0 / np.sqrt(n)
        assert abs(z.var() - 1.0) < 6.0 * np.sqrt(2.0 / n)
        assert stats.kstest(z, "norm").pvalue > 1e-4
    # the two outputs of one block are uncorrelated
    assert abs(np.corrcoef(z0, z1)[0, 1]) < 6.0 / np.sqrt(n)


def test_stream_separation_by_counter_words():
    a = P.standard_normals(0, np.arange(4096), seed=99, pid=0)[0]
    b = P.standard_normals(0, np.arange(4096), seed=99, pid=1)[0]
    c = P.standard_normals(1, np.arange(4096), seed=99, pid=0)[0]
    d = P.standard_normals(0, np.arange(4096), seed=100, pid=0)[0]
    for other in (b, c, d):
        assert abs(np.corrcoef(a, other)[0, 1]) < 0.1
        assert not np.any(a == other)


def test_sampled_controls_respect_box_and_zero_noise_limit():
    U = np.array([[0.5, -1.9], [1.99, 0.0], [-3.0, 3.0]])
    u = P.sampled_controls(U, np.arange(2000), 5, (0.5, 0.8), (-2, -2), (2, 2))
    assert u.min() >= -2.0 and u.max() <= 2.0
    u0 = P.sampled_controls(U, np.arange(10), 5, (0.0, 0.0), (-2, -2), (2, 2))
    np.testing.assert_array_equal(u0, np.broadcast_to(np.clip(U, -2, 2)[:, None, :], u0.shape))
