"""Pins for the oracle's random words, uniforms and normals (CPU only)."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import special, stats

from oracle import rng
from oracle.model import inv_cdf

HERE = os.path.dirname(os.path.abspath(__file__))


def _random_counters(n, seed=7):
    g = np.random.default_rng(seed)
    c = g.integers(0, 2**32, size=(n, 6), dtype=np.uint64)
    c[:, 1] >>= 3          # rocRAND addresses counter words 0-1 by a 64-bit offset*4
    c[:8] = 0
    c[1, 0] = 1
    c[2, 2] = 1
    c[3, :] = 2**32 - 1
    c[3, 1] = 2**29 - 1
    c[4, 4] = 42
    c[5, 1] = 1
    return c


def test_philox_numpy_matches_scalar():
    cs = _random_counters(300)
    for row in cs[:300]:
        a = rng.philox4x32_10(row[:4], row[4:])
        b = rng.philox4x32_10_np(*[np.array([x]) for x in row[:4]], row[4], row[5])
        assert a == tuple(int(x[0]) for x in b)


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand_engine(tmp_path):
    """Library pin: rocRAND's Philox4x32-10 engine (host-callable header) gives
    the same blocks as the oracle for arbitrary counters and keys."""
    exe = tmp_path / "philox_ref"
    subprocess.run(["hipcc", "-O1", "-I/opt/rocm/include", os.path.join(HERE, "rocrand_philox_words.cpp"),
                    "-o", str(exe)], check=True, capture_output=True)
    cs = _random_counters(500)
    inp = "\n".join(" ".join(str(int(x)) for x in row) for row in cs) + "\n"
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    for row, line in zip(cs, out):
        ref = tuple(int(x) for x in line.split())
        assert rng.philox4x32_10(row[:4], row[4:]) == ref


def test_philox_stream_layout():
    # word w of a path is element w % 4 of block (path, w // 4, instance, 0)
    words = rng.philox_path_words(path=5, n_words=10, instance=3, seed=42 + (7 << 32))
    for w in range(10):
        blk = rng.philox4x32_10((5, w // 4, 3, 0), (42, 7))
        assert words[w] == blk[w % 4]
    arr = rng.philox_words([5, 6], 10, instance=3, seed=42 + (7 << 32))
    assert list(arr[0]) == words


def test_philox_words_look_uniform():
    w = rng.philox_words(np.arange(4096), 16).reshape(-1)
    # chi-square on the top 8 bits and a lag-1 correlation test
    counts = np.bincount((w >> 24).astype(np.int64), minlength=256)
    chi2 = ((counts - w.size / 256) ** 2 / (w.size / 256)).sum()
    assert stats.chi2.sf(chi2, 255) > 1e-4
    u = rng.uniform_f64(w)
    r = np.corrcoef(u[:-1], u[1:])[0, 1]
    assert abs(r) < 5 / math.sqrt(u.size)


def test_sobol_first_dimension_is_van_der_corput():
    # Gray-code order of dim 0: 0, 1/2, 3/4, 1/4, 3/8, 7/8, 5/8, 1/8
    w = rng.sobol_words(np.arange(8), 3)
    exp = [0, 0.5, 0.75, 0.25, 0.375, 0.875, 0.625, 0.125]
    assert [x / 2**32 for x in w[:, 0]] == exp


def test_sobol_matches_rocrand_direction_vectors():
    """Library pin: Gray-code Sobol points built from rocRAND's Joe-Kuo
    direction vectors equal scipy's for 15 dimensions and 4096 points."""
    import ctypes
    try:
        lib = ctypes.CDLL("/opt/rocm/lib/librocrand.so")
    except OSError:
        pytest.skip("librocrand not available")
    p = ctypes.POINTER(ctypes.c_uint)()
    assert lib.rocrand_get_direction_vectors32(ctypes.byref(p), 101) == 0
    D, N = 15, 4096
    v = np.ctypeslib.as_array(p, shape=(D * 32,)).reshape(D, 32).astype(np.uint32)
    ours = rng.sobol_words(np.arange(N), D)
    for i in (0, 1, 2, 3, 100, 1023, 1024, 4095):
        g = i ^ (i >> 1)
        x = np.zeros(D, dtype=np.uint32)
        for b in range(32):
            if (g >> b) & 1:
                x ^= v[:, b]
        assert np.array_equal(x, ours[i]), i


def test_sobol_subset_indexing():
    a = rng.sobol_words(np.arange(64), 5)
    b = rng.sobol_words(np.array([63, 7, 0]), 5)
    assert np.array_equal(b, a[[63, 7, 0]])


def test_uniform_maps_exact_and_symmetric():
    x = np.array([0, 1, 255, 256, 2**31, 2**32 - 1], dtype=np.uint64)
    u64 = rng.uniform_f64(x)
    assert u64[0] == 2.0**-33 and u64[-1] == 1 - 2.0**-33
    u32 = rng.uniform_f32(x)
    assert u32[0] == 2.0**-24 and u32[-1] == 1 - 2.0**-24
    assert np.all(u32.astype(np.float32).astype(np.float64) == u32)   # exact in binary32
    g = np.random.default_rng(3).integers(0, 2**32, size=10000, dtype=np.uint64)
    comp = (~g) & np.uint64(0xFFFFFFFF)
    assert np.all(rng.uniform_f64(g) + rng.uniform_f64(comp) == 1.0)
    assert np.all(rng.uniform_f32(g) + rng.uniform_f32(comp) == 1.0)
    assert np.all((u64 > 0) & (u64 < 1)) and np.all((u32 > 0) & (u32 < 1))


def test_inv_cdf_matches_scipy_and_invariants():
    g = np.random.default_rng(5)
    u = np.concatenate([g.random(5000), rng.uniform_f64(np.arange(0, 2**32, 2**22, dtype=np.uint64)),
                        [2.0**-33, 1 - 2.0**-33, 2.0**-25, 0.5]])
    z = inv_cdf(u)
    ref = special.ndtri(u)
    assert np.max(np.abs(z - ref) / np.maximum(1.0, np.abs(ref))) < 1e-14
    assert np.allclose(special.ndtr(z), u, rtol=1e-12, atol=0)
    mid = u[(u > 1e-6) & (u < 1 - 1e-6)]
    assert np.allclose(inv_cdf(1 - mid), -inv_cdf(mid), rtol=1e-9, atol=1e-12)
    assert inv_cdf(0.5) == 0.0
