"""Pins for the oracle's random numbers and directions.

Philox4x32-10 (Salmon et al., SC'11) is checked bit for bit against rocRAND's
independent header implementation; the direction sampler (uniform exit from a
sphere, Sec. 2 of the paper: the exit point of a ball centred at the start is
uniform on its surface) against its first two moments and the mean-value
property of harmonic functions.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import wos

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("rr") / "philox_ref")
    subprocess.run([HIPCC, "-O1", os.path.join(HERE, "rocrand_philox_ref.cpp"), "-o", exe],
                   check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand(rocrand_ref):
    rng = np.random.default_rng(7)
    n = 3000
    ctr = rng.integers(0, 2 ** 32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:, 1] &= 0x3FFFFFFF  # keep the engine's offset*4 within 64 bits
    ctr[:10] = 0
    ctr[10:20, 0] = np.arange(10)
    seeds = rng.integers(0, 2 ** 63, size=n, dtype=np.uint64)
    seeds[:5] = [0, 1, 2, 2 ** 32, 2 ** 63 - 1]
    lines = "".join(f"{int(s)} {c[0]} {c[1]} {c[2]} {c[3]}\n" for s, c in zip(seeds, ctr))
    out = subprocess.run([rocrand_ref], input=lines, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(v) for v in ln.split()] for ln in out.strip().splitlines()], dtype=np.uint64)
    got = np.concatenate([wos.philox(c[None, :], int(s)) for s, c in zip(seeds, ctr)]).astype(np.uint64)
    assert ref.shape == (n, 4)
    np.testing.assert_array_equal(got, ref)


def test_philox_uniformity_and_independence():
    n = 1 << 16
    ctr = np.zeros((n, 4), dtype=np.uint32)
    ctr[:, 0] = np.arange(n)
    ctr[:, 2] = 3
    ctr[:, 3] = 11
    out = wos.philox(ctr, 1)
    # top byte of each word: chi^2 with 255 dof
    for k in range(4):
        hist = np.bincount(out[:, k] >> 24, minlength=256)
        chi2 = np.sum((hist - n / 256) ** 2 / (n / 256))
        assert 150 < chi2 < 380, (k, chi2)
    u = (out.astype(np.float64) + 0.5) / 2 ** 32
    # words within a block and consecutive counters are uncorrelated
    c = np.corrcoef(np.column_stack([u, np.roll(u[:, 0], 1)]).T)
    off = c[~np.eye(5, dtype=bool)]
    assert np.max(np.abs(off)) < 5.0 / np.sqrt(n)
    # a one-bit change of the counter flips about half the output bits
    ctr2 = ctr.copy()
    ctr2[:, 2] ^= 1
    flips = np.unpackbits((out ^ wos.philox(ctr2, 1)).view(np.uint8)).mean()
    assert abs(flips - 0.5) < 0.01


def test_direction_moments_and_norm():
    n = 200_000
    ctr = np.zeros((n, 4), dtype=np.uint32)
    ctr[:, 0] = np.arange(n)
    r = wos.philox(ctr, 99)
    u = (r[:, :2].astype(np.float64) + 0.5) / 2 ** 32
    w = wos.direction(u)
    np.testing.assert_allclose(np.linalg.norm(w, axis=1), 1.0, atol=1e-15)
    tol = 5.0 / np.sqrt(n)
    assert np.max(np.abs(w.mean(0))) < tol
    S = (w[:, :, None] * w[:, None, :]).mean(0)
    assert np.max(np.abs(S - np.eye(3) / 3)) < tol
    # known reduction: z = 1 - 2 u1 exactly, and the azimuth is 2 pi u2
    np.testing.assert_array_equal(w[:, 2], 1.0 - 2.0 * u[:, 0])
    ang = np.mod(np.arctan2(w[:, 1], w[:, 0]), 2 * np.pi)
    np.testing.assert_allclose(ang, 2 * np.pi * u[:, 1], atol=1e-9)


def test_mean_value_property():
    """The mean of a harmonic function over a sphere is its centre value."""
    n = 400_000
    ctr = np.zeros((n, 4), dtype=np.uint32)
    ctr[:, 0] = np.arange(n)
    ctr[:, 3] = 5
    r = wos.philox(ctr, 3)
    u = (r[:, :2].astype(np.float64) + 0.5) / 2 ** 32
    w = wos.direction(u)
    x0 = np.array([0.3, -0.2, 0.4])
    rad = 0.35
    s = np.array([1.2, 0.9, -0.7])
    f = lambda p: 1.0 / np.linalg.norm(p - s, axis=-1) + p[..., 0] ** 2 - p[..., 2] ** 2
    vals = f(x0 + rad * w)
    se = vals.std() / np.sqrt(n)
    assert abs(vals.mean() - f(x0)) < 4 * se
