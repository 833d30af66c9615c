"""Pins for the oracle's Philox-4x32-10 (CPU only)."""

import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import assign, philox

HERE = os.path.dirname(os.path.abspath(__file__))


def test_numpy_matches_scalar():
    rng = np.random.default_rng(1)
    ctr = rng.integers(0, 2 ** 32, size=(200, 4), dtype=np.uint64)
    key = rng.integers(0, 2 ** 32, size=(200, 2), dtype=np.uint64)
    for c, k in zip(ctr, key):
        ref = philox.philox4x32_10(tuple(int(x) for x in c), tuple(int(x) for x in k))
        got = philox.philox4x32_10_np(*(np.array([x]) for x in c), int(k[0]), int(k[1]))
        assert tuple(int(g[0]) for g in got) == ref


def test_round_structure_changes_every_word():
    # Flipping any counter or key bit changes every output word (a dropped or misrouted
    # term in the round would leave some word unchanged for some input bit).
    base_c, base_k = (0x01234567, 0x89ABCDEF, 0xDEADBEEF, 0x0BADF00D), (0x11111111, 0x22222222)
    ref = philox.philox4x32_10(base_c, base_k)
    for w in range(4):
        for bit in (0, 7, 31):
            c = list(base_c)
            c[w] ^= 1 << bit
            out = philox.philox4x32_10(c, base_k)
            assert all(a != b for a, b in zip(out, ref))
    for w in range(2):
        k = list(base_k)
        k[w] ^= 1 << 13
        out = philox.philox4x32_10(base_c, k)
        assert all(a != b for a, b in zip(out, ref))


@pytest.fixture(scope="module")
def rocrand_pin(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = tmp_path_factory.mktemp("pin") / "rocrand_philox_pin"
    subprocess.run([hipcc, "-O1", os.path.join(HERE, "rocrand_philox_pin.cpp"), "-o", str(exe)],
                   check=True, capture_output=True)
    return str(exe)


def test_matches_rocrand(rocrand_pin):
    """rocRAND's Philox-4x32-10, run (not read), with (seed, subsequence = draw index,
    offset = 4 * block) must give the oracle's block for counter (j, 0, lo b, hi b) and
    key (lo seed, hi seed)."""
    rng = np.random.default_rng(7)
    triples = [(0, 0, 0), (2 ** 64 - 1, 2 ** 64 - 1, 0)]
    for _ in range(40):
        triples.append((int(rng.integers(0, 2 ** 63)) * 2 + 1, int(rng.integers(0, 2 ** 63)),
                        4 * int(rng.integers(0, 2 ** 20))))
    inp = "".join(f"{s} {b} {o}\n" for s, b, o in triples)
    out = subprocess.run([rocrand_pin], input=inp, capture_output=True, text=True, check=True)
    lines = out.stdout.strip().splitlines()
    assert len(lines) == len(triples)
    for (s, b, o), line in zip(triples, lines):
        j = o // 4
        ref = philox.philox4x32_10((j & 0xFFFFFFFF, j >> 32, b & 0xFFFFFFFF, b >> 32),
                                   (s & 0xFFFFFFFF, s >> 32))
        assert tuple(int(x) for x in line.split()) == ref


def test_unit_keys_follow_block_layout(rocrand_pin):
    """Unit i of draw b reads word (i // 64) % 4 of block 64 (i // 256) + i % 64."""
    seed, b, n = 0xFEEDFACE12345678, 987654321, 600
    u = assign.unit_keys(seed, b, n)
    blocks = sorted({assign.unit_block_word(i)[0] for i in range(n)})
    inp = "".join(f"{seed} {b} {4 * j}\n" for j in blocks)
    out = subprocess.run([rocrand_pin], input=inp, capture_output=True, text=True, check=True)
    words = {j: tuple(int(x) for x in line.split())
             for j, line in zip(blocks, out.stdout.strip().splitlines())}
    for i in range(n):
        j, r = assign.unit_block_word(i)
        assert u[i] == words[j][r]
