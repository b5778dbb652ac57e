"""Pins of the oracle's random-number layer.

* Philox4x32-10 block vs the engine in the rocRAND headers (a library routine
  written by others, compiled here for the host).
* The uniform pick floor(w*k/2^32): exact preimage sizes for every k <= 24
  (closed form) and the boundary words of every bucket.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("hipcc / rocRAND headers not available")
    d = tmp_path_factory.mktemp("philox")
    exe = str(d / "philox_ref")
    subprocess.run([hipcc, "-O1", "-o", exe, os.path.join(HERE, "philox_ref.cpp")], check=True,
                   capture_output=True)
    return exe


def test_philox_matches_rocrand(orc, rocrand_ref):
    rng = np.random.default_rng(7)
    cases = [[0, 0, 0, 0, 0, 0], [0xFFFFFFFF] * 6]
    cases += rng.integers(0, 2**32, size=(300, 6), dtype=np.uint64).tolist()
    # the counter layouts the method uses: small step/playout/leaf/tree values
    for g in range(24):
        cases.append([g, 5, 77, 3, 2, 0])
        cases.append([g >> 2, 0x80000000 + g % 16, 1999, 0, 1, 0])
        cases.append([g, 0xC0000000, 12, 2047, 3, 0])
        cases.append([g, 0xFFFFFFFF, 0xFFFFFFFF, 4095, 2, 0])
    inp = "\n".join(" ".join("%x" % int(v) for v in c) for c in cases) + "\n"
    out = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True, check=True).stdout
    ref = [[int(x, 16) for x in line.split()] for line in out.strip().splitlines()]
    assert len(ref) == len(cases)
    for c, r in zip(cases, ref):
        got = orc.philox(c[:4], c[4:]).tolist()
        assert got == r, (c, got, r)


def test_philox_counter_sensitivity(orc):
    # every counter word and every key word changes every output word (avalanche)
    base = orc.philox([1, 2, 3, 4], [5, 6])
    for i in range(6):
        v = [1, 2, 3, 4, 5, 6]
        v[i] ^= 1
        o = orc.philox(v[:4], v[4:])
        assert np.all(o != base)


@pytest.mark.parametrize("k", list(range(1, 25)))
def test_mulshift_preimages(orc, k):
    # bucket j receives the words w with j*2^32 <= w*k < (j+1)*2^32, i.e.
    # w in [ceil(j*2^32/k), ceil((j+1)*2^32/k)): sizes differ by at most one
    two32 = 1 << 32
    starts = [-(-j * two32 // k) for j in range(k + 1)]
    sizes = [starts[j + 1] - starts[j] for j in range(k)]
    assert sum(sizes) == two32
    assert max(sizes) - min(sizes) <= 1
    for j in range(k):
        assert orc.mulshift(starts[j], k) == j
        assert orc.mulshift(starts[j + 1] - 1, k) == j
        if starts[j] > 0:
            assert orc.mulshift(starts[j] - 1, k) == j - 1
    assert orc.mulshift(0xFFFFFFFF, k) == k - 1
