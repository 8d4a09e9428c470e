"""The oracle's Philox4x32-10 noise blocks against rocRAND's open-source
Philox4x32-10 engine (a third implementation of the SC'11 generator), built
here as a host-only program from tests/aux/rocrand_philox_dump.cpp and run, not
copied."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def dump_exe(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("rr") / "rr_dump")
    subprocess.run([hipcc, "-O1", "--offload-arch=gfx950", "-x", "hip",
                    os.path.join(HERE, "aux", "rocrand_philox_dump.cpp"), "-o", out],
                   check=True, capture_output=True)
    return out


def test_oracle_philox_matches_rocrand(dump_exe, oracle):
    rng = np.random.default_rng(2309)
    triples = [(0, 0, 0), (230910292, 0, 0), (230910292, 999, 33554431),
               (2 ** 64 - 1, 2 ** 32 + 7, 2 ** 40 - 1)]
    triples += [(int(rng.integers(0, 2 ** 63)), int(rng.integers(0, 2 ** 40)), int(rng.integers(0, 2 ** 40)))
                for _ in range(200)]
    inp = "".join(f"{s} {t} {q}\n" for s, t, q in triples)
    res = subprocess.run([dump_exe], input=inp, capture_output=True, text=True, check=True)
    lines = res.stdout.strip().splitlines()
    assert len(lines) == len(triples)
    for (s, t, q), line in zip(triples, lines):
        ref = [int(x) for x in line.split()]
        ctr = [q & 0xFFFFFFFF, q >> 32, t & 0xFFFFFFFF, t >> 32]
        key = [s & 0xFFFFFFFF, s >> 32]
        assert oracle.philox4x32_10(ctr, key) == ref, (s, t, q)
        # and the noise values of the four cells of that block
        for j in range(4):
            w = ref[j] - (1 << 32) if ref[j] >= 1 << 31 else ref[j]
            assert oracle.noise_r(s, t, 4 * q + j) == (w + 0.5) / 2.0 ** 31
