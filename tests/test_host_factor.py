"""CPU checks of the library's host factorisation (csrc/factor.cpp, compiled
into a small test program with g++): the two-chain band factor of a long star
solves the same system as its single envelope factor (the direct local solves
of Sec. 4.1, in another elimination order), its separator comes out the same
in both chains, and every band position is owned by exactly one chain."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2207_07488_amd", "csrc")


@pytest.fixture(scope="module")
def prog(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    out = str(tmp_path_factory.mktemp("host") / "twin_factor_check")
    cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-pthread", "-I", CSRC,
           os.path.join(HERE, "host", "twin_factor_check.cpp"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return out


@pytest.mark.parametrize("nx,ny,seed", [(30, 20, 1), (60, 40, 2), (25, 25, 3), (100, 10, 4), (45, 45, 5)])
def test_two_chain_factor_solves_the_same_system(prog, nx, ny, seed):
    r = subprocess.run([prog, str(nx), str(ny), str(seed)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    m, K, s, err, sepdiff, missing, res = r.stdout.split()
    assert float(res) <= 1e-11  # the single envelope factor solves the system
    assert int(K) > 0 and int(K) % 64 == 0 and int(K) + int(s) <= 0.75 * int(m)
    assert float(err) <= 1e-12  # the two chains give the same solution
    assert float(sepdiff) == 0.0  # both chains finish the separator with the same bits
    assert int(missing) == 0


def test_short_star_has_no_two_chain_factor(prog):
    r = subprocess.run([prog, "20", "20", "6"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0
    m, K = r.stdout.split()[:2]
    assert int(m) == 400 and int(K) == 0  # below 512 positions
