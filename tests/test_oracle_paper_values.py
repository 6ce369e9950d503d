"""The oracle against values the paper prints (long runs, opt-in with --runslow).

Example 4.4 (Sec. 4): Gaussian hill, 400 x 400, t = 10; GRE printed for three
diffusion tensors (tests/golden/ex44_gaussian_hill_gre.txt).
"""
import os

import pytest

from oracle import Oracle
from paper_1906_11036_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "ex44_gaussian_hill_gre.txt")


def rows():
    out = []
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            kxx, kxy, kyy, gre = line.split()
            out.append(([[float(kxx) * 1e-3, float(kxy) * 1e-3],
                         [float(kxy) * 1e-3, float(kyy) * 1e-3]], float(gre)))
    return out


@pytest.mark.slow
@pytest.mark.parametrize("K,paper_gre", rows())
def test_oracle_reproduces_example_4_4(K, paper_gre):
    p = W.gaussian_hill_problem(400, u=(0.01, 0.01), D=1e-3, sigma0=0.01, K=K)
    o = Oracle(p, openmp=True)
    nst = int(round(10.0 / o.dt))
    o.step(nst)
    X, Y = p.mesh()
    gre, _ = o.errors(p.exact(X, Y, o.time))
    print(f"paper {paper_gre:.4e} oracle {gre:.4e}")
    assert abs(gre - paper_gre) <= 0.15 * paper_gre
