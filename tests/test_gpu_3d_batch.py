"""Three-dimensional batches (``dugks3_batch``): one launch a step over D3Q15 or
D3Q19 instances of different sizes, walls and coefficients gives each D3Q19
instance bitwise what it gets alone, and each D3Q15 one the same up to the
grouping of its face sums (through the C ABI of include/dugks3d.h)."""
import numpy as np
import pytest

import paper_1906_11036_amd as dg
from paper_1906_11036_amd import workloads as W

pytestmark = pytest.mark.gpu
P, M, D = W.PERIODIC, W.MIRROR, W.DIRICHLET


def say(*a):
    print(*a, flush=True)


def members(q, specs, seed):
    out = []
    for k, (nx, ny, nz, bc, bdeg) in enumerate(specs):
        out.append(W.random_problem3d(seed + k, nx, ny, nz, q=q, bc=bc, stretched=any(v != P for v in bc),
                                      bdeg=bdeg))
    return out


def run_alone(p, storage, steps, launch):
    s = dg.Solver3D(p, storage=storage, launch=launch)
    s.set_phi(p.phi0)
    if D in p.bc:
        s.set_dirichlet(p.rings(steps))
    s.step(steps)
    f = s.get_f()
    s.close()
    return f


CASES = [
    (19, [(70, 9, 7, (P, P, P), 1), (33, 5, 11, (M, P, M), 2), (20, 13, 6, (D, M, P), 2),
          (130, 4, 5, (P, P, P), 3)]),
    (15, [(64, 7, 9, (P, P, P), 1), (17, 11, 6, (P, P, P), 2)]),
]


@pytest.mark.parametrize("storage,launch", [("f64", (2, 4)), ("f32", (4, 3)), ("f32", (2, 32))])
@pytest.mark.parametrize("q,specs", CASES)
def test_batch_equals_instances_alone(storage, launch, q, specs):
    probs = members(q, specs, 1200 + q)
    say(f"case 3-D batch {storage} q={q} launch={launch} sizes {[s[:3] for s in specs]}")
    steps = 4
    solvers = []
    for p in probs:
        s = dg.Solver3D(p, storage=storage)
        s.set_phi(p.phi0)
        if D in p.bc:
            s.set_dirichlet(p.rings(steps))
        solvers.append(s)
    b = dg.Batch3D(solvers, launch=launch)
    inf = b.info()
    assert inf["cells"] == sum(p.cells for p in probs)
    b.step(steps)
    eps = 1e-15 if storage == "f64" else 1e-6
    for p, s in zip(probs, solvers):
        ref = run_alone(p, storage, steps, launch)
        got = s.get_f()
        if q == 15:   # the face sums in two parts (the walled instantiation) or four
            assert np.abs(got - ref).max() <= eps * np.abs(ref).max()
        else:
            assert np.array_equal(got, ref), (q, p.nx, p.ny, p.nz, p.bc)
    b.close()


def test_batch_refuses_unequal_steps_and_sources():
    probs = members(19, [(30, 6, 5, (P, P, P), 1), (25, 7, 4, (P, P, P), 1)], 1300)
    solvers = [dg.Solver3D(p, storage="f64") for p in probs]
    for p, s in zip(probs, solvers):
        s.set_phi(p.phi0)
    solvers[0].step(1)
    b = dg.Batch3D(solvers)
    with pytest.raises(dg.DugksError):
        b.step(1)                      # the instances are at different steps
    solvers[1].step(1)
    b.step(2)
    probs[1].src_terms = W.random_source_terms3d(1301, probs[1], nterms=1)
    solvers[1].set_source_terms(probs[1].src_terms)
    with pytest.raises(dg.DugksError):
        b.step(1)                      # sources are not batched
    b.close()
