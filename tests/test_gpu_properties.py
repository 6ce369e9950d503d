"""Property tests of the GPU path against the oracle: mesh sizes, lattices,
wall kinds, stretched or uniform meshes, coefficient degrees, launch shapes
and step counts drawn by hypothesis.  The draws are derandomized (the same
cases every run) and no example database is kept.  Binary64 storage must
equal the oracle to 1e-12 relative to max |f~|."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import paper_1906_11036_amd as dg
from oracle import Oracle, Oracle1D, Oracle3D
from paper_1906_11036_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
PROPS = settings(max_examples=60, derandomize=True, database=None, deadline=None,
                 suppress_health_check=[HealthCheck.too_slow])


def say(*a):
    print(*a, flush=True)


def rel_max(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@PROPS
@given(seed=st.integers(0, 10**6), nx=st.integers(1, 140), ny=st.integers(1, 40),
       q=st.sampled_from([9, 5]), bcx=st.sampled_from([W.PERIODIC, W.DIRICHLET, W.MIRROR]),
       bcy=st.sampled_from([W.PERIODIC, W.DIRICHLET, W.MIRROR]), stretched=st.booleans(),
       bdeg=st.integers(1, 4), ddeg=st.integers(1, 4), rows=st.sampled_from([2, 4, 8, 16, 64]),
       wpb=st.sampled_from([1, 2, 4]), sched=st.sampled_from([dg.SCHED_GRID, dg.SCHED_PERSISTENT]),
       steps=st.integers(1, 4))
def test_2d_fp64_random(seed, nx, ny, q, bcx, bcy, stretched, bdeg, ddeg, rows, wpb, sched, steps):
    if (bcx != W.PERIODIC and nx < 2) or (bcy != W.PERIODIC and ny < 2):
        return   # walls need two cells per axis for distinct ghosts
    p = W.random_problem(seed, nx, ny, q=q, bcx=bcx, bcy=bcy, stretched=stretched, bdeg=bdeg, ddeg=ddeg)
    say(f"case 2d seed={seed} {nx}x{ny} q={q} bc=({bcx},{bcy}) stretched={stretched} "
        f"deg=({bdeg},{ddeg}) launch=({rows},{wpb},{sched}) steps={steps}")
    s = dg.Solver(p, storage="f64", launch=(rows, wpb, sched, 1))
    s.set_phi(p.phi0)
    rings = p.rings(steps)
    if rings is not None:
        s.set_dirichlet(rings)
    s.step(steps)
    o = Oracle(p)
    o.step(steps, rings)
    assert rel_max(s.get_f(), o.get_f()) <= TOL64


@PROPS
@given(seed=st.integers(0, 10**6), nx=st.integers(1, 130), ny=st.integers(1, 12), nz=st.integers(1, 10),
       q=st.sampled_from([19, 15, 7]),
       bc=st.tuples(*[st.sampled_from([W.PERIODIC, W.MIRROR, W.DIRICHLET])] * 3),
       stretched=st.booleans(), bdeg=st.integers(1, 4), rows=st.sampled_from([1, 2]),
       planes=st.integers(1, 16), steps=st.integers(1, 3))
def test_3d_fp64_random(seed, nx, ny, nz, q, bc, stretched, bdeg, rows, planes, steps):
    p = W.random_problem3d(seed, nx, ny, nz, q=q, bc=bc, stretched=stretched, bdeg=bdeg, ddeg=2)
    say(f"case 3d seed={seed} {nx}x{ny}x{nz} q={q} bc={bc} stretched={stretched} bdeg={bdeg} "
        f"launch=({rows},{planes}) steps={steps}")
    s = dg.Solver3D(p, storage="f64")
    s.set_launch(rows, planes)
    s.set_phi(p.phi0)
    rings = p.rings(steps)
    if rings is not None:
        s.set_dirichlet(rings)
    s.step(steps)
    o = Oracle3D(p)
    o.step(steps, rings)
    assert rel_max(s.get_f(), o.get_f()) <= TOL64


@PROPS
@given(seed=st.integers(0, 10**6), n=st.integers(1, 400), bc=st.sampled_from([W.PERIODIC, W.DIRICHLET1]),
       stretched=st.booleans(), steps=st.integers(1, 9))
def test_1d_fp64_random(seed, n, bc, stretched, steps):
    p = W.random_problem1d(seed, n, bc=bc, stretched=stretched)
    say(f"case 1d seed={seed} n={n} bc={bc} stretched={stretched} steps={steps}")
    s = dg.Solver1D(p, "f64")
    s.set_phi(p.phi0)
    s.step(steps)
    o = Oracle1D(p)
    o.step(steps)
    assert rel_max(s.get_f(), o.get_f()) <= TOL64
    assert rel_max(s.get_phi_prev(), o.get_phi_prev()) <= TOL64


@settings(max_examples=25, derandomize=True, database=None, deadline=None,
          suppress_health_check=[HealthCheck.too_slow])
@given(seed=st.integers(0, 10**6), nx=st.integers(1, 130), ny=st.integers(1, 14), nz=st.integers(1, 10),
       q=st.sampled_from([19, 15, 7]),
       bc=st.tuples(*[st.sampled_from([W.PERIODIC, W.MIRROR, W.DIRICHLET])] * 3),
       bdeg=st.integers(1, 4), rows=st.tuples(st.integers(2, 4), st.integers(2, 4)),
       planes=st.tuples(st.integers(1, 16), st.integers(1, 16)), steps=st.integers(1, 3))
def test_3d_fp32_launch_shapes_bitwise(seed, nx, ny, nz, q, bc, bdeg, rows, planes, steps):
    """Binary32: two random launch shapes (two or four waves a row, one or two
    staging slots, chunk lengths) give bitwise the same distributions."""
    p = W.random_problem3d(seed, nx, ny, nz, q=q, bc=bc, stretched=True, bdeg=bdeg, ddeg=2)
    say(f"case 3d f32 seed={seed} {nx}x{ny}x{nz} q={q} bc={bc} bdeg={bdeg} rows={rows} planes={planes}")
    out = []
    for r, pl in zip(rows, planes):
        s = dg.Solver3D(p, storage="f32")
        s.set_launch(r, pl)
        s.set_phi(p.phi0)
        if p.rings(1) is not None:
            s.set_dirichlet(p.rings(steps))
        s.step(steps)
        out.append(s.get_f())
        s.close()
    assert np.array_equal(out[0], out[1])
