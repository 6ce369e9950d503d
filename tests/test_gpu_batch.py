"""GPU batches: one launch over many instances must give each instance exactly
what it gets alone, match the oracle in binary64, and replay identically from
the captured hipGraph."""
import numpy as np
import pytest

import paper_1906_11036_amd as dg
from oracle import Oracle
from paper_1906_11036_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def mixed_batch():
    """Uneven sizes (ragged strips and chunks), both lattices' D2Q9 member,
    periodic and mirror walls, equilibrium degrees 1, 3 and 7."""
    out = []
    specs = [(64, 64, 0, 1, 1), (300, 41, 0, 2, 2), (62, 17, 2, 1, 1), (125, 130, 0, 4, 3),
             (7, 9, 0, 2, 1), (200, 3, 2, 3, 1), (1, 5, 0, 1, 1), (129, 64, 0, 3, 2)]
    for k, (nx, ny, bc, bdeg, ddeg) in enumerate(specs):
        p = W.random_problem(500 + k, nx, ny, bcx=bc, bcy=bc, stretched=(bc == W.MIRROR),
                             bdeg=bdeg, ddeg=ddeg)
        if bc == W.MIRROR:
            p.bx, p.by = (0.0,), (0.0,)
        out.append(p)
    return out


def test_batch_fp64_matches_oracle():
    probs = mixed_batch()
    say("case batch fp64 vs oracle")
    b = dg.Batch(probs, storage="f64")
    b.set_all_phi()
    b.step(5)
    for i, p in enumerate(probs):
        o = Oracle(p)
        o.step(5)
        ref = o.get_phi()
        err = np.abs(b.get_phi(i) - ref).max() / np.abs(ref).max()
        assert err <= 1e-12, (i, err)


@pytest.mark.parametrize("storage", ["f64", "f32", "f16neq", "bf16neq"])
def test_batch_equals_single_instances_bitwise(storage):
    """Same kernel, same per-instance data: the batch reproduces each instance
    run alone bit for bit (the 16-bit scale is per instance)."""
    probs = mixed_batch()
    say(f"case batch vs single {storage}")
    b = dg.Batch(probs, storage=storage)
    b.set_all_phi()
    b.step(9)
    for i, p in enumerate(probs):
        s = dg.Solver(p, storage=storage)
        s.set_phi(p.phi0)
        s.step(9)
        assert np.array_equal(b.get_phi(i), s.get_phi()), (storage, i)


def symmetric(p):
    """p with B_y = B_x and D_yy = D_xx (x<->y symmetric equilibrium)."""
    p.by, p.dyy = p.bx, p.dxx
    return p


@pytest.mark.parametrize("storage", ["f32", "f16neq", "bf16neq"])
@pytest.mark.parametrize("q", [9, 5])
def test_xy_symmetric_kernel_gives_the_general_kernels_values(storage, q):
    """Instances with B_x = B_y and D_xx = D_yy run alone in the kernel that evaluates
    one equilibrium polynomial per x<->y pair of directions (binary32 and 16-bit storage,
    no source); in a batch with an asymmetric instance the general kernel runs them.
    Bitwise the same (ragged strips, mirror walls)."""
    specs = [(70, 33, W.PERIODIC, 3), (64, 64, W.MIRROR, 2), (130, 9, W.PERIODIC, 1)]
    syms = []
    for k, (nx, ny, bc, bdeg) in enumerate(specs):
        p = symmetric(W.random_problem(700 + k, nx, ny, q=q, bcx=bc, bcy=bc, stretched=(bc == W.MIRROR),
                                       bdeg=bdeg, ddeg=2))
        if bc == W.MIRROR:
            p.bx = p.by = (0.0,)
        syms.append(p)
    asym = W.random_problem(710, 50, 30, q=q, bdeg=2)
    assert asym.bx != asym.by
    say(f"case xy-symmetric kernel {storage} q={q}")
    b = dg.Batch(syms + [asym], storage=storage)
    assert b.info(0)["xy_symmetric"] == 0
    b.set_all_phi()
    b.step(9)
    for i, p in enumerate(syms):
        s = dg.Solver(p, storage=storage)
        assert s.info()["xy_symmetric"] == 1
        s.set_phi(p.phi0)
        s.step(9)
        assert np.array_equal(b.get_phi(i), s.get_phi()), (storage, q, i)
        s.close()


@pytest.mark.parametrize("storage", ["f32", "f16neq"])
def test_graph_replays_match_eager_steps(storage):
    """dugks_batch_step replays a captured hipGraph of 32 steps; single steps
    launch eagerly.  Checked after every replay, with host reads in between."""
    probs = W.batch_problems(count=6, nmin=64, nmax=300)
    say(f"case graph replay {storage}")
    a = dg.Batch(probs, storage=storage)
    e = dg.Batch(probs, storage=storage)
    a.set_all_phi()
    e.set_all_phi()
    for rep in range(4):
        a.step(32)
        for _ in range(32):
            e.step(1)
        for i in range(len(probs)):
            assert np.array_equal(a.get_phi(i), e.get_phi(i)), (rep, i)


def test_batch_recipe_subset_against_oracle():
    """A few instances of the benchmark batch recipe (smallest sizes), FP32
    storage, against the binary64 oracle over 100 steps."""
    probs = [p for p in W.batch_problems() if p.nx <= 80][:4]
    say("case batch recipe subset", [p.nx for p in probs])
    b = dg.Batch(probs, storage="f32")
    b.set_all_phi()
    b.step(100)
    for i, p in enumerate(probs):
        o = Oracle(p)
        o.step(100)
        ref = o.get_phi()
        l2 = np.sqrt(((b.get_phi(i) - ref) ** 2).sum() / (ref ** 2).sum())
        say(f"  instance {i} n={p.nx}: rel-L2 {l2:.2e}")
        assert l2 <= 2 * 100 * np.finfo(np.float32).eps


def test_autotune_keeps_state():
    probs = mixed_batch()
    b = dg.Batch(probs, storage="f32")
    b.set_all_phi()
    b.step(3)
    before = [b.get_phi(i) for i in range(len(probs))]
    b.autotune(1)
    after = [b.get_phi(i) for i in range(len(probs))]
    for x, y in zip(before, after):
        assert np.array_equal(x, y)


def test_per_instance_reset_of_a_stepped_batch():
    """One clock for the batch: after an odd number of steps, setting one
    instance again leaves the others stale (another step, buffer parity and
    16-bit scale phase), so stepping and reading them are refused until each
    instance is set again; then the batch equals a fresh one."""
    probs = mixed_batch()[:4]
    for storage in ("f32", "bf16neq"):
        say(f"case per-instance reset {storage}")
        b = dg.Batch(probs, storage=storage)
        b.set_all_phi()
        b.step(3)
        b.set_phi(1, probs[1].phi0)
        with pytest.raises(dg.DugksError) as ei:
            b.step(1)
        assert ei.value.code == dg._lib.E_STATE
        with pytest.raises(dg.DugksError):
            b.get_phi(0)
        with pytest.raises(dg.DugksError):
            b.autotune(1)
        assert b.get_phi(1).shape == probs[1].phi0.shape   # the re-set instance is readable
        for i, p in enumerate(probs):
            if i != 1:
                b.set_phi(i, p.phi0)
        b.step(5)
        fresh = dg.Batch(probs, storage=storage)
        fresh.set_all_phi()
        fresh.step(5)
        for i in range(len(probs)):
            assert np.array_equal(b.get_phi(i), fresh.get_phi(i)), (storage, i)


def test_graph_replay_any_step_count():
    """Runs of 4 or more steps from a step divisible by 4 replay captured graphs
    (32 and 4 steps); the rest launch one by one.  Every split gives the eager
    result bit for bit, and the launch counters say which path ran."""
    probs = W.batch_problems(count=5, nmin=64, nmax=200)
    for storage in ("f32", "f16neq"):
        say(f"case graph any count {storage}")
        a = dg.Batch(probs, storage=storage)
        e = dg.Batch(probs, storage=storage)
        a.set_all_phi()
        e.set_all_phi()
        done = 0
        for n in (4, 8, 3, 1, 20, 36, 5):
            a.step(n)
            for _ in range(n):
                e.step(1)
            done += n
            for i in range(len(probs)):
                assert np.array_equal(a.get_phi(i), e.get_phi(i)), (storage, n, i)
        info = a.info()
        assert info["graph_steps"] + info["eager_steps"] >= done
        # 4 + 8 from step 0, then 3 + 1 eager, then 20 + 36 from step 16, then 4 of the last 5
        assert info["graph_steps"] >= 4 + 8 + 20 + 36 + 4
        assert e.info()["graph_steps"] == 0
