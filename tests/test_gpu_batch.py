"""Batched persistent launches, hipGraph replay, launch-shape invariance,
the autotuner and the non-physical-state latch, through the C ABI."""
import numpy as np
import pytest

import oracle
from paper_2201_12193_amd import inputs as I
from tests.parity_util import comp_scale, rel_state_err

pytestmark = pytest.mark.gpu


def _t(U):
    import torch
    return torch.from_numpy(np.ascontiguousarray(U)).to("cuda:0")


def _small_batch(seed=3):
    """uneven 1D and 2D Euler instances (transmissive 1D, periodic 2D)"""
    rng = np.random.default_rng(seed)
    out = []
    for n in (128, 300, 1000, 2049):
        prob, U, _ = I.euler_riemann_1d(int(rng.integers(1 << 30)), n=n)
        out.append((prob, U))
    for n in (40, 66, 130):
        prob, U, _ = I.euler_quadrants_2d(int(rng.integers(1 << 30)), n=n, nq=2)
        out.append((prob, U))
    prob, U, _ = I.burgers_smooth_1d(seed=7, n=200)
    out.append((prob, U))
    return out


def test_batched_equals_standalone_bitwise():
    from paper_2201_12193_amd.mrhweno import Solver
    batch = _small_batch()
    Ub = [_t(U) for _, U in batch]
    sb = Solver([p for p, _ in batch], Ub)
    sb.step(5)
    tb, nb, _ = sb.sync()
    for q, (p, U) in enumerate(batch):
        Us = _t(U)
        ss = Solver([p], [Us])
        ss.step(5)
        ts, ns, _ = ss.sync()
        assert ts[0] == tb[q] and ns[0] == nb[q]
        assert np.array_equal(Us.cpu().numpy(), Ub[q].cpu().numpy()), q
        ss.close()
    sb.close()


def test_batched_instances_match_oracle():
    from paper_2201_12193_amd.mrhweno import Solver
    batch = _small_batch(seed=4)
    Ub = [_t(U) for _, U in batch]
    sb = Solver([p for p, _ in batch], Ub)
    prev = [U.copy() for _, U in batch]
    for _ in range(2):
        sb.step(1)
        dts = sb.last_dt()
        sb.sync()
        for q, (p, U) in enumerate(batch):
            got = Ub[q].cpu().numpy()
            ref = oracle.rk3_step(p, prev[q], dts[q])
            assert rel_state_err(p, got, ref, comp_scale(p, U)) <= 1e-12, q
            prev[q] = got
    sb.close()


def test_graph_replay_equals_eager():
    """hipGraph replays (step) and one-kernel-at-a-time launches (profile)
    give bitwise identical states, replay after replay."""
    from paper_2201_12193_amd.mrhweno import Solver
    prob, U, _ = I.euler_quadrants_2d(seed=21, n=96, nq=2)
    A, B = _t(U), _t(U)
    sa, sb = Solver([prob], [A]), Solver([prob], [B])
    for _ in range(4):
        sa.step(2)
        sb.profile(2)
        sa.sync()
        sb.sync()
        assert np.array_equal(A.cpu().numpy(), B.cpu().numpy())
    sa.close()
    sb.close()


@pytest.mark.parametrize("rows", [8, 13, 64, 200])
def test_launch_shape_invariance(rows):
    from paper_2201_12193_amd.mrhweno import Solver
    prob, U, _ = I.euler_quadrants_2d(seed=22, n=130, nq=2)
    A, B = _t(U), _t(U)
    sa, sb = Solver([prob], [A]), Solver([prob], [B])
    sb.set_launch(rows, 0 if rows != 13 else 37)   # also a persistent grid smaller than the work list
    sa.step(3)
    sb.step(3)
    sa.sync()
    sb.sync()
    assert np.array_equal(A.cpu().numpy(), B.cpu().numpy())
    sa.close()
    sb.close()


def test_autotune_keeps_state_and_results():
    from paper_2201_12193_amd.mrhweno import Solver
    prob, U, _ = I.euler_quadrants_2d(seed=23, n=256, nq=2)
    A, B = _t(U), _t(U)
    sa, sb = Solver([prob], [A]), Solver([prob], [B])
    rows, grid, ms = sa.autotune(rows=(8, 32, 64), grids=(0, 512), reps=2)
    assert rows in (8, 32, 64) and grid in (0, 512) and ms > 0
    sa.sync()
    assert np.array_equal(A.cpu().numpy(), U)     # tuning does not touch the state
    sa.step(2)
    sb.step(2)
    sa.sync()
    sb.sync()
    assert np.array_equal(A.cpu().numpy(), B.cpu().numpy())
    sa.close()
    sb.close()


def test_indicator_strip_height_keeps_results():
    """The KXRCF pass's strip height (set, or tuned on the current states)
    changes neither the state nor any step's result: a batch of a walled
    and a periodic instance steps bit for bit alike at heights 8, 46, 200 and
    the tuned one, and as with the per-problem default."""
    from paper_2201_12193_amd.mrhweno import Solver
    p1, U1, _ = I.euler_quadrants_2d(seed=25, n=300, nq=2)
    p2, U2, _ = I.euler_quadrants_2d(seed=26, n=130, nq=2)
    p2 = p2.replace(bc_x=I.REFLECTIVE, bc_y=I.TRANSMISSIVE)
    ref = [_t(U1), _t(U2)]
    s0 = Solver([p1, p2], ref)
    s0.step(3)
    s0.sync()
    want = [x.cpu().numpy() for x in ref]
    s0.close()
    for rows in (8, 46, 200, None):
        A = [_t(U1), _t(U2)]
        s = Solver([p1, p2], A)
        if rows is None:
            r, ms = s.autotune_indicator(rows=(8, 20, 46), reps=2)
            assert r in (8, 20, 46) and ms > 0
            s.sync()
            assert np.array_equal(A[0].cpu().numpy(), U1) and np.array_equal(A[1].cpu().numpy(), U2)
        else:
            s.set_indicator_launch(rows)
        s.step(3)
        s.sync()
        for a, w in zip(A, want):
            assert np.array_equal(a.cpu().numpy(), w), rows
        s.close()


def test_nonphysical_state_is_latched():
    """A negative density (forced from the host) is reported by sync, no step
    is taken and the state is left as it was; other instances go on."""
    from paper_2201_12193_amd.mrhweno import Solver, ERR_NONPHYSICAL
    prob, U, _ = I.euler_quadrants_2d(seed=24, n=32, nq=2)
    bad = U.copy()
    bad[0, 0, 5, 7] = -0.1
    A, B = _t(bad), _t(U)
    s = Solver([prob, prob], [A, B])
    s.step(3)
    t, steps, st = s.sync(raise_on_error=False)
    assert st == ERR_NONPHYSICAL
    assert steps[0] == 0 and t[0] == 0.0 and np.array_equal(A.cpu().numpy(), bad)
    assert steps[1] == 3 and t[1] > 0.0
    s.close()


@pytest.mark.slow
def test_configured_batch_equals_standalone_and_oracle():
    """The configured batch (256 Euler instances, 192 1D with N log-uniform
    in [128, 16384] and 64 2D with side log-uniform in [64, 1024], the
    benchmark's seed) advanced 8 steps in one context: a sample of instances
    of both dimensions (the smallest and largest of each, instances that
    meet a non-physical state within those steps, and a spread between)
    equals the same instance run alone bit for bit, with the same time and
    step count; the smallest instances' first step matches the oracle."""
    from paper_2201_12193_amd.mrhweno import Solver
    pairs = I.batched_instances(2048)
    probs = [p.replace(t_final=float("inf")) for p, _ in pairs]
    Ub = [_t(U) for _, U in pairs]
    sb = Solver(probs, Ub)
    sb.step(1)
    dts = sb.last_dt()
    t1, n1, _ = sb.sync(raise_on_error=False)
    first = [U.cpu().numpy() for U in Ub]
    sb.step(7)
    tb, nb, st = sb.sync(raise_on_error=False)
    sb.close()
    latched = [q for q in range(len(probs)) if nb[q] < 8]
    assert latched, "the configured batch has instances that stop within 8 steps"
    one = [q for q in range(len(probs)) if probs[q].dim == 1]
    two = [q for q in range(len(probs)) if probs[q].dim == 2]
    size = lambda q: probs[q].ncell
    sample = {min(one, key=size), max(one, key=size), min(two, key=size), max(two, key=size)}
    sample |= set(one[::48]) | set(two[::16]) | set(latched[:3])
    print(f"configured batch: {len(probs)} instances, latched {latched}, sample {sorted(sample)}", flush=True)
    for q in sorted(sample):
        Us = _t(pairs[q][1])
        ss = Solver([probs[q]], [Us])
        ss.step(8)
        ts, ns, _ = ss.sync(raise_on_error=False)
        ss.close()
        assert ts[0] == tb[q] and ns[0] == nb[q], q
        assert np.array_equal(Us.cpu().numpy(), Ub[q].cpu().numpy()), q
    for q in (min(one, key=size), min(two, key=size)):
        if n1[q] == 1:
            ref = oracle.rk3_step(probs[q], pairs[q][1], dts[q])
            assert rel_state_err(probs[q], first[q], ref, comp_scale(probs[q], pairs[q][1])) <= 1e-12, q
