"""GPU tests of the batched launch (several uneven instances advanced by one
launch per phase), the sweep autotuner and the hipGraph replay.

The batched kernels run the same per-node arithmetic as the single-instance
ones, so their fields must agree bit for bit; the oracle checks each instance
as well.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2003_12186_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B(require_gpu):
    from paper_2003_12186_amd import binding
    binding.load()
    return binding


def _small_batch(n=6, math_=W.MATH_FP64):
    ws = W.membrane_batch_uneven(n_inst=64)
    ws = sorted(ws, key=lambda w: w.problem.nx)       # a spread of sizes
    pick = [ws[int(i)] for i in np.linspace(0, 63, n)]
    for w in pick:
        w.problem.math = math_
    return pick


@pytest.mark.parametrize("math_", [W.MATH_FP32, W.MATH_FP64])
def test_batched_equals_single_and_oracle(B, math_):
    ws = _small_batch(6, math_)
    _say("batched membranes, sizes " + ", ".join(str(w.problem.nx) for w in ws) +
         f", math={math_}, 300 steps")
    sim = B.Sim([w.problem for w in ws], [w.X0 for w in ws])
    tune = sim.autotune(3)
    _say(f"  autotune: {tune}")
    sim.step(300)
    for j, w in enumerate(ws):
        g = sim.fields(B.F_DISTRIB, inst=j, dtype=np.float32)
        one = B.Sim([w.problem], [w.X0])
        one.step(300)
        s1 = one.fields(B.F_DISTRIB, dtype=np.float32)
        assert np.array_equal(g, s1), f"instance {j} differs from its single-instance run"
        assert np.array_equal(sim.markers(j)[0], one.markers()[0])
        one.close()
        p = O.make_problem(w.problem)
        f = O.rest_state(p)
        X = w.X0.copy()
        O.run(p, f, X, 300)
        _, ux, uy = O.moments(p, f)
        gg = sim.fields(B.F_UX | B.F_UY, inst=j)
        err = np.sqrt(((gg[0] - ux) ** 2 + (gg[1] - uy) ** 2).sum() / (ux ** 2 + uy ** 2).sum())
        _say(f"  instance {j} (L={w.problem.nx}, N={w.problem.n_markers}): rel L2 u vs oracle {err:.2e}")
        assert err <= 1e-6
    assert all(sim.diag(j)["error_bits"] == 0 for j in range(len(ws)))
    sim.close()


@pytest.mark.parametrize("math_", [W.MATH_FP32, W.MATH_FP64])
def test_fp16_batched_equals_single(B, math_):
    # FP16 storage: the batched sweep (one launch over the slices of every
    # instance) and the single-instance row-segment sweep of a 512-wide
    # lattice run the same per-node arithmetic and agree bit for bit.
    ws = [W.membrane_seeded(L=512, seed=s, storage=W.STORE_FP16) for s in (0, 2)]
    for w in ws:
        w.problem.math = math_
    _say(f"FP16 512x512 membranes (seeds 0, 2), math={math_}: batched vs single, 200 steps")
    sim = B.Sim([w.problem for w in ws], [w.X0 for w in ws])
    sim.step(200)
    for j, w in enumerate(ws):
        one = B.Sim([w.problem], [w.X0])
        one.step(200)
        assert np.array_equal(sim.fields(B.F_DISTRIB, inst=j, dtype=np.float32),
                              one.fields(B.F_DISTRIB, dtype=np.float32))
        assert np.array_equal(sim.markers(j)[0], one.markers()[0])
        one.close()
    assert all(sim.diag(j)["error_bits"] == 0 for j in range(len(ws)))
    sim.close()


def test_batched_binning_of_longest_chords_equals_single(B):
    # The longest chords an initial curve may have (4 lu) on a wavy membrane:
    # each chord's box meets up to four tiles (all counted in the batched
    # geometry pass's LDS table), and the one block of 256 chords meets about
    # ninety tiles (the table holds 128).  The tile lists differ from the
    # single-instance pass in order only, so the fields agree bit for bit.
    L, n = 512, 256
    th = 2.0 * np.pi * np.arange(n) / n
    r = 130.0 + 12.0 * np.sin(8.0 * th)
    X = np.stack([L / 2.0 + r * np.cos(th), L / 2.0 + r * np.sin(th)], axis=1)
    chords = np.hypot(*(np.roll(X, -1, axis=0) - X).T)
    assert 3.9 < chords.max() <= 4.0
    probs = [W.Problem(nx=L, ny=L, tau=0.8, interface=W.IF_MEMBRANE, n_markers=n, kappa=kappa,
                       dX=2.0) for kappa in (2e-3, 5e-3)]
    _say(f"batched binning of {n} chords up to {chords.max():.2f} lu long on {L}^2, "
         "50 steps vs single runs")
    sim = B.Sim(probs, [X, X])
    sim.step(50)
    for j in range(2):
        one = B.Sim([probs[j]], [X])
        one.step(50)
        assert np.array_equal(sim.fields(B.F_DISTRIB, inst=j, dtype=np.float32),
                              one.fields(B.F_DISTRIB, dtype=np.float32))
        assert np.array_equal(sim.markers(j)[0], one.markers()[0])
        assert one.diag()["error_bits"] == 0
        one.close()
    assert all(sim.diag(j)["error_bits"] == 0 for j in range(2))
    sim.close()


@pytest.mark.parametrize("math_", [W.MATH_FP32, W.MATH_FP64])
def test_batched_ragged_lattices_equal_single_and_oracle(B, math_):
    # Lattices whose sides are not multiples of the 16-node tile (partial
    # tiles on two sides) nor of the sweep's slices (slices run across row
    # ends): the batched passes clip as the single-instance ones do.
    shapes = [(72, 56, 20.0, 14.0), (100, 84, 30.0, 24.0), (45, 61, 12.0, 17.0)]
    probs, X0 = [], []
    for j, (nx, ny, a, b) in enumerate(shapes):
        n = int(round(W.ramanujan_perimeter(a, b) / 0.8))
        probs.append(W.Problem(nx=nx, ny=ny, tau=0.7 + 0.1 * j, interface=W.IF_MEMBRANE,
                               n_markers=n, kappa=0.02, dX=W.membrane_dX(a, b, n), math=math_))
        X0.append(W.ellipse_markers(nx / 2.0, ny / 2.0, a, b, n))
    _say(f"batched membranes on ragged lattices {[(p.nx, p.ny) for p in probs]}, math={math_}, "
         "300 steps")
    sim = B.Sim(probs, X0)
    sim.autotune(2)
    sim.step(300)
    for j, p in enumerate(probs):
        one = B.Sim([p], [X0[j]])
        one.step(300)
        assert np.array_equal(sim.fields(B.F_DISTRIB, inst=j, dtype=np.float32),
                              one.fields(B.F_DISTRIB, dtype=np.float32))
        assert np.array_equal(sim.markers(j)[0], one.markers()[0])
        one.close()
        q = O.make_problem(p)
        f = O.rest_state(q)
        X = X0[j].copy()
        O.run(q, f, X, 300)
        _, ux, uy = O.moments(q, f)
        g = sim.fields(B.F_UX | B.F_UY, inst=j)
        err = np.sqrt(((g[0] - ux) ** 2 + (g[1] - uy) ** 2).sum() / (ux ** 2 + uy ** 2).sum())
        _say(f"  {p.nx}x{p.ny}: rel L2 u vs oracle {err:.2e}, max |dX| "
             f"{np.abs(sim.markers(j)[0] - X).max():.1e}")
        assert err <= 1e-6
    assert all(sim.diag(j)["error_bits"] == 0 for j in range(len(probs)))
    sim.close()


@pytest.mark.parametrize("case", ["membrane", "membrane_batch", "rigid"])
def test_graph_replay_equals_direct_launches(B, case):
    _say(f"graph replay vs direct launches, {case}")
    ws = {"membrane": lambda: [W.membrane_ellipse64()], "membrane_batch": lambda: _small_batch(3),
          "rigid": lambda: [W.cylinder_channel(small=True)]}[case]()
    probs, X0 = [w.problem for w in ws], [w.X0 for w in ws]
    a = B.Sim(probs, X0)
    b = B.Sim(probs, X0)
    b.set_graph(True)
    # several replays with eager work in between: pair graphs only (10), long
    # graphs of 16 steps plus pairs (37, 16) and an odd count's direct step
    # (37, 3)
    done = 0
    for rep, n in enumerate((10, 37, 16, 10, 3)):
        a.step(n)
        b.step(n)
        done += n
        for j in range(len(ws)):
            fa = a.fields(B.F_DISTRIB, inst=j, dtype=np.float32)
            fb = b.fields(B.F_DISTRIB, inst=j, dtype=np.float32)
            assert np.array_equal(fa, fb), (rep, j)
            assert np.array_equal(a.markers(j)[0], b.markers(j)[0])
    assert b.diag()["step"] == done
    b.set_graph(True, steps=4)            # another long-graph length
    a.step(9)
    b.step(9)
    for j in range(len(ws)):
        assert np.array_equal(a.fields(B.F_DISTRIB, inst=j, dtype=np.float32),
                              b.fields(B.F_DISTRIB, inst=j, dtype=np.float32))
    assert b.diag()["step"] == done + 9
    a.close()
    b.close()


@pytest.mark.parametrize("batched", [False, True])
def test_overlap_modes_are_bit_identical(B, batched):
    _say(f"overlap modes serial / full / interp-first, batched={batched}")
    ws = _small_batch(3) if batched else [W.membrane_ellipse64()]
    probs, X0 = [w.problem for w in ws], [w.X0 for w in ws]
    out = []
    for mode in (B.OVERLAP_SERIAL, B.OVERLAP_FULL, B.OVERLAP_INTERP_FIRST):
        s = B.Sim(probs, X0)
        s.set_overlap(mode)
        s.step(57)
        out.append([(s.fields(B.F_DISTRIB, inst=j, dtype=np.float32), s.markers(j)[0])
                    for j in range(len(ws))])
        s.close()
    for other in out[1:]:
        for (fa, xa), (fb, xb) in zip(out[0], other):
            assert np.array_equal(fa, fb) and np.array_equal(xa, xb)


def test_tile_footprint_and_autotune_keep_results(B):
    # The tile pass's blocks per CU change only the schedule, and the
    # autotuner's whole-step trials leave the state as they found it.
    _say("tile-pass footprint 0 / 1 / 4 / 16 blocks per CU, then autotune mid-run")
    ws = _small_batch(4)
    probs, X0 = [w.problem for w in ws], [w.X0 for w in ws]
    out = []
    for per_cu in (0, 1, 4, 16):
        s = B.Sim(probs, X0)
        s.set_tile_blocks(per_cu)
        assert s.schedule()["tile_blocks_per_cu"] == per_cu
        s.step(41)
        out.append([(s.fields(B.F_DISTRIB, inst=j, dtype=np.float32), s.markers(j)[0])
                    for j in range(len(ws))])
        s.close()
    for other in out[1:]:
        for (fa, xa), (fb, xb) in zip(out[0], other):
            assert np.array_equal(fa, fb) and np.array_equal(xa, xb)
    s = B.Sim(probs, X0)
    s.step(20)
    tune = s.autotune(2)
    _say(f"  autotune: {tune}")
    assert tune["tile_blocks_per_cu"] in (0, 24, 16, 12, 8, 4, 2, 1) and tune["step_us"] > 0.0
    s.step(21)
    for j in range(len(ws)):
        assert np.array_equal(s.fields(B.F_DISTRIB, inst=j, dtype=np.float32), out[0][j][0])
        assert np.array_equal(s.markers(j)[0], out[0][j][1])
    s.close()


def test_batch_rejects_mixed_storage(B):
    ws = _small_batch(2)
    ws[1].problem.storage = W.STORE_FP16
    with pytest.raises(B.IILBMError) as e:
        B.Sim([w.problem for w in ws], [w.X0 for w in ws])
    assert e.value.code == B.EINVAL


def test_batch_mixing_membranes_and_plain_fluid(B):
    # Instances without an interface ride along in a membrane batch.
    ws = _small_batch(2)
    plain = W.Problem(nx=48, ny=80, tau=0.7, math=W.MATH_FP64)
    probs = [ws[0].problem, plain, ws[1].problem]
    X0 = [ws[0].X0, None, ws[1].X0]
    _say("batch: membrane, plain 48x80 fluid, membrane; 120 steps")
    sim = B.Sim(probs, X0)
    f_plain = np.ascontiguousarray(
        O.d2q9()[2][:, None, None] * (1.0 + 1e-3 * W.seeded_noise((9, 80, 48), 60, 0)))
    sim.set_distrib(f_plain, inst=1)
    sim.step(120)
    for j, (p, x) in enumerate(zip(probs, X0)):
        one = B.Sim([p], [x])
        if j == 1:
            one.set_distrib(f_plain)
        one.step(120)
        assert np.array_equal(sim.fields(B.F_DISTRIB, inst=j, dtype=np.float32),
                              one.fields(B.F_DISTRIB, dtype=np.float32)), j
        one.close()
    sim.close()


def test_full_batch512_sampled_instances_match_oracle(B):
    # The 512-instance workload in the launch configuration the bench times
    # (autotuned table, HIP graphs): 20 steps, then the smallest, the largest
    # and two other instances against the oracle.
    ws = W.membrane_batch_uneven(512)
    for w in ws:
        w.problem.math = W.MATH_FP64
    _say("batch of 512 uneven membranes, 20 steps (graphs, autotuned), 4 sampled vs oracle")
    sim = B.Sim([w.problem for w in ws], [w.X0 for w in ws])
    sim.autotune(2)
    sim.set_graph(True)
    sim.step(20)
    sizes = [w.problem.nx for w in ws]
    picks = [int(np.argmin(sizes)), int(np.argmax(sizes)), 137, 400]
    for j in picks:
        w = ws[j]
        p = O.make_problem(w.problem)
        f = O.rest_state(p)
        X = w.X0.copy()
        O.run(p, f, X, 20)
        _, ux, uy = O.moments(p, f)
        g = sim.fields(B.F_UX | B.F_UY, inst=j)
        err = np.sqrt(((g[0] - ux) ** 2 + (g[1] - uy) ** 2).sum() / (ux ** 2 + uy ** 2).sum())
        dX = np.abs(sim.markers(j)[0] - X).max()
        _say(f"  instance {j} (L={w.problem.nx}, N={w.problem.n_markers}): rel L2 u {err:.2e}, |dX| {dX:.1e}")
        assert err <= 1e-6 and dX <= 1e-9
    assert all(sim.diag(j)["error_bits"] == 0 for j in picks)
    sim.close()


def test_isolation_keeps_the_other_instances_running(B):
    # a non-finite state in one instance of a batch: with isolation on, that
    # instance carries the error bits and the others evolve exactly as alone
    w = W.membrane_ellipse64()
    _say("isolation: NaN in instance 1 of 3; instances 0 and 2 vs a clean batch")
    sims = [B.Sim([w.problem] * 3, [w.X0] * 3) for _ in range(2)]
    bad, clean = sims
    bad.set_isolation(True)
    p = O.make_problem(w.problem)
    f = O.rest_state(p)
    f[3, 30, 40] = np.nan          # next to the membrane: reaches the markers
    bad.set_distrib(f, inst=1)
    bad.step(20)
    clean.step(20)
    bits = bad.instance_errors()
    _say(f"  error bits {bits.tolist()}")
    assert bits[1] != 0 and bits[0] == 0 and bits[2] == 0
    bad.step(30)                   # the handle keeps stepping
    clean.step(30)
    for j in (0, 2):
        assert np.array_equal(bad.fields(B.F_DISTRIB, inst=j), clean.fields(B.F_DISTRIB, inst=j))
        assert np.array_equal(bad.markers(j)[0], clean.markers(j)[0])
    # without isolation the same state stops the handle
    stop = B.Sim([w.problem] * 3, [w.X0] * 3)
    stop.set_distrib(f, inst=1)
    stop.step(20)
    with pytest.raises(B.IILBMError) as e:
        stop.sync()
    assert e.value.code == B.EUNSTABLE
    for s in (bad, clean, stop):
        s.close()
