"""GPU parity of the learned-correction kernels (through the C ABI) against
the FP64 oracle in ``oracle/learned.py``.

The network runs on BF16 MFMA with FP32 accumulation and BF16 activations,
so its outputs and gradients are compared with the oracle evaluated on the
same BF16-rounded weights and inputs, to BF16 accuracy (relative L2 1e-2 for
outputs, 3e-2 for gradients).  Features and targets use FP32/FP64
arithmetic and are compared to their rounding; flags are exact away from
ties (|sd| within 1e-4 of 0 or of the band edge 4).
"""
import sys

import numpy as np
import pytest

import oracle as O
import oracle.learned as OL
from paper_2003_12186_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mods(require_gpu):
    from paper_2003_12186_amd import binding, learned
    binding.load()
    learned.lib()
    return binding, learned


def _bf16(a):
    import torch
    return torch.tensor(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).float().numpy().astype(np.float64)


def _rel(a, b):
    return np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300)


def _params(seed, bias=0.05):
    Wt, b = OL.init_params(seed=seed)
    rng = np.random.default_rng(seed + 100)
    b = [rng.normal(scale=bias, size=x.shape) for x in b]
    return Wt, b


def _net(LN, Wt, b):
    p = LN.flatten_params(Wt, b)
    net = LN.Net(p)
    Wq = [_bf16(w) for w in Wt]                         # what the kernels multiply with
    bq = [np.asarray(x, dtype=np.float32).astype(np.float64) for x in b]
    return net, Wq, bq


def _inputs(n, seed):
    import torch
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(n, 24, 24, 4)).astype(np.float32)
    t = torch.tensor(x).to(torch.bfloat16).cuda()
    return t, t.float().cpu().numpy().astype(np.float64)


def test_forward_matches_oracle(mods):
    _, LN = mods
    _say("CNN forward, 6 random patches, BF16 MFMA vs FP64 oracle")
    Wt, b = _params(1)
    net, Wq, bq = _net(LN, Wt, b)
    xg, xo = _inputs(6, 2)
    out, _ = net.forward(xg)
    got = out.cpu().numpy().astype(np.float64)
    want = OL.forward(Wq, bq, xo)[4]
    r = _rel(got, want)
    _say(f"  rel L2 {r:.3e}  max|d| {np.abs(got - want).max():.3e} of max {np.abs(want).max():.3e}")
    assert got.shape == want.shape
    assert r <= 1e-2
    assert np.abs(got - want).max() <= 3e-2 * np.abs(want).max()


def test_backward_matches_oracle(mods):
    import torch
    _, LN = mods
    _say("CNN backward (masked MSE), 5 patches, per-layer gradients vs FP64 oracle")
    Wt, b = _params(3)
    net, Wq, bq = _net(LN, Wt, b)
    xg, xo = _inputs(5, 4)
    rng = np.random.default_rng(5)
    tgt = rng.normal(size=(5, 16, 16, 9)).astype(np.float32)
    mask = (rng.random((5, 16, 16)) < 0.6).astype(np.uint8)
    out, sv = net.forward(xg, save=True)
    grad, loss = net.backward(xg, sv, out, torch.tensor(tgt).cuda(), torch.tensor(mask).cuda())
    g = grad.cpu().numpy().astype(np.float64)
    acts = OL.forward(Wq, bq, xo)
    gW, gb = OL.backward(Wq, bq, acts, tgt.astype(np.float64), mask.astype(bool))
    lo = OL.loss(acts[4], tgt.astype(np.float64), mask.astype(bool))
    gw2, gb2 = LN.split_params(g)
    for l in range(4):
        rw, rb = _rel(gw2[l], gW[l]), _rel(gb2[l], gb[l])
        _say(f"  layer {l + 1}: rel L2 dW {rw:.3e}  db {rb:.3e}")
        assert rw <= 3e-2 and rb <= 3e-2
    _say(f"  loss {loss.item():.6e} vs {lo:.6e}")
    assert abs(loss.item() - lo) <= 1e-2 * lo


def test_backward_is_deterministic(mods):
    import torch
    _, LN = mods
    Wt, b = _params(6)
    net, _, _ = _net(LN, Wt, b)
    xg, _ = _inputs(7, 7)
    tgt = torch.randn((7, 16, 16, 9), device="cuda")
    mask = torch.ones((7, 16, 16), dtype=torch.uint8, device="cuda")
    out, sv = net.forward(xg, save=True)
    g1, _ = net.backward(xg, sv, out, tgt, mask)
    g2, _ = net.backward(xg, sv, out, tgt, mask)
    assert torch.equal(g1, g2)


def test_adam_matches_oracle_and_repacks(mods):
    import torch
    _, LN = mods
    _say("Adam: three FP32 steps vs FP64 oracle, then forward with the new weights")
    Wt, b = _params(8)
    p0 = LN.flatten_params(Wt, b)
    net = LN.Net(p0)
    rng = np.random.default_rng(9)
    ref = p0.astype(np.float64).copy()
    opt = OL.Adam([ref], lr=1e-3)
    for _ in range(3):
        g = rng.normal(size=LN.NPARAM).astype(np.float32)
        net.adam(torch.tensor(g).cuda(), lr=1e-3)
        opt.step([ref], [g.astype(np.float64)])
    got = net.numpy().astype(np.float64)
    assert np.abs(got - ref).max() <= 1e-6 * max(1.0, np.abs(ref).max())
    # the packed copy follows the master weights
    xg, xo = _inputs(2, 10)
    out, _ = net.forward(xg)
    Wn, bn = LN.split_params(net.numpy())
    want = OL.forward([_bf16(w) for w in Wn], bn, xo)[4]
    assert _rel(out.cpu().numpy().astype(np.float64), want) <= 1e-2


def _pair(steps_c=40, L=64, n=128, seed=10003):
    c, f = W.learned_pair_coarse_fine(seed, L=L, n_markers=n)
    c.problem.math = W.MATH_FP64
    f.problem.math = W.MATH_FP64
    return c, f, steps_c


SC = dict(in_scale=(1e3, 1e3, 1e3, 0.125), out_scale=1e-4)


def test_band_tiles_and_patches_match_oracle(mods):
    B, LN = mods
    c, _, steps = _pair()
    _say(f"band tiles + patches: coarse {c.problem.nx}^2, N={c.problem.n_markers}, {steps} steps")
    sim = B.Sim([c.problem], [c.X0])
    sim.step(steps)
    band = LN.Band(sim)
    sc = LN.make_scales(**SC)
    band.find()
    band.patches(sc)
    f = sim.fields(B.F_DISTRIB)
    X = sim.markers()[0]
    feat, sd = OL.node_features(f, X)
    want_tiles = OL.band_tiles(sd)
    slots = band.slots()
    got_tiles = [band.tile_of(s) for s in slots]
    _say(f"  {len(got_tiles)} GPU tiles, {len(want_tiles)} oracle band tiles")
    assert set(want_tiles) <= set(got_tiles)
    assert got_tiles == sorted(got_tiles, key=lambda t: (t[1], t[0]))
    inp = band.inp.float().cpu().numpy().astype(np.float64)
    fl = band.flags.cpu().numpy()
    ps = band.pscale.cpu().numpy().astype(np.float64)
    scale = np.array(SC["in_scale"])
    for s, (tx, ty) in zip(slots, got_tiles):
        fo = OL.extract_patch(feat, tx, ty)
        so = OL.extract_patch(sd, tx, ty)
        amp = OL.patch_amplitude(fo, scale)
        assert abs(ps[s] - amp) <= 1e-4 * amp, (tx, ty, ps[s], amp)
        g = inp[s] / scale
        g[..., :3] *= ps[s]
        for ch in range(3):
            assert np.all(np.abs(g[..., ch] - fo[..., ch]) <= 5e-3 * np.abs(fo[..., ch]) + 1e-9), (tx, ty, ch)
        assert np.all(np.abs(g[..., 3] - fo[..., 3]) <= 5e-3 * np.abs(fo[..., 3]) + 1e-4)
        away0 = np.abs(so) > 1e-4
        assert np.array_equal((fl[s] & 1)[away0] == 1, (so < 0)[away0]), (tx, ty)
        away4 = np.abs(np.abs(so) - 4.0) > 1e-4
        assert np.array_equal((fl[s] & 2)[away4] == 2, (np.abs(so) <= 4.0)[away4]), (tx, ty)
    sim.close()


def test_targets_match_oracle(mods):
    B, LN = mods
    c, f, steps = _pair()
    _say(f"targets: coarse {c.problem.nx}^2 x {steps} steps vs fine {f.problem.nx}^2 x {4 * steps}")
    sc_ = B.Sim([c.problem], [c.X0])
    sf = B.Sim([f.problem], [f.X0])
    sc_.step(steps)
    sf.step(4 * steps)
    band = LN.Band(sc_)
    sc = LN.make_scales(**SC)
    band.find()
    band.patches(sc)
    tg, mk = band.targets(sf, sc)
    fc, ff = sc_.fields(B.F_DISTRIB), sf.fields(B.F_DISTRIB)
    want = OL.targets(fc, ff)
    _, sd = OL.node_features(fc, sc_.markers()[0])
    tg = tg.cpu().numpy().astype(np.float64) * SC["out_scale"]
    tg *= band.pscale.cpu().numpy().astype(np.float64)[:, None, None, None]
    mk = mk.cpu().numpy()
    scale = np.abs(want).max()
    n = 0
    for s in band.slots():
        tx, ty = band.tile_of(s)
        wo = want[ty * 16:(ty + 1) * 16, tx * 16:(tx + 1) * 16]
        so = sd[ty * 16:(ty + 1) * 16, tx * 16:(tx + 1) * 16]
        m = mk[s].astype(bool)
        away4 = np.abs(np.abs(so) - 4.0) > 1e-4
        assert np.array_equal(m[away4], (np.abs(so) <= 4.0)[away4])
        assert np.abs(tg[s][m] - wo[m]).max(initial=0.0) <= 1e-5 * scale
        n += int(m.sum())
    _say(f"  {n} band nodes, max |target| {scale:.3e}")
    assert n > 100
    sc_.close()
    sf.close()


def test_correction_matches_oracle(mods):
    B, LN = mods
    c, _, steps = _pair()
    _say("fused correction (patches -> network -> masked add) vs oracle network on the same patches")
    sim = B.Sim([c.problem], [c.X0])
    sim.step(steps)
    Wt, b = _params(11, bias=0.2)
    net, Wq, bq = _net(LN, Wt, b)
    band = LN.Band(sim)
    sc = LN.make_scales(**SC)
    f0 = sim.fields(B.F_DISTRIB)
    band.correct(net, sc)
    f1 = sim.fields(B.F_DISTRIB)
    got = f1 - f0
    inp = band.inp.float().cpu().numpy().astype(np.float64)
    fl = band.flags.cpu().numpy()
    slots = band.slots()
    out = OL.forward(Wq, bq, inp[slots])[4] * SC["out_scale"]
    out *= band.pscale.cpu().numpy().astype(np.float64)[slots][:, None, None, None]
    ex, ey, _ = O.d2q9()
    want = np.zeros_like(got)
    for q, s in enumerate(slots):
        tx, ty = band.tile_of(s)
        for oy in range(16):
            for ox in range(16):
                fq = fl[s, oy + 4, ox + 4]
                if not fq & 2:
                    continue
                for i in range(9):
                    if i and (fl[s, oy + 4 - ey[i], ox + 4 - ex[i]] & 1) != (fq & 1):
                        continue
                    want[i, ty * 16 + oy, tx * 16 + ox] = out[q, oy, ox, i]
    _say(f"  max |df| {np.abs(want).max():.3e}, rel L2 {_rel(got, want):.3e}")
    assert np.array_equal(got == 0.0, want == 0.0)
    assert _rel(got, want) <= 1e-2
    assert np.abs(got - want).max() <= 3e-2 * np.abs(want).max()
    sim.close()


def test_infer_over_many_tiles_matches_forward_and_apply(mods):
    B, LN = mods
    # a 512^2 instance lists more band tiles than one block per instance
    # strides over, next to a 256^2 one
    pairs = [W.learned_pair_coarse_fine(10003, L=256, n_markers=512), W.learned_pair_coarse_fine(10004, L=512, n_markers=1024)]
    for c, _ in pairs:
        c.problem.math = W.MATH_FP64
    _say("correct == tiles + patches + infer (bit-exact) == training forward + apply, 256^2 and 512^2")
    sims = [B.Sim([c.problem for c, _ in pairs], [c.X0 for c, _ in pairs]) for _ in range(3)]
    for s in sims:
        s.step(30)
    Wt, b = _params(12, bias=0.2)
    net, _, _ = _net(LN, Wt, b)
    sc = LN.make_scales(**SC)
    bands = [LN.Band(s) for s in sims]
    bands[0].correct(net, sc)
    bands[1].find()
    bands[1].patches(sc)
    bands[1].infer(net, sc)
    bands[2].find()
    bands[2].patches(sc)
    out, _ = net.forward(bands[2].inp)
    bands[2].apply(out, sc)
    cnt = bands[0].count.cpu().numpy()
    _say(f"  band tiles per instance {cnt.tolist()}")
    assert cnt[1] > 64 and np.array_equal(cnt, bands[1].count.cpu().numpy())
    f0 = [sims[0].fields(B.F_DISTRIB, inst=j) for j in range(2)]
    for j in range(2):
        assert np.array_equal(sims[1].fields(B.F_DISTRIB, inst=j), f0[j])
    ref = [B.Sim([pairs[j][0].problem], [pairs[j][0].X0]) for j in range(2)]
    for j, r in enumerate(ref):
        r.step(30)
        base = r.fields(B.F_DISTRIB)
        d0 = f0[j] - base
        d2 = sims[2].fields(B.F_DISTRIB, inst=j) - base
        _say(f"  inst {j}: max |df| {np.abs(d0).max():.3e}, max diff {np.abs(d0 - d2).max():.3e}")
        assert np.abs(d0).max() > 0
        assert np.abs(d0 - d2).max() <= 1e-6 * np.abs(d0).max()
        # every listed tile with a band node received a correction (its rest population)
        sl = slice(j * bands[0].cap, j * bands[0].cap + cnt[j])
        tl = bands[0].tiles.view(-1, 2).cpu().numpy()[sl]
        has = (bands[0].flags.cpu().numpy()[sl, 4:20, 4:20] & 2).reshape(cnt[j], -1).any(axis=1)
        hit = np.abs(d0[0]).reshape(r.problems[0].ny // 16, 16, r.problems[0].nx // 16, 16).max(axis=(1, 3))
        assert has.sum() > 0.8 * cnt[j]
        assert (hit[tl[has, 1], tl[has, 0]] > 0).all()
        r.close()
    for s in sims:
        s.close()


@pytest.mark.parametrize("mode", ["full", "interp_first", "serial"])
def test_registered_correction_matches_manual_steps(mods, mode):
    B, LN = mods
    # the handle applying the correction inside its steps (other streams,
    # graph replays) gives the same state as step + correct called in turn
    pairs = [W.learned_pair_coarse_fine(s, L=64, n_markers=128) for s in (10003, 10006)]
    for c, _ in pairs:
        c.problem.math = W.MATH_FP64
    modes = {"full": B.OVERLAP_FULL, "interp_first": B.OVERLAP_INTERP_FIRST, "serial": B.OVERLAP_SERIAL}
    _say(f"registered correction vs step + correct, overlap {mode}, 2 instances, 8 steps")
    Wt, b = _params(13, bias=0.2)
    net, _, _ = _net(LN, Wt, b)
    sc = LN.make_scales(**SC)
    sims = [B.Sim([c.problem for c, _ in pairs], [c.X0 for c, _ in pairs]) for _ in range(3)]
    for sm in sims:
        sm.set_overlap(modes[mode])
    manual, reg, plain = sims
    bm = LN.Band(manual)
    for _ in range(8):
        manual.step(1)
        bm.correct(net, sc)
    br = LN.Band(reg)
    br.attach(net, sc)
    reg.step(2)
    reg.set_graph(True)
    reg.step(6)
    plain.step(8)
    for j in range(2):
        fm = manual.fields(B.F_DISTRIB, inst=j)
        assert np.array_equal(reg.fields(B.F_DISTRIB, inst=j), fm)
        assert np.array_equal(reg.markers(j)[0], manual.markers(j)[0])
        assert np.abs(fm - plain.fields(B.F_DISTRIB, inst=j)).max() > 0
    # unregistered, the handle steps without the correction again
    br.detach()
    reg.step(2)
    manual.step(2)
    assert np.array_equal(reg.fields(B.F_DISTRIB, inst=1), manual.fields(B.F_DISTRIB, inst=1))
    for sm in sims:
        sm.close()


def test_fp16_storage_correction_paths_agree(mods):
    B, LN = mods
    # FP16 deviation storage: the registered correction, the host-called one
    # and the training forward + masked add give the same lattice
    pairs = [W.learned_pair_coarse_fine(s, L=64, n_markers=128) for s in (10003, 10006)]
    for c, _ in pairs:
        c.problem.storage = W.STORE_FP16
        c.problem.math = W.MATH_FP32
    _say("FP16 storage: registered == step + correct (bit-exact) ~ step + forward + apply")
    Wt, b = _params(14, bias=0.2)
    net, _, _ = _net(LN, Wt, b)
    sc = LN.make_scales(**SC)
    sims = [B.Sim([c.problem for c, _ in pairs], [c.X0 for c, _ in pairs]) for _ in range(4)]
    reg, manual, fwd, plain = sims
    br = LN.Band(reg)
    br.attach(net, sc)
    reg.step(6)
    bm, bf = LN.Band(manual), LN.Band(fwd)
    for _ in range(6):
        manual.step(1)
        bm.correct(net, sc)
        fwd.step(1)
        bf.find()
        bf.patches(sc)
        out, _ = net.forward(bf.inp)
        bf.apply(out, sc)
    plain.step(6)
    for j in range(2):
        fr = reg.fields(B.F_DISTRIB, inst=j)
        assert np.array_equal(fr, manual.fields(B.F_DISTRIB, inst=j))
        d_reg = fr - plain.fields(B.F_DISTRIB, inst=j)
        d_fwd = fwd.fields(B.F_DISTRIB, inst=j) - plain.fields(B.F_DISTRIB, inst=j)
        _say(f"  inst {j}: max |df| {np.abs(d_reg).max():.3e}, rel L2 reg vs fwd {_rel(d_reg, d_fwd):.3e}")
        assert np.abs(d_reg).max() > 0
        # both round every corrected value to FP16 once, in the same way
        assert _rel(d_reg, d_fwd) <= 1e-3
    for sm in sims:
        sm.close()


def test_training_reduces_the_loss(mods):
    import torch
    B, LN = mods
    _say("training: 2 coarse/fine pairs 64^2/128^2, patches every 20 coarse steps, 150 Adam steps")
    sc = LN.make_scales(**SC)
    pairs = [W.learned_pair_coarse_fine(s, L=64, n_markers=128) for s in (0, 1)]
    sc_ = B.Sim([p[0].problem for p in pairs], [p[0].X0 for p in pairs])
    sf = B.Sim([p[1].problem for p in pairs], [p[1].X0 for p in pairs])
    band = LN.Band(sc_)
    X, T, M = [], [], []
    for _ in range(5):
        sc_.step(20)
        sf.step(80)
        band.find()
        band.patches(sc)
        tg, mk = band.targets(sf, sc)
        sl = torch.tensor(band.slots(), device="cuda")
        X.append(band.inp[sl].clone())
        T.append(tg[sl].clone())
        M.append(mk[sl].clone())
    X, T, M = torch.cat(X), torch.cat(T), torch.cat(M)
    Wt, b = OL.init_params(seed=12)
    net = LN.Net(LN.flatten_params(Wt, b))
    losses = []
    for it in range(150):
        out, sv = net.forward(X, save=True)
        g, loss = net.backward(X, sv, out, T, M)
        net.adam(g, lr=1e-3)
        losses.append(loss.item())
    _say(f"  {X.shape[0]} patches; loss {losses[0]:.4e} -> {losses[-1]:.4e}")
    assert np.isfinite(losses).all()
    assert losses[-1] < 0.5 * losses[0]
    sc_.close()
    sf.close()


def test_trained_network_gains_over_no_correction(mods):
    # Ablation on held-out seeds with the committed weights: the one-step
    # band error of the network against the fine run's targets, next to the
    # error of applying no correction (the plain coarse method).
    import os
    _, LN = mods
    from paper_2003_12186_amd import train_learned as TL
    d = np.load(os.path.join(os.path.dirname(LN.__file__), "data", "cnn_coarse256.npz"))
    net = LN.Net(d["params"])
    sc = LN.make_scales(d["in_scale"], float(d["out_scale"]))
    held = list(W.LEARNED_HELDOUT_SEEDS)[:8]
    l_net, l_zero = TL.heldout_loss(net, sc, held, per_seed=2)
    _say(f"held-out seeds {held[0]}..{held[-1]}: one-step band loss network {l_net:.4e} "
         f"vs no correction {l_zero:.4e}")
    assert l_net < 0.7 * l_zero


def test_ceiling_gap_is_acoustic_and_band_bound(mods):
    # The ceiling study on 16 held-out seeds to coarse step 1000: the plain
    # coarse run's error against the fine run is at least 95 % curl-free
    # (acoustic) in energy; the exact targets applied every step on the band
    # leave it above 1e-2, on the whole lattice below.  This is why the
    # learned band correction cannot reach a 1e-2 rollout (measured on 200
    # seeds: 16.7 % / 8.9 % / 0.08 % medians at step 1000).
    import os
    _, LN = mods
    from paper_2003_12186_amd import train_learned as TL
    d = np.load(os.path.join(os.path.dirname(LN.__file__), "data", "cnn_coarse256.npz"))
    net = LN.Net(d["params"])
    sc = LN.make_scales(d["in_scale"], float(d["out_scale"]))
    held = list(W.LEARNED_HELDOUT_SEEDS)[:16]
    res = TL.ceiling(net, sc, held, alphas=(0.1,), checkpoints=(500, 1000))
    r = res["runs"]
    tot = np.array(r["plain"]["total"][-1])
    div = np.array(r["plain"]["div_free"][-1])
    band = np.median(r["exact_band"]["total"][-1])
    whole = np.median(r["exact_whole"]["total"][-1])
    share = np.median(div ** 2 / tot ** 2)
    _say(f"16 held-out seeds, coarse step 1000: plain {np.median(tot):.4f} (divergence-free energy "
         f"share {share:.4f}), exact band {band:.4f}, exact whole lattice {whole:.2e}")
    assert share < 0.05
    assert whole < 1e-2 < band < np.median(tot)
