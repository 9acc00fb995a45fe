"""Training data, training and evaluation of the learned coarse correction.

Coarse/fine pairs are membrane runs of the seeded membrane generator at 256^2 and
512^2 in diffusive scaling (``workloads.learned_pair_coarse_fine``); both advance on
the GPU through the library, many instances per handle.  Training patches
are the band tiles of the uncorrected coarse run at seeded snapshot steps,
with the equilibrium-change targets of the fine run at the same physical
time.  Evaluation runs held-out seeds three ways (fine, coarse, coarse with
the correction after every coarse step) and compares the coarse velocity
with the fine one restricted to the coarse nodes (times 2).

    python -m paper_2003_12186_amd.train_learned --train 2000 --heldout 200 \
        --out paper_2003_12186_amd/data/cnn_coarse256.npz
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import binding as B
from . import learned as LN
from . import workloads as W

COARSE_STEPS = 2000
FINE_PER_COARSE = 4


def log(msg: str) -> None:
    print(f"[learned] {msg}", flush=True)


def _sims(seeds, L=256, n_markers=512):
    pairs = [W.learned_pair_coarse_fine(s, L=L, n_markers=n_markers) for s in seeds]
    sc = B.Sim([c.problem for c, _ in pairs], [c.X0 for c, _ in pairs])
    sf = B.Sim([f.problem for _, f in pairs], [f.X0 for _, f in pairs])
    return sc, sf


def snapshot_steps(seed: int, k: int, spacing: str = "uniform"):
    """k distinct coarse steps drawn from stream (5, seed): uniform in
    [50, 2000), or log-uniform in [1, 2000) so that the early transient is
    sampled as densely per decade as the late decay."""
    rng = W.SplitMix64(5, seed)
    out = set()
    while len(out) < k:
        u = rng.uniform()
        if spacing == "log":
            out.add(max(1, min(COARSE_STEPS - 1, int(np.exp(u * np.log(COARSE_STEPS))))))
        else:
            out.add(50 + int(u * (COARSE_STEPS - 50)))
    return sorted(out)


def generate(seeds, sc: LN.Scales, per_seed: int = 4, batch: int = 128, L: int = 256,
             n_markers: int = 512, spacing: str = "uniform", net=None, alpha: float = 0.0,
             teacher: bool = False):
    """Patches, targets and masks (device tensors) of the band tiles of the
    coarse runs at `per_seed` snapshot steps per seed.  All instances of a
    batch share the union of their snapshot steps; a seed keeps only its own.
    With `net`, the coarse runs are corrected by it (scaled by `alpha`) after
    every step, so the patches come from the states the corrected run visits;
    a batch whose corrected run fails stops contributing.

    With `teacher`, the coarse runs are corrected after every step by the
    exact targets of that step (the fine run advances in lockstep).  A target
    is then the one-step drift of the coarse scheme from a state that agrees
    with the fine run, which is what the correction meets when it is applied
    every step; targets of the uncorrected run instead hold the drift
    accumulated since the start."""
    import torch
    X, T, M = [], [], []
    seeds = list(seeds)
    for b0 in range(0, len(seeds), batch):
        sb = seeds[b0:b0 + batch]
        t0 = time.perf_counter()
        sc_, sf = _sims(sb, L, n_markers)
        sc_.set_graph(True)
        sf.set_graph(True)
        band = LN.Band(sc_)
        want = {s: set(snapshot_steps(s, per_seed, spacing)) for s in sb}
        stops = sorted(set().union(*want.values()))
        now = 0
        corr = None
        if net is not None:
            corr = LN.Band(sc_)
            sca = LN.make_scales(list(sc.in_scale), sc.out_scale * alpha)
        failed = False
        if teacher:
            last = stops[-1]
            for n in range(1, last + 1):
                sc_.step(1)
                sf.step(FINE_PER_COARSE)
                band.find()
                band.patches(sc)
                tg, mk = band.targets(sf, sc)
                keep = []
                if n in stops:
                    cnt = band.count.cpu().numpy()
                    keep = [j * band.cap + r for j, s in enumerate(sb) if n in want[s]
                            for r in range(int(cnt[j]))]
                if keep:
                    idx = torch.tensor(keep, device=band.inp.device)
                    X.append(band.inp[idx].clone())
                    T.append(tg[idx].clone())
                    M.append(mk[idx].clone())
                band.apply(tg, sc)
            stops = []
        for st in stops:
            if corr is None:
                sc_.step(st - now)
            else:
                try:
                    for _ in range(st - now):
                        sc_.step(1)
                        corr.correct(net, sca)
                    sc_.sync()
                except B.IILBMError as e:
                    log(f"corrected collection failed at step {st}: {e}")
                    failed = True
                    break
            sf.step(FINE_PER_COARSE * (st - now))
            now = st
            band.find()
            band.patches(sc)
            tg, mk = band.targets(sf, sc)
            cnt = band.count.cpu().numpy()
            keep = [j * band.cap + r for j, s in enumerate(sb) if st in want[s] for r in range(int(cnt[j]))]
            if keep:
                idx = torch.tensor(keep, device=band.inp.device)
                X.append(band.inp[idx].clone())
                T.append(tg[idx].clone())
                M.append(mk[idx].clone())
        if not failed:
            sc_.sync()
        sf.sync()
        sc_.close()
        sf.close()
        log(f"seeds {sb[0]}..{sb[-1]}: {sum(x.shape[0] for x in X)} patches so far "
            f"({time.perf_counter() - t0:.1f} s)")
    return torch.cat(X), torch.cat(T), torch.cat(M)


IN_SCALE = (1.0, 3.0 ** 0.5, 3.0 ** 0.5, 0.125)


def fit_scales(seeds, per_seed=2, L=256, n_markers=512, teacher: bool = False) -> LN.Scales:
    """Fixed input scales (rho - 1 against sqrt(3) u, the acoustic balance
    c_s drho = u, and sd / 8) and the output scale: the standard deviation
    of the band targets over the patch amplitude, from a few seeds."""
    unit = LN.make_scales(IN_SCALE, 1.0)
    _, T, M = generate(seeds, unit, per_seed=per_seed, batch=len(seeds), L=L, n_markers=n_markers,
                       teacher=teacher)
    s_out = max(float(T[M.bool()].std()), 1e-12)
    return LN.make_scales(IN_SCALE, s_out)


def fit(X, T, M, steps: int, batch: int = 512, lr: float = 1e-3, seed: int = 0, log_every: int = 500,
        init=None):
    """Adam on random mini-batches of patches; returns the network and the
    loss history (one value per step)."""
    import torch
    from .learned import Net
    n = X.shape[0]
    p0 = init if init is not None else he_init(seed)
    net = Net(p0)
    g = torch.Generator(device="cpu").manual_seed(seed)
    hist = []
    t0 = time.perf_counter()
    for it in range(steps):
        idx = torch.randint(0, n, (min(batch, n),), generator=g).to(X.device)
        xb, tb, mb = X[idx], T[idx], M[idx]
        out, sv = net.forward(xb, save=True)
        grad, loss = net.backward(xb, sv, out, tb, mb)
        net.adam(grad, lr=lr)
        hist.append(loss)
        if (it + 1) % log_every == 0:
            ls = torch.stack(hist[-log_every:]).mean().item()
            log(f"step {it + 1}/{steps}: loss {ls:.4e} ({time.perf_counter() - t0:.1f} s)")
    return net, torch.cat(hist).cpu().numpy()


def he_init(seed: int) -> np.ndarray:
    """He-normal weights (std sqrt(2 / fan_in)), zero biases, from stream
    (5, 1000000 + seed)."""
    rng = W.SplitMix64(5, 1000000 + seed)
    parts = []
    for ci, co in zip(LN.CHANNELS[:-1], LN.CHANNELS[1:]):
        parts.append(rng.normal_array(9 * ci * co) * np.sqrt(2.0 / (9 * ci)))
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)


def _err(sc_, sf, j):
    gc = sc_.fields(B.F_UX | B.F_UY, inst=j)
    gf = sf.fields(B.F_UX | B.F_UY, inst=j)
    r = 2.0 * gf[:, ::2, ::2]
    return float(np.sqrt(((gc - r) ** 2).sum() / (r ** 2).sum()))


def heldout_loss(net, sc: LN.Scales, seeds, per_seed: int = 4, teacher: bool = False):
    """One-step metric on held-out seeds: masked MSE of the network against
    the targets, and of the zero correction (the method without it)."""
    X, T, M = generate(seeds, sc, per_seed=per_seed, batch=len(seeds), teacher=teacher)
    out, _ = net.forward(X)
    m = M.unsqueeze(-1).float()
    den = 9.0 * float(M.sum().item())
    return (float((m * (out - T) ** 2).sum().item()) / den, float((m * T ** 2).sum().item()) / den)


def evaluate(net, sc: LN.Scales, seeds, L: int = 256, n_markers: int = 512, checkpoints=(500, 1000, 2000),
             alpha: float = 1.0):
    """Per-seed relative L2 velocity error of the coarse run against the fine
    one, without and with the correction (times `alpha`, applied by the
    handle inside every step), and the wall time of each run (all seeds
    batched in one handle; HIP graphs for the plain runs)."""
    sc = LN.make_scales(list(sc.in_scale), sc.out_scale * alpha)
    import torch
    seeds = list(seeds)
    res = {"seeds": seeds, "checkpoints": list(checkpoints)}
    # fine reference
    pairs = [W.learned_pair_coarse_fine(s, L=L, n_markers=n_markers) for s in seeds]
    sf = B.Sim([f.problem for _, f in pairs], [f.X0 for _, f in pairs])
    sp = B.Sim([c.problem for c, _ in pairs], [c.X0 for c, _ in pairs])
    sl = B.Sim([c.problem for c, _ in pairs], [c.X0 for c, _ in pairs])
    band = LN.Band(sl)
    band.attach(net, sc)   # the handle corrects inside every step (direct launches)
    for s in (sf, sp):
        s.set_graph(True)
    t_f = t_p = t_l = 0.0
    now = 0
    e_plain, e_learn = [], []
    for cp in checkpoints:
        n = cp - now
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sf.step(FINE_PER_COARSE * n)
        sf.sync()
        t_f += time.perf_counter() - t0
        t0 = time.perf_counter()
        sp.step(n)
        sp.sync()
        t_p += time.perf_counter() - t0
        t0 = time.perf_counter()
        if sl is not None:
            try:
                sl.step(n)
                sl.sync()
            except B.IILBMError as e:
                log(f"corrected run failed before coarse step {cp}: {e}")
                sl.close()
                sl = None
        t_l += time.perf_counter() - t0
        now = cp
        e_plain.append([_err(sp, sf, j) for j in range(len(seeds))])
        e_learn.append([_err(sl, sf, j) if sl is not None else float("nan") for j in range(len(seeds))])
        log(f"coarse step {cp}: median rel L2 plain {np.median(e_plain[-1]):.3e} "
            f"learned {np.median(e_learn[-1]):.3e}")
    res.update(err_plain=e_plain, err_learned=e_learn, t_fine=t_f, t_coarse=t_p,
               t_coarse_learned=t_l, learned_stable=sl is not None)
    for s in (sf, sp, sl):
        if s is not None:
            s.close()
    return res


def _split_divfree(u, v):
    """Divergence-free part of a periodic 2-D field (Helmholtz split by FFT)."""
    k = np.fft.fftfreq(u.shape[0]) * 2 * np.pi
    ky, kx = np.meshgrid(k, k, indexing="ij")
    k2 = kx ** 2 + ky ** 2
    k2[0, 0] = 1.0
    U, V = np.fft.fft2(u), np.fft.fft2(v)
    dv = kx * U + ky * V
    return u - np.real(np.fft.ifft2(kx * dv / k2)), v - np.real(np.fft.ifft2(ky * dv / k2))


def ceiling(net, sc: LN.Scales, seeds, alphas=(1.0, 0.1), checkpoints=(250, 500, 1000, 2000)):
    """What a correction of this form can reach, on held-out seeds: the plain
    coarse run, the exact targets of the fine run applied every coarse step
    on the band (|sd| <= 4) and on the whole lattice, and the network at each
    alpha; at every checkpoint the relative L2 velocity error against the
    fine run, split into its curl-free (acoustic) and divergence-free parts
    (each over the norm of the whole fine field)."""
    import torch
    seeds = list(seeds)
    n = len(seeds)
    pairs = [W.learned_pair_coarse_fine(s) for s in seeds]
    mk = lambda k: B.Sim([p[k].problem for p in pairs], [p[k].X0 for p in pairs])
    sf, sp, sb, sw = mk(1), mk(0), mk(0), mk(0)
    nets = {}
    for a in alphas:
        s = mk(0)
        s.set_isolation(True)
        bd = LN.Band(s)
        bd.attach(net, LN.make_scales(list(sc.in_scale), sc.out_scale * a))
        nets[a] = (s, bd)
    unit = LN.make_scales(IN_SCALE, 1.0)
    bb, bw = LN.Band(sb), LN.Band(sw)
    tx, ty = np.meshgrid(np.arange(16), np.arange(16))
    every = np.stack([tx.ravel(), ty.ravel()], 1).astype(np.int32).ravel()
    bw.tiles.copy_(torch.tensor(np.tile(every, n), dtype=torch.int32, device=bw.tiles.device))
    bw.count.fill_(256)

    def errs(s, j, ref, rs, ok=True):
        g = s.fields(B.F_UX | B.F_UY, inst=j)
        if not ok or not np.isfinite(g).all():
            return (float("nan"),) * 3
        d = g - ref
        gs = _split_divfree(g[0], g[1])
        nrm = np.sqrt((ref ** 2).sum())
        sol = np.sqrt(((gs[0] - rs[0]) ** 2 + (gs[1] - rs[1]) ** 2).sum()) / nrm
        tot = np.sqrt((d ** 2).sum()) / nrm
        return float(tot), float(np.sqrt(max(tot ** 2 - sol ** 2, 0.0))), float(sol)

    names = ["plain", "exact_band", "exact_whole"] + [f"net_alpha_{a}" for a in alphas]
    res = {"seeds": seeds, "kappa": [c.problem.kappa for c, _ in pairs],
           "tau": [c.problem.tau for c, _ in pairs], "checkpoints": list(checkpoints),
           "runs": {k: {"total": [], "curl_free": [], "div_free": []} for k in names}}
    step = 0
    for cp in checkpoints:
        while step < cp:
            sf.step(FINE_PER_COARSE)
            for s in (sp, sb, sw):
                s.step(1)
            for s, _ in nets.values():
                s.step(1)
            bb.find()
            bb.patches(unit)
            tg, _ = bb.targets(sf, unit)
            bb.apply(tg, unit)
            bw.patches(unit)
            bw.flags |= 2                       # every node of every tile
            tg, _ = bw.targets(sf, unit)
            bw.apply(tg, unit)
            step += 1
        bits = {a: s.instance_errors() for a, (s, _) in nets.items()}
        rows = {k: [] for k in names}
        for j in range(n):
            ref = 2.0 * sf.fields(B.F_UX | B.F_UY, inst=j)[:, ::2, ::2]
            rs = _split_divfree(ref[0], ref[1])
            rows["plain"].append(errs(sp, j, ref, rs))
            rows["exact_band"].append(errs(sb, j, ref, rs))
            rows["exact_whole"].append(errs(sw, j, ref, rs))
            for a, (s, _) in nets.items():
                rows[f"net_alpha_{a}"].append(errs(s, j, ref, rs, bits[a][j] == 0))
        for k in names:
            arr = np.array(rows[k])
            for q, key in enumerate(("total", "curl_free", "div_free")):
                res["runs"][k][key].append(arr[:, q].tolist())
        log(f"ceiling, coarse step {cp}: " + "; ".join(
            f"{k} {np.nanmedian(np.array(rows[k])[:, 0]) if np.isfinite(np.array(rows[k])[:, 0]).any() else float('nan'):.4f}"
            for k in names))
    for s in [sf, sp, sb, sw] + [s for s, _ in nets.values()]:
        s.close()
    summ = {}
    for k in names:
        r = res["runs"][k]
        summ[k] = {}
        for key in ("total", "div_free"):
            fin = np.array(r[key][-1])
            summ[k][key] = {
                "median": [float(np.nanmedian(x)) if np.isfinite(x).any() else None for x in map(np.array, r[key])],
                "p95_at_end": float(np.nanpercentile(fin, 95)) if np.isfinite(fin).any() else None,
                "frac_within_1e-2_at_end": float((fin <= 1e-2).mean()),
                "finite_at_end": int(np.isfinite(fin).sum())}
    res["summary"] = summ
    return res


def main(argv=None) -> int:
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=2000, help="training seeds 0..n-1")
    ap.add_argument("--heldout", type=int, default=200, help="held-out seeds 10000..")
    ap.add_argument("--per-seed", type=int, default=4)
    ap.add_argument("--steps", type=int, default=6000)
    ap.add_argument("--batch", type=int, default=512)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--gen-batch", type=int, default=128)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(__file__), "data", "cnn_coarse256.npz"))
    ap.add_argument("--report", default=None, help="JSON summary path")
    ap.add_argument("--alpha", type=float, nargs="*", default=[1.0],
                    help="evaluate the correction scaled by each factor")
    ap.add_argument("--spacing", choices=["uniform", "log"], default="uniform",
                    help="snapshot steps: uniform in [50, 2000) or log-uniform in [1, 2000)")
    ap.add_argument("--teacher", action="store_true",
                    help="targets from coarse runs kept on the fine run by the exact correction "
                         "every step (one-step drift) instead of from uncorrected runs")
    ap.add_argument("--dagger", default=None, metavar="NPZ",
                    help="start from these weights and add patches from runs corrected by them")
    ap.add_argument("--dagger-alpha", type=float, default=0.1)
    ap.add_argument("--eval-only", default=None, metavar="NPZ",
                    help="skip data generation and training; evaluate these weights")
    ap.add_argument("--ceiling", default=None, metavar="JSON",
                    help="with --eval-only: run the ceiling study on the held-out seeds (exact "
                         "band and whole-lattice targets, the network at each --alpha, errors "
                         "split into curl-free and divergence-free parts) and write it here")
    a = ap.parse_args(argv)
    B.load()
    LN.lib()
    if a.eval_only:
        d = np.load(a.eval_only)
        net = LN.Net(d["params"])
        sc = LN.make_scales(d["in_scale"], float(d["out_scale"]))
        hist = d["loss"]
        t_gen = t_train = 0.0
    else:
        t0 = time.perf_counter()
        init = None
        if a.dagger:
            d0 = np.load(a.dagger)
            sc = LN.make_scales(d0["in_scale"], float(d0["out_scale"]))
            init = d0["params"]
        else:
            sc = fit_scales(range(a.train)[:8], teacher=a.teacher)
        log(f"scales in {list(sc.in_scale)} out {sc.out_scale:.3e}")
        X, T, M = generate(range(a.train), sc, per_seed=a.per_seed, batch=a.gen_batch,
                           spacing=a.spacing, teacher=a.teacher)
        if a.dagger:
            X2, T2, M2 = generate(range(a.train), sc, per_seed=a.per_seed, batch=a.gen_batch,
                                  spacing=a.spacing, net=LN.Net(init), alpha=a.dagger_alpha)
            X, T, M = torch.cat([X, X2]), torch.cat([T, T2]), torch.cat([M, M2])
            del X2, T2, M2
        t_gen = time.perf_counter() - t0
        log(f"{X.shape[0]} training patches, {int(M.sum().item())} band nodes ({t_gen:.1f} s)")
        t1 = time.perf_counter()
        net, hist = fit(X, T, M, a.steps, batch=a.batch, lr=a.lr, init=init)
        t_train = time.perf_counter() - t1
        del X, T, M
        torch.cuda.empty_cache()
        os.makedirs(os.path.dirname(a.out), exist_ok=True)
        np.savez(a.out, params=net.numpy(), in_scale=np.array(list(sc.in_scale), np.float32),
                 out_scale=np.float32(sc.out_scale), loss=hist.astype(np.float32),
                 meta=json.dumps({"train_seeds": a.train, "per_seed": a.per_seed, "steps": a.steps,
                                  "batch": a.batch, "lr": a.lr, "spacing": a.spacing,
                                  "teacher": a.teacher}))
        log(f"saved {a.out}")
    held = list(W.LEARNED_HELDOUT_SEEDS)[:a.heldout]
    if a.ceiling:
        res = ceiling(net, sc, held, alphas=tuple(a.alpha))
        with open(a.ceiling, "w") as fh:
            json.dump(res, fh)
        log(json.dumps(res["summary"]))
        return 0
    teacher = a.teacher
    if a.eval_only:
        teacher = bool(json.loads(str(d["meta"])).get("teacher", False)) if "meta" in d else False
    l_net, l_zero = heldout_loss(net, sc, held[:32], teacher=teacher)
    log(f"held-out one-step loss: network {l_net:.4e}, no correction {l_zero:.4e}")
    runs = {}
    for al in a.alpha:
        ev = evaluate(net, sc, held, alpha=al)
        fin_p = np.array(ev["err_plain"][-1])
        fin_l = np.array(ev["err_learned"][-1])
        runs[str(al)] = {
            "median_err_plain": [float(np.median(e)) for e in ev["err_plain"]],
            "median_err_learned": [float(np.nanmedian(e)) if np.isfinite(e).any() else None
                                   for e in ev["err_learned"]],
            "checkpoints": ev["checkpoints"], "stable": ev["learned_stable"],
            "frac_within_1e-2_learned": float((fin_l <= 1e-2).mean()),
            "frac_improved": float((fin_l < fin_p).mean()),
            "t_fine": ev["t_fine"], "t_coarse": ev["t_coarse"], "t_coarse_learned": ev["t_coarse_learned"],
            "speedup_learned_vs_fine": ev["t_fine"] / ev["t_coarse_learned"],
        }
    summary = {"heldout": a.heldout, "heldout_loss_network": l_net, "heldout_loss_zero": l_zero,
               "runs": runs, "t_generate": t_gen, "t_train": t_train,
               "final_loss": float(hist[-200:].mean())}
    ev = runs
    log(json.dumps(summary))
    if a.report:
        with open(a.report, "w") as fh:
            json.dump({"summary": summary, "eval": ev}, fh)
    return 0


if __name__ == "__main__":
    sys.exit(main())
