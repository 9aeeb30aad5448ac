"""Train the warm-start network on converged fluxes produced by the GPU solver, then
measure warm vs cold solves on held-out seeds.

Data: problems of the 17 x 17 lattice family (fixed mesh, material map and cross
sections redrawn per seed); each is solved by libmoc (FP32 sweep) to `--tol-data`,
its flux rasterised to log(phi) targets. Training: MSE on the 7 output channels, Adam,
all on the project's HIP kernels; each batch is rotated / mirrored by a random element of
the square's symmetry group, and the weights of the epoch with the lowest validation loss
are kept. Evaluation: iterations and wall time to `--tol`,
cold start vs the network's guess (averaged over the lattice's 8 symmetries, and
without that average) vs a non-learned guess (flat homogenised spectrum).

python -m paper_2607_01591_amd.train_warmstart --train 160 --val 32 --test 16 \
    --out paper_2607_01591_amd/weights/warmstart_17x17.npz --report warmstart_report.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def log(msg):
    print(f"[warmstart] {msg}", flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=160)
    ap.add_argument("--val", type=int, default=32)
    ap.add_argument("--test", type=int, default=16)
    ap.add_argument("--tol-data", type=float, default=1e-5)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--out", default=None)
    ap.add_argument("--report", default=None)
    ap.add_argument("--weights", default=None, help="skip training, load these weights")
    ap.add_argument("--train-budget", type=float, default=0.0,
                    help="seconds: stop after the epoch that exceeds this (0 = no limit)")
    ap.add_argument("--no-cmfd", action="store_true",
                    help="generate the training data without CMFD acceleration")
    ap.add_argument("--no-augment", action="store_true", help="train without the rotations and mirror images")
    ap.add_argument("--data-budget", type=float, default=0.0,
                    help="seconds: stop generating training problems once this is spent (0 = no limit)")
    a = ap.parse_args(argv)
    if a.train > 1800 or a.val > 200:
        ap.error("training seeds are 100000..101799 and validation seeds 101800..101999")

    import torch
    from . import cnn, moc
    from . import problems as P
    from .warmstart import C_OUT_PAD, CHANNELS, DILATIONS, C_IN, WarmStart, homogenized_guess, load_net

    dev = torch.device("cuda:0")
    base = P.config(5, seed=100000)
    solver = moc.Solver(base, precision="f32", max_iter=20000, check_every=10)
    n_cells, region_cell = P.coarse_cells(base, 17, 17)
    V = solver.volumes()
    ws = WarmStart(solver, base, dev)
    log(f"mesh: {solver.R} regions, {solver.S} segments; image 128x128")

    def make_data(seeds, tag, budget=0.0):
        X = torch.empty((len(seeds), 128, 128, 32), dtype=torch.bfloat16, device=dev)
        T = torch.empty((len(seeds), 128, 128, C_OUT_PAD), dtype=torch.float32, device=dev)
        t0 = time.perf_counter()
        iters = []
        if not a.no_cmfd:
            solver.set_coarse_mesh(n_cells, region_cell)
        for i, sd in enumerate(seeds):
            if budget > 0 and time.perf_counter() - t0 > budget:
                log(f"{tag}: data budget spent after {i} problems")
                return X[:i], T[:i], iters
            p = P.config(5, seed=sd)
            solver.set_materials(p)
            r = solver.solve(a.tol_data)
            iters.append(r["iterations"])
            ws.rasterize(p, out=X[i:i + 1])
            ws.target(solver.flux(), out=T[i:i + 1])
            cnn.center(T[i:i + 1], base.n_groups)
            if i % 8 == 0 or i == len(seeds) - 1:
                log(f"{tag} {i + 1}/{len(seeds)} seed {sd}: {r['iterations']} it, k={r['k']:.5f}, "
                    f"{time.perf_counter() - t0:.0f} s")
        return X, T, iters

    report = {"tol": a.tol, "tol_data": a.tol_data}
    if a.weights:
        ws.net = load_net(a.weights, dev, base.n_groups)
        log(f"loaded {a.weights}")
    else:
        Xva, Tva, _ = make_data(list(range(101800, 101800 + a.val)), "val")
        Xtr, Ttr, it_tr = make_data(list(range(100000, 100000 + a.train)), "train", a.data_budget)
        n_train = int(Xtr.shape[0])
        report["n_train"], report["n_val"] = n_train, a.val
        report["data_iterations_mean"] = float(np.mean(it_tr))
        net = ws.net
        G = base.n_groups
        rng = np.random.default_rng(0)
        t0 = time.perf_counter()
        hist = []
        best = (np.inf, -1, None)
        for ep in range(a.epochs):
            lr = a.lr * (0.5 ** (ep // max(1, a.epochs // 4)))
            perm = rng.permutation(n_train)
            tl = []
            for b0 in range(0, n_train - a.batch + 1, a.batch):
                idx = torch.as_tensor(perm[b0:b0 + a.batch], device=dev)
                xb, tb = Xtr[idx], Ttr[idx]
                if not a.no_augment:
                    # the lattice's square symmetry: a rotated or mirrored material map is
                    # another valid problem whose flux is the same map of the flux
                    rot, flip = int(rng.integers(4)), bool(rng.integers(2))
                    xb, tb = torch.rot90(xb, rot, dims=(1, 2)), torch.rot90(tb, rot, dims=(1, 2))
                    if flip:
                        xb, tb = torch.flip(xb, dims=(2,)), torch.flip(tb, dims=(2,))
                tl.append(net.train_step(xb.contiguous(), tb.contiguous(), G, lr=lr))
            vl = []
            for b0 in range(0, a.val, a.batch):
                y = net.forward(Xva[b0:b0 + a.batch].contiguous())
                vl.append(float(((y[..., :G] - Tva[b0:b0 + a.batch, ..., :G]) ** 2).mean().item()))
            hist.append((float(np.mean(tl)), float(np.mean(vl))))
            if hist[-1][1] < best[0]:
                best = (hist[-1][1], ep, net.state())
            log(f"epoch {ep + 1}/{a.epochs} lr {lr:.1e}: train {hist[-1][0]:.4e} val {hist[-1][1]:.4e} "
                f"({time.perf_counter() - t0:.0f} s)")
            if a.train_budget > 0 and time.perf_counter() - t0 > a.train_budget:
                log(f"training budget spent after {ep + 1} epochs")
                break
        # keep the weights of the epoch with the lowest validation loss
        net.load(best[2])
        log(f"best validation loss {best[0]:.4e} at epoch {best[1] + 1}")
        report["best_val"], report["best_epoch"] = best[0], best[1] + 1
        report["train_history"] = hist
        report["train_seconds"] = time.perf_counter() - t0
        if a.out:
            os.makedirs(os.path.dirname(a.out), exist_ok=True)
            st = net.state()
            np.savez(a.out, **{f"W{i}": w for i, w in enumerate(st["W"])},
                     **{f"b{i}": b for i, b in enumerate(st["b"])}, chans=np.array(CHANNELS),
                     dil=np.array(DILATIONS))
            log(f"saved {a.out}")

    # ---------------------------------------------------------------- evaluation
    # per test seed: cold start, CMFD, the network's guess, the network's guess with CMFD,
    # and the non-learned homogenised guess (all to the same residual)
    rows = []
    for sd in range(200000, 200000 + a.test):
        p = P.config(5, seed=sd)
        solver.set_coarse_mesh(0)
        solver.set_materials(p)
        cold = solver.solve(a.tol)
        phi_ref = solver.flux().cpu().numpy()
        warm = ws.solve_warm(p, a.tol)
        phi_w = solver.flux().cpu().numpy()
        plain = ws.solve_warm(p, a.tol, symmetrize=False)
        solver.set_initial_guess(homogenized_guess(p, V, dev), -1.0)
        hom = solver.solve(a.tol)
        solver.set_coarse_mesh(n_cells, region_cell)
        cm = solver.solve(a.tol)
        wcm = ws.solve_warm(p, a.tol)
        err = float(np.max(np.abs(phi_w - phi_ref) / phi_ref))
        rows.append({"seed": sd, "cold_it": cold["iterations"], "cold_ms": cold["wall_ms"],
                     "warm_it": warm["iterations"], "warm_sweeps": warm["sweeps"], "warm_ms": warm["total_ms"],
                     "warm_predict_ms": warm["predict_ms"], "warm_plain_sweeps": plain["sweeps"],
                     "warm_plain_ms": plain["total_ms"], "hom_it": hom["iterations"], "hom_sweeps": hom["sweeps"],
                     "hom_ms": hom["wall_ms"], "cmfd_sweeps": cm["sweeps"], "cmfd_ms": cm["wall_ms"],
                     "warm_cmfd_sweeps": wcm["sweeps"], "warm_cmfd_ms": wcm["total_ms"],
                     "dk_warm_cold": abs(warm["k"] - cold["k"]), "dk_cmfd_cold": abs(cm["k"] - cold["k"]),
                     "flux_err_warm_vs_cold": err, "fell_back": bool(warm["flags"] & moc.FLAG_FELL_BACK_TO_COLD)})
        log(f"test seed {sd}: cold {cold['iterations']} it {cold['wall_ms']:.0f} ms | warm {warm['sweeps']} sweeps "
            f"{warm['total_ms']:.0f} ms (unsymmetrised {plain['sweeps']}) | homogenised {hom['sweeps']} | "
            f"CMFD {cm['sweeps']} sweeps {cm['wall_ms']:.0f} ms "
            f"| warm+CMFD {wcm['sweeps']} sweeps {wcm['total_ms']:.0f} ms | dk {rows[-1]['dk_warm_cold']:.1e}")

    def stat(key):
        v = np.array([r[key] for r in rows], float)
        return {"median": float(np.median(v)), "q1": float(np.percentile(v, 25)), "q3": float(np.percentile(v, 75))}

    report["test"] = rows
    report["summary"] = {k: stat(k) for k in ("cold_it", "warm_sweeps", "warm_plain_sweeps", "hom_sweeps", "cmfd_sweeps",
                                              "warm_cmfd_sweeps", "cold_ms", "warm_ms", "warm_plain_ms", "hom_ms",
                                              "cmfd_ms", "warm_cmfd_ms")}
    report["totals"] = {k: float(np.sum([r[k] for r in rows])) for k in report["summary"]}
    log(json.dumps(report["summary"]))
    if a.report:
        os.makedirs(os.path.dirname(a.report) or ".", exist_ok=True)
        with open(a.report, "w") as f:
            json.dump(report, f, indent=1)
    return report


if __name__ == "__main__":
    main()
    sys.exit(0)
