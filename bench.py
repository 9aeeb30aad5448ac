"""Benchmark: segment-group updates per second of the planar-MOC power iteration on one
MI355X, plus time to a 1e-6 residual, beside the FP64 CPU oracle.

A step is one power iteration of the whole path: source update, transport sweep (the
dominant kernel), scalar-flux finalisation, FP64 eigenvalue update, normalisation and
residual. The workload is the 51 x 51 pin lattice (about 1.2M triangular regions,
7 groups, 128 azimuthal x 3 polar directions, 0.01 cm spacing, vacuum on two sides),
synthetic seeded inputs. `value` = U / (wall time per step), U = 2 P G S segment-group
updates per sweep.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published HBM peak; FP32 vector peak from 256 CUs x 64 lanes x FMA at 2.4 GHz
HBM_PEAK_GBS = 8000.0
N_CU, CLOCK_GHZ = 256, 2.4
FP32_NONPACKED_TFLOPS = N_CU * 64 * 2 * CLOCK_GHZ / 1000.0      # FMA = 2 flops, no packed FP32
DG_FLOPS_PER_UPDATE = 44   # DGMOC segment solution per (segment, polar, group); 1 - e^-a and the reciprocal count one each
FLOPS_PER_UPDATE = 7     # tau mul, 1 - e^-tau (1), psi - q, * F, psi -= d, tally fma (2)
COUNTERS = os.path.join(ROOT, "profiles", "k_sweep_f32_lattice51x51_counters.txt")


def kernel_sources_hash():
    """sha256 over the sources that decide what the sweep kernel reads and writes (its code,
    the segment packing and the launch set-up: every moc_* source but the CMFD kernels,
    which run between sweeps); measured counters are only reported while this hash matches
    the one recorded with them."""
    csrc = os.path.join(ROOT, "paper_2607_01591_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(csrc)):
        if name.startswith("moc_") and name.endswith((".hip", ".h", ".cpp")) and name != "moc_cmfd.hip":
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per sweep launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary, each scaled by what the same counter reads for a 1 GiB device copy; None when
    there is no summary or the kernel sources changed since it was taken."""
    if not os.path.exists(COUNTERS):
        return None, "no counter summary"
    kv = {}
    with open(COUNTERS) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_sources_sha256") != kernel_sources_hash():
        return None, "kernel changed since the counters were taken"
    return float(kv["traffic_bytes_per_launch"]), os.path.relpath(COUNTERS, ROOT)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", type=int, default=3, help="problem recipe (3 = 51x51 lattice)")
    ap.add_argument("--no-f64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-full", action="store_true",
                    help="also time the oracle on the hexagon, the whole 51x51 lattice and to 1e-6 on the 17x17 lattice")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-hex", action="store_true")
    ap.add_argument("--solve-seeds", type=int, default=16)
    ap.add_argument("--no-cmfd", action="store_true", help="skip the CMFD time-to-tolerance legs")
    ap.add_argument("--no-dg", action="store_true", help="skip the DGMOC (extruded 3D) leg")
    ap.add_argument("--dg-only", action="store_true", help="run only the DGMOC leg (profiling)")
    ap.add_argument("--dg-steps", type=int, default=5)
    ap.add_argument("--no-sn", action="store_true", help="skip the DFEM-SN leg")
    ap.add_argument("--sn-only", action="store_true", help="run only the DFEM-SN leg (profiling)")
    ap.add_argument("--no-hfem", action="store_true", help="skip the HFEM leg")
    ap.add_argument("--no-cnn", action="store_true", help="skip the warm-start network leg")
    ap.add_argument("--cnn-only", action="store_true", help="run only the warm-start network leg (profiling)")
    ap.add_argument("--hfem-only", action="store_true", help="run only the HFEM leg (profiling)")
    ap.add_argument("--hfem-max-iter", type=int, default=5000, help="iteration cap of the HFEM solve")
    ap.add_argument("--exp-mode", default="poly")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also launch a plain 1 GiB device copy (counter calibration under rocprofv3 --pmc)")
    return ap.parse_args()


def time_iterations(s, steps, warmup):
    import torch
    s.run_iterations(warmup)
    torch.cuda.synchronize()
    s.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = s.run_iterations(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = s.profile()
    s.set_profiling(False)
    return (t1 - t0) * 1e3 / steps, prof, r


def algorithmic_bytes(info, precision):
    """Bytes one sweep launch must move at minimum: the segment stream once
    (length + region id), Sigma_t and qhat read once, the tally read-modify-written once,
    boundary fluxes read and written once."""
    R, G, P, T, S = (info["n_regions"], info["n_groups"], info["n_polar"], info["n_tracks"],
                     info["n_segments"])
    rb = 8 if precision == "f64" else 4
    seg = S * (rb + 4)
    xs = 2 * R * G * rb
    tally = 2 * R * G * 8
    psi = 2 * T * 2 * P * G * rb
    return seg + xs + tally + psi


def host_cpus():
    """Sockets, physical cores and logical CPUs of the host (/proc/cpuinfo), and the CPUs
    this process may run on (its affinity mask)."""
    sockets, cores, logical = set(), set(), 0
    phys = core = None
    with open("/proc/cpuinfo") as f:
        for line in f.read().splitlines() + [""]:
            key, _, val = line.partition(":")
            key = key.strip()
            if key == "processor":
                logical += 1
            elif key == "physical id":
                phys = val.strip()
            elif key == "core id":
                core = val.strip()
            elif not line.strip() and phys is not None:
                sockets.add(phys)
                cores.add((phys, core))
                phys = core = None
    allowed = len(os.sched_getaffinity(0))
    return {"sockets": len(sockets) or 1, "physical_cores": len(cores) or logical, "logical_cpus": logical,
            "allowed_cpus": allowed}


def _oracle_rate(prob, threads, reps):
    """Median FP64 oracle sweep rate (updates/s) over `reps` sweeps after one warm-up."""
    import numpy as np
    from oracle.oracle import Oracle
    o = Oracle.from_problem(prob, threads=threads)
    o.set_threads(threads)
    src = np.ones((o.R, o.G))
    o.sweep(src)
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        o.sweep(src)
        ts.append(time.perf_counter() - t0)
    U = 2 * o.P * o.G * o.S
    return U / float(np.median(ts)), U, float(np.median(ts))


def cpu_baseline(workload, full=False):
    """The FP64 oracle as it stands, built -O3 -march=native (no fast-math) for this host,
    timed on bounded samples: one thread and all usable physical cores (at most 16, the
    host share of one GPU), median sweep time after one warm-up. Samples: a 6 x 6 pin window
    of the 51 x 51 lattice (same pin template, A = 128, P = 3, 0.01 cm: the `value`), the
    17 x 17 lattice in full, and the oracle's time to a 1e-6 residual on the pin cell.
    full=True adds the 271-pin hexagon, the whole 51 x 51 lattice (all cores, one sweep) and
    the time to 1e-6 on the 17 x 17 lattice (minutes)."""
    import tempfile
    from oracle import oracle as O
    from paper_2607_01591_amd import problems as P
    host = host_cpus()
    threads = max(1, min(16, host["physical_cores"], host["allowed_cpus"]))
    so = os.path.join(tempfile.mkdtemp(prefix="oracle_native_"), "liboracle_native.so")
    O.build(force=True, native=True, out=so)
    O.lib(so)
    out = {"kind": "oracle", "unit": "updates/s", "cores": threads, "host": host,
           "build": "gcc -O3 -march=native -fopenmp (no fast-math)"}
    win = P.square_lattice(6, 6, seed=3, m=5, n_fuel_rings=5, n_mod_rings=7, n_azim=128, spacing=0.01,
                           bc=(1, 0, 1, 0), name="cfg3_window6x6")
    r1, U, t1 = _oracle_rate(win, 1, 3)
    rn, _, tn = _oracle_rate(win, threads, 5)
    out.update(value=rn, value_1core=r1, value_allcores=rn,
               sample=f"FP64 oracle sweeps of a 6x6-pin window of the 51x51 lattice (same template, A=128, P=3, "
                      f"0.01 cm; U={U:.3e} per sweep): median of 3 on 1 thread ({t1:.2f} s) and of 5 on {threads} "
                      f"threads ({tn:.2f} s), each after one warm-up")
    log(f"oracle window: {r1:.3e} updates/s on 1 thread, {rn:.3e} on {threads}")
    lat = P.config(2)
    a1, U2, _ = _oracle_rate(lat, 1, 3)
    an, _, _ = _oracle_rate(lat, threads, 5)
    out["lattice17x17"] = {"updates_per_sweep": U2, "value_1core": a1, "value_allcores": an}
    log(f"oracle 17x17: {a1:.3e} updates/s on 1 thread, {an:.3e} on {threads}")
    pin = P.config(1)
    o = O.Oracle.from_problem(pin)
    t0 = time.perf_counter()
    r = o.solve(tol=1e-6)
    out["pincell_time_to_1e-6_s"] = time.perf_counter() - t0
    out["pincell_iterations"] = r["iterations"]
    if full:
        hx = P.config(4)
        h1, U4, _ = _oracle_rate(hx, 1, 1)
        hn, _, _ = _oracle_rate(hx, threads, 3)
        out["hexagon_g33"] = {"updates_per_sweep": U4, "value_1core": h1, "value_allcores": hn}
        log(f"oracle hexagon: {h1:.3e} updates/s on 1 thread, {hn:.3e} on {threads}")
        o2 = O.Oracle.from_problem(lat, threads=threads)
        o2.set_threads(threads)
        # in chunks of 100 iterations, each continuing from the last (the oracle keeps its
        # boundary fluxes), so the run reports its progress as it goes
        t0 = time.perf_counter()
        phi, k, its = None, 1.0, 0
        while True:
            r2 = o2.solve(tol=1e-6, max_iter=100, phi0=phi, k0=k)
            phi, k, its = r2["phi"], r2["k"], its + r2["iterations"]
            log(f"oracle 17x17: {its} iterations, residual {r2['residual']:.2e}, {time.perf_counter() - t0:.0f} s")
            if r2["converged"] or its >= 20000:
                break
        out["lattice17x17_time_to_1e-6_s"] = time.perf_counter() - t0
        out["lattice17x17_iterations"] = its
        log(f"oracle 17x17 to 1e-6: {out['lattice17x17_time_to_1e-6_s']:.1f} s, {its} iterations")
        del o2
        big = P.config(3)
        o3 = O.Oracle.from_problem(big, threads=threads)
        o3.set_threads(threads)
        import numpy as np
        src = np.ones((o3.R, o3.G))
        t0 = time.perf_counter()
        o3.sweep(src)
        dt = time.perf_counter() - t0
        out["lattice51x51"] = {"updates_per_sweep": 2 * o3.P * o3.G * o3.S, "value_allcores": 2 * o3.P * o3.G * o3.S / dt,
                               "sweep_s": dt}
        log(f"oracle 51x51: one sweep {dt:.1f} s on {threads} threads")
    return out


def dg_leg(args):
    """DGMOC on the extruded 17 x 17 workload: FP32 (and FP64) iteration and sweep times."""
    import torch
    from paper_2607_01591_amd import dgmoc
    from paper_2607_01591_amd import problems as P
    ext = P.config_3d(6)
    out = {"workload": f"{ext.name}: {ext.base.n_regions} regions x {ext.n_planes} planes, "
                       f"{ext.base.n_groups} groups, A={ext.base.n_azim} x P={ext.base.n_polar} per hemisphere, "
                       f"spacing {ext.base.spacing} cm, linear axial DG; bottom reflective, top vacuum"}
    for prec in ("f32",) if args.no_f64 else ("f32", "f64"):
        log(f"DGMOC {prec}: creating context")
        s = dgmoc.DGSolver(ext, precision=prec, check_every=1 << 30)
        steps = args.dg_steps if prec == "f32" else max(2, args.dg_steps // 2)
        ms, prof, r = time_iterations(s, steps, 1)
        sw = prof["sweep_ms"] / max(1, prof["sweeps"])
        out[prec] = {"updates_per_sweep": s.U, "updates_per_s": s.U / (ms * 1e-3), "ms_per_iteration": ms,
                     "sweep_ms": sw, "device_GiB": s.info["device_bytes"] / 2**30, "k_after": r["k"]}
        if prec == "f32":
            ach = s.U * DG_FLOPS_PER_UPDATE / (sw * 1e-3) / 1e12
            out["roofline"] = {"bound": "alu", "achieved": ach, "peak": FP32_NONPACKED_TFLOPS, "unit": "TFLOP/s",
                               "frac": ach / FP32_NONPACKED_TFLOPS, "flops_per_update": DG_FLOPS_PER_UPDATE,
                               "note": "whole sweep (driven-flux and plane-sweep kernels) from HIP events"}
        log(f"DGMOC {prec}: {ms:.2f} ms/iteration, sweep {sw:.2f} ms, {s.U / (ms * 1e-3):.3e} updates/s")
        del s
        torch.cuda.empty_cache()
    return out


def sn_leg(args):
    """DFEM-SN on the 17 x 17 lattice mesh: sweep time and local solves per second, level by
    level and tile by tile (pin-cell tiles)."""
    import torch
    from paper_2607_01591_amd import dfem
    from paper_2607_01591_amd import problems as P
    prob = P.config(2)
    out = {"workload": f"{prob.name}: {len(prob.tri)} triangles (linear elements), {prob.n_groups} groups, "
                       f"{prob.n_azim} azimuths x {prob.n_polar} polar = {prob.n_azim * prob.n_polar} directions, reflective"}
    n_tiles, tile = P.grid_tiles(prob, 17, 17)
    out["tiles"] = f"{n_tiles} pin cells"
    for prec in ("f32",) if args.no_f64 else ("f32", "f64"):
        log(f"DFEM-SN {prec}: creating context")
        s = dfem.SNSolver(prob, precision=prec, check_every=1 << 30)
        n_solves = s.info["n_tasks"] * prob.n_groups
        # level by level (one dependent launch per level: bound by the per-level latency)
        ms, prof, r = time_iterations(s, 5, 1)
        sw = prof["sweep_ms"] / max(1, prof["sweeps"])
        lev = {"ms_per_iteration": ms, "sweep_ms": sw, "levels": s.info["n_levels"], "bound": "latency",
               "us_per_level": sw * 1e3 / max(1, s.info["n_levels"]), "slots": s.info["n_slots"]}
        log(f"DFEM-SN {prec}, level by level: {ms:.2f} ms/iteration, sweep {sw:.2f} ms, "
            f"{n_solves / (sw * 1e-3):.3e} solves/s, {s.info['n_levels']} levels, {s.info['n_slots']} slots")
        # tile by tile (pin cells): one launch per tile level
        s.set_tiles(tile)
        ms_t, prof_t, r_t = time_iterations(s, 5, 1)
        sw_t = prof_t["sweep_ms"] / max(1, prof_t["sweeps"])
        inf = s.info
        out[prec] = {"local_solves_per_sweep": n_solves, "solves_per_s": n_solves / (sw_t * 1e-3),
                     "ms_per_iteration": ms_t, "sweep_ms": sw_t, "schedule": "tiles",
                     "tile_levels": inf["n_tile_levels"], "max_inner_levels": inf["max_inner_levels"],
                     "tile_lds_bytes": inf["tile_lds_bytes"], "tile_slots": inf["n_tile_slots"],
                     "bound": "latency", "levels_schedule": lev, "tasks": inf["n_tasks"],
                     "device_GiB": inf["device_bytes"] / 2**30, "k_after": r_t["k"]}
        log(f"DFEM-SN {prec}, pin-cell tiles: {ms_t:.2f} ms/iteration, sweep {sw_t:.2f} ms, "
            f"{n_solves / (sw_t * 1e-3):.3e} solves/s, {inf['n_tile_levels']} tile levels, "
            f"{inf['tile_lds_bytes']} B of LDS per block")
        del s
        torch.cuda.empty_cache()
    # time to a 1e-6 residual, tile by tile, FP32 (convergence checked every 10 iterations)
    s = dfem.SNSolver(prob, precision="f32", max_iter=20000, check_every=10)
    s.set_tiles(tile)
    s.run_iterations(1)
    r = s.solve(1e-6)
    out["f32_solve"] = {"tol": 1e-6, "converged": r["converged"], "iterations": r["iterations"],
                        "wall_ms": r["wall_ms"], "k": r["k"]}
    log(f"DFEM-SN f32 tiles, solve to 1e-6: k = {r['k']:.6f}, {r['iterations']} iterations, {r['wall_ms']:.0f} ms")
    del s
    torch.cuda.empty_cache()
    return out


def cnn_leg(args):
    """Warm-start network on the matrix cores: BF16 forward of the 7-layer dilated network
    on a batch of 128 x 128 lattice images (FP32 accumulation) and one training step
    (forward, input and weight gradients, Adam), against the dense BF16 MFMA peak."""
    import torch
    from paper_2607_01591_amd import cnn
    from paper_2607_01591_amd.warmstart import C_IN, CHANNELS, DILATIONS, IMG
    dev = torch.device("cuda:0")
    N = 8
    net = cnn.ConvNet(CHANNELS, dev, seed=0, in_used=C_IN, out_used=7, dilations=DILATIONS)
    g = torch.Generator(device="cpu").manual_seed(0)
    x = torch.randn((N, IMG, IMG, CHANNELS[0]), generator=g).to(dev).to(torch.bfloat16)
    t = torch.randn((N, IMG, IMG, CHANNELS[-1]), generator=g).to(dev)
    flops_fwd = sum(2 * 9 * ci * co * N * IMG * IMG for ci, co in zip(CHANNELS[:-1], CHANNELS[1:]))
    for _ in range(3):
        net.forward(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    e0.record()
    for _ in range(reps):
        net.forward(x)
    e1.record()
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1) / reps
    for _ in range(2):
        net.train_step(x, t, 7, lr=1e-4)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        net.train_step(x, t, 7, lr=1e-4)
    e1.record()
    torch.cuda.synchronize()
    step_ms = e0.elapsed_time(e1) / reps
    # a training step: forward, input gradient of every layer but the first, weight gradient
    flops_step = flops_fwd + 2 * flops_fwd - 2 * 9 * CHANNELS[0] * CHANNELS[1] * N * IMG * IMG
    peak = 2500.0
    out = {"workload": f"{len(CHANNELS) - 1}-layer 3x3 network {CHANNELS}, dilations {DILATIONS}, batch {N} x "
                       f"{IMG} x {IMG}, BF16 operands, FP32 accumulation",
           "forward_ms": fwd_ms, "forward_TFLOPs": flops_fwd / (fwd_ms * 1e-3) / 1e12,
           "train_step_ms": step_ms, "train_step_TFLOPs": flops_step / (step_ms * 1e-3) / 1e12,
           "roofline": {"bound": "mfma", "unit": "TFLOP/s", "peak": peak,
                        "achieved": flops_fwd / (fwd_ms * 1e-3) / 1e12,
                        "frac": flops_fwd / (fwd_ms * 1e-3) / 1e12 / peak, "kernel": "k_conv_fwd (whole forward)"}}
    log(f"CNN: forward {fwd_ms:.3f} ms ({out['forward_TFLOPs']:.1f} TFLOP/s), training step {step_ms:.3f} ms "
        f"({out['train_step_TFLOPs']:.1f} TFLOP/s)")
    return out


def copy_probe():
    """Two plain 1 GiB device-to-device copies: their HBM counters calibrate the scale of
    the counters of the kernels measured in the same run."""
    import torch
    src_c = torch.ones(1 << 28, dtype=torch.float32, device="cuda")     # 1 GiB
    dst_c = torch.empty_like(src_c)
    for _ in range(2):
        dst_c.copy_(src_c)
    torch.cuda.synchronize()
    log("copy probe: 2 x 1 GiB device-to-device copies")
    del src_c, dst_c


def hfem_leg(args):
    """Diffusion HFEM on the 51 x 51 x 32 pin-cell core (7 groups, volume order 2, face
    order 1): device preassembly time, red-black sweep time against the HBM roofline, and
    the eigenvalue solve to 1e-6."""
    import torch
    from paper_2607_01591_amd import hfem
    from paper_2607_01591_amd import problems as P
    g = P.brick_core()
    log("HFEM: creating context (host checks, uploads, device preassembly)")
    s = hfem.HFEMSolver(g, volume_order=2, face_order=1, inner_iterations=2, check_every=1 << 30)
    inf = s.info
    N, G, Np, Nft = inf["n_nodes"], inf["n_groups"], inf["n_moments"], inf["n_face_dofs"]
    ms, prof, r = time_iterations(s, 20, 2)
    rb_ms = prof["sweep_ms"] / max(1, prof["sweeps"])
    # per node-group and red-black iteration: R once, B s once, the gathered J- and the
    # written J+ (FP64)
    per_pg = 8 * (Nft * Nft + 3 * Nft)
    alg = N * G * per_pg
    gbs = alg / (rb_ms * 1e-3) / 1e9
    out = {"workload": f"{g.name}: {N} pin-cell nodes ({len(g.edges[0]) - 1} x {len(g.edges[1]) - 1} x "
                       f"{len(g.edges[2]) - 1}), {G} groups, volume order 2 ({Np} moments), face order 1 "
                       f"({Nft} face DoFs), per-node cross sections, 2 red-black iterations per outer iteration",
           "setup_ms": inf["setup_ms"], "assemble_ms": inf["assemble_ms"], "device_GiB": inf["device_bytes"] / 2**30,
           "ms_per_iteration": ms, "rb_iteration_ms": rb_ms, "dof_updates_per_s": N * G * Nft / (rb_ms * 1e-3),
           "roofline": {"bound": "hbm", "kernel": "moc::k_hf_rb", "algorithmic_bytes": alg, "bytes_per_node_group": per_pg,
                        "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}}
    log(f"HFEM: preassembly {inf['assemble_ms']:.1f} ms, {ms:.3f} ms/iteration, red-black iteration {rb_ms:.3f} ms "
        f"= {gbs:.0f} GB/s ({gbs / HBM_PEAK_GBS:.2f} of HBM peak)")
    del s
    torch.cuda.empty_cache()
    # the same with R and A^-1 stored in FP32 (half the bytes of the sweep)
    s = hfem.HFEMSolver(g, volume_order=2, face_order=1, inner_iterations=2, check_every=1 << 30, fp32_matrices=True)
    ms32, prof32, _ = time_iterations(s, 20, 2)
    rb32 = prof32["sweep_ms"] / max(1, prof32["sweeps"])
    per_pg32 = 4 * Nft * Nft + 8 * 3 * Nft
    out["fp32_matrices"] = {"ms_per_iteration": ms32, "rb_iteration_ms": rb32, "bytes_per_node_group": per_pg32,
                            "achieved_GBs": N * G * per_pg32 / (rb32 * 1e-3) / 1e9,
                            "dof_updates_per_s": N * G * Nft / (rb32 * 1e-3)}
    log(f"HFEM, FP32 matrices: {ms32:.3f} ms/iteration, red-black iteration {rb32:.3f} ms")
    del s
    torch.cuda.empty_cache()
    s = hfem.HFEMSolver(g, volume_order=2, face_order=1, inner_iterations=2, max_iter=args.hfem_max_iter,
                        check_every=10)
    r = s.solve(1e-6)
    out["solve"] = {"tol": 1e-6, "k": r["k"], "iterations": r["iterations"], "converged": r["converged"],
                    "wall_ms": r["wall_ms"]}
    log(f"HFEM: solve to 1e-6: k = {r['k']:.6f}, {r['iterations']} iterations, {r['wall_ms']:.0f} ms, "
        f"converged {r['converged']}")
    del s
    torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); sharding by azimuthal "
              "angle across GPUs is designed but not built", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2607_01591_amd import moc
    from paper_2607_01591_amd import problems as P

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.dg_only:
        print(json.dumps({"dgmoc": dg_leg(args)}), flush=True)
        return
    if args.sn_only:
        print(json.dumps({"dfem_sn": sn_leg(args)}), flush=True)
        return
    if args.cnn_only:
        print(json.dumps({"cnn": cnn_leg(args)}), flush=True)
        return
    if args.hfem_only:
        hf = hfem_leg(args)
        if args.copy_probe:
            copy_probe()
        print(json.dumps({"hfem": hf}), flush=True)
        return
    log(f"generating workload {args.workload}")
    prob = P.config(args.workload)
    log("creating FP32 context (host tracking + upload)")
    s32 = moc.Solver(prob, precision="f32", exp_mode=args.exp_mode, check_every=1 << 30)
    info = s32.info
    log(f"R={info['n_regions']} T={info['n_tracks']} S={info['n_segments']} U={info['n_updates']} "
        f"setup {info['setup_ms']:.0f} ms, device {info['device_bytes'] / 2**30:.2f} GiB")
    ms, prof, r = time_iterations(s32, args.steps, args.warmup)
    U = info["n_updates"]
    if args.copy_probe:
        copy_probe()
    sweep_ms = prof["sweep_ms"] / max(1, prof["sweeps"])
    log(f"FP32: {ms:.3f} ms/iteration, sweep kernel {sweep_ms:.3f} ms avg over {prof['sweeps']}, "
        f"k={r['k']:.6f}")
    value = U / (ms * 1e-3)
    achieved = U * FLOPS_PER_UPDATE / (sweep_ms * 1e-3) / 1e12
    traffic, traffic_src = measured_traffic()
    roofline = {"bound": "alu", "achieved": achieved, "peak": FP32_NONPACKED_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / FP32_NONPACKED_TFLOPS, "traffic": traffic,
                "traffic_source": traffic_src, "kernel": "moc::k_sweep<float, 3, 7, 0, false>", "kernel_ms": sweep_ms,
                "flops_per_update": FLOPS_PER_UPDATE, "updates_per_launch": U}
    alg_bytes = algorithmic_bytes(info, "f32")
    hbm = {"algorithmic_bytes": alg_bytes, "achieved_GBs": alg_bytes / (sweep_ms * 1e-3) / 1e9,
           "frac_of_8TBs": alg_bytes / (sweep_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    if traffic is not None:
        hbm["measured_GBs"] = traffic / (sweep_ms * 1e-3) / 1e9
    del s32
    torch.cuda.empty_cache()

    fp64 = None
    if not args.no_f64:
        log("creating FP64 context")
        s64 = moc.Solver(prob, precision="f64", check_every=1 << 30)
        ms64, prof64, r64 = time_iterations(s64, max(3, args.steps // 4), 1)
        sw64 = prof64["sweep_ms"] / max(1, prof64["sweeps"])
        fp64 = {"updates_per_s": U / (ms64 * 1e-3), "ms_per_step": ms64, "sweep_kernel_ms": sw64}
        log(f"FP64: {ms64:.3f} ms/iteration, sweep kernel {sw64:.3f} ms")
        del s64
        torch.cuda.empty_cache()

    hexa = None
    if not args.no_hex:
        log("hexagonal assembly (33 groups): FP32 sweep throughput")
        ph = P.config(4)
        sh = moc.Solver(ph, precision="f32", check_every=1 << 30)
        msh, profh, _ = time_iterations(sh, 5, 1)
        swh = profh["sweep_ms"] / max(1, profh["sweeps"])
        hexa = {"workload": f"{ph.name}: {sh.R} regions, 33 groups", "updates_per_sweep": sh.U,
                "updates_per_s": sh.U / (msh * 1e-3), "ms_per_step": msh, "sweep_kernel_ms": swh}
        log(f"hexagon: {msh:.3f} ms/iteration, sweep {swh:.3f} ms, {sh.U / (msh * 1e-3):.3e} updates/s")
        del sh
        torch.cuda.empty_cache()

    cmfd3 = None
    if not args.no_cmfd:
        log("51x51 lattice: time to a 1e-6 residual with CMFD on the 51 x 51 pin cells (cold start)")
        s3 = moc.Solver(prob, precision="f32", max_iter=2000, check_every=1)
        n_cells, region_cell = P.coarse_cells(prob, 51, 51)
        s3.set_coarse_mesh(n_cells, region_cell)
        s3.run_iterations(1)     # first-use costs (code objects) outside the timing
        s3.set_profiling(True)
        r3 = s3.solve(1e-6)
        pr3 = s3.profile()
        s3.set_profiling(False)
        ci = s3.coarse_info()
        cmfd3 = {"workload": f"{prob.name}, FP32 sweep, CMFD on {n_cells} pin cells, residual 1e-6",
                 "converged": r3["converged"], "iterations": r3["iterations"], "wall_ms": r3["wall_ms"],
                 "ms_per_iteration": r3["wall_ms"] / max(1, r3["iterations"]), "k": r3["k"],
                 "sweep_ms_avg": pr3["sweep_ms"] / max(1, pr3["sweeps"]),
                 "cmfd_step_ms_avg": pr3["cmfd_ms"] / max(1, pr3["cmfd_steps"]),
                 "coarse_surfaces": ci["n_surfaces"], "crossing_entries": ci["n_crossings"],
                 "last_coarse_outer": ci["last_outer"], "last_coarse_inner": ci["last_inner"]}
        log(f"CMFD 51x51: {cmfd3}")
        del s3
        torch.cuda.empty_cache()

    solve = None
    if not args.no_solve:
        import numpy as np
        weights = os.path.join(ROOT, "paper_2607_01591_amd", "weights", "warmstart_17x17.npz")
        log("time to 1e-6 on 17x17 lattices (held-out seeds): cold, CMFD, warm start, warm start + CMFD")
        base = P.config(5, seed=100000)
        s5 = moc.Solver(base, precision="f32", max_iter=20000, check_every=10)
        n5, rc5 = P.coarse_cells(base, 17, 17)
        ws = None
        if os.path.exists(weights):
            from paper_2607_01591_amd.warmstart import WarmStart, load_net
            dev0 = torch.device("cuda:0")
            ws = WarmStart(s5, base, dev0, net=load_net(weights, dev0, base.n_groups))
        from paper_2607_01591_amd.warmstart import homogenized_guess
        V5 = s5.volumes()
        s5.run_iterations(1)     # first-use costs (code objects) outside the timed solves
        rows = []
        for sd in range(200000, 200000 + args.solve_seeds):
            p5 = P.config(5, seed=sd)
            s5.set_coarse_mesh(0)
            s5.set_materials(p5)
            c = s5.solve(1e-6)
            row = {"seed": sd, "cold_iterations": c["iterations"], "cold_ms": c["wall_ms"]}
            s5.set_initial_guess(homogenized_guess(p5, V5, torch.device("cuda:0")), -1.0)
            h = s5.solve(1e-6)
            row.update(nonlearned_sweeps=h["sweeps"], nonlearned_ms=h["wall_ms"])
            if ws is not None:
                w = ws.solve_warm(p5, 1e-6)
                row.update(warm_sweeps=w["sweeps"], warm_iterations=w["iterations"], warm_ms=w["total_ms"],
                           warm_predict_ms=w["predict_ms"], warm_converged=w["converged"],
                           warm_fell_back=bool(w["flags"] & moc.FLAG_FELL_BACK_TO_COLD))
            if not args.no_cmfd:
                s5.set_coarse_mesh(n5, rc5)
                cm = s5.solve(1e-6)
                row.update(cmfd_iterations=cm["iterations"], cmfd_ms=cm["wall_ms"])
                if ws is not None:
                    wc = ws.solve_warm(p5, 1e-6)
                    row.update(warm_cmfd_sweeps=wc["sweeps"], warm_cmfd_ms=wc["total_ms"])
            rows.append(row)
            log(f"seed {sd}: {row}")
        def stat(k):
            if not rows or k not in rows[0]:
                return None
            v = np.array([r[k] for r in rows], float)
            return {"median": float(np.median(v)), "q1": float(np.percentile(v, 25)),
                    "q3": float(np.percentile(v, 75)), "total": float(v.sum())}
        solve = {"workload": f"17x17 lattice family (31k regions), FP32 sweep, residual 1e-6, "
                             f"{len(rows)} held-out seeds from 200000; median, quartiles and total",
                 "cold_iterations": stat("cold_iterations"), "cold_ms": stat("cold_ms"),
                 "nonlearned_sweeps": stat("nonlearned_sweeps"), "nonlearned_ms": stat("nonlearned_ms"),
                 "warm_sweeps": stat("warm_sweeps"), "warm_ms": stat("warm_ms"),
                 "cmfd_iterations": stat("cmfd_iterations"), "cmfd_ms": stat("cmfd_ms"),
                 "warm_cmfd_sweeps": stat("warm_cmfd_sweeps"), "warm_cmfd_ms": stat("warm_cmfd_ms"),
                 "runs": rows}

    dg = None
    if not args.no_dg:
        dg = dg_leg(args)

    sn = None
    if not args.no_sn:
        sn = sn_leg(args)

    hf = None
    if not args.no_hfem:
        hf = hfem_leg(args)

    cn = None
    if not args.no_cnn:
        cn = cnn_leg(args)

    cpu = None
    if not args.no_cpu:
        log("timing the FP64 CPU oracle on a bounded sample")
        cpu = cpu_baseline(args.workload, full=args.cpu_full)
        log(f"oracle: {cpu['value']:.3e} updates/s on {cpu['cores']} threads")

    out = {
        "metric": "segment-group updates/s (FP32 sweep power iteration)",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{prob.name}: {info['n_regions']} regions, {info['n_groups']} groups, "
                               f"A={prob.n_azim} x P={prob.n_polar}, spacing {prob.spacing} cm",
                   "regions": info["n_regions"], "groups": info["n_groups"], "tracks": info["n_tracks"],
                   "segments": info["n_segments"], "updates_per_sweep": U},
        "roofline": roofline,
        "hbm_view": hbm,
        "fp64": fp64,
        "time_to_tol": solve,
        "cmfd_51x51": cmfd3,
        "hexagon_g33": hexa,
        "dgmoc_3d": dg,
        "dfem_sn": sn,
        "hfem": hf,
        "cnn": cn,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
