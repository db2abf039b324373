"""Throughput of the coupled LBM + IB step on one MI355X, and iterations to steady state.

A step is one pass of the whole hot path (lattice pass with force spreading and velocity
interpolation, membrane advection / forces / source map, per-tile node lists) over the
2048 x 2048 lattice with 2000 Voronoi cells.  The second half of the metric counts the
iterations the species lattice alone needs to reach steady state on held-out 256 x 256
static-tissue samples.  Prints one JSON line (rank 0).

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload large|tissue|tiny]
                  [--storage fp32|fp16|bf16] [--ade-samples N] [--sweep-sims N] [--sweep-steps K]
                  [--no-cpu-baseline]

The batched sweep (64 uneven simulations in one batch, against the same simulations run one
after another) is reported beside the headline number.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "coupled LBM+IB MLUPS at 2048²/2000 cells (% HBM peak); ADE iters-to-steady"
HBM_PEAK_GBS = 8000.0
GOLD = os.path.join(ROOT, "tests", "golden")
# HBM bytes one launch of the lattice pass moves at the large workload in FP32, from two
# rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE, each scaled by what the counter reads for a
# copy of known size; profiles/k_lattice_large_2048x2048_2000cells_fp32_hbm_bytes.md), with the
# SHA-256 of the kernel's sources when they were taken: reported only while the sources match.
LATTICE_TRAFFIC = {"bytes": 524912684,
                   "sources_sha256": "0b8c4622d26274e08557f17ca46256e296260b8f4a8709b4bdbf4e2f6014c83a"}
LATTICE_SOURCES = ("paper_1503_06726_amd/csrc/k_lattice.hip", "paper_1503_06726_amd/csrc/lbib_device.h")


def lattice_sources_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in LATTICE_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


POP_BYTES = {"fp32": 4, "fp16": 2, "bf16": 2}


def lattice_bytes_per_update(S: int, mask: bool, pop_bytes: int = 4) -> float:
    """Algorithmic bytes per lattice node of one lattice pass: every population read once and
    written once, plus the node's inside-any-cell bit read when a source term needs it."""
    return pop_bytes * 2 * (9 + 5 * S) + (0.125 if mask else 0.0)


def step_bytes_per_update(S: int, mask: bool, n_nodes: int, nn: int, pop_bytes: int = 4) -> float:
    """Algorithmic bytes per lattice node of a whole step: the lattice pass plus the node
    positions read and written (16 B per node, FP64 x and y)."""
    return lattice_bytes_per_update(S, mask, pop_bytes) + 16.0 * n_nodes / nn


ADE_TOL = 1e-6
ADE_CAP = 1_000_000


def ade_samples(n: int):
    """The held-out static-tissue samples (generated on the host in a process pool, before the
    GPU is touched)."""
    from paper_1503_06726_amd import warmstart as WS
    if n <= 0:
        return []
    return WS.generate(range(n), held_out=True, workers=min(8, os.cpu_count() or 1))


def ade_half(samples, lbib, stream):
    """Iterations to steady state of the species alone (u = 0, frozen membranes), in FP64,
    stopping at ||phi^k - phi^{k-1}|| <= 1e-6 ||phi^k||: from zero, and from the trained
    surrogate's prediction."""
    import numpy as np
    from paper_1503_06726_amd import warmstart as WS
    src, _, feat = WS.prepare(samples, stream)
    t0 = time.perf_counter()
    k0, phi_z = WS.solve(samples, src, tol=ADE_TOL, max_iters=ADE_CAP, stream=stream)
    t_zero = time.perf_counter() - t0
    params, meta = WS.load()
    net = lbib.Net(samples[0].ny, samples[0].nx, 16, stream=stream)
    net.set_params(params)
    t0 = time.perf_counter()
    phi_hat = WS.predict(net, feat, samples)
    t_pred = time.perf_counter() - t0
    net.close()
    t0 = time.perf_counter()
    kw, phi_w = WS.solve(samples, src, phi0=phi_hat, tol=ADE_TOL, max_iters=ADE_CAP, stream=stream)
    t_warm = time.perf_counter() - t0

    def stats(k):
        kk = np.where(k > 0, k, ADE_CAP)
        return {"median_iters": float(np.median(kk)), "mean_iters": round(float(kk.mean()), 1),
                "unconverged": int((k == 0).sum())}
    z, wm = stats(k0), stats(kw)
    true_err = ade_true_error(samples, phi_zero=phi_z, phi_warm=phi_w)
    return {"workload": "static tissue 256x256 walls-y, 50-300 Voronoi cells, seeded source cells, "
                        "D ~ U(0.02, 0.5), decay ~ U(1e-5, 1e-3), source 1e-3; held-out seeds",
            "samples": len(samples), "tol": ADE_TOL, "cap": ADE_CAP, "precision": "f64",
            "zero_start": z, "warm_start": wm,
            "speedup_median": round(z["median_iters"] / wm["median_iters"], 3),
            "speedup_mean": round(z["mean_iters"] / wm["mean_iters"], 3),
            "seconds": {"zero_start_solves": round(t_zero, 2), "prediction": round(t_pred, 3),
                        "warm_start_solves": round(t_warm, 2)},
            "net": f"BF16 U-Net, {meta['samples']} training samples, {meta['epochs']} epochs",
            "true_error": true_err}


def ade_true_error(samples, phi_zero, phi_warm):
    """Relative L2 distance of the iterated steady states from the fixed points a sparse direct
    solve of the D2Q5 equations gives (stored for the first held-out samples by
    tests/golden/make_ade_goldens.py), against the asymptotic size tol / lambda of the error
    the stopping rule leaves (slow modes decay by about 1 - lambda per iteration)."""
    import numpy as np
    path = os.path.join(GOLD, "ade_fixed_points.npz")
    if not os.path.exists(path):
        return None
    g = np.load(path)
    n = min(int(g["samples"]), len(samples))
    rows = []
    for i in range(n):
        ref = g[f"phi_{i}"].astype(np.float64)
        bound = ADE_TOL / float(g[f"decay_{i}"])
        ez = float(np.linalg.norm(phi_zero[i] - ref) / np.linalg.norm(ref))
        ew = float(np.linalg.norm(phi_warm[i] - ref) / np.linalg.norm(ref))
        rows.append((ez, ew, ez / bound, ew / bound))
    a = np.array(rows)
    return {"samples": n, "reference": "sparse direct solve of the D2Q5 fixed point (FP64)",
            "zero_start_rel_l2": {"median": float(np.median(a[:, 0])), "max": float(a[:, 0].max())},
            "warm_start_rel_l2": {"median": float(np.median(a[:, 1])), "max": float(a[:, 1].max())},
            "max_error_over_tol_per_decay": {"zero_start": float(a[:, 2].max()), "warm_start": float(a[:, 3].max())}}


def sweep_workloads(n: int):
    """The sweep's simulations (host geometry, in a process pool before the GPU is touched)."""
    import concurrent.futures as cf
    from paper_1503_06726_amd import workloads as W
    if n <= 0:
        return []
    with cf.ProcessPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        return list(ex.map(W.sweep_member, range(n)))


def sweep_half(ws, steps: int, lbib, stream):
    """Batched parameter sweep: every simulation advanced `steps` steps by one batch (tile
    height autotuned, whole 16-step periods replayed from one graph), against the same
    simulations stepped one after another with lbib_step.  Total MLUPS of both."""
    import numpy as np
    import torch
    steps = max(16, steps - steps % 16)
    A = [lbib.from_workload(w, stream=stream) for w in ws]
    B = [lbib.from_workload(w, stream=stream) for w in ws]
    nn = sum(w.nx * w.ny for w in ws)
    for s in A:                                     # warm-up: one period each (captures graphs)
        s.step(16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in A:
        s.step(steps)
    for s in A:
        s.sync()
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    log(f"sweep: sequential {steps} steps of {len(ws)} simulations: {t_seq:.3f} s")
    batch = lbib.Batch(B, stream=stream)
    rows, groups, tune = batch.autotune(periods=4)
    log(f"sweep: autotuned tile height {rows} rows, {groups} groups; ms per step {tune}")
    batch.step(16)
    batch.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.step(steps)
    batch.sync()
    torch.cuda.synchronize()
    t_bat = time.perf_counter() - t0
    log(f"sweep: batched {steps} steps: {t_bat:.3f} s")
    # both sets have now taken 16 + steps steps; at the default tile height they agree bit for bit
    same = None
    if rows == 8:                          # (either grouping)
        i = int(np.argmin([w.nx * w.ny for w in ws]))
        fa, fb = A[i].get_fields(mask=False), B[i].get_fields(mask=False)
        same = all(np.array_equal(fa[k], fb[k]) for k in ("rho", "u", "phi", "xy"))
    batch.close()
    for s in A + B:
        s.close()
    bat = nn * steps / t_bat / 1e6
    seq = nn * steps / t_seq / 1e6
    b_up = lattice_bytes_per_update(1, True)
    return {"workload": f"{len(ws)} simulations, nx and ny log-uniform in [128, 1024], walls-y, "
                        "min(U{10..500}, nx ny / 100) Voronoi cells, tau ~ U(0.55, 1.2), k ~ U(0.005, 0.05), "
                        "body 1e-6 x, 1 D2Q5 species (source/decay)",
            "sims": len(ws), "lattice_nodes": nn, "membrane_nodes": int(sum(w.n_nodes for w in ws)),
            "cells": int(sum(w.n_cells for w in ws)), "steps": steps, "storage": "fp32",
            "batched_mlups": round(bat, 1), "sequential_mlups": round(seq, 1), "speedup": round(bat / seq, 3),
            "batched_ms_per_step": round(t_bat / steps * 1e3, 4),
            "sequential_ms_per_step": round(t_seq / steps * 1e3, 4),
            "batched_lattice_bytes_frac_of_hbm": round(b_up * bat * 1e6 / 1e9 / HBM_PEAK_GBS, 4),
            "tile_rows": rows, "groups": groups,
            "autotune_ms_per_step": {f"{g} groups, {h} rows": round(v, 4) for (g, h), v in tune.items()},
            "smallest_member_bit_identical": same}


def storage_half(w, ref, warmup: int, steps: int, kt_steps: int, mlups32: float, lbib, stream):
    """The same run with FP16 and BF16 population storage (collision in FP32): MLUPS, the
    lattice kernel's time, and the relative L2 distance of each field from the FP32 run after
    the same steps (ref: the FP32 run's fields)."""
    import numpy as np
    import torch
    out = {}
    nn = w.nx * w.ny

    def rel(a, b):
        nb = float(np.linalg.norm(b))
        return float(np.linalg.norm(np.asarray(a) - np.asarray(b))) / (nb if nb > 0 else 1.0)
    for name, st in (("fp16", lbib.STORAGE_FP16), ("bf16", lbib.STORAGE_BF16)):
        sim = lbib.from_workload(w, stream=stream, storage=st)
        sim.step(warmup)
        sim.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        sim.sync()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        sim.set_timing(True)
        sim.step(kt_steps)
        ms, n = sim.get_timing(lbib.K_LATTICE)
        sim.set_timing(False)
        F = sim.get_fields(mask=False)
        sim.close()
        mlups = nn * steps / dt / 1e6
        b_lat = lattice_bytes_per_update(w.n_species, w.mask_needed(), 2)
        out[name] = {"value": round(mlups, 1), "speedup_vs_fp32": round(mlups / mlups32, 3),
                     "lattice_us": round(ms / n * 1e3, 2),
                     "lattice_frac_of_hbm": round(b_lat * nn / (ms / n / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                     "rel_l2_vs_fp32": {"rho-rho0": rel(F["rho"] - w.rho0, ref["rho"] - w.rho0), "u": rel(F["u"], ref["u"]),
                                        "phi": rel(F["phi"], ref["phi"]), "X-X0": rel(F["xy"] - w.xy, ref["xy"] - w.xy)}}
        log(f"storage {name}: {out[name]}")
    out["steps_compared"] = warmup + steps + kt_steps
    return out


# the surrogate network's convolutions (input, output channels and resolution divisor of the 15
# layers; the first layer's eight feature channels as the network defines them)
NET_CIN = (8, 32, 32, 64, 64, 128, 128, 256, 256, 128, 128, 64, 64, 32, 32)
NET_COUT = (32, 32, 64, 64, 128, 128, 256, 256, 128, 128, 64, 64, 32, 32, 16)
NET_DIV = (1, 1, 2, 2, 4, 4, 8, 8, 4, 4, 2, 2, 1, 1, 1)
BF16_PEAK_TFLOPS = 2500.0


def net_flops(h: int, w: int, batch: int):
    """(forward, training step) FLOPs of the 3x3 convolutions: 2 x 9 Cin Cout per output
    pixel; a training step is the forward pass, the data gradient of every layer but the first
    and the weight gradient of every layer."""
    f = [2 * 9 * ci * co * (h // d) * (w // d) for ci, co, d in zip(NET_CIN, NET_COUT, NET_DIV)]
    return batch * sum(f), batch * (3 * sum(f) - f[0])


def net_half(lbib, stream, h: int = 256, w: int = 256, batch: int = 16, steps: int = 20):
    """Training steps and predictions of the warm-start network at the warm-start workload's
    size (256 x 256, batch 16), random weights and inputs."""
    import numpy as np
    import torch
    net = lbib.Net(h, w, batch, stream=stream)
    rng = np.random.default_rng(1503)
    net.set_params((0.05 * rng.standard_normal(net.n_params)).astype(np.float32))
    x = torch.tensor(rng.random((batch, h, w, 8)), dtype=torch.float32, device="cuda")
    y = torch.tensor(rng.random((batch, h, w)), dtype=torch.float32, device="cuda")
    out = torch.empty((batch, h, w), dtype=torch.float32, device="cuda")
    for _ in range(3):
        net.train_step(x.data_ptr(), y.data_ptr(), batch, 1e-4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        net.train_step(x.data_ptr(), y.data_ptr(), batch, 1e-4)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    t0 = time.perf_counter()
    for _ in range(steps):
        net.predict(x.data_ptr(), batch, out.data_ptr())
    torch.cuda.synchronize()
    dp = (time.perf_counter() - t0) / steps
    net.close()
    fw, tr = net_flops(h, w, batch)
    return {"shape": f"{batch} x {h} x {w}", "train_step_ms": round(dt * 1e3, 3),
            "train_TFLOPs": round(tr / dt / 1e12, 1), "train_frac_bf16_peak": round(tr / dt / 1e12 / BF16_PEAK_TFLOPS, 4),
            "predict_ms": round(dp * 1e3, 3), "predict_TFLOPs": round(fw / dp / 1e12, 1),
            "predict_frac_bf16_peak": round(fw / dp / 1e12 / BF16_PEAK_TFLOPS, 4),
            "flops_count": "2 x 9 Cin Cout per output pixel of the 15 convolutions; training = forward + "
                           "data gradients (all but the first layer) + weight gradients"}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, budget_s: float = 12.0, max_steps: int = 30):
    """The FP64 oracle on the host: a bounded sample of the same workload on all the threads
    OpenMP gives it and on one thread, and the tiny workload's whole 200-step run on both."""
    from oracle import oracle as O
    from paper_1503_06726_amd import workloads as W
    log("cpu baseline: oracle on the same workload")
    cores = O.threads()

    def timed(wl, n_max, budget):
        o = O.from_workload(wl)
        t0 = time.perf_counter()
        n = 0
        while n < n_max:
            o.step(1)
            n += 1
            if time.perf_counter() - t0 > budget:
                break
        return n, time.perf_counter() - t0

    n, dt = timed(w, max_steps, budget_s)
    O.set_threads(1)
    n1, dt1 = timed(w, 3, 8.0)
    tiny = W.tiny_cell()
    nt1, tt1 = timed(tiny, tiny.steps, 60.0)
    O.set_threads(cores)
    ntc, ttc = timed(tiny, tiny.steps, 60.0)
    mlups = w.nx * w.ny * n / dt / 1e6
    return {"value": round(mlups, 3), "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"{n} steps of the same {w.nx}x{w.ny} workload ({w.n_cells} cells) in FP64, "
                      f"{dt:.1f} s, OpenMP lattice loops on {cores} threads",
            "cpu_model": cpu_model(),
            "single_thread": {"value": round(w.nx * w.ny * n1 / dt1 / 1e6, 3), "unit": "MLUPS", "cores": 1,
                              "sample": f"{n1} steps of the same workload, {dt1:.1f} s"},
            "tiny_full_run": {"workload": tiny.name, "steps": nt1,
                              "seconds_one_thread": round(tt1, 3), "seconds_all_threads": round(ttc, 3),
                              "mlups_one_thread": round(tiny.nx * tiny.ny * nt1 / tt1 / 1e6, 3),
                              "mlups_all_threads": round(tiny.nx * tiny.ny * ntc / ttc / 1e6, 3)}}


def oracle_field_errors(w, lbib, stream):
    """Per-field error against the FP64 oracle after 100 and 1,000 steps of the large workload
    for each population storage, on the seeded samples of tests/golden/horizon_large.npz (the
    oracle's checkpoints): relative L2 of u, phi and X - X0, and of rho - rho0."""
    import numpy as np
    path = os.path.join(GOLD, "horizon_large.npz")
    if not os.path.exists(path):
        return None
    g = np.load(path)
    lat, nodes = g["lat_idx"], g["node_idx"]

    def rel(a, b):
        nb = float(np.linalg.norm(b))
        return float(np.linalg.norm(a - b)) / (nb if nb > 0 else 1.0)
    out = {"checkpoints": [100, 1000], "samples": {"lattice_nodes": int(lat.size), "membrane_nodes": int(nodes.size)}}
    for name, st in (("fp32", lbib.STORAGE_FP32), ("fp16", lbib.STORAGE_FP16), ("bf16", lbib.STORAGE_BF16)):
        sim = lbib.from_workload(w, stream=stream, storage=st)
        res, done = {}, 0
        for k in (100, 1000):
            sim.step(k - done)
            done = k
            F = sim.get_fields(mask=False)
            res[str(k)] = {"u": rel(F["u"].reshape(2, -1)[:, lat], g[f"u_{k}"]),
                           "phi": rel(F["phi"].reshape(w.n_species, -1)[:, lat], g[f"phi_{k}"]),
                           "X-X0": rel(F["xy"][nodes] - w.xy[nodes], g[f"dX_{k}"]),
                           "rho-rho0": rel(F["rho"].reshape(-1)[lat] - w.rho0, g[f"drho_{k}"])}
        sim.close()
        out[name] = res
        log(f"oracle errors {name}: {res}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="large", choices=["large", "tissue", "tiny"])
    ap.add_argument("--storage", default="fp32", choices=["fp32", "fp16", "bf16"],
                    help="population storage (collision always in FP32)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--ade-samples", type=int, default=256,
                    help="held-out static-tissue samples for the iterations-to-steady half (0 skips)")
    ap.add_argument("--no-storage-variants", action="store_true",
                    help="skip the FP16 / BF16 storage runs reported beside the FP32 number")
    ap.add_argument("--sweep-sims", type=int, default=64,
                    help="simulations of the batched sweep (0 skips)")
    ap.add_argument("--sweep-steps", type=int, default=2000)
    ap.add_argument("--copy-probe", action="store_true",
                    help="run only a plain device copy of 1 GiB (calibrates the HBM byte counters)")
    ap.add_argument("--net-only", action="store_true",
                    help="run only the warm-start network's training and prediction timing")
    ap.add_argument("--no-net", action="store_true", help="skip the warm-start network's timing")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the lattice would shard into "
              "y-slabs across GPUs, which this build does not implement.", file=sys.stderr)
        sys.exit(2)

    only = args.copy_probe or args.net_only
    samples = [] if only else ade_samples(args.ade_samples)
    sweep = [] if only else sweep_workloads(args.sweep_sims)

    import torch
    from paper_1503_06726_amd import lbib, workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_probe:
        # a copy of known size: 2^30 bytes read and 2^30 bytes written per launch
        a = torch.ones(2 ** 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        log("copy probe: 5 copies of 2^30 bytes")
        return
    if args.net_only:
        r = net_half(lbib, torch.cuda.current_stream().cuda_stream)
        log(f"warm-start network: {r}")
        print(json.dumps({"warmstart_net": r}), flush=True)
        return
    w = W.WORKLOADS[args.workload]()
    S = w.n_species
    mask = w.mask_needed()
    log(f"workload: {w.name}, {w.n_nodes} nodes")
    stream = torch.cuda.current_stream().cuda_stream
    storage = {"fp32": lbib.STORAGE_FP32, "fp16": lbib.STORAGE_FP16, "bf16": lbib.STORAGE_BF16}[args.storage]
    pb = POP_BYTES[args.storage]
    sim = lbib.from_workload(w, stream=stream, storage=storage)
    log(f"device memory: {sim.device_bytes() / 2**20:.1f} MiB")
    sim.step(args.warmup)
    sim.sync()
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} steps done")

    # timed region: the production path (whole 16-step periods replay captured graphs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    sim.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log(f"timed {args.steps} steps: {dt:.3f} s")

    # kernel durations: HIP events around every launch on the library's stream (direct
    # launches; a kernel runs the same whether launched directly or from a graph)
    kt_steps = min(args.steps, 256)
    sim.set_timing(True)
    sim.step(kt_steps)
    timings = {lbib.KERNEL_NAMES[k]: sim.get_timing(k) for k in range(len(lbib.KERNEL_NAMES))}
    sim.set_timing(False)
    for k, (ms, n) in timings.items():
        if n:
            log(f"  {k:12s} {ms / n * 1e3:9.2f} us/launch  ({n} launches)")

    # the FP64 sums of the monitor (lbib_reduce_device: the same two kernels), 50 enqueued back
    # to back on the library's stream between two synchronisations (launch gaps included)
    out_sums = torch.zeros(3 + S, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    sim.reduce_device(out_sums.data_ptr())
    sim.sync()
    t0 = time.perf_counter()
    for _ in range(50):
        sim.reduce_device(out_sums.data_ptr())
    sim.sync()
    reduce_us = (time.perf_counter() - t0) / 50 * 1e6

    # sanity: the state is finite after the timed run
    red = sim.reduce()
    ref = sim.get_fields(mask=False) if args.storage == "fp32" and not args.no_storage_variants else None
    sim.close()

    nn = w.nx * w.ny
    mlups = nn * args.steps / dt / 1e6
    lat_ms, lat_n = timings["lattice"]
    lat_s = lat_ms / lat_n / 1e3
    b_lat = lattice_bytes_per_update(S, mask, pb)
    achieved = b_lat * nn / lat_s / 1e9
    b_step = step_bytes_per_update(S, mask, w.n_nodes, nn, pb)
    traffic = None
    if (args.storage == "fp32" and args.workload == "large" and LATTICE_TRAFFIC["bytes"]
            and LATTICE_TRAFFIC["sources_sha256"] == lattice_sources_sha()):
        traffic = LATTICE_TRAFFIC["bytes"]
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": "k_lattice", "bytes_per_update": b_lat, "us_per_launch": round(lat_s * 1e6, 2),
            "step_bytes_per_update": round(b_step, 2),
            "step_frac": round(b_step * mlups * 1e6 / 1e9 / HBM_PEAK_GBS, 4)}
    # the whole step against the same roofline (the survey's "% roofline": algorithmic bytes of
    # the step, lattice pass plus node positions, times the measured update rate)
    step_roof = {"bytes_per_update": round(b_step, 2), "achieved_GBs": round(b_step * mlups * 1e6 / 1e9, 1),
                 "peak_GBs": HBM_PEAK_GBS, "frac": round(b_step * mlups * 1e6 / 1e9 / HBM_PEAK_GBS, 4),
                 "bytes_count": "8 (9 + 5 S) population bytes + 1/8 source bit + 16 N / (nx ny) node-position bytes"}
    out = {"metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 5), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic (seeded Voronoi tissue, SeedSequence(1503))",
           "config": {"workload": w.name, "nx": w.nx, "ny": w.ny, "n_cells": w.n_cells, "n_nodes": w.n_nodes,
                      "species": S, "tau": w.tau, "storage": f"{args.storage} population deviations, fp64 node positions"},
           "roofline": roof, "step_roofline": step_roof,
           "kernels_us": {k: round(ms / n * 1e3, 2) for k, (ms, n) in timings.items() if n},
           "monitor_reduction_us": round(reduce_us, 2),
           "mass": red[0]}
    if ref is not None:
        out["storage_variants"] = storage_half(w, ref, args.warmup, args.steps, kt_steps, mlups, lbib, stream)
        errs = oracle_field_errors(w, lbib, stream) if args.workload == "large" else None
        if errs is not None:
            out["storage_variants"]["rel_l2_vs_fp64_oracle"] = errs
    if samples:
        log(f"iterations to steady: {len(samples)} samples")
        out["ade_iters_to_steady"] = ade_half(samples, lbib, stream)
        log(f"  {out['ade_iters_to_steady']}")
    if sweep:
        out["batched_sweep"] = sweep_half(sweep, args.sweep_steps, lbib, stream)
        log(f"  {out['batched_sweep']}")
    if not args.no_net:
        out["warmstart_net"] = net_half(lbib, stream)
        log(f"  warm-start network: {out['warmstart_net']}")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
