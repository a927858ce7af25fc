"""Throughput of the Kubo-formula Hall conductivity on one MI355X.

Workload (default): the n_orb = 32 random tight-binding model on R in
{-3..3}^3 (343 lattice vectors), a uniform 100^3 k-grid (10^6 k-points), 64
Fermi levels spread evenly over the band range, eta = 1e-3, Fermi-Dirac
occupation at kT = 0.01, all in FP64.  One step = sigma_xy for every Fermi
level over the whole grid (Bloch sums, eigensolves, velocity rotations,
curvature and Fermi sums, reduction), with the hoppings already in HBM.

Prints one JSON line: k-points/s, the roofline position of the dominant
kernel (timed with HIP events on its own stream through the library's timing
records) and the CPU oracle timed on a bounded sample of the same workload.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6  # 256 CU x 2.4 GHz x 128 FP64 flop/clk


def nominal_flops_per_k(n: int, n_R: int, n_f: int, fermi_dirac: bool) -> float:
    """Algorithmic FP64 flops per k-point of the forward path.

    Direct Bloch sum of H, v_x, v_y over the upper triangles (12 n_R n(n+1)),
    a Hermitian eigensolve counted as Householder + QR with vectors (24 n^3),
    two rotations U^+ v U (32 n^3), the band-pair curvature (5 n^2) and the
    Fermi sums (24 n N_F with Fermi-Dirac, 2 n N_F with a step)."""
    return 12.0 * n_R * n * (n + 1) + 24.0 * n**3 + 32.0 * n**3 + 5.0 * n * n + \
        (24.0 if fermi_dirac else 2.0) * n * n_f


def fermi_levels(cfg: int, wl):
    from paper_2309_06675_amd import synth

    if cfg == 0:
        return np.zeros((1, 1))
    with open(os.path.join(ROOT, "tests", "golden", "fermi_ranges.json")) as f:
        ranges = json.load(f)["ranges"][str(cfg)]
    return np.array([synth.fermi_levels(lo, hi, wl.n_fermi) for lo, hi in ranges])


def measure_batched(steps: int, warmup: int):
    """The 200-model workload: one batched plan replayed as a hipGraph vs one plan per model."""
    import torch

    from paper_2309_06675_amd import kubo, synth

    wl = synth.workload(2)
    ef = fermi_levels(2, wl)
    dev = "cuda:0"
    s = torch.cuda.Stream(dev)
    t_all = kubo.to_device_t(wl.models, dev)
    efd = torch.from_numpy(ef).to(dev)
    total_k = len(wl.models) * wl.n_k
    flops = sum(nominal_flops_per_k(m.n, m.n_R, wl.n_fermi, wl.kT > 0) for m in wl.models) * wl.n_k
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    out = {}
    with torch.cuda.stream(s):
        os.environ["KUBO_CHUNK_MB"] = "4096"
        plan = kubo.Plan(wl.models, grid=wl.grid, n_fermi=wl.n_fermi,
                         flags=kubo.KUBO_F_GRAPH | kubo.KUBO_F_FORWARD_ONLY, device=dev)
        sig = torch.empty(len(wl.models), wl.n_fermi, dtype=torch.float64, device=dev)
        for _ in range(warmup):
            plan.forward(t_all, efd, wl.eta, wl.kT, out=sig)
        torch.cuda.synchronize()
        start.record(s)
        for _ in range(steps):
            plan.forward(t_all, efd, wl.eta, wl.kT, out=sig)
        stop.record(s)
        torch.cuda.synchronize()
        ms_b = start.elapsed_time(stop) / steps
        st = plan.device_status()
        if st != kubo.KUBO_OK:
            raise SystemExit(f"batched device status: {kubo.kubo_status_string(st)}")
        sig_b = sig.cpu().numpy()
        del plan
        # plain path: one plan (and workspace) per model, launched one after another
        plans, ts, sigs = [], [], []
        off = 0
        os.environ["KUBO_CHUNK_MB"] = "256"
        for i, m in enumerate(wl.models):
            plans.append(kubo.Plan([m], grid=wl.grid, n_fermi=wl.n_fermi,
                                   flags=kubo.KUBO_F_FORWARD_ONLY, device=dev))
            cnt = m.t.size
            ts.append(t_all[off:off + cnt])
            off += cnt
            sigs.append(torch.empty(1, wl.n_fermi, dtype=torch.float64, device=dev))
        for _ in range(warmup):
            for i, p in enumerate(plans):
                p.forward(ts[i], efd[i:i + 1], wl.eta, wl.kT, out=sigs[i])
        torch.cuda.synchronize()
        start.record(s)
        for _ in range(steps):
            for i, p in enumerate(plans):
                p.forward(ts[i], efd[i:i + 1], wl.eta, wl.kT, out=sigs[i])
        stop.record(s)
        torch.cuda.synchronize()
        ms_p = start.elapsed_time(stop) / steps
        sig_p = torch.cat(sigs).cpu().numpy()
        os.environ.pop("KUBO_CHUNK_MB", None)
    out["workload"] = wl.name
    out["models"] = len(wl.models)
    out["k_points_per_step"] = total_k
    out["batched_graph"] = {"ms_per_step": ms_b, "k_points_per_s": total_k / (ms_b / 1e3),
                            "tflops_nominal": flops / (ms_b / 1e3) / 1e12,
                            "frac": flops / (ms_b / 1e3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS}
    out["plain_per_model"] = {"ms_per_step": ms_p, "k_points_per_s": total_k / (ms_p / 1e3),
                              "tflops_nominal": flops / (ms_p / 1e3) / 1e12,
                              "frac": flops / (ms_p / 1e3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS}
    out["batched_over_plain"] = ms_p / ms_b
    out["max_abs_diff_batched_vs_plain"] = float(np.abs(sig_b - sig_p).max())
    return out


def measure_large(adjoint: bool = True, parts: int = 16):
    """The n_orb = 128 workload (729 R, 128^3 grid, 256 Fermi levels): the forward at
    eta = 1e-3 and the adjoint at eta = 1e-2 over the whole grid, enqueued as `parts`
    consecutive k-slabs (slabs add up exactly; each slab prints a progress line)."""
    import torch

    from paper_2309_06675_amd import kubo, synth

    wl = synth.workload(4)
    m = wl.models[0]
    ef = fermi_levels(4, wl)
    dev = "cuda:0"
    t = kubo.to_device_t([m], dev)
    efd = torch.from_numpy(ef).to(dev)
    stream = torch.cuda.current_stream(dev)
    cuts = [wl.n_k * i // parts for i in range(parts + 1)]
    plans = [kubo.Plan([m], grid=wl.grid, n_fermi=wl.n_fermi, device=dev,
                       slabs=[(cuts[i], cuts[i + 1] - cuts[i])]) for i in range(parts)]
    warm = kubo.Plan([m], grid=wl.grid, n_fermi=wl.n_fermi, slabs=[(0, 4 * wl.grid[0])],
                     device=dev)
    warm.forward(t, efd, wl.eta, wl.kT)
    warm.backward(t, efd, wl.eta_adjoint, wl.kT, torch.ones(1, wl.n_fermi, dtype=torch.float64,
                                                            device=dev))
    torch.cuda.synchronize()

    def timed(fn):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        r = fn()
        b.record(stream)
        torch.cuda.synchronize()
        return r, a.elapsed_time(b)

    sig = torch.zeros(1, wl.n_fermi, dtype=torch.float64, device=dev)
    fms = 0.0
    for i, p in enumerate(plans):
        s_i, ms = timed(lambda: p.forward(t, efd, wl.eta, wl.kT))
        assert p.device_status() == kubo.KUBO_OK
        sig += s_i
        fms += ms
        print(f"large forward slab {i + 1}/{parts}: {ms:.1f} ms", file=sys.stderr, flush=True)
    fpk = nominal_flops_per_k(m.n, m.n_R, wl.n_fermi, True)
    out = {"workload": wl.name, "k_points": wl.n_k, "forward_ms": fms,
           "forward_k_points_per_s": wl.n_k / (fms / 1e3),
           "forward_frac_nominal": fpk * wl.n_k / (fms / 1e3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS,
           "sigma_sum": float(sig.sum().item())}
    if adjoint:
        sbar = torch.ones(1, wl.n_fermi, dtype=torch.float64, device=dev)
        g = torch.zeros_like(t)
        bms = 0.0
        for i, p in enumerate(plans):
            g_i, ms = timed(lambda: p.backward(t, efd, wl.eta_adjoint, wl.kT, sbar))
            assert p.device_status() == kubo.KUBO_OK
            g += g_i
            bms += ms
            print(f"large adjoint slab {i + 1}/{parts}: {ms:.1f} ms", file=sys.stderr, flush=True)
        out.update({"adjoint_ms": bms, "adjoint_k_points_per_s": wl.n_k / (bms / 1e3),
                    "adjoint_forward_ratio": bms / fms,
                    "grad_abs_sum": float(g.abs().sum().item())})
    return out


def kernel_source_digest() -> str:
    """sha256 of the sources of the dominant kernel (the one-wavefront per-k kernel)."""
    import hashlib

    h = hashlib.sha256()
    for f in ("kubo_wave.hip", "kubo_cplx.h", "kubo_internal.h", "kubo_launch.h"):
        with open(os.path.join(ROOT, "paper_2309_06675_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic():
    """HBM bytes per launch of the dominant kernel from the committed counter runs
    (profiles/traffic_k_forward_wave_n32.json), or None if the kernel changed since."""
    path = os.path.join(ROOT, "profiles", "traffic_k_forward_wave_n32.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha256") != kernel_source_digest():
        return None
    return rec.get("bytes_per_launch")


def copy_calibration(mbytes: int):
    """One device-to-device copy of a known size (to scale the FETCH/WRITE counters)."""
    import torch

    n = mbytes * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n * 8, "read_bytes": n * 8, "write_bytes": n * 8}), flush=True)
    return 0


def cpu_baseline(model, wl, ef, sample: int):
    """The CPU oracle, untuned, on a contiguous slab of `sample` k-points."""
    from oracle import oracle as O

    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
    kb = (wl.n_k // 2) - sample // 2
    t0 = time.perf_counter()
    O.ahc(model.t, model.R, wl.grid, ef, wl.eta, wl.kT, k_begin=kb, k_count=sample,
          nthreads=threads)
    dt = time.perf_counter() - t0
    return {"value": sample / dt, "unit": "k-points/s", "cores": threads, "kind": "oracle",
            "sample": f"{sample} consecutive k-points (flat index {kb}..{kb + sample - 1}) of the "
                      f"same model, grid and Fermi levels; {dt:.2f} s wall on {threads} threads"}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-sample", type=int, default=4096,
                    help="k-points the CPU oracle is timed on (0 skips it)")
    ap.add_argument("--k-block", type=int, default=0, help="override the k-block of the plan")
    ap.add_argument("--threads", type=int, default=0,
                    help="per-k kernel: 64 = one wavefront, 256 = one workgroup (0 = default)")
    ap.add_argument("--adjoint-steps", type=int, default=1,
                    help="timed backward passes for the adjoint/forward ratio (0 skips)")
    ap.add_argument("--batched-steps", type=int, default=1,
                    help="timed steps of the 200-model batched workload (0 skips)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="only run one device copy of MB megabytes (counter calibration)")
    ap.add_argument("--large", action="store_true",
                    help="only run the n_orb = 128 workload (forward + adjoint) and print it")
    args = ap.parse_args(argv)
    if args.copy_calibration > 0:
        return copy_calibration(args.copy_calibration)
    if args.large:
        if args.gpus != 1:
            print("bench.py measures one GPU", file=sys.stderr)
            return 2
        print(json.dumps(measure_large()), flush=True)
        return 0
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(k-slabs shard across GPUs by design, but this build runs on one GPU only)",
              file=sys.stderr)
        return 2

    import torch

    from paper_2309_06675_amd import kubo, synth

    cfg = 1
    wl = synth.workload(cfg)
    model = wl.models[0]
    ef = fermi_levels(cfg, wl)
    dev = "cuda:0"
    torch.cuda.set_device(0)
    tiles = "auto"
    if args.k_block > 0 or args.threads > 0:
        tiles = [(model.n, args.threads, args.k_block if args.k_block > 0 else 32)]
    plan = kubo.Plan([model], grid=wl.grid, n_fermi=wl.n_fermi, flags=kubo.KUBO_F_TIMING,
                     tiles=tiles, device=dev)
    t = kubo.to_device_t([model], dev)
    efd = torch.from_numpy(ef).to(dev)
    sigma = torch.empty(1, wl.n_fermi, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)

    for _ in range(args.warmup):
        plan.forward(t, efd, wl.eta, wl.kT, out=sigma)
    torch.cuda.synchronize()
    if args.warmup > 0:
        st = plan.device_status()
        if st != kubo.KUBO_OK:
            raise SystemExit(f"device status after warm-up: {kubo.kubo_status_string(st)}")
    plan.kernel_time(0, reset=True)

    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for i in range(args.steps):
        plan.forward(t, efd, wl.eta, wl.kT, out=sigma)
    stop.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    st = plan.device_status()
    if st != kubo.KUBO_OK:
        raise SystemExit(f"device status: {kubo.kubo_status_string(st)}")
    k_ms, launches, kpts = plan.kernel_time(0)
    total_k = plan.total_k * args.steps
    value = total_k / (ms / 1e3)

    fpk = nominal_flops_per_k(model.n, model.n_R, wl.n_fermi, wl.kT > 0)
    achieved = fpk * kpts / (k_ms / 1e3) / 1e12
    out = {
        "metric": "k-points/s for sigma_xy (n_orb=32, FP64) at 1 MI355X",
        "value": value,
        "unit": "k-points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "n32_R343_k100^3_F64_kT0.01_eta1e-3", "n_orb": model.n,
                   "n_R": model.n_R, "grid": list(wl.grid), "n_fermi": wl.n_fermi,
                   "eta": wl.eta, "kT": wl.kT, "model_seed": 1000, "parallelism": "single-gpu"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                     "traffic": recorded_traffic(), "kernel": "k_forward_wave<32> (per-k fused)",
                     "flops_per_k": fpk, "kernel_ms_per_step": k_ms / args.steps,
                     "launches_per_step": launches / args.steps},
        "sigma_checksum": float(sigma.sum().item()),
    }
    if args.adjoint_steps > 0:
        # adjoint of sum_j sbar_j sigma_j over the same grid (all hoppings), same stream
        sbar = torch.ones(1, wl.n_fermi, dtype=torch.float64, device=dev)
        grad = torch.empty_like(t)
        plan.backward(t, efd, wl.eta, wl.kT, sbar, out=grad)
        torch.cuda.synchronize()
        plan.kernel_time(1, reset=True)
        start.record(stream)
        for _ in range(args.adjoint_steps):
            plan.backward(t, efd, wl.eta, wl.kT, sbar, out=grad)
        stop.record(stream)
        torch.cuda.synchronize()
        st = plan.device_status()
        if st != kubo.KUBO_OK:
            raise SystemExit(f"device status (backward): {kubo.kubo_status_string(st)}")
        bms = start.elapsed_time(stop) / args.adjoint_steps
        out["adjoint"] = {"ms_per_step": bms, "k_points_per_s": plan.total_k / (bms / 1e3),
                          "adjoint_forward_ratio": bms / (ms / args.steps),
                          "kernel_ms_per_step": plan.kernel_time(1)[0] / args.adjoint_steps,
                          "grad_checksum": float(grad.abs().sum().item())}
    if args.batched_steps > 0:
        out["batched"] = measure_batched(args.batched_steps, 1)
    if args.cpu_sample > 0:
        out["cpu_baseline"] = cpu_baseline(model, wl, ef[0], args.cpu_sample)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
