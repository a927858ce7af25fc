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
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def bloch_flops_per_k(n: int, n_R: int, nR0: int, N0: int) -> float:
    """FP64 flops per k-point of the Bloch sums of H, v_x, v_y as the kernels execute them
    (sum-factorised over kx pencils).  Per pencil of N0 k-points: T_rho and Ty_rho, one
    complex multiply-add each per lattice vector and matrix element (16 n_R n^2); per
    k-point: the nR0-term rho-sums of H, v_x and v_y over the upper triangles
    (3 x 8 x nR0 x n(n+1)/2)."""
    return 16.0 * n_R * n * n / N0 + 12.0 * nR0 * n * (n + 1)


def direct_bloch_flops_per_k(n: int, n_R: int) -> float:
    """The same sums taken directly over all lattice vectors (upper triangles): 12 n_R n(n+1)."""
    return 12.0 * n_R * n * (n + 1)


def forward_flops_per_k(n: int, n_R: int, nR0: int, N0: int, n_f: int, fermi_dirac: bool,
                        direct: bool = False) -> float:
    """Algorithmic FP64 flops per k-point of the forward path: the Bloch sums (sum-factorised
    as executed, or direct), a Hermitian eigensolve counted as Householder + QR with vectors
    (24 n^3), two rotations U^+ v U (32 n^3), the band-pair curvature (5 n^2) and the Fermi
    sums (24 n N_F with Fermi-Dirac, 2 n N_F with a step)."""
    s2 = direct_bloch_flops_per_k(n, n_R) if direct else bloch_flops_per_k(n, n_R, nR0, N0)
    return s2 + 24.0 * n**3 + 32.0 * n**3 + 5.0 * n * n + \
        (24.0 if fermi_dirac else 2.0) * n * n_f


def adjoint_flops_per_k(n: int, n_R: int, nR0: int, N0: int, n_f: int, k_block: int) -> float:
    """Algorithmic FP64 flops per k-point of the backward pass: the forward recomputed, the
    cotangents ((20 + 24 N_F) n), back through the eigendecomposition and the rotations
    (ten complex products, 80 n^3), the per-k pencil sums of Hbar, vbar_x, vbar_y (3 x 8 x
    nR0 x n^2) and the transposed Bloch sum per k-block of k_block points (16 n_R n^2)."""
    return forward_flops_per_k(n, n_R, nR0, N0, n_f, True) + (20.0 + 24.0 * n_f) * n + \
        80.0 * n**3 + 24.0 * nR0 * n * n + 16.0 * n_R * n * n / k_block


def n_rx(model) -> int:
    return len(set(int(x) for x in model.R[:, 0]))


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
    flops = sum(forward_flops_per_k(m.n, m.n_R, n_rx(m), wl.grid[0], wl.n_fermi, wl.kT > 0)
                for m in wl.models) * wl.n_k
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
                            "tflops": flops / (ms_b / 1e3) / 1e12,
                            "frac": flops / (ms_b / 1e3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS}
    out["plain_per_model"] = {"ms_per_step": ms_p, "k_points_per_s": total_k / (ms_p / 1e3),
                              "tflops": flops / (ms_p / 1e3) / 1e12,
                              "frac": flops / (ms_p / 1e3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS}
    out["batched_over_plain"] = ms_p / ms_b
    out["max_abs_diff_batched_vs_plain"] = float(np.abs(sig_b - sig_p).max())
    return out


def _timed_median(fn, reps: int, stream):
    """Median over `reps` calls of fn() of the HIP-event time on `stream` (ms)."""
    import torch

    out = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        torch.cuda.synchronize()
        out.append(a.elapsed_time(b))
    return float(np.median(out)), out


def measure_adjoint_cfg3(reps: int = 5):
    """The adjoint workload at its own shape: the n_orb = 32 model on its 64^3 grid, 16 Fermi
    levels, eta = 1e-2, kT = 0.01; gradient of sum_j sigma_j w.r.t. all 343 x 32 x 32
    hoppings.  Forward and backward each timed as the median of `reps` passes."""
    import torch

    from paper_2309_06675_amd import kubo, synth

    wl = synth.workload(3)
    m = wl.models[0]
    ef = fermi_levels(3, wl)
    dev = "cuda:0"
    stream = torch.cuda.current_stream(dev)
    plan = kubo.Plan([m], grid=wl.grid, n_fermi=wl.n_fermi, flags=kubo.KUBO_F_TIMING,
                     device=dev)
    t = kubo.to_device_t([m], dev)
    efd = torch.from_numpy(ef).to(dev)
    sig = torch.empty(1, wl.n_fermi, dtype=torch.float64, device=dev)
    sbar = torch.ones(1, wl.n_fermi, dtype=torch.float64, device=dev)
    grad = torch.empty_like(t)
    plan.forward(t, efd, wl.eta_adjoint, wl.kT, out=sig)
    plan.backward(t, efd, wl.eta_adjoint, wl.kT, sbar, out=grad)
    torch.cuda.synchronize()
    plan.kernel_time(0, reset=True)
    plan.kernel_time(1, reset=True)
    fms, fall = _timed_median(lambda: plan.forward(t, efd, wl.eta_adjoint, wl.kT, out=sig), reps,
                              stream)
    bms, ball = _timed_median(lambda: plan.backward(t, efd, wl.eta_adjoint, wl.kT, sbar,
                                                    out=grad), reps, stream)
    st = plan.device_status()
    if st != kubo.KUBO_OK:
        raise SystemExit(f"adjoint workload device status: {kubo.kubo_status_string(st)}")
    kb = int(np.ceil(wl.grid[0] / np.ceil(wl.grid[0] / 32)))
    ffk = forward_flops_per_k(m.n, m.n_R, n_rx(m), wl.grid[0], wl.n_fermi, True)
    bfk = adjoint_flops_per_k(m.n, m.n_R, n_rx(m), wl.grid[0], wl.n_fermi, kb)
    bk_ms, _, bk_k = plan.kernel_time(1)
    return {"workload": wl.name, "k_points": wl.n_k, "reps": reps,
            "forward_ms_median": fms, "backward_ms_median": bms,
            "forward_ms_all": fall, "backward_ms_all": ball,
            "forward_k_points_per_s": wl.n_k / (fms / 1e3),
            "backward_k_points_per_s": wl.n_k / (bms / 1e3),
            "adjoint_forward_ratio": bms / fms,
            "backward_kernel_ms_per_pass": bk_ms / reps,
            "flops_per_k": {"forward": ffk, "backward": bfk},
            "frac": {"forward": ffk * wl.n_k / (fms / 1e3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS,
                     "backward": bfk * wl.n_k / (bms / 1e3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS},
            "grad_checksum": float(grad.abs().sum().item())}


def measure_cfg4_slab(planes: int = 2, reps: int = 2):
    """The n_orb = 128 workload (729 R, 128^3 grid, 256 Fermi levels; eta = 1e-3 forward,
    1e-2 adjoint) on a slab of `planes` consecutive k_z planes from the middle of the grid
    (planes x 128^2 k-points); median of `reps` passes each way."""
    import torch

    from paper_2309_06675_amd import kubo, synth

    wl = synth.workload(4)
    m = wl.models[0]
    ef = fermi_levels(4, wl)
    dev = "cuda:0"
    stream = torch.cuda.current_stream(dev)
    per_plane = wl.grid[0] * wl.grid[1]
    kb = (wl.grid[2] // 2) * per_plane
    kc = planes * per_plane
    plan = kubo.Plan([m], grid=wl.grid, n_fermi=wl.n_fermi, slabs=[(kb, kc)], device=dev)
    t = kubo.to_device_t([m], dev)
    efd = torch.from_numpy(ef).to(dev)
    sbar = torch.ones(1, wl.n_fermi, dtype=torch.float64, device=dev)
    warm = kubo.Plan([m], grid=wl.grid, n_fermi=wl.n_fermi, slabs=[(kb, 2 * wl.grid[0])],
                     device=dev)
    warm.forward(t, efd, wl.eta, wl.kT)
    warm.backward(t, efd, wl.eta_adjoint, wl.kT, sbar)
    torch.cuda.synchronize()
    del warm
    print(f"cfg4 slab: {kc} k-points", file=sys.stderr, flush=True)
    fms, fall = _timed_median(lambda: plan.forward(t, efd, wl.eta, wl.kT), reps, stream)
    print(f"cfg4 slab forward {fms:.1f} ms", file=sys.stderr, flush=True)
    bms, ball = _timed_median(lambda: plan.backward(t, efd, wl.eta_adjoint, wl.kT, sbar), reps,
                              stream)
    print(f"cfg4 slab backward {bms:.1f} ms", file=sys.stderr, flush=True)
    st = plan.device_status()
    if st != kubo.KUBO_OK:
        raise SystemExit(f"cfg4 slab device status: {kubo.kubo_status_string(st)}")
    kbb = int(np.ceil(wl.grid[0] / np.ceil(wl.grid[0] / 32)))
    ffk = forward_flops_per_k(m.n, m.n_R, n_rx(m), wl.grid[0], wl.n_fermi, True)
    bfk = adjoint_flops_per_k(m.n, m.n_R, n_rx(m), wl.grid[0], wl.n_fermi, kbb)
    return {"workload": wl.name, "slab": {"k_begin": kb, "k_count": kc,
                                          "what": f"{planes} k_z planes from the middle"},
            "reps": reps, "forward_ms_median": fms, "backward_ms_median": bms,
            "forward_k_points_per_s": kc / (fms / 1e3),
            "backward_k_points_per_s": kc / (bms / 1e3),
            "adjoint_forward_ratio": bms / fms,
            "flops_per_k": {"forward": ffk, "backward": bfk},
            "frac": {"forward": ffk * kc / (fms / 1e3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS,
                     "backward": bfk * kc / (bms / 1e3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS}}


def gf_flops_per_k(n: int, n_R: int, nr0: int, n0: int, n_fermi: int, n_omega: int) -> float:
    """Algorithmic flops per k-point of the Green's-function form: the pencil sums
    (16 n_R n^2 per pencil, spread over its n0 points) and the full-matrix rho-sums of H, v_x,
    v_y (24 nR0 n^2), then per Fermi level and node one inverse (8 n^3), four products
    (32 n^3) and two traces (16 n^2)."""
    return (16.0 * n_R * n * n / n0 + 24.0 * nr0 * n * n
            + n_fermi * n_omega * (40.0 * n**3 + 16.0 * n * n))


def measure_gf(reps: int = 3, n_fermi: int = 8, n_omega: int = 16, gamma: float = 0.01):
    """The Green's-function form on the n_orb = 32 model (343 R) on a 32^3 grid: n_fermi of the
    workload's Fermi levels, n_omega Gauss-Legendre nodes on (0, inf) (w = tan(pi (u + 1)/4)),
    scattering rate gamma; median of `reps` passes."""
    import torch

    from paper_2309_06675_amd import kubo, synth

    wl = synth.workload(1)
    m = wl.models[0]
    grid = (32, 32, 32)
    nk = grid[0] * grid[1] * grid[2]
    ef_all = fermi_levels(1, wl)[0]
    ef = np.ascontiguousarray(ef_all[:: len(ef_all) // n_fermi][:n_fermi]).reshape(1, n_fermi)
    u, c = np.polynomial.legendre.leggauss(n_omega)
    th = 0.25 * np.pi * (u + 1.0)
    om, wt = np.tan(th), 0.25 * np.pi * c / np.cos(th) ** 2
    dev = "cuda:0"
    stream = torch.cuda.current_stream(dev)
    plan = kubo.Plan([m], grid=grid, n_fermi=n_fermi,
                     flags=kubo.KUBO_F_FORWARD_ONLY | kubo.KUBO_F_TIMING, device=dev)
    t = kubo.to_device_t([m], dev)
    efd = torch.from_numpy(ef).to(dev)
    omd = torch.from_numpy(om).to(dev)
    wtd = torch.from_numpy(wt).to(dev)
    sig = torch.empty(1, n_fermi, dtype=torch.float64, device=dev)
    plan.gf(t, efd, gamma, omd, wtd, out=sig)
    torch.cuda.synchronize()
    plan.kernel_time(3, reset=True)
    ms, alls = _timed_median(lambda: plan.gf(t, efd, gamma, omd, wtd, out=sig), reps, stream)
    st = plan.device_status()
    if st != kubo.KUBO_OK:
        raise SystemExit(f"gf device status: {kubo.kubo_status_string(st)}")
    k_ms, launches, kpts = plan.kernel_time(3)
    fpk = gf_flops_per_k(m.n, m.n_R, n_rx(m), grid[0], n_fermi, n_omega)
    fpk_kernel = fpk - 16.0 * m.n_R * m.n**2 / grid[0]
    achieved = fpk_kernel * kpts / (k_ms / 1e3) / 1e12
    print(f"gf {ms:.1f} ms", file=sys.stderr, flush=True)
    return {"workload": f"gf_n32_R343_k32^3_F{n_fermi}_W{n_omega}_gamma{gamma:g}",
            "k_points": nk, "reps": reps, "ms_median": ms, "ms_all": alls,
            "k_points_per_s": nk / (ms / 1e3),
            "kernel": "k_gf (one workgroup per k-point)",
            "kernel_ms_per_pass": k_ms / reps, "flops_per_k": fpk,
            "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS},
            "sigma_checksum": float(sig.sum().item())}


def big_reduction_bytes_per_k(n: int) -> int:
    """HBM bytes per k-point the large-n Householder reduction has to move: at step k the
    lower triangle (diagonal included) of rows/columns k+2.. is read and written once
    (16-byte complex elements), and step 0 reads the whole matrix once."""
    tri = sum(m * (m + 1) // 2 for m in range(1, n - 1))
    return 16 * (2 * tri + n * n)


def measure_large_n(reps: int = 3, n: int = 256, grid=(16, 16, 16), n_fermi: int = 16):
    """The large-n path (128 < n <= 512: many workgroups per k-point): a random n = 256 model
    on R in {-1..1}^3 (27 lattice vectors), a 16^3 grid, 16 Fermi levels over [-3, 3],
    eta = 1e-3, kT = 0.01; median of `reps` forward passes."""
    import torch

    from paper_2309_06675_amd import kubo, synth

    m = synth.random_model(n, 1, 1.0, 4000 + n)
    nk = grid[0] * grid[1] * grid[2]
    ef = np.linspace(-3.0, 3.0, n_fermi).reshape(1, n_fermi)
    dev = "cuda:0"
    stream = torch.cuda.current_stream(dev)
    plan = kubo.Plan([m], grid=grid, n_fermi=n_fermi,
                     flags=kubo.KUBO_F_FORWARD_ONLY | kubo.KUBO_F_TIMING, device=dev)
    t = kubo.to_device_t([m], dev)
    efd = torch.from_numpy(ef).to(dev)
    sig = torch.empty(1, n_fermi, dtype=torch.float64, device=dev)
    plan.forward(t, efd, 1e-3, 0.01, out=sig)
    torch.cuda.synchronize()
    plan.kernel_time(4, reset=True)
    ms, alls = _timed_median(lambda: plan.forward(t, efd, 1e-3, 0.01, out=sig), reps, stream)
    st = plan.device_status()
    if st != kubo.KUBO_OK:
        raise SystemExit(f"large-n device status: {kubo.kubo_status_string(st)}")
    fpk = forward_flops_per_k(m.n, m.n_R, n_rx(m), grid[0], n_fermi, True)
    # the reduction kernel (bound by HBM bandwidth): HIP events around each of its launches
    red_ms, red_launches, red_k = plan.kernel_time(4)
    bpk = big_reduction_bytes_per_k(n)
    red_gbs = bpk * red_k / (red_ms / 1e3) / 1e9 if red_ms > 0 else None
    print(f"large n={n} {ms:.1f} ms", file=sys.stderr, flush=True)
    return {"workload": f"n{n}_R27_k16^3_F{n_fermi}_kT0.01", "k_points": nk, "reps": reps,
            "ms_median": ms, "ms_all": alls, "k_points_per_s": nk / (ms / 1e3),
            "flops_per_k": fpk,
            "tflops": fpk * nk / (ms / 1e3) / 1e12,
            "frac": fpk * nk / (ms / 1e3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS,
            "reduction_roofline": {
                "bound": "hbm", "kernel": "k_big_tridiag", "achieved": red_gbs,
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": red_gbs / HBM_PEAK_GBS if red_gbs else None,
                "bytes_per_k": bpk, "launches": red_launches,
                "k_points_per_launch": red_k / red_launches if red_launches else None,
                "ms_per_launch": red_ms / red_launches if red_launches else None,
                "bytes_model": "lower triangle of the trailing matrix read and written once per step, "
                               "the whole matrix read once at step 0"},
            "sigma_checksum": float(sig.sum().item())}


def measure_large(adjoint: bool = True, parts: int = 16):
    """The n_orb = 128 workload over its whole 128^3 grid (forward at eta = 1e-3, adjoint at
    eta = 1e-2), enqueued as `parts` consecutive k-slabs (slabs add up exactly; each slab
    prints a progress line).  Not part of the default run (about three minutes)."""
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
    sbar = torch.ones(1, wl.n_fermi, dtype=torch.float64, device=dev)
    sig = torch.zeros(1, wl.n_fermi, dtype=torch.float64, device=dev)
    fms = 0.0
    for i, p in enumerate(plans):
        ms, _ = _timed_median(lambda: sig.add_(p.forward(t, efd, wl.eta, wl.kT)), 1, stream)
        assert p.device_status() == kubo.KUBO_OK
        fms += ms
        print(f"large forward slab {i + 1}/{parts}: {ms:.1f} ms", file=sys.stderr, flush=True)
    fpk = forward_flops_per_k(m.n, m.n_R, n_rx(m), wl.grid[0], wl.n_fermi, True)
    out = {"workload": wl.name, "k_points": wl.n_k, "forward_ms": fms,
           "forward_k_points_per_s": wl.n_k / (fms / 1e3),
           "forward_frac": fpk * wl.n_k / (fms / 1e3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS,
           "sigma_sum": float(sig.sum().item())}
    if adjoint:
        g = torch.zeros_like(t)
        bms = 0.0
        for i, p in enumerate(plans):
            ms, _ = _timed_median(lambda: g.add_(p.backward(t, efd, wl.eta_adjoint, wl.kT,
                                                            sbar)), 1, stream)
            assert p.device_status() == kubo.KUBO_OK
            bms += ms
            print(f"large adjoint slab {i + 1}/{parts}: {ms:.1f} ms", file=sys.stderr,
                  flush=True)
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


def recorded_counters():
    """The committed counter record of the dominant kernel
    (profiles/counters_k_forward_wave_n32.json: HBM bytes per launch from FETCH_SIZE and
    WRITE_SIZE scaled by a plain copy, executed FP64 flops per launch, LDS bank conflicts),
    or None if the kernel's sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "counters_k_forward_wave_n32.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha256") != kernel_source_digest():
        return None
    return rec


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


def flop_calibration(mbytes: int):
    """Elementwise FP64 kernels of known work (counter calibration): a + b (one add per
    element) and a + b * c (one multiply-add per element) over mbytes of doubles each."""
    import torch

    n = mbytes * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.full_like(a, 0.5)
    c = torch.full_like(a, 0.25)
    torch.cuda.synchronize()
    d = a + b
    e = torch.addcmul(a, b, c)
    torch.cuda.synchronize()
    print(json.dumps({"elements": n, "add_flops": n, "fma_flops": 2 * n,
                      "check": float(d[0] + e[0])}), flush=True)
    return 0


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(model, wl, ef, sample: int, single_sample: int):
    """The CPU oracle, untuned, on a contiguous slab of `sample` k-points from the middle of
    the grid with all threads the process may use, and on `single_sample` k-points with one
    thread.  Cost per k-point is the same everywhere on the grid, so k-points/s extrapolates
    linearly to the full grid."""
    from oracle import oracle as O

    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    kb = (wl.n_k // 2) - sample // 2
    t0 = time.perf_counter()
    O.ahc(model.t, model.R, wl.grid, ef, wl.eta, wl.kT, k_begin=kb, k_count=sample,
          nthreads=threads)
    dt = time.perf_counter() - t0
    out = {"value": sample / dt, "unit": "k-points/s", "cores": threads, "kind": "oracle",
           "sample": f"{sample} consecutive k-points (flat index {kb}..{kb + sample - 1}) of the "
                     f"same model, grid and Fermi levels; {dt:.2f} s wall on {threads} threads; "
                     f"extrapolated: the full {wl.n_k}-point grid would take "
                     f"{wl.n_k / (sample / dt):.0f} s",
           "cpu_model": cpu_model(), "nproc": os.cpu_count(),
           "affinity_cpus": len(os.sched_getaffinity(0))}
    if single_sample > 0:
        t0 = time.perf_counter()
        O.ahc(model.t, model.R, wl.grid, ef, wl.eta, wl.kT, k_begin=kb, k_count=single_sample,
              nthreads=1)
        d1 = time.perf_counter() - t0
        out["single_core"] = {"value": single_sample / d1, "unit": "k-points/s",
                              "sample": f"{single_sample} k-points from flat index {kb}; "
                                        f"{d1:.2f} s wall on 1 thread (extrapolated)"}
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-sample", type=int, default=20480,
                    help="k-points the CPU oracle is timed on with all threads (0 skips it)")
    ap.add_argument("--cpu-single-sample", type=int, default=1024,
                    help="k-points the CPU oracle is timed on with one thread (0 skips it)")
    ap.add_argument("--k-block", type=int, default=0, help="override the k-block of the plan")
    ap.add_argument("--threads", type=int, default=0,
                    help="per-k kernel: 64 = one wavefront, 256 = one workgroup (0 = default)")
    ap.add_argument("--adjoint-reps", type=int, default=5,
                    help="timed passes (median) of the adjoint workload, each way (0 skips)")
    ap.add_argument("--large-reps", type=int, default=2,
                    help="timed passes (median) of the n_orb = 128 slab, each way (0 skips)")
    ap.add_argument("--batched-steps", type=int, default=1,
                    help="timed steps of the 200-model batched workload (0 skips)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="only run one device copy of MB megabytes (counter calibration)")
    ap.add_argument("--flop-calibration", type=int, default=0, metavar="MB",
                    help="only run two elementwise FP64 kernels on MB megabytes (counter calibration)")
    ap.add_argument("--large", action="store_true",
                    help="only run the n_orb = 128 workload over its full grid and print it")
    ap.add_argument("--large-n-reps", type=int, default=3,
                    help="timed passes (median) of the n = 256 large-n workload (0 skips)")
    ap.add_argument("--gf-reps", type=int, default=3,
                    help="timed passes (median) of the Green's-function form (0 skips)")
    ap.add_argument("--legs", default="forward,adjoint,n128,batched,gf,large_n,cpu",
                    help="comma-separated legs to run (forward is always run; for profiling)")
    args = ap.parse_args(argv)
    legs = set(args.legs.split(","))
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(k-slabs shard across GPUs by design, but this build runs on one GPU only)",
              file=sys.stderr)
        return 2
    if args.copy_calibration > 0:
        return copy_calibration(args.copy_calibration)
    if args.flop_calibration > 0:
        return flop_calibration(args.flop_calibration)
    if args.large:
        print(json.dumps(measure_large()), flush=True)
        return 0

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
    plan = kubo.Plan([model], grid=wl.grid, n_fermi=wl.n_fermi,
                     flags=kubo.KUBO_F_TIMING | kubo.KUBO_F_FORWARD_ONLY, tiles=tiles, device=dev)
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

    nr0 = n_rx(model)
    fpk = forward_flops_per_k(model.n, model.n_R, nr0, wl.grid[0], wl.n_fermi, wl.kT > 0)
    fpk_direct = forward_flops_per_k(model.n, model.n_R, nr0, wl.grid[0], wl.n_fermi,
                                     wl.kT > 0, direct=True)
    # the per-k kernel executes everything but the pencil sums (a separate kernel)
    fpk_kernel = fpk - 16.0 * model.n_R * model.n**2 / wl.grid[0]
    achieved = fpk_kernel * kpts / (k_ms / 1e3) / 1e12
    rec = recorded_counters()
    traffic = rec["bytes_per_launch"] if rec else None
    per_launch_k = kpts / max(launches, 1)
    counters = None
    if rec:
        # executed FP64 work from the counters (issued lanes, MFMA at 512 flops per MOP),
        # over the live launch time of this run
        exe = rec["fp64_flops_per_k_point"] * kpts / (k_ms / 1e3) / 1e12
        counters = {"executed_fp64_tflops": exe, "executed_frac": exe / FP64_VECTOR_PEAK_TFLOPS,
                    "executed_flops_per_k": rec["fp64_flops_per_k_point"],
                    "lds_bank_conflicts_per_access": rec["lds_bank_conflicts_per_access"],
                    "hbm_bytes_per_k": rec["bytes_per_launch"] / rec["k_points_per_launch_mean"],
                    "source": "profiles/" + rec["summary"]}
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
                     "traffic": traffic, "traffic_unit": "HBM bytes per launch",
                     "traffic_per_step": (traffic * launches / args.steps) if traffic else None,
                     "kernel": "k_forward_wave<32> (per-k fused)",
                     "flop_model": "sum-factorised Bloch sums as executed + 24n^3 eigensolve + "
                                   "32n^3 rotations + 5n^2 curvature + 24 n N_F Fermi sums",
                     "flops_per_k_kernel": fpk_kernel, "flops_per_k_step": fpk,
                     "k_points_per_launch": per_launch_k,
                     "kernel_ms_per_step": k_ms / args.steps,
                     "launches_per_step": launches / args.steps,
                     "direct_sum_model": {"flops_per_k": fpk_direct,
                                          "tflops": fpk_direct * total_k / (ms / 1e3) / 1e12,
                                          "note": "Bloch sums counted as the direct sum over "
                                                  "all lattice vectors; not executed"},
                     "counters": counters},
        "step_tflops": fpk * total_k / (ms / 1e3) / 1e12,
        "sigma_checksum": float(sigma.sum().item()),
    }
    del plan
    if args.adjoint_reps > 0 and "adjoint" in legs:
        out["adjoint"] = measure_adjoint_cfg3(args.adjoint_reps)
    if args.large_reps > 0 and "n128" in legs:
        out["n128_slab"] = measure_cfg4_slab(reps=args.large_reps)
    if args.gf_reps > 0 and "gf" in legs:
        out["gf"] = measure_gf(args.gf_reps)
    if args.large_n_reps > 0 and "large_n" in legs:
        out["large_n"] = measure_large_n(args.large_n_reps)
    if args.batched_steps > 0 and "batched" in legs:
        out["batched"] = measure_batched(args.batched_steps, 1)
    if args.cpu_sample > 0 and "cpu" in legs:
        out["cpu_baseline"] = cpu_baseline(model, wl, ef[0], args.cpu_sample,
                                           args.cpu_single_sample)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
