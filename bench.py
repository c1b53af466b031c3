#!/usr/bin/env python3
"""Energyscape throughput on one MI355X.

Workload: one sensor, 32 microphones x 16384 samples (float32) per recording,
1500 directions on a Fibonacci hemisphere grid, 20-85 kHz matched-filter band,
envelope low-pass + decimation by 10 (1639 range bins); a step is one pass of
the whole pipeline (matched filter, beamformer, envelope) over a batch of
--frames recordings that share the plan.  Inputs are seeded synthetic echoes
of point reflectors, resident in HBM before timing starts.

Every beamformer path is timed and checked against the FP64 oracle on sampled
directions of every benchmarked energyscape:
  fp32_td       time-domain linear-interpolation DAS, FP32 (oracle mode td, bar 1e-5)
  bf16_mfma_fd  frequency-domain exact-delay DAS, per-bin GEMM on BF16 MFMA (oracle mode fd, bar 1e-3)
  fp32_fd       frequency-domain DAS with the per-bin GEMM on FP32 MFMA (oracle mode fd, bar 1e-5)
  bf16_mfma_td  time-domain DAS as a dense product on BF16 MFMA, weights and samples split (oracle
                mode td, bar 1e-3)
  bf16x2_mfma_td  the same with single-term BF16 samples: two products instead of three (bar 1e-3)
  f16_mfma_td   time-domain DAS on FP16 MFMA: fractional delays on a 1/2048-sample grid (exact FP16
                weights), FP16 samples scaled per frame: one product (oracle mode td, bar 1e-3)
The headline `value` is the fastest BF16-MFMA or FP32 path (the arithmetic the metric names)
whose error meets the metric's bar (rel. L2 <= 1e-3); the FP16 path is reported beside it.  `roofline` describes that path's dominant kernel, timed
live with HIP events on the stream it runs on; `cpu_baseline` is the oracle
itself on the host.
"""

from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "energyscapes/s at 32mic×16k×1500dir, BF16-MFMA vs FP32 path, rel err ≤1e-3"
METRIC_BAR = 1e-3
PEAK_FP32_VECTOR_TFLOPS = 157.3      # MI355X published FP32 vector peak (packed FP32)
PEAK_FP32_NOPACK_TFLOPS = 78.6       # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz, plain FMA
PEAK_BF16_MFMA_TFLOPS = 2500.0       # MI355X published dense BF16 matrix-core peak
CSRC = "paper_2208_10839_amd/csrc/"
PATHS = {
    # name: (mode, oracle mode, bar, dtype, dominant kernel(s) of beamform_envelope, kernel sources)
    "fp32_td": ("td", "td", 1e-5, "f32", "das_td_env_kernel",
                [CSRC + "k_das_td.hip", CSRC + "plan.hpp"]),
    "bf16_mfma_fd": ("fd_bf16", "fd", 1e-3, "bf16", "fd_gemm_kernel<bf16> + fd_ifft_env_kernel",
                     [CSRC + "k_fd.hip", CSRC + "fft_lds.hpp", CSRC + "plan.hpp"]),
    "fp32_fd": ("fd_fp32", "fd", 1e-5, "f32", "fd_gemm_kernel<fp32> + fd_ifft_env_kernel",
                [CSRC + "k_fd.hip", CSRC + "fft_lds.hpp", CSRC + "plan.hpp"]),
    "bf16_mfma_td": ("td_bf16", "td", 1e-3, "bf16", "das_mfma_env_kernel",
                     [CSRC + "k_das_mfma.hip", CSRC + "plan.hpp"]),
    "bf16x2_mfma_td": ("td_bf16x2", "td", 1e-3, "bf16", "das_mfma_env_kernel<single-term samples>",
                       [CSRC + "k_das_mfma.hip", CSRC + "plan.hpp"]),
    "f16_mfma_td": ("td_f16", "td", 1e-3, "f16", "das_mfma_env_kernel<FP16>",
                    [CSRC + "k_das_mfma.hip", CSRC + "plan.hpp"]),
}


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--frames", type=int, default=16, help="recordings per step (batch)")
    ap.add_argument("--paths", default=",".join(PATHS), help="comma-separated subset of " + ",".join(PATHS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-dirs", type=int, default=1500, help="directions in the oracle timing sample")
    ap.add_argument("--check-dirs", type=int, default=6, help="sampled directions per frame for the error")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="after timing, copy this many MiB device-to-device (a plain copy kernel of known "
                         "size for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    return ap.parse_args()


def sources_hash(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_record(kernel, kernel_hash):
    """HBM bytes per launch from rocprofv3 counters, if they were taken on this exact kernel source."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_c2_f16.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    k = rec.get("kernels", {}).get(kernel)
    if not k or k.get("kernel_sources_sha256_16") != kernel_hash:
        return None
    return k.get("hbm_bytes_per_launch")


def cpu_baseline(w, plan_P, n_dirs):
    """The FP64 oracle, as it is, on one recording: full matched filter + n_dirs directions (TD mode)."""
    import threadpoolctl

    import oracle
    with threadpoolctl.threadpool_limits(1):
        x = w.x[0].astype(np.float64)
        t0 = time.perf_counter()
        yhat = oracle.matched_filter(x, w.chirp, plan_P, w.fs, w.cfg.band)
        t_mf = time.perf_counter() - t0
        idx = np.linspace(0, w.dirs.shape[0] - 1, n_dirs).astype(int)
        R = w.cfg.decim
        h = oracle.default_lowpass(R)
        Q = oracle.num_range_bins(0, x.shape[1], R)
        t0 = time.perf_counter()
        Dl = oracle.delays(w.mic_pos, w.dirs[idx], w.fs, w.c)
        b = oracle.das_td(yhat, Dl, oracle.beam_window_indices(0, Q, R, h.size))
        oracle.envelope(b, h, Q, R)
        t_bf = time.perf_counter() - t0
    t_one = t_mf + t_bf * w.dirs.shape[0] / n_dirs
    return {"value": round(1.0 / t_one, 4), "unit": "energyscapes/s", "cores": 1, "kind": "oracle",
            "sample": (f"1 recording: full matched filter ({t_mf:.2f} s) + time-domain beamformer/envelope for "
                       f"{n_dirs} of {w.dirs.shape[0]} directions ({t_bf:.2f} s), scaled to all directions; "
                       f"numpy FP64, 1 thread"),
            "host_cpu": _cpu_name(), "host_nproc": os.cpu_count()}


def _cpu_name():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def sampled_errors(E, w, P, n_check, omode):
    import oracle
    rng = np.random.default_rng(11)
    errs = []
    for f in range(E.shape[0]):
        idx = np.sort(rng.choice(w.dirs.shape[0], n_check, replace=False))
        Eo = oracle.energyscape(w.x[f].astype(np.float64), w.chirp, w.mic_pos, w.dirs, fs=w.fs, c=w.c,
                                P=P, R=w.cfg.decim, band=w.cfg.band, mode=omode, dir_index=idx)
        errs.append(float(np.linalg.norm(E[f][idx] - Eo) / np.linalg.norm(Eo)))
    return errs


def time_calls(fn, K, stream):
    import torch
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(K):
        fn()
    ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / K


def run_path(name, w, x, args, stream):
    import torch

    from paper_2208_10839_amd import binding
    mode, omode, bar, dtype, kernel, srcs = PATHS[name]
    F, K, W = args.frames, args.steps, args.warmup
    M, N, D = w.x.shape[1], w.x.shape[2], w.dirs.shape[0]
    plan = binding.Plan(w.mic_pos, w.chirp, w.dirs, N, fs=w.fs, c=w.c, band=w.cfg.band,
                        decim=w.cfg.decim, mode=mode, max_frames=F)
    E = torch.empty((F, D, plan.Q), dtype=torch.float32, device=x.device)
    for _ in range(W):
        plan.energyscape(x, out=E)
    ms_step = time_calls(lambda: plan.energyscape(x, out=E), K, stream)
    mf = plan.matched_filter(x)
    for _ in range(2):
        plan.beamform_envelope(mf, out=E)
    ms_be = time_calls(lambda: plan.beamform_envelope(mf, out=E), K, stream)
    ms_mf = time_calls(lambda: plan.matched_filter(x, out=mf), K, stream)
    plan.energyscape(x, out=E)
    errs = sampled_errors(E.cpu().numpy(), w, plan.P, args.check_dirs, omode)
    G, Q, Kt, P = plan.G, plan.Q, plan.K, plan.P
    if omode == "td":
        flops = F * (8.0 * D * G * M + 2.0 * Kt * D * Q)
    else:
        # per-bin GEMM over the stored bins + one P-point inverse transform per direction + FIR
        flops = F * (8.0 * D * M * plan.band_bins + 5.0 * P * np.log2(P) * D + 2.0 * Kt * D * Q)
    achieved = flops / (ms_be / 1e3) / 1e12
    khash = sources_hash(srcs)
    # dense BF16 and FP16 matrix-core peaks are the same (2.5 PFLOP/s)
    mfma = mode.startswith("td_bf16") or mode == "td_f16"
    bound, peak = ("mfma", PEAK_BF16_MFMA_TFLOPS) if mfma else ("alu", PEAK_FP32_VECTOR_TFLOPS)
    roof = {"bound": bound, "kernel": kernel, "achieved": round(achieved, 3),
            "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4),
            "frac_of_plain_fma_peak": round(achieved / PEAK_FP32_NOPACK_TFLOPS, 4),
            "traffic": traffic_record(kernel, khash),
            "flop_per_launch": flops, "launch_ms": round(ms_be, 4), "kernel_sources_sha256_16": khash}
    mflop = plan.query(binding.Q_MATRIX_FLOP_PER_FRAME) * F
    if mflop:
        roof["matrix_flop_per_launch"] = mflop
        roof["matrix_pipe_frac"] = round(mflop / (ms_be / 1e3) / 1e12 / PEAK_BF16_MFMA_TFLOPS, 4)
    out = {"value": round(F / (ms_step / 1e3), 2), "unit": "energyscapes/s", "ms_per_step": round(ms_step, 4),
           "dtype": dtype, "mode": mode, "oracle_mode": omode, "bar": bar,
           "rel_err_sampled_max": max(errs), "rel_err_sampled_per_frame": [float(f"{e:.3e}") for e in errs],
           "meets_bar": max(errs) <= bar, "stages_ms_per_step": {"matched_filter": round(ms_mf, 4),
                                                                "beamform_envelope": round(ms_be, 4)},
           "roofline": roof}
    plan.close()
    return out


def plain_path(w, x, args, stream):
    """The plain single-sensor GPU path: F = 1, stage by stage, beam materialised in HBM, FP32 TD."""
    from paper_2208_10839_amd import binding
    plan1 = binding.Plan(w.mic_pos, w.chirp, w.dirs, w.x.shape[2], fs=w.fs, c=w.c, band=w.cfg.band,
                         decim=w.cfg.decim, mode="td", max_frames=1)
    x1 = x[:1].contiguous()
    mf1 = plan1.matched_filter(x1)
    b1 = plan1.beamform(mf1)
    e1 = plan1.envelope(b1)

    def step():
        plan1.matched_filter(x1, out=mf1)
        plan1.beamform(mf1, out=b1)
        plan1.envelope(b1, out=e1)
    ms = time_calls(step, args.steps, stream)
    plan1.close()
    return {"value": round(1e3 / ms, 2), "unit": "energyscapes/s",
            "what": "F=1, matched filter -> beam in HBM -> envelope, FP32 time-domain path"}


def network_path(args, stream):
    """The heterogeneous sensor network (8 sensors x 4 frames, own geometry, N in {8192, 16384, 32768},
    91-azimuth or 1500-direction grids) through sonar_energyscape_multi, eager and replayed from a graph,
    on the headline path's mode (TD_BF16X2: every sensor has 32 microphones)."""
    import torch

    from paper_2208_10839_amd import binding
    from workloads import synth
    net = synth.make_network()
    plans = [binding.Plan(w.mic_pos, w.chirp, w.dirs, w.x.shape[2], fs=w.fs, c=w.c, band=w.cfg.band,
                          max_frames=w.x.shape[0], mode="td_bf16x2") for w in net]
    xs = [torch.from_numpy(w.x).cuda() for w in net]
    outs = [torch.empty((w.x.shape[0], w.dirs.shape[0], pl.Q), dtype=torch.float32, device="cuda")
            for w, pl in zip(net, plans)]
    n_es = sum(w.x.shape[0] for w in net)
    for _ in range(3):
        binding.energyscape_multi(plans, xs, outs)
    ms_eager = time_calls(lambda: binding.energyscape_multi(plans, xs, outs), args.steps, stream)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        binding.energyscape_multi(plans, xs, outs)
    torch.cuda.synchronize()
    ms_graph = time_calls(g.replay, args.steps, torch.cuda.current_stream())
    for pl in plans:
        pl.close()
    return {"energyscapes_per_call": n_es, "mode": "td_bf16x2",
            "eager": {"value": round(n_es / (ms_eager / 1e3), 2), "unit": "energyscapes/s", "ms_per_call": round(ms_eager, 4)},
            "graph_replay": {"value": round(n_es / (ms_graph / 1e3), 2), "unit": "energyscapes/s",
                             "ms_per_call": round(ms_graph, 4)},
            "shapes": [[int(w.x.shape[2]), int(w.dirs.shape[0])] for w in net]}


def adjoint_path(args, stream):
    """One self-calibration step on the 32 mic x 16384 sample x 1500 direction x 10 frame workload
    (exact-phase plan): new positions, beamform + envelope, and dL/dp through sonar_energyscape_vjp."""
    import torch

    from paper_2208_10839_amd import binding
    from workloads import synth
    w = synth.make_calibration()
    F = w.x.shape[0]
    plan = binding.Plan(w.start_pos, w.chirp, w.dirs, w.x.shape[2], fs=w.fs, c=w.c, band=w.band,
                        decim=w.decim, mode="fd_fp32", max_frames=F)
    x = torch.from_numpy(w.x).cuda()
    mf = plan.matched_filter(x)
    beam = plan.beamform(mf)
    E = plan.envelope(beam)
    dE = torch.zeros_like(E)
    for f, fc in enumerate(w.cells):
        for d, q in fc:
            dE[f, d, q] = -1.0
    dpos = torch.empty((plan.M, 3), dtype=torch.float64, device="cuda")
    lib = binding.load()
    sh = binding._stream_handle(stream)
    pos = np.ascontiguousarray(w.start_pos)
    plan.enable_gradients()

    def step():
        binding._check(lib.sonar_plan_set_positions(plan._h, binding._ptr(pos), sh), "set_positions")
        plan.beamform(mf, out=beam)
        plan.envelope(beam, out=E)
        binding._check(lib.sonar_energyscape_vjp(plan._h, ctypes.c_void_p(mf.data_ptr()),
                                                 ctypes.c_void_p(beam.data_ptr()), ctypes.c_void_p(dE.data_ptr()),
                                                 F, None, None, ctypes.c_void_p(dpos.data_ptr()), sh), "vjp")
    for _ in range(2):
        step()
    ms = time_calls(step, args.steps, stream)
    plan.close()
    return {"what": "set_positions + beamform + envelope + dL/dp (FD exact-phase, FP32), 10 frames",
            "value": round(F / (ms / 1e3), 2), "unit": "frames/s", "ms_per_step": round(ms, 4)}


def pdm_path(args, stream, x_shape):
    """The PDM front end on the headline batch: 16 frames x 32 mics x 16384 samples x 10 ticks of packed
    1-bit words -> FP32 samples (sonar_pdm_demodulate), alone and followed by the headline energyscape."""
    import torch

    from paper_2208_10839_amd import binding
    from workloads import synth
    F, M, N = x_shape
    D = 10
    rng = np.random.default_rng(np.random.SeedSequence([7, 9, 9, 9]))
    words = torch.from_numpy(rng.integers(0, 2**32, size=(F, N * D, 1), dtype=np.uint64)
                             .astype(np.uint32).view(np.int32)).cuda()
    dem = binding.Pdm(M, N, D, max_frames=F)
    x = dem.demodulate(words)
    ms = time_calls(lambda: dem.demodulate(words, out=x), args.steps, stream)
    w = synth.make_workload("c2", frames=1)
    plan = binding.Plan(w.mic_pos, w.chirp, w.dirs, N, fs=w.fs, c=w.c, band=w.cfg.band, decim=w.cfg.decim,
                        mode="td_bf16x2", max_frames=F)
    E = torch.empty((F, w.dirs.shape[0], plan.Q), dtype=torch.float32, device="cuda")

    def step():
        dem.demodulate(words, out=x)
        plan.energyscape(x, out=E)
    for _ in range(2):
        step()
    ms_e2e = time_calls(step, args.steps, stream)
    algo_bytes = F * N * D * 4 + F * M * N * 4
    dem.close()
    plan.close()
    return {"what": "sonar_pdm_demodulate: 16 frames x 32 mics x 16384 samples x 10 PDM ticks, 321-tap FIR",
            "ms_per_call": round(ms, 4), "achieved_GBps": round(algo_bytes / (ms / 1e3) / 1e9, 1),
            "algorithmic_bytes": algo_bytes,
            "end_to_end_from_pdm": {"value": round(F / (ms_e2e / 1e3), 2), "unit": "energyscapes/s",
                                    "ms_per_step": round(ms_e2e, 4), "mode": "td_bf16x2"}}


def variants_path(w, x, args, stream):
    """The variant readings on the headline batch: integer delays (TD_NEAREST), 4-point Lagrange delays
    (TD_CUBIC) and the Butterworth IIR envelope (order 4, beam window in HBM, chunked scan), energyscapes/s."""
    from paper_2208_10839_amd import binding
    import torch
    F, N, D = x.shape[0], x.shape[2], w.dirs.shape[0]
    out = {}
    for name, mode, iir in (("td_nearest_fir", "td_nearest", 0), ("td_cubic_fir", "td_cubic", 0),
                            ("td_linear_iir4", "td", 2)):
        plan = binding.Plan(w.mic_pos, w.chirp, w.dirs, N, fs=w.fs, c=w.c, band=w.cfg.band, decim=w.cfg.decim,
                            mode=mode, max_frames=F)
        if iir:
            plan.set_envelope_iir(iir)
        E = torch.empty((F, D, plan.Q), dtype=torch.float32, device=x.device)
        for _ in range(2):
            plan.energyscape(x, out=E)
        ms = time_calls(lambda: plan.energyscape(x, out=E), args.steps, stream)
        out[name] = {"value": round(F / (ms / 1e3), 2), "unit": "energyscapes/s", "ms_per_step": round(ms, 4)}
        plan.close()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark measures one GPU; runs on several GPUs are not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    from workloads import synth

    F, K, W = args.frames, args.steps, args.warmup
    print(f"[bench] building workload c2 x {F} frames", file=sys.stderr, flush=True)
    w = synth.make_workload("c2", frames=F)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    x = torch.from_numpy(w.x).to(dev)
    torch.cuda.synchronize()

    results = {}
    for name in [p for p in args.paths.split(",") if p]:
        print(f"[bench] path {name}: warmup {W}, timing {K} steps, checking against the oracle",
              file=sys.stderr, flush=True)
        results[name] = run_path(name, w, x, args, stream)
    plain = plain_path(w, x, args, stream)
    print("[bench] sensor network batch", file=sys.stderr, flush=True)
    network = network_path(args, stream)
    print("[bench] self-calibration step (adjoint)", file=sys.stderr, flush=True)
    adjoint = adjoint_path(args, stream)
    print("[bench] PDM front end", file=sys.stderr, flush=True)
    pdm_fe = pdm_path(args, stream, tuple(x.shape))
    print("[bench] variant readings", file=sys.stderr, flush=True)
    variants = variants_path(w, x, args, stream)

    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * 1024 * 1024 // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # headline: the metric names the BF16-MFMA path against FP32, so FP16 paths are reported beside it
    ok = {k: v for k, v in results.items() if v["rel_err_sampled_max"] <= METRIC_BAR and v["dtype"] in ("bf16", "f32")}
    best = max(ok, key=lambda k: ok[k]["value"]) if ok else max(results, key=lambda k: results[k]["value"])
    head = results[best]
    fast = {k: v for k, v in results.items() if v["rel_err_sampled_max"] <= METRIC_BAR}
    fastest = max(fast, key=lambda k: fast[k]["value"]) if fast else best

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on the host", file=sys.stderr, flush=True)
        cpu = cpu_baseline(w, 32768, args.cpu_dirs)

    out = {
        "metric": METRIC, "value": head["value"], "unit": "energyscapes/s", "n_gpus": 1,
        "steps": K, "warmup": W, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": head["dtype"], "data": "synthetic",
        "config": {"workload": "32 mics x 16384 samples (f32) x 1500 Fibonacci directions, band 20-85 kHz, "
                               "R=10 (1639 range bins)",
                   "frames_per_step": F, "path": best, "fft_len": 32768},
        "roofline": head["roofline"],
        "cpu_baseline": cpu,
        "rel_err_sampled": {"max": head["rel_err_sampled_max"], "bar": METRIC_BAR,
                            "dirs_per_frame": args.check_dirs},
        "fastest_path_within_bar": {"path": fastest, "value": results[fastest]["value"],
                                    "dtype": results[fastest]["dtype"],
                                    "rel_err_sampled_max": results[fastest]["rel_err_sampled_max"]},
        "paths": results,
        "plain_single_sensor_gpu_path": plain,
        "sensor_network_batch": network,
        "self_calibration_step": adjoint,
        "pdm_front_end": pdm_fe,
        "variant_readings": variants,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
