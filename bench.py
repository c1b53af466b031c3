#!/usr/bin/env python3
"""Energyscape throughput on one MI355X.

Workload (the default, `--config c2`): one sensor, 32 microphones x 16384 samples (float32) per
recording, 1500 directions on a Fibonacci hemisphere grid, 20-85 kHz matched-filter band, envelope
low-pass + decimation by 10 (1639 range bins); a step is one pass of the whole pipeline (matched
filter, beamformer, envelope) over a batch of --frames recordings that share the plan.  Inputs are
seeded synthetic echoes of point reflectors, resident in HBM before timing starts.

Timing follows the paper's protocol (§5, Table 2: 100 measurements, mean (std)): per batch size
F in --sweep, --warmup untimed batches then --steps timed batches, each bracketed by HIP events on
the launch stream; energyscapes/s = F * steps / elapsed, latency per batch as mean (std), p50, p99.

Beamformer paths (each with its own oracle reading and bar):
  fp32_td         time-domain linear-interpolation DAS, FP32 (oracle td, bar 1e-5)
  bf16_mfma_fd    frequency-domain exact-delay DAS, per-bin GEMM on BF16 MFMA (oracle fd, bar 1e-3)
  fp32_fd         frequency-domain DAS, per-bin GEMM on FP32 MFMA (oracle fd, bar 1e-5)
  bf16x3_mfma_fd  the same GEMM on BF16 MFMA with split operands (hi*hi + hi*lo + lo*hi), the guaranteed-accuracy
                  BF16 mode (oracle fd, bar 1e-3; errors near FP32)
  bf16_mfma_td    time-domain DAS as a dense product on BF16 MFMA, weights and samples split (td, 1e-3)
  bf16x2_mfma_td  the same with single-term BF16 samples: two products instead of three (td, 1e-3)
  f16_mfma_td     time-domain DAS on FP16 MFMA, delays on a 1/2048-sample grid (td, 3e-4)
  bf16g_mfma_td   time-domain DAS on BF16 MFMA, delays on a 1/256-sample grid so both weights are exact
                  single BF16 terms: one product per sample plane (td, 1e-3)
The headline `value` is the fastest BF16-MFMA or FP32 path (the arithmetic the metric names) whose
error meets its own bar, at --frames recordings per batch; FP16 is reported beside it.
`roofline` describes that path's dominant kernel, timed live with HIP events on its stream.

`cpu_baseline` is the FP64 oracle on the host: one process on one thread over a bounded sample, and
a process pool over the frames of the batch (the paper's worker processes, §3); the energyscapes the
oracle computes there are the references of every error record (all directions of the first and
last frame of the batch for every path, every direction of every frame for the time-domain paths
when the pool ran over all frames, sampled directions otherwise; each record says which).

`--config c5` runs the stress configuration instead: 64 microphones in 7 cm, 65536 samples, 10000
directions, 16 recordings per batch; BF16-MFMA frequency-domain against FP32 time-domain.
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
PEAK_BF16_MFMA_TFLOPS = 2500.0       # MI355X published dense BF16 (and FP16) matrix-core peak
PEAK_FP32_MFMA_TFLOPS = 157.3        # MI355X published dense FP32 matrix-core peak
PEAK_HBM_GBPS = 8000.0
CSRC = "paper_2208_10839_amd/csrc/"
PATHS = {
    # name: (mode, oracle reading, bar, dtype, dominant kernel(s) of beamform_envelope, kernel sources)
    "fp32_td": ("td", "td", 1e-5, "f32", "das_td_env_kernel",
                [CSRC + "k_das_td.hip", CSRC + "plan.hpp"]),
    "bf16_mfma_fd": ("fd_bf16", "fd", 1e-3, "bf16", "fd_gemm_kernel<bf16> + fd_ifft_env_kernel",
                     [CSRC + "k_fd.hip", CSRC + "fft_lds.hpp", CSRC + "plan.hpp"]),
    "fp32_fd": ("fd_fp32", "fd", 1e-5, "f32", "fd_gemm_kernel<fp32> + fd_ifft_env_kernel",
                [CSRC + "k_fd.hip", CSRC + "fft_lds.hpp", CSRC + "plan.hpp"]),
    "bf16x3_mfma_fd": ("fd_bf16x3", "fd", 1e-3, "bf16", "fd_gemm_kernel<bf16x3> + fd_ifft_env_kernel",
                       [CSRC + "k_fd.hip", CSRC + "fft_lds.hpp", CSRC + "plan.hpp"]),
    "bf16_mfma_td": ("td_bf16", "td", 1e-3, "bf16", "das_mfma_env_kernel",
                     [CSRC + "k_das_mfma.hip", CSRC + "plan.hpp"]),
    "bf16x2_mfma_td": ("td_bf16x2", "td", 1e-3, "bf16", "das_mfma_env_kernel<single-term samples>",
                       [CSRC + "k_das_mfma.hip", CSRC + "plan.hpp"]),
    "f16_mfma_td": ("td_f16", "td", 3e-4, "f16", "das_mfma_env_kernel<FP16>",
                    [CSRC + "k_das_mfma.hip", CSRC + "plan.hpp"]),
    "bf16g_mfma_td": ("td_bf16g", "td", 1e-3, "bf16", "das_mfma_env_kernel<BF16, gridded single-term weights>",
                      [CSRC + "k_das_mfma.hip", CSRC + "plan.hpp"]),
}
# Table 2 of the paper (ms per measurement, mean (std), 100 measurements, other hardware; its chain
# also includes PDM demodulation): context for the direction-count lines, never a target
PAPER_TABLE2_MS = {
    "GTX 1080 Ti": {"90": [5.93, 0.66], "1850": [51.58, 6.38], "3000": [77.02, 7.81]},
    "GTX 1050": {"90": [23.03, 2.38], "1850": [202.37, 20.85], "3000": [323.83, 33.18]},
    "Jetson TX2": {"90": [68.40, 13.40], "1850": [585.24, 61.02], "3000": [911.47, 91.97]},
    "i7-7567U (NumPy/SciPy)": {"90": [132.53, 4.89], "1850": [976.33, 14.54], "3000": [1541.41, 20.30]},
}


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100, help="timed batches per measurement")
    ap.add_argument("--warmup", type=int, default=10, help="untimed batches before each measurement")
    ap.add_argument("--frames", type=int, default=16, help="recordings per batch of the headline figure")
    ap.add_argument("--sweep", default="1,4,16,64", help="batch sizes F timed for every path")
    ap.add_argument("--config", default="c2", choices=("c2", "c5"))
    ap.add_argument("--paths", default=",".join(PATHS), help="comma-separated subset of " + ",".join(PATHS))
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle (then no error records are available)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the sensor network, self-calibration, PDM, variant and direction-count lines")
    ap.add_argument("--cpu-dirs", type=int, default=300, help="directions in the single-thread oracle sample")
    ap.add_argument("--pool-workers", type=int, default=0, help="oracle pool processes (0: host CPUs, at most 16)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="after timing, copy this many MiB device-to-device (a plain copy kernel of known "
                         "size for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    return ap.parse_args()


def say(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


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


def _cpu_name():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# ----------------------------------------------------------------------------------------------
# GPU timing
# ----------------------------------------------------------------------------------------------

def time_batches(fn, K, W, stream):
    """W untimed calls, then K calls each bracketed by HIP events on `stream` (enqueued back to
    back).  Returns per-call milliseconds (numpy array) and the elapsed milliseconds over all K."""
    import torch
    for _ in range(W):
        fn()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(K + 1)]
    torch.cuda.synchronize()
    evs[0].record(stream)
    for i in range(K):
        fn()
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    per = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(K)])
    return per, float(evs[0].elapsed_time(evs[K]))


def stats(per, total_ms, F):
    return {"energyscapes_per_s": round(F * len(per) / (total_ms / 1e3), 2),
            "batch_ms": {"mean": round(float(per.mean()), 4), "std": round(float(per.std()), 4),
                         "p50": round(float(np.percentile(per, 50)), 4),
                         "p99": round(float(np.percentile(per, 99)), 4)},
            "batches": len(per)}


def time_calls(fn, K, stream):
    per, total = time_batches(fn, K, 0, stream)
    return total / K


def make_plan(binding, w, mode, F, dirs=None, **kw):
    return binding.Plan(w.mic_pos, w.chirp, w.dirs if dirs is None else dirs, w.x.shape[2], fs=w.fs, c=w.c,
                        band=w.cfg.band, decim=w.cfg.decim, mode=mode, max_frames=F, **kw)


def run_path(name, w, x, args, stream, sweep):
    """Throughput sweep over batch sizes, stage times and roofline at --frames, and the energyscapes
    of the --frames batch (host copy, for the error records)."""
    import torch

    from paper_2208_10839_amd import binding
    mode, omode, bar, dtype, kernel, srcs = PATHS[name]
    F, K, W = args.frames, args.steps, args.warmup
    M, N, D = w.x.shape[1], w.x.shape[2], w.dirs.shape[0]
    Fmax = max(sweep + [F])
    plan = make_plan(binding, w, mode, Fmax)
    E = torch.empty((Fmax, D, plan.Q), dtype=torch.float32, device=x.device)
    by_f = {}
    for Fb in sweep:
        xb, Eb = x[:Fb], E[:Fb]
        per, tot = time_batches(lambda: plan.energyscape(xb, out=Eb), K, W, stream)
        by_f[str(Fb)] = stats(per, tot, Fb)
    xf, Ef = x[:F], E[:F]
    per, tot = time_batches(lambda: plan.energyscape(xf, out=Ef), K, W, stream)
    head = stats(per, tot, F)
    mf = plan.matched_filter(xf)
    ms_be = time_batches(lambda: plan.beamform_envelope(mf, out=Ef), K, 2, stream)[1] / K
    ms_mf = time_batches(lambda: plan.matched_filter(xf, out=mf), K, 2, stream)[1] / K
    plan.energyscape(xf, out=Ef)
    E_host = Ef.cpu().numpy()
    G, Q, Kt, P = plan.G, plan.Q, plan.K, plan.P
    if omode == "td":
        flops = F * (8.0 * D * G * M + 2.0 * Kt * D * Q)
    else:
        # per-bin GEMM over the stored bins + one P-point inverse transform per direction + FIR
        flops = F * (8.0 * D * M * plan.band_bins + 5.0 * P * np.log2(P) * D + 2.0 * Kt * D * Q)
    achieved = flops / (ms_be / 1e3) / 1e12
    khash = sources_hash(srcs)
    mfma = mode.startswith("td_bf16") or mode == "td_f16"   # td_bf16, td_bf16x2, td_bf16g, td_f16
    bound, peak = ("mfma", PEAK_BF16_MFMA_TFLOPS) if mfma else ("alu", PEAK_FP32_VECTOR_TFLOPS)
    roof = {"bound": bound, "kernel": kernel, "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4), "frac_of_plain_fma_peak": round(achieved / PEAK_FP32_NOPACK_TFLOPS, 4),
            "traffic": traffic_record(kernel, khash), "flop_per_launch": flops, "launch_ms": round(ms_be, 4),
            "kernel_sources_sha256_16": khash}
    if omode == "fd":
        # the two kernels of beamform_envelope against their own roofs: the per-bin GEMM alone
        # (sonar_beam_spectrum) on the matrix cores, the inverse + envelope (the rest) on the vector ALUs
        Bs = plan.beam_spectrum(mf)
        ms_gemm = time_batches(lambda: plan.beam_spectrum(mf, out=Bs), K, 2, stream)[1] / K
        ms_inv = max(ms_be - ms_gemm, 1e-6)
        gemm_flops = F * 8.0 * D * M * plan.band_bins
        inv_flops = F * (5.0 * P * np.log2(P) * D + 2.0 * Kt * D * Q)
        gpeak = PEAK_FP32_MFMA_TFLOPS if mode == "fd_fp32" else PEAK_BF16_MFMA_TFLOPS
        roof["kernels"] = {
            "fd_gemm_kernel": {"bound": "mfma", "achieved": round(gemm_flops / (ms_gemm / 1e3) / 1e12, 3),
                               "peak": gpeak, "unit": "TFLOP/s",
                               "frac": round(gemm_flops / (ms_gemm / 1e3) / 1e12 / gpeak, 4),
                               "flop_per_launch": gemm_flops, "launch_ms": round(ms_gemm, 4),
                               "input_bytes": int(F * plan.band_bins * M * 8),
                               "output_bytes": int(F * D * plan.query(binding.Q_BEAM_SPEC_STRIDE) * 8)},
            "fd_ifft_env_kernel": {"bound": "alu", "achieved": round(inv_flops / (ms_inv / 1e3) / 1e12, 3),
                                   "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                                   "frac": round(inv_flops / (ms_inv / 1e3) / 1e12 / PEAK_FP32_VECTOR_TFLOPS, 4),
                                   "flop_per_launch": inv_flops, "launch_ms": round(ms_inv, 4),
                                   "timing": "beamform_envelope minus the GEMM alone",
                                   "phase_len": plan.query(binding.Q_FD_PHASE_LEN),
                                   "fused": bool(plan.query(binding.Q_FD_FUSED))}}
        del Bs
    mflop = plan.query(binding.Q_MATRIX_FLOP_PER_FRAME) * F
    if mflop:
        roof["matrix_flop_per_launch"] = mflop
        roof["matrix_pipe_frac"] = round(mflop / (ms_be / 1e3) / 1e12 / PEAK_BF16_MFMA_TFLOPS, 4)
    out = {"value": head["energyscapes_per_s"], "unit": "energyscapes/s",
           "ms_per_step": head["batch_ms"]["mean"], "latency": head, "sweep": by_f,
           "dtype": dtype, "mode": mode, "oracle_mode": omode, "bar": bar,
           "stages_ms_per_step": {"matched_filter": round(ms_mf, 4), "beamform_envelope": round(ms_be, 4)},
           "roofline": roof}
    plan.close()
    return out, E_host


def pcie_path(name, w, x, args, stream):
    """End to end with the host: pinned H2D copy of x, the energyscape, D2H copy of E, per batch of
    --frames recordings on one stream (serial: the copies are not overlapped with compute)."""
    import torch

    from paper_2208_10839_amd import binding
    mode = PATHS[name][0]
    F = args.frames
    plan = make_plan(binding, w, mode, F)
    xh = torch.from_numpy(np.ascontiguousarray(w.x[:F])).pin_memory()
    Eh = torch.empty((F, w.dirs.shape[0], plan.Q), dtype=torch.float32).pin_memory()
    xd = torch.empty_like(xh, device=x.device)
    Ed = torch.empty(tuple(Eh.shape), dtype=torch.float32, device=x.device)

    def step():
        xd.copy_(xh, non_blocking=True)
        plan.energyscape(xd, out=Ed)
        Eh.copy_(Ed, non_blocking=True)
    per, tot = time_batches(step, args.steps, args.warmup, stream)
    plan.close()
    out = stats(per, tot, F)
    out.update({"path": name, "frames_per_batch": F,
                "bytes_h2d_per_batch": int(xh.numel() * 4), "bytes_d2h_per_batch": int(Eh.numel() * 4),
                "what": "pinned H2D of x, energyscape, D2H of E, serial on one stream"})
    return out


def plain_path(w, x, args, stream):
    """The plain single-sensor GPU path: F = 1, stage by stage, beam materialised in HBM, FP32 TD."""
    from paper_2208_10839_amd import binding
    plan1 = make_plan(binding, w, "td", 1)
    x1 = x[:1]
    mf1 = plan1.matched_filter(x1)
    b1 = plan1.beamform(mf1)
    e1 = plan1.envelope(b1)

    def step():
        plan1.matched_filter(x1, out=mf1)
        plan1.beamform(mf1, out=b1)
        plan1.envelope(b1, out=e1)
    per, tot = time_batches(step, args.steps, args.warmup, stream)
    plan1.close()
    out = stats(per, tot, 1)
    out.update({"value": out["energyscapes_per_s"], "unit": "energyscapes/s",
                "what": "F=1, matched filter -> beam in HBM -> envelope, FP32 time-domain path"})
    return out


def ctx_grids():
    from workloads import synth
    return {"91": synth.azimuth_grid(91), "1850": synth.restricted_grid(1850), "3000": synth.fibonacci_hemisphere(3000)}


def direction_count_lines(w, x, args, stream, names, grids):
    """The direction counts of Table 2 (90 -> 91 azimuths, 1850 within +-45 deg, 3000 on the
    hemisphere) for the given paths, at F = 1 (one measurement at a time, as in the paper) and at
    --frames; the energyscapes of frame 0 are kept for the error records."""
    import torch

    from paper_2208_10839_amd import binding
    out, keep = {}, {}
    for name in names:
        mode = PATHS[name][0]
        out[name] = {}
        for g, dirs in grids.items():
            plan = make_plan(binding, w, mode, args.frames, dirs=dirs)
            E = torch.empty((args.frames, dirs.shape[0], plan.Q), dtype=torch.float32, device=x.device)
            rec = {}
            for Fb in (1, args.frames):
                xb, Eb = x[:Fb], E[:Fb]
                per, tot = time_batches(lambda: plan.energyscape(xb, out=Eb), args.steps, args.warmup, stream)
                rec[f"F{Fb}"] = stats(per, tot, Fb)
            plan.energyscape(x[:1], out=E[:1])
            keep[(name, g)] = E[0].cpu().numpy()
            out[name][g] = {"directions": int(dirs.shape[0]), **rec}
            plan.close()
    return out, keep


def network_path(args, stream, mode):
    """The heterogeneous sensor network (8 sensors x 4 frames, own geometry, N in {8192, 16384, 32768},
    91-azimuth or 1500-direction grids) through sonar_energyscape_multi (one persistent beamformer launch
    for the MFMA time-domain modes), eager and replayed from a graph, on the headline candidate's mode
    (every sensor has 32 microphones); beside it the items one by one (sonar_energyscape_batch per item on
    one stream) and the network with FP16 samples."""
    import torch

    from paper_2208_10839_amd import binding
    from workloads import synth
    net = synth.make_network()
    plans = [binding.Plan(w.mic_pos, w.chirp, w.dirs, w.x.shape[2], fs=w.fs, c=w.c, band=w.cfg.band,
                          max_frames=w.x.shape[0], mode=mode) for w in net]
    xs = [torch.from_numpy(w.x).cuda() for w in net]
    outs = [torch.empty((w.x.shape[0], w.dirs.shape[0], pl.Q), dtype=torch.float32, device="cuda")
            for w, pl in zip(net, plans)]
    n_es = sum(w.x.shape[0] for w in net)
    per, tot = time_batches(lambda: binding.energyscape_multi(plans, xs, outs), args.steps, args.warmup, stream)
    eager = stats(per, tot, n_es)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        binding.energyscape_multi(plans, xs, outs)
    torch.cuda.synchronize()
    per, tot = time_batches(g.replay, args.steps, 2, torch.cuda.current_stream())
    graph = stats(per, tot, n_es)

    def one_by_one():
        for pl, x, o in zip(plans, xs, outs):
            pl.energyscape(x, out=o)
    per, tot = time_batches(one_by_one, args.steps, args.warmup, stream)
    single = stats(per, tot, n_es)
    for pl in plans:
        pl.close()
    # FP16 samples (the configuration's input precision) on the same mode
    plans16 = [binding.Plan(w.mic_pos, w.chirp, w.dirs, w.x.shape[2], fs=w.fs, c=w.c, band=w.cfg.band,
                            max_frames=w.x.shape[0], mode=mode, sample_dtype="f16") for w in net]
    xs16 = [x.half() for x in xs]
    per, tot = time_batches(lambda: binding.energyscape_multi(plans16, xs16, outs), args.steps, args.warmup, stream)
    eager16 = stats(per, tot, n_es)
    for pl in plans16:
        pl.close()
    return {"energyscapes_per_call": n_es, "mode": mode,
            "items_one_by_one": {"value": single["energyscapes_per_s"], "unit": "energyscapes/s", **single},
            "fp16_samples_eager": {"value": eager16["energyscapes_per_s"], "unit": "energyscapes/s", **eager16},
            "eager": {"value": eager["energyscapes_per_s"], "unit": "energyscapes/s", **eager},
            "graph_replay": {"value": graph["energyscapes_per_s"], "unit": "energyscapes/s", **graph},
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
    ms = time_calls(step, max(3, args.steps // 10), stream)

    # the same loss read from its cells only (sonar_energyscape_cells): E at the reflector cells and
    # dL/dp without the beam window
    cl = [(f, d, q) for f, fc in enumerate(w.cells) for d, q in fc]
    cells = torch.tensor(cl, dtype=torch.int32, device="cuda")
    wts = torch.full((len(cl),), -1.0, dtype=torch.float32, device="cuda")
    Ec = torch.empty((len(cl),), dtype=torch.float32, device="cuda")

    def step_cells():
        binding._check(lib.sonar_plan_set_positions(plan._h, binding._ptr(pos), sh), "set_positions")
        binding._check(lib.sonar_energyscape_cells(plan._h, ctypes.c_void_p(mf.data_ptr()),
                                                   ctypes.c_void_p(cells.data_ptr()), len(cl),
                                                   ctypes.c_void_p(wts.data_ptr()), F, ctypes.c_void_p(Ec.data_ptr()),
                                                   ctypes.c_void_p(dpos.data_ptr()), sh), "cells")
    for _ in range(2):
        step_cells()
    ms_c = time_calls(step_cells, max(10, args.steps // 2), stream)
    plan.close()
    return {"what": "set_positions + beamform + envelope + dL/dp (FD exact-phase, FP32), 10 frames",
            "value": round(F / (ms / 1e3), 2), "unit": "frames/s", "ms_per_step": round(ms, 4),
            "cells_path": {"what": f"set_positions + E and dL/dp at the {len(cl)} reflector cells only "
                                   "(sonar_energyscape_cells), same loss", "value": round(F / (ms_c / 1e3), 2),
                           "unit": "frames/s", "ms_per_step": round(ms_c, 4)}}


def pdm_path(args, stream, x_shape, mode):
    """The PDM front end on the headline batch: F frames x 32 mics x 16384 samples x 10 ticks of packed
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
    plan = make_plan(binding, w, mode, F)
    E = torch.empty((F, w.dirs.shape[0], plan.Q), dtype=torch.float32, device="cuda")

    def step():
        dem.demodulate(words, out=x)
        plan.energyscape(x, out=E)
    per, tot = time_batches(step, args.steps, 2, stream)
    e2e = stats(per, tot, F)
    algo_bytes = F * N * D * 4 + F * M * N * 4
    dem.close()
    plan.close()
    return {"what": f"sonar_pdm_demodulate: {F} frames x {M} mics x {N} samples x {D} PDM ticks, 321-tap FIR",
            "ms_per_call": round(ms, 4), "achieved_GBps": round(algo_bytes / (ms / 1e3) / 1e9, 1),
            "algorithmic_bytes": algo_bytes,
            "end_to_end_from_pdm": {"value": e2e["energyscapes_per_s"], "unit": "energyscapes/s",
                                    "ms_per_step": e2e["batch_ms"]["mean"], "mode": mode}}


def variants_path(w, x, args, stream):
    """The variant readings on the headline batch: integer delays (TD_NEAREST), 4-point Lagrange delays
    (TD_CUBIC) and the Butterworth IIR envelope (order 4, beam window in HBM, chunked scan), energyscapes/s."""
    import torch

    from paper_2208_10839_amd import binding
    F, D = args.frames, w.dirs.shape[0]
    xf = x[:F]
    out = {}
    for name, mode, iir in (("td_nearest_fir", "td_nearest", 0), ("td_cubic_fir", "td_cubic", 0),
                            ("td_linear_iir4", "td", 2)):
        plan = make_plan(binding, w, mode, F)
        if iir:
            plan.set_envelope_iir(iir)
        E = torch.empty((F, D, plan.Q), dtype=torch.float32, device=x.device)
        per, tot = time_batches(lambda: plan.energyscape(xf, out=E), max(10, args.steps // 5), 2, stream)
        s = stats(per, tot, F)
        out[name] = {"value": s["energyscapes_per_s"], "unit": "energyscapes/s", "ms_per_step": s["batch_ms"]["mean"]}
        plan.close()
    return out


# ----------------------------------------------------------------------------------------------
# The oracle on the host (the only part of this script that runs it)
# ----------------------------------------------------------------------------------------------

def cpu_baseline_leg(w, P, F, args, ctx):
    """The FP64 oracle as it stands, timed on the host:
      * one process, one thread: frame 0, full matched filter + a stratified sample of --cpu-dirs
        directions in each reading (td, fd), stage by stage, scaled to all directions; also the
        direction counts of Table 2 (91 / 1850 / 3000) on a sample of 24 directions each;
      * a process pool over the F frames of the batch (time-domain reading, every direction):
        frames/s of the pool, per-frame seconds mean (std);
      * frequency-domain reading, every direction of frames 0 and F-1 and 24 directions of the others
        (pool, split by directions), for the error records.
    Returns (cpu_baseline record, references) with references[(reading, frame)] = (dir_index or None, E)."""
    import threadpoolctl

    import oracle
    from oracle import pool
    R, band = w.cfg.decim, w.cfg.band
    D = w.dirs.shape[0]
    refs = {}
    single = {}
    with threadpoolctl.threadpool_limits(1):
        x0 = w.x[0].astype(np.float64)
        idx = np.linspace(0, D - 1, min(args.cpu_dirs, D)).astype(int)
        for reading in ("td", "fd"):
            t = {}
            t0 = time.perf_counter()
            E = oracle.energyscape(x0, w.chirp, w.mic_pos, w.dirs, fs=w.fs, c=w.c, P=P, R=R, band=band,
                                   mode=reading, dir_index=idx, timings=t)
            wall = time.perf_counter() - t0
            scale = D / idx.size
            per_es = t["matched_filter"] + (t["beamform"] + t["envelope"]) * scale
            single[reading] = {"s_per_energyscape": round(per_es, 3),
                               "value": round(1.0 / per_es, 4), "unit": "energyscapes/s",
                               "stages_s": {"matched_filter": round(t["matched_filter"], 3),
                                            "beamform": round(t["beamform"] * scale, 3),
                                            "envelope": round(t["envelope"] * scale, 3)},
                               "sample": f"frame 0: full matched filter, {idx.size} of {D} directions "
                                         f"({wall:.1f} s), beamformer and envelope scaled to all directions"}
            refs[("s_" + reading, 0)] = (idx, E)
        ctx_single = {}
        for g, dirs in ctx.items():
            cidx = np.linspace(0, dirs.shape[0] - 1, min(24, dirs.shape[0])).astype(int)
            t = {}
            E = oracle.energyscape(x0, w.chirp, w.mic_pos, dirs, fs=w.fs, c=w.c, P=P, R=R, band=band, mode="td",
                                   dir_index=cidx, timings=t)
            scale = dirs.shape[0] / cidx.size
            ms = 1e3 * (t["matched_filter"] + (t["beamform"] + t["envelope"]) * scale)
            ctx_single[g] = {"directions": int(dirs.shape[0]), "ms_per_energyscape": round(ms, 1),
                             "sample": f"{cidx.size} directions, scaled"}
            refs[("ctx_" + g, 0)] = (cidx, E)
    nw = args.pool_workers or pool.default_workers()
    jobs = [pool.Job(x=w.x[f], chirp=w.chirp, mic_pos=w.mic_pos, dirs=w.dirs, fs=w.fs, c=w.c, P=P, R=R,
                     band=band, mode="td") for f in range(F)]
    say(f"oracle pool: {F} frames x {D} directions (td) on {nw} processes")
    Es, times, wall = pool.run(jobs, workers=nw, split=1 if F >= nw else max(1, nw // F))
    for f in range(F):
        refs[("td", f)] = (None, Es[f])
    per_frame = np.array([t["total"] for t in times])
    stage_mean = {k: round(float(np.mean([t[k] for t in times])), 3) for k in ("matched_filter", "beamform", "envelope")}
    pool_rec = {"value": round(F / wall, 4), "unit": "energyscapes/s", "cores": nw, "frames": F,
                "wall_s": round(wall, 2),
                "s_per_energyscape_in_a_worker": {"mean": round(float(per_frame.mean()), 3),
                                                  "std": round(float(per_frame.std()), 3)},
                "stages_s_mean": stage_mean,
                "sample": f"all {F} frames of the batch, every direction, time-domain reading, one frame per task"}
    fd_jobs, fd_keys = [], []
    sidx = np.sort(np.random.default_rng(11).choice(D, min(24, D), replace=False))
    for f in range(F):
        full = f in (0, F - 1)
        fd_jobs.append(pool.Job(x=w.x[f], chirp=w.chirp, mic_pos=w.mic_pos, dirs=w.dirs, fs=w.fs, c=w.c, P=P, R=R,
                                band=band, mode="fd", dir_index=None if full else sidx))
        fd_keys.append((f, None if full else sidx))
    say(f"oracle pool: frequency-domain reading for the error records on {nw} processes")
    Efd, _, wall_fd = pool.run(fd_jobs, workers=nw, split=max(1, nw // 2))
    for (f, ix), E in zip(fd_keys, Efd):
        refs[("fd", f)] = (ix, E)
    rec = {"value": single["td"]["value"], "unit": "energyscapes/s", "cores": 1, "kind": "oracle",
           "sample": single["td"]["sample"] + "; numpy FP64, 1 thread (time-domain reading)",
           "single_thread": single, "pool": pool_rec, "direction_counts_single_thread_td": ctx_single,
           "fd_reference_wall_s": round(wall_fd, 2),
           "host_cpu": _cpu_name(), "host_nproc": os.cpu_count(), "pool_processes": nw}
    return rec, refs


def error_record(E, refs, reading, F, bar):
    """Relative L2 per frame against the oracle references of that reading (the bar applies to it),
    and the largest error over the largest reference value, max|E - E_ref| / max|E_ref|; says which
    frames were checked on every direction and which on sampled directions."""
    per, peak, full, sampled = [], [], [], []
    for f in range(F):
        if (reading, f) not in refs:
            continue
        ix, Eo = refs[(reading, f)]
        got = E[f] if ix is None else E[f][ix]
        ref = float(np.linalg.norm(Eo))
        per.append(float(np.linalg.norm(got - Eo)) / ref if ref > 0 else float(np.linalg.norm(got - Eo)))
        top = float(np.max(np.abs(Eo)))
        dev = float(np.max(np.abs(got - Eo)))
        peak.append(dev / top if top > 0 else dev)
        (full if ix is None else sampled).append(f)
    if not per:
        return None
    return {"max": max(per), "per_frame": [float(f"{e:.3e}") for e in per], "bar": bar,
            "meets_bar": max(per) <= bar, "max_abs_over_max_ref": float(f"{max(peak):.3e}"),
            "frames_all_directions": full,
            "frames_sampled_directions": sampled,
            "sampled_directions_per_frame": int(len(refs[(reading, sampled[0])][0])) if sampled else 0}


# ----------------------------------------------------------------------------------------------

def main_c2(args):
    import torch

    from workloads import synth
    F, K, W = args.frames, args.steps, args.warmup
    sweep = sorted(set(int(s) for s in args.sweep.split(",") if s))
    Fmax = max(sweep + [F])
    say(f"building workload c2 x {Fmax} frames")
    w = synth.make_workload("c2", frames=Fmax)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    x = torch.from_numpy(w.x).to(dev)
    torch.cuda.synchronize()

    results, outputs = {}, {}
    for name in [p for p in args.paths.split(",") if p]:
        say(f"path {name}: F in {sweep}, {W} warm-up + {K} timed batches each")
        results[name], outputs[name] = run_path(name, w, x, args, stream, sweep)
    extras = {}
    say("plain single-sensor path")
    extras["plain_single_sensor_gpu_path"] = plain_path(w, x, args, stream)
    # the extras run on the fastest BF16 path (the headline candidate; its error is checked below)
    bf16_paths = [n for n in results if results[n]["dtype"] == "bf16"]
    fast_bf16 = max(bf16_paths, key=lambda n: results[n]["value"]) if bf16_paths else None
    ok0 = [n for n in (fast_bf16, "fp32_td") if n in results]
    xmode = PATHS[fast_bf16][0] if fast_bf16 else "td_bf16x2"
    ctx = ctx_grids()
    ctx_keep = {}
    if not args.no_extras:
        say("PCIe-inclusive end to end")
        extras["end_to_end_pcie"] = pcie_path(ok0[0] if ok0 else next(iter(results)), w, x, args, stream)
        say("direction counts of Table 2")
        extras["direction_counts"], ctx_keep = direction_count_lines(w, x, args, stream, ok0, ctx)
        say("sensor network batch")
        extras["sensor_network_batch"] = network_path(args, stream, xmode)
        say("self-calibration step (adjoint)")
        extras["self_calibration_step"] = adjoint_path(args, stream)
        say("PDM front end")
        extras["pdm_front_end"] = pdm_path(args, stream, (F, w.x.shape[1], w.x.shape[2]), xmode)
        say("variant readings")
        extras["variant_readings"] = variants_path(w, x, args, stream)

    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * 1024 * 1024 // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    cpu, refs = None, {}
    if not args.no_cpu_baseline:
        say("FP64 oracle on the host (single thread, then a process pool)")
        cpu, refs = cpu_baseline_leg(w, 32768, F, args, ctx)
    for name, r in results.items():
        r["rel_err"] = error_record(outputs[name], refs, r["oracle_mode"], F, r["bar"])
    for name, lines in extras.get("direction_counts", {}).items():
        for g, rec in lines.items():
            if ("ctx_" + g, 0) in refs:
                ix, Eo = refs[("ctx_" + g, 0)]
                e = float(np.linalg.norm(ctx_keep[(name, g)][ix] - Eo) / np.linalg.norm(Eo))
                rec["rel_err_frame0_sampled"] = {"value": float(f"{e:.3e}"), "directions": int(len(ix)),
                                                 "bar": PATHS[name][2], "meets_bar": e <= PATHS[name][2]}
    if extras.get("direction_counts"):
        extras["direction_counts"]["paper_table2_ms_context"] = PAPER_TABLE2_MS

    def meets(r):
        return r["rel_err"] is None or r["rel_err"]["meets_bar"]
    ok = {k: v for k, v in results.items() if meets(v) and v["dtype"] in ("bf16", "f32")}
    best = max(ok, key=lambda k: ok[k]["value"]) if ok else max(results, key=lambda k: results[k]["value"])
    head = results[best]
    fast = {k: v for k, v in results.items() if meets(v)}
    fastest = max(fast, key=lambda k: fast[k]["value"]) if fast else best

    out = {
        "metric": METRIC, "value": head["value"], "unit": "energyscapes/s", "n_gpus": 1,
        "steps": K, "warmup": W, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": head["dtype"], "data": "synthetic",
        "config": {"workload": "32 mics x 16384 samples (f32) x 1500 Fibonacci directions, band 20-85 kHz, "
                               "R=10 (1639 range bins)",
                   "frames_per_step": F, "path": best, "fft_len": 32768},
        "roofline": head["roofline"],
        "cpu_baseline": cpu,
        "rel_err": head["rel_err"],
        "latency": head["latency"],
        "fastest_path_within_bar": {"path": fastest, "value": results[fastest]["value"],
                                    "dtype": results[fastest]["dtype"],
                                    "rel_err_max": (results[fastest]["rel_err"] or {}).get("max")},
        "paths": results,
        **extras,
    }
    print(json.dumps(out), flush=True)


def main_c5(args):
    """Stress configuration: 64 mics x 65536 samples x 10000 directions, 16 recordings per batch:
    BF16-MFMA frequency-domain path against the FP32 time-domain path, with the error of frame 0
    against the oracle on a stated direction subset."""
    import torch

    from paper_2208_10839_amd import binding
    from workloads import synth
    F = 16
    K, W = min(args.steps, 10), min(args.warmup, 2)
    say(f"building workload c5 x {F} frames")
    w = synth.make_workload("c5", frames=F)
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    x = torch.from_numpy(w.x).cuda()
    D = w.dirs.shape[0]
    res, outs = {}, {}
    for name in [p for p in args.paths.split(",") if p in PATHS]:
        mode = PATHS[name][0]
        try:
            plan = make_plan(binding, w, mode, F)
        except binding.SonarError as e:
            res[name] = {"error": str(e)}
            continue
        E = torch.empty((F, D, plan.Q), dtype=torch.float32, device="cuda")
        say(f"c5 path {name}: {W} warm-up + {K} timed batches of {F}")
        per, tot = time_batches(lambda: plan.energyscape(x, out=E), K, W, stream)
        res[name] = {"mode": mode, "bar": PATHS[name][2], "dtype": PATHS[name][3], "oracle_mode": PATHS[name][1],
                     **stats(per, tot, F), "fft_len": plan.P}
        outs[name] = E[0].cpu().numpy()
        plan.close()
    cpu = None
    if not args.no_cpu_baseline:
        import threadpoolctl

        import oracle
        from oracle import pool
        idx = np.sort(np.random.default_rng(5).choice(D, 1000, replace=False))
        refs = {}
        nw = args.pool_workers or pool.default_workers()
        for reading in ("td", "fd"):
            job = pool.Job(x=w.x[0], chirp=w.chirp, mic_pos=w.mic_pos, dirs=w.dirs, fs=w.fs, c=w.c, P=131072,
                           R=w.cfg.decim, band=w.cfg.band, mode=reading, dir_index=idx)
            say(f"c5 oracle {reading}: frame 0, {idx.size} directions on {nw} processes")
            Es, times, wall = pool.run([job], workers=nw, split=nw)
            refs[reading] = Es[0]
            cpu = cpu or {}
            cpu[reading] = {"wall_s": round(wall, 2), "cores": nw,
                            "sample": f"frame 0, {idx.size} of {D} directions",
                            "value": round(idx.size / D / wall, 5), "unit": "energyscapes/s (scaled)"}
        with threadpoolctl.threadpool_limits(1):
            t = {}
            sub = idx[:40]
            oracle.energyscape(w.x[0].astype(np.float64), w.chirp, w.mic_pos, w.dirs, fs=w.fs, c=w.c, P=131072,
                               R=w.cfg.decim, band=w.cfg.band, mode="td", dir_index=sub, timings=t)
            s = t["matched_filter"] + (t["beamform"] + t["envelope"]) * D / sub.size
            cpu["single_thread_td"] = {"value": round(1.0 / s, 6), "unit": "energyscapes/s", "cores": 1,
                                       "sample": f"frame 0, full matched filter + {sub.size} directions, scaled"}
        for name, E0 in outs.items():
            Eo = refs[res[name]["oracle_mode"]]
            e = float(np.linalg.norm(E0[idx] - Eo) / np.linalg.norm(Eo))
            res[name]["rel_err_frame0"] = {"value": float(f"{e:.3e}"), "directions": int(idx.size),
                                           "bar": res[name]["bar"], "meets_bar": e <= res[name]["bar"]}
    ok = {k: v for k, v in res.items() if "energyscapes_per_s" in v and v["dtype"] in ("bf16", "f32")
          and v.get("rel_err_frame0", {"meets_bar": True})["meets_bar"]}
    best = max(ok, key=lambda k: ok[k]["energyscapes_per_s"]) if ok else None
    out = {"metric": "energyscapes/s at 64mic×64k×10000dir (stress configuration)",
           "value": ok[best]["energyscapes_per_s"] if best else None, "unit": "energyscapes/s", "n_gpus": 1,
           "steps": K, "warmup": W, "ms_per_step": ok[best]["batch_ms"]["mean"] if best else None,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": ok[best]["dtype"] if best else None, "data": "synthetic",
           "config": {"workload": "64 mics in 7 cm x 65536 samples (f32) x 10000 Fibonacci directions, band "
                                  "20-85 kHz, R=10 (6554 range bins), 50 reflectors at 10 dB SNR",
                      "frames_per_step": F, "path": best, "fft_len": 131072},
           "paths": res, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark measures one GPU; runs on several GPUs are not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.config == "c5":
        main_c5(args)
    else:
        main_c2(args)


if __name__ == "__main__":
    main()
