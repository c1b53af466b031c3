"""Heterogeneous sensor network in one call (GPU): 8 sensors x 4 frames, each sensor with its
own array geometry, recording length (8192 / 16384 / 32768) and direction grid (91-azimuth 2D
or 1500-direction 3D), through sonar_energyscape_multi; replayed from a HIP graph; and the
mode chosen by sonar_plan_create_tuned.  Every energyscape is compared with the FP64 oracle
(all directions of the 2D grids, 12 sampled directions of the 3D grids)."""

import sys

import numpy as np
import pytest

import oracle as O
from workloads import synth

pytestmark = pytest.mark.gpu

BARS = {"td": 1e-5, "td_bf16": 1e-3, "td_bf16x2": 1e-3, "td_f16": 3e-4, "fd_fp32": 1e-5, "fd_bf16x3": 1e-5, "fd_bf16": 1e-3,
        "td_bf16g": 1e-3}


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    return torch


@pytest.fixture(scope="module")
def network():
    return synth.make_network()


def _plan(gpu, w, **kw):
    return gpu.Plan(w.mic_pos, w.chirp, w.dirs, w.x.shape[2], fs=w.fs, c=w.c, band=w.cfg.band,
                    max_frames=w.x.shape[0], **kw)


def _sample(w):
    D = w.dirs.shape[0]
    if D <= 128:
        return np.arange(D)
    return np.sort(np.random.default_rng(D).choice(D, 12, replace=False))


def _check_against_oracle(w, E, P, mode, label):
    idx = _sample(w)
    omode = "fd" if mode.startswith("fd") else "td"
    errs = []
    for f in range(w.x.shape[0]):
        Eo = O.energyscape(w.x[f].astype(np.float64), w.chirp, w.mic_pos, w.dirs, fs=w.fs, c=w.c, P=P,
                           R=w.cfg.decim, band=w.cfg.band, mode=omode, dir_index=idx)
        errs.append(rel_l2(E[f][idx], Eo))
    _say(f"  {label}: N={w.x.shape[2]} D={w.dirs.shape[0]} {mode}: max rel L2 over frames = {max(errs):.3e}")
    assert max(errs) <= BARS[mode]


@pytest.mark.parametrize("mode", ["td", "td_bf16", "td_bf16x2", "td_f16", "td_bf16g"])
def test_network_multi(gpu, torch_mod, network, mode):
    torch = torch_mod
    _say(f"case network multi {mode}: 8 sensors x 4 frames")
    plans = [_plan(gpu, w, mode=mode) for w in network]
    xs = [torch.from_numpy(w.x).cuda() for w in network]
    Es = gpu.energyscape_multi(plans, xs)
    singles = [pl.energyscape(x) for pl, x in zip(plans, xs)]
    torch.cuda.synchronize()
    for s, (w, pl, E, E1) in enumerate(zip(network, plans, Es, singles)):
        assert torch.equal(E, E1)          # same kernels, same order: bit-identical
        _check_against_oracle(w, E.cpu().numpy(), pl.P, mode, f"sensor {s}")


def test_network_multi_shared_plan(gpu, torch_mod, network):
    """Items that share a plan (and so its workspace) stay ordered on one stream while the
    other items run beside them: every result equals its own single call."""
    torch = torch_mod
    _say("case network multi with a shared plan: td")
    plans = [_plan(gpu, w, mode="td") for w in network[:3]]
    xs = [torch.from_numpy(w.x).cuda() for w in network[:3]]
    x0b = (xs[0] * 0.5).contiguous()
    items_p = [plans[0], plans[1], plans[0], plans[2], plans[0]]
    items_x = [xs[0], xs[1], x0b, xs[2], xs[0][:2].contiguous()]
    Es = gpu.energyscape_multi(items_p, items_x)
    singles = [pl.energyscape(x) for pl, x in zip(items_p, items_x)]
    torch.cuda.synchronize()
    for E, E1 in zip(Es, singles):
        assert torch.equal(E, E1)


@pytest.mark.parametrize("mode", ["td_bf16", "td_bf16x2", "td_f16", "td_bf16g"])
def test_network_graph_replay(gpu, torch_mod, network, mode):
    """The multi call captured once in a graph, replayed on new inputs: every replay equals the
    eager result for the same inputs."""
    torch = torch_mod
    _say(f"case network graph replay: {mode}")
    plans = [_plan(gpu, w, mode=mode) for w in network]
    xs = [torch.from_numpy(w.x).cuda() for w in network]
    outs = [torch.empty((w.x.shape[0], w.dirs.shape[0], pl.Q), dtype=torch.float32, device="cuda")
            for w, pl in zip(network, plans)]
    gpu.energyscape_multi(plans, xs, outs)           # warm-up outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        gpu.energyscape_multi(plans, xs, outs)
    torch.cuda.synchronize()
    rng = np.random.default_rng(9)
    for rep in range(3):
        for x in xs:                                   # eager work between replays: new inputs
            x.copy_(torch.from_numpy((rng.standard_normal(tuple(x.shape)) * 0.1).astype(np.float32)))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = [o.clone() for o in outs]
        ref = gpu.energyscape_multi(plans, xs)
        torch.cuda.synchronize()
        for a, b in zip(got, ref):
            assert torch.equal(a, b)
        _say(f"  replay {rep}: {len(got)} items equal to the eager call")


@pytest.mark.parametrize("tune", ["fp32", "bf16"])
def test_tuned_plan(gpu, torch_mod, network, tune):
    torch = torch_mod
    w = network[3]                                     # 16384 samples, 1500 directions
    pl = _plan(gpu, w, tune=tune)
    allowed = {"fp32": {"td", "fd_fp32", "fd_bf16x3"}, "bf16": {"td", "fd_fp32", "fd_bf16x3", "td_bf16", "fd_bf16", "td_bf16x2", "td_f16", "td_bf16g"}}
    waves = pl.query(gpu.Q_MT_WAVES)
    _say(f"case tuned {tune}: chose {pl.mode} (MFMA workgroup waves: {waves})")
    assert pl.mode in allowed[tune]
    assert waves in ((4, 8) if pl.mode.startswith("td_bf16") or pl.mode == "td_f16" else (0,))
    if pl.mode.startswith("fd"):
        assert pl.query(gpu.Q_FD_PHASE_LEN) >= 16
    E = pl.energyscape(torch.from_numpy(w.x).cuda()).cpu().numpy()
    _check_against_oracle(w, E, pl.P, pl.mode, f"tuned {tune}")


def test_network_eager_call_while_another_stream_captures(gpu, torch_mod, network):
    """A multi call captured on one stream leaves the library's side streams joined to that capture
    until it ends; an eager multi call on another stream in that window must neither land in the
    graph nor fail: it runs (in order, on its own stream) and gives the single-call results, and
    the graph still replays the captured call."""
    torch = torch_mod
    _say("case network: eager multi on a second stream during a capture")
    sub = network[:3]
    plans_a = [_plan(gpu, w, mode="td_bf16x2") for w in sub]
    plans_b = [_plan(gpu, w, mode="td_bf16x2") for w in sub]
    xs = [torch.from_numpy(w.x).cuda() for w in sub]
    outs_a = [torch.empty((w.x.shape[0], w.dirs.shape[0], pl.Q), dtype=torch.float32, device="cuda")
              for w, pl in zip(sub, plans_a)]
    outs_b = [torch.zeros_like(o) for o in outs_a]
    gpu.energyscape_multi(plans_a, xs, outs_a)
    torch.cuda.synchronize()
    s2 = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        gpu.energyscape_multi(plans_a, xs, outs_a)
        gpu.energyscape_multi(plans_b, xs, outs_b, stream=s2)
    torch.cuda.synchronize()
    ref = [pl.energyscape(x) for pl, x in zip(plans_b, xs)]
    torch.cuda.synchronize()
    for a, b in zip(outs_b, ref):
        assert torch.equal(a, b)
    for o in outs_a:
        o.zero_()
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    for a, b in zip(outs_a, ref):
        assert torch.equal(a, b)


def test_tune_cache_persists_the_choice(gpu, torch_mod, network, tmp_path):
    """sonar_tune_cache: the first tuned creation times the candidates and appends its choice as one
    JSON line; the second finds it and creates the same plan without timing (no new line); a
    different descriptor gets its own line."""
    import json
    torch = torch_mod
    path = tmp_path / "tune.jsonl"
    gpu.tune_cache(str(path))
    try:
        w = network[3]
        _say("case tune cache: tuned plan twice, then another direction grid")
        p1 = _plan(gpu, w, tune="bf16")
        lines = path.read_text().splitlines()
        assert len(lines) == 1
        rec = json.loads(lines[0])
        assert gpu.BF_MODES[p1.mode] == rec["mode"]
        p2 = _plan(gpu, w, tune="bf16")
        assert len(path.read_text().splitlines()) == 1
        assert p2.mode == p1.mode
        for q in (gpu.Q_MT_WAVES, gpu.Q_FD_PHASE_LEN):
            assert p2.query(q) == p1.query(q)
        x = torch.from_numpy(w.x).cuda()
        assert torch.equal(p1.energyscape(x), p2.energyscape(x))
        _say(f"  chose {p1.mode} ({rec})")
        p3 = gpu.Plan(w.mic_pos, w.chirp, w.dirs[:700], w.x.shape[2], fs=w.fs, c=w.c, band=w.cfg.band,
                      max_frames=w.x.shape[0], tune="fp32")
        assert len(path.read_text().splitlines()) == 2
        assert p3.mode in ("td", "fd_fp32", "fd_bf16x3")
    finally:
        gpu.tune_cache(None)


C3_SUBSET = 250   # directions of each 1500-direction energyscape checked against the oracle (all of the 2D grids)


@pytest.mark.parametrize("mode", ["td_bf16x2", "td_bf16g", "fd_bf16"])
def test_network_fp16_samples(gpu, torch_mod, network, mode):
    """The sensor network as configured: FP16 samples, BF16 matrix-core beamforming (the persistent
    time-domain launch, or the per-bin GEMM with each sensor's 4 frames as its N dimension).  All 32
    energyscapes against the oracle on the rounded samples (compute-only error, bar 1e-3): every
    direction of the 91-azimuth grids, a seeded subset of 250 of the 1500-direction grids; the
    end-to-end error against the oracle on the FP32 samples is printed beside it."""
    from oracle import pool
    torch = torch_mod
    _say(f"case network FP16 samples: {mode}, 8 sensors x 4 frames")
    plans = [_plan(gpu, w, mode=mode, sample_dtype="f16") for w in network]
    xh = [w.x.astype(np.float16) for w in network]
    Es = gpu.energyscape_multi(plans, [torch.from_numpy(x).cuda() for x in xh])
    Es = [E.cpu().numpy() for E in Es]
    omode = "fd" if mode.startswith("fd") else "td"
    jobs, keys = [], []
    for s, (w, pl, x) in enumerate(zip(network, plans, xh)):
        D = w.dirs.shape[0]
        idx = None if D <= 128 else np.sort(np.random.default_rng(100 + s).choice(D, C3_SUBSET, replace=False))
        for f in range(w.x.shape[0]):
            for src, tag in ((x[f], "rounded"), (w.x[f], "fp32")):
                jobs.append(pool.Job(x=src, chirp=w.chirp, mic_pos=w.mic_pos, dirs=w.dirs, fs=w.fs, c=w.c, P=pl.P,
                                     R=w.cfg.decim, band=w.cfg.band, mode=omode, dir_index=idx))
                keys.append((s, f, tag, idx))
    refs, _, wall = pool.run(jobs, workers=pool.default_workers())
    _say(f"  oracle: {len(jobs)} energyscapes in {wall:.1f} s")
    worst = {"rounded": 0.0, "fp32": 0.0}
    for (s, f, tag, idx), Eo in zip(keys, refs):
        got = Es[s][f] if idx is None else Es[s][f][idx]
        e = rel_l2(got, Eo)
        worst[tag] = max(worst[tag], e)
        if tag == "rounded":
            assert e <= BARS[mode], (s, f, e)
    _say(f"  max compute-only rel L2 over 32 energyscapes = {worst['rounded']:.3e}; "
         f"end to end (vs FP32 samples) = {worst['fp32']:.3e}")
