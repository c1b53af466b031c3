"""The entry point that allocates nothing (sonar_energyscape_batch_static) against
sonar_energyscape_batch (GPU): the same kernels on buffers carved from the library's static
device scratch instead of the plan's workspace, so the energyscapes must be bit-identical.
Two calls in a row per case, the second with a smaller input, since every call shares the
device's scratch and finds the previous call's contents there."""

import sys

import numpy as np
import pytest

from workloads import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    return torch


# (mode, N, D, frames of the first call, frames of the second, extra plan arguments)
CASES = [
    ("td", 4000, 96, 3, 1, {}),
    ("td_bf16x2", 16384, 1500, 8, 2, {}),
    ("td_f16", 3000, 70, 4, 2, {}),
    ("td_bf16", 2500, 40, 2, 1, {}),
    ("fd_bf16", 4000, 96, 3, 1, {}),
    ("fd_fp32", 16384, 50, 2, 1, {"band": None}),    # 16385 bins: unfused inverse, beam window in scratch
    ("td", 40000, 20, 2, 1, {}),                      # P = 65536: four-step matched filter scratch
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-N{c[1]}-D{c[2]}" for c in CASES])
def test_static_scratch_equals_batch(gpu, torch_mod, case):
    torch = torch_mod
    mode, N, D, F1, F2, extra = case
    w = synth.make_workload("c2", frames=F1, n_samples=N, n_dirs=D)
    band = extra.get("band", w.cfg.band)
    _say(f"case static scratch: {mode} N={N} D={D} F={F1} then a smaller input")
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, N, fs=w.fs, c=w.c, band=band, max_frames=F1, mode=mode)
    x = torch.from_numpy(w.x).cuda()
    ref1 = plan.energyscape(x)
    E1 = plan.energyscape_static(x)
    torch.cuda.synchronize()
    assert torch.equal(E1, ref1)
    # second call: fewer frames, other samples (the scratch still holds the first call's data)
    x2 = (x[F1 - F2:] * -0.75).contiguous()
    ref2 = plan.energyscape(x2)
    E2 = plan.energyscape_static(x2)
    torch.cuda.synchronize()
    assert torch.equal(E2, ref2)
    assert not torch.equal(E2, E1[:F2])


def test_static_scratch_second_plan_smaller(gpu, torch_mod):
    """A call on a smaller plan after a large one on the same device's scratch."""
    torch = torch_mod
    _say("case static scratch: large plan then a small plan")
    wa = synth.make_workload("c2", frames=4, n_samples=16384, n_dirs=1500)
    wb = synth.make_workload("c1", frames=1)
    pa = gpu.Plan(wa.mic_pos, wa.chirp, wa.dirs, 16384, fs=wa.fs, c=wa.c, band=wa.cfg.band, max_frames=4,
                  mode="td_bf16x2")
    pb = gpu.Plan(wb.mic_pos, wb.chirp, wb.dirs, 4096, fs=wb.fs, c=wb.c, mode="td_bf16x2")
    xa, xb = torch.from_numpy(wa.x).cuda(), torch.from_numpy(wb.x).cuda()
    Ea, Eb = pa.energyscape_static(xa), pb.energyscape_static(xb)
    torch.cuda.synchronize()
    assert torch.equal(Ea, pa.energyscape(xa))
    assert torch.equal(Eb, pb.energyscape(xb))


def test_static_scratch_rejects_batches_beyond_its_size(gpu, torch_mod):
    """F frames that need more than the static scratch are refused before anything is enqueued."""
    torch = torch_mod
    w = synth.make_workload("c2", frames=1)
    _say("case static scratch: batch beyond the scratch size is refused")
    F = 16
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, 16384, fs=w.fs, c=w.c, band=w.cfg.band, max_frames=F, mode="fd_bf16")
    x = torch.zeros((F, 32, 16384), dtype=torch.float32, device="cuda")
    E = torch.full((F, plan.D, plan.Q), 7.0, dtype=torch.float32, device="cuda")
    with pytest.raises(gpu.SonarError) as ei:
        plan.energyscape_static(x, out=E)
    assert ei.value.status == gpu.SONAR_E_INVALID
    assert "static scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((E == 7.0).all())          # nothing was enqueued
