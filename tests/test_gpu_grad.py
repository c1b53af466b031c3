"""Reverse-mode derivatives on the GPU (sonar_energyscape_vjp) against the FP64 oracle.

The library's gradients are compared with the oracle's chain rule (energyscape_vjp_td /
energyscape_vjp_fd and their steps) on the same seeded inputs: the envelope gradient
G_b, the matched-filter gradient, dL/dx and dL/dp.  The GPU computes them in FP32 from
its own FP32 forward buffers.  Bars (relative L2): 1e-5 for one step given the GPU's
input of that step, 1e-4 for dx and dp against the oracle's whole chain (the FP32
forward error, ~1e-6 relative, is amplified where |b| is small by the b/|b| factor of
the envelope's derivative and by the cancelling difference of neighbouring samples in
the TD delay derivative).  A central difference of the GPU's own forward pass through
sonar_plan_set_positions checks dL/dp end to end, and the self-calibration workload
(32 mics, 16384 samples, 1500 directions, 10 frames of 5 reflectors, positions perturbed
by 0.5 mm) is solved with these gradients.
"""

import sys

import numpy as np
import pytest

import oracle as O
from workloads import synth

pytestmark = pytest.mark.gpu

TOL_GRAD = 1e-4   # end results (dx, dp) against the oracle's whole chain
TOL_STEP = 1e-5   # one step against the oracle applied to the GPU's input of that step


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    return torch


def _plan(gpu, w, mode, **kw):
    return gpu.Plan(w.mic_pos, w.chirp, w.dirs, w.x.shape[2], fs=w.fs, c=w.c, band=w.cfg.band,
                    decim=w.cfg.decim, mode={"td": "td", "fd": "fd_fp32", "cubic": "td_cubic"}[mode], **kw)


def _oracle_steps(w, frame, plan, mode):
    """Oracle forward of one frame: (R, h, Q, Dl, n_idx, y or Y, b)."""
    x = w.x[frame].astype(np.float64)
    R, P = w.cfg.decim, plan.P
    h = O.default_lowpass(R)
    Q = O.num_range_bins(0, x.shape[1], R)
    Dl = O.delays(w.mic_pos, w.dirs, w.fs, w.c)
    n_idx = O.beam_window_indices(0, Q, R, h.size)
    if mode in ("td", "cubic"):
        y = O.matched_filter(x, w.chirp, P, w.fs, w.cfg.band)
        b = O.das_td(y, Dl, n_idx) if mode == "td" else O.das_td_cubic(y, Dl, n_idx)
    else:
        y = O.matched_filter_spectrum(x, w.chirp, P, w.fs, w.cfg.band)
        b = O.das_fd(y, Dl, n_idx)
    return R, h, Q, Dl, n_idx, y, b


def _oracle_back(w, plan, mode, steps, G_b):
    """Oracle backward from G_b: (G_mf over Z_P, dx, dpos)."""
    R, h, Q, Dl, n_idx, y, b = steps
    N = w.x.shape[2]
    if mode in ("td", "cubic"):
        G_y, dDl = (O.das_td_vjp if mode == "td" else O.das_td_cubic_vjp)(y, Dl, n_idx, G_b)
        dx = O.matched_filter_vjp(G_y, w.chirp, plan.P, N, w.fs, w.cfg.band)
    else:
        G_y, dDl = O.das_fd_vjp(y, Dl, n_idx, G_b)
        dx = O.matched_filter_spectrum_vjp(G_y, w.chirp, plan.P, N, w.fs, w.cfg.band)
    return G_y, dx, O.delays_vjp(dDl, w.dirs, w.fs, w.c)


@pytest.mark.parametrize("mode", ["td", "fd", "cubic"])
def test_vjp_matches_oracle(gpu, torch_mod, mode):
    """Each step against the oracle applied to the GPU's own input of that step (the
    envelope derivative b/|b| is ill-conditioned where |b| is small, so G_b is checked on
    the GPU's forward beam), and the end results dx, dp against the oracle's whole chain."""
    _check_vjp(gpu, torch_mod, mode, n_dirs=37, fft_len=0)


@pytest.mark.parametrize("mode,fft_len", [("fd", 65536), ("td", 65536), ("fd", 131072)])
def test_vjp_long_fft_matches_oracle(gpu, torch_mod, mode, fft_len):
    """FFT lengths above 32768: the adjoint's P-point transforms run as P / 16384 phase
    transforms of 16384 points and dx through the four-step inverse; same bars as above."""
    _check_vjp(gpu, torch_mod, mode, n_dirs=11, fft_len=fft_len)


def test_vjp_chunked_scratch_matches_per_frame(gpu, torch_mod):
    """The adjoint's transform scratch holds at most 4 GiB (4096 channels of P = 131072): 2 frames
    of 2100 directions run as two chunks in one call and as one chunk per frame in two calls; dx
    agrees bit for bit and dL/dp is the sum of the per-frame ones (same FP64 reduction, other order)."""
    torch = torch_mod
    w = synth.make_workload("c2", frames=2, n_samples=4096, n_dirs=2100)
    _say("case vjp chunked scratch: M=32 N=4096 D=2100 F=2 P=131072 fd_fp32")
    plan = _plan(gpu, w, "fd", max_frames=2, fft_len=131072)
    x = torch.from_numpy(w.x).cuda()
    mf = plan.matched_filter(x)
    dE = torch.from_numpy(np.random.default_rng(np.random.SeedSequence([4, 2, 1, 0]))
                          .standard_normal((2, plan.D, plan.Q)).astype(np.float32)).cuda()
    _, dx, dpos = plan.vjp(mf, plan.beamform(mf), dE)
    parts = [plan.vjp(mf[f:f + 1].contiguous(), plan.beamform(mf[f:f + 1].contiguous()), dE[f:f + 1].contiguous())
             for f in range(2)]
    torch.cuda.synchronize()
    for f in range(2):
        assert torch.equal(dx[f], parts[f][1][0]), f
    err = rel_l2(dpos, parts[0][2] + parts[1][2])
    _say(f"chunked vs per-frame: dx equal, dpos rel {err:.2e}")
    assert err <= 1e-12


def _check_vjp(gpu, torch_mod, mode, n_dirs, fft_len):
    torch = torch_mod
    w = synth.make_workload("c2", frames=2, n_samples=4096, n_dirs=n_dirs)
    _say(f"case vjp {mode}: M=32 N=4096 D={n_dirs} F=2 fft_len={fft_len or 'default'}")
    plan = _plan(gpu, w, mode, max_frames=2, fft_len=fft_len)
    if fft_len:
        assert plan.P == fft_len
    x = torch.from_numpy(w.x).cuda()
    mf = plan.matched_filter(x)
    beam = plan.beamform(mf)
    b_gpu = beam.cpu().numpy().astype(np.complex128)
    rng = np.random.default_rng(np.random.SeedSequence([4, 0, 0, 5]))
    dE = rng.standard_normal((2, plan.D, plan.Q)).astype(np.float32)
    dy, dx, dpos = plan.vjp(mf, beam, torch.from_numpy(dE).cuda())
    torch.cuda.synchronize()
    gb, dy, dx = beam.cpu().numpy(), dy.cpu().numpy(), dx.cpu().numpy()
    lo, kb = plan.band_lo_bin, plan.band_bins
    dpos_o = np.zeros((plan.M, 3))
    for f in range(2):
        steps = _oracle_steps(w, f, plan, mode)
        R, h, Q = steps[:3]
        dEf = dE[f].astype(np.float64)
        # steps on the GPU's own inputs
        G_b_own = O.envelope_vjp(b_gpu[f], h, dEf, Q, R)
        G_y_own, _, _ = _oracle_back(w, plan, mode, steps, gb[f].astype(np.complex128))
        # the whole chain
        G_b = O.envelope_vjp(steps[6], h, dEf, Q, R)
        G_y, dx_o, dp = _oracle_back(w, plan, mode, steps, G_b)
        dpos_o += dp
        if mode == "fd":
            G_y_own, G_y = G_y_own[:, lo:lo + kb].T, G_y[:, lo:lo + kb].T
        step_errs = dict(G_b=rel_l2(gb[f], G_b_own), G_mf=rel_l2(dy[f], G_y_own))
        chain_errs = dict(G_b=rel_l2(gb[f], G_b), G_mf=rel_l2(dy[f], G_y), dx=rel_l2(dx[f], dx_o))
        _say(f"vjp {mode} frame {f}: steps " + " ".join(f"{k}={v:.2e}" for k, v in step_errs.items()) +
             "; chain " + " ".join(f"{k}={v:.2e}" for k, v in chain_errs.items()))
        for k, v in step_errs.items():
            assert v <= TOL_STEP, (k, v)
        assert chain_errs["dx"] <= TOL_GRAD
    err = rel_l2(dpos, dpos_o)
    _say(f"vjp {mode} dpos rel L2 = {err:.2e}")
    assert err <= TOL_GRAD


def test_vjp_positions_only_matches_full_call(gpu, torch_mod):
    """dpos does not depend on whether the matched-filter gradient is also requested."""
    torch = torch_mod
    w = synth.make_workload("c1", n_dirs=19)
    _say("case vjp dpos-only: c1 D=19")
    plan = _plan(gpu, w, "fd")
    x = torch.from_numpy(w.x).cuda()
    mf = plan.matched_filter(x)
    beam = plan.beamform(mf)
    dE = torch.ones((1, plan.D, plan.Q), dtype=torch.float32, device="cuda")
    _, _, dpos_a = plan.vjp(mf, beam.clone(), dE, want_dx=False)
    _, _, dpos_b = plan.vjp(mf, beam.clone(), dE, want_dx=True)
    assert np.array_equal(dpos_a, dpos_b)


@pytest.mark.parametrize("mode", ["td", "fd"])
def test_set_positions_matches_a_new_plan(gpu, torch_mod, mode):
    torch = torch_mod
    w = synth.make_workload("c1", n_dirs=31)
    _say(f"case set_positions {mode}: c1 D=31")
    rng = np.random.default_rng(np.random.SeedSequence([4, 0, 0, 6]))
    pos2 = w.mic_pos + rng.normal(0.0, 0.5e-3, size=w.mic_pos.shape)
    plan = _plan(gpu, w, mode)
    x = torch.from_numpy(w.x).cuda()
    plan.set_positions(pos2)
    E1 = plan.energyscape(x).cpu().numpy()
    w2 = synth.Workload(w.cfg, w.x, w.chirp, pos2, w.dirs, w.reflectors)
    E2 = _plan(gpu, w2, mode).energyscape(x).cpu().numpy()
    err = rel_l2(E1, E2)
    _say(f"set_positions {mode}: rel L2 vs new plan = {err:.2e}")
    if mode == "fd":
        assert np.array_equal(E1, E2)   # same tables from the same kernels
    else:
        assert err <= 1e-6            # same sums; the row offsets of the two plans differ
    if mode == "td":
        with pytest.raises(gpu.SonarError):
            plan.set_positions(w.mic_pos * 4.0)   # beyond the TD plan's delay range
    else:
        plan.set_positions(w.mic_pos * 4.0)       # exact phases: any geometry


@pytest.mark.parametrize("mode,bar", [("td_bf16", 1e-3), ("td_bf16x2", 1e-3), ("td_f16", 3e-4), ("td_bf16g", 1e-3)])
def test_set_positions_rebuilds_mfma_tiles(gpu, torch_mod, mode, bar):
    """MFMA TD modes: new positions rebuild the direction tiles, tap groups and weights.  The result
    matches the oracle at the new positions and a plan created there; going back to the old
    positions gives the old energyscape bit for bit; positions beyond the plan's delay range are
    refused and leave the plan as it was."""
    torch = torch_mod
    w = synth.make_workload("c1", n_dirs=97)          # 4 direction tiles
    _say(f"case set_positions {mode}: c1 D=97")
    rng = np.random.default_rng(np.random.SeedSequence([4, 0, 0, 7]))
    pos2 = w.mic_pos + rng.normal(0.0, 0.5e-3, size=w.mic_pos.shape)
    N = w.x.shape[2]
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, N, fs=w.fs, c=w.c, mode=mode)
    x = torch.from_numpy(w.x).cuda()
    E0 = plan.energyscape(x).cpu().numpy()
    plan.set_positions(pos2)
    E1 = plan.energyscape(x).cpu().numpy()[0]
    E2 = gpu.Plan(pos2, w.chirp, w.dirs, N, fs=w.fs, c=w.c, mode=mode).energyscape(x).cpu().numpy()[0]
    Eo = O.energyscape(w.x[0].astype(np.float64), w.chirp, pos2, w.dirs, fs=w.fs, c=w.c, P=plan.P, R=10,
                       mode="td")
    e_new, e_or = rel_l2(E1, E2), rel_l2(E1, Eo)
    _say(f"  moved plan vs new plan {e_new:.2e}, vs oracle {e_or:.2e} (bar {bar:.0e})")
    # the two plans sum the same products; their K-chunks may group the taps differently
    assert e_new <= 1e-5
    assert e_or <= bar
    plan.set_positions(w.mic_pos)
    assert np.array_equal(plan.energyscape(x).cpu().numpy(), E0)
    with pytest.raises(gpu.SonarError) as ei:
        plan.set_positions(w.mic_pos * 4.0)           # beyond the plan's delay range
    assert ei.value.status == gpu.SONAR_E_UNSUPPORTED
    assert np.array_equal(plan.energyscape(x).cpu().numpy(), E0)


def test_autograd_function_matches_vjp(gpu, torch_mod):
    """Energyscape.apply: backward gives the sonar_energyscape_vjp results for x and positions."""
    torch = torch_mod
    w = synth.make_workload("c1", n_dirs=23)
    _say("case autograd: c1 D=23, fd_fp32")
    plan = _plan(gpu, w, "fd")
    x = torch.from_numpy(w.x).cuda().requires_grad_(True)
    pos = torch.from_numpy(w.mic_pos.copy()).requires_grad_(True)
    wts = torch.from_numpy(np.random.default_rng(np.random.SeedSequence([4, 0, 0, 8]))
                           .standard_normal((1, plan.D, plan.Q)).astype(np.float32)).cuda()
    E = gpu.Energyscape.apply(x, pos, plan)
    (E * wts).sum().backward()
    mf = plan.matched_filter(x.detach())
    beam = plan.beamform(mf)
    _, dx, dpos = plan.vjp(mf, beam, wts)
    torch.cuda.synchronize()
    assert torch.equal(x.grad, dx)
    assert np.array_equal(pos.grad.numpy(), dpos)


def test_autograd_backward_uses_its_own_forward_geometry(gpu, torch_mod):
    """Two forwards on one plan at different positions, then backward of the first: its gradients
    are those of the first geometry (the plan's delay tables were moved by the second forward)."""
    torch = torch_mod
    w = synth.make_workload("c1", n_dirs=23)
    _say("case autograd two geometries: c1 D=23, fd_fp32")
    plan = _plan(gpu, w, "fd")
    wts = torch.from_numpy(np.random.default_rng(np.random.SeedSequence([4, 0, 0, 10]))
                           .standard_normal((1, plan.D, plan.Q)).astype(np.float32)).cuda()
    pos1 = w.mic_pos.copy()
    pos2 = pos1 + np.random.default_rng(np.random.SeedSequence([4, 0, 0, 11])).normal(0.0, 1e-3, pos1.shape)
    x1 = torch.from_numpy(w.x).cuda().requires_grad_(True)
    p1 = torch.from_numpy(pos1.copy()).requires_grad_(True)
    x2 = torch.from_numpy(w.x).cuda().requires_grad_(True)
    p2 = torch.from_numpy(pos2.copy()).requires_grad_(True)
    E1 = gpu.Energyscape.apply(x1, p1, plan)
    E2 = gpu.Energyscape.apply(x2, p2, plan)
    (E1 * wts).sum().backward()
    plan.set_positions(pos1)
    mf = plan.matched_filter(x1.detach())
    _, dx, dpos = plan.vjp(mf, plan.beamform(mf), wts)
    torch.cuda.synchronize()
    assert torch.equal(x1.grad, dx)
    assert np.array_equal(p1.grad.numpy(), dpos)
    (E2 * wts).sum().backward()
    plan.set_positions(pos2)
    mf = plan.matched_filter(x2.detach())
    _, dx2, dpos2 = plan.vjp(mf, plan.beamform(mf), wts)
    torch.cuda.synchronize()
    assert torch.equal(x2.grad, dx2)
    assert np.array_equal(p2.grad.numpy(), dpos2)
    assert not np.array_equal(dpos, dpos2)


@pytest.mark.parametrize("mode", ["td", "fd", "cubic"])
def test_backward_from_samples_matches_vjp(gpu, torch_mod, mode):
    """sonar_energyscape_backward (x -> dx, dp in one call) equals matched filter + beamform + VJP."""
    torch = torch_mod
    w = synth.make_workload("c1", frames=2, n_dirs=19)
    _say(f"case backward {mode}: c1 D=19 F=2")
    plan = _plan(gpu, w, mode, max_frames=2)
    x = torch.from_numpy(w.x).cuda()
    dE = torch.from_numpy(np.random.default_rng(np.random.SeedSequence([4, 0, 0, 9]))
                          .standard_normal((2, plan.D, plan.Q)).astype(np.float32)).cuda()
    dx, dpos = plan.backward(x, dE)
    mf = plan.matched_filter(x)
    _, dx2, dpos2 = plan.vjp(mf, plan.beamform(mf), dE)
    torch.cuda.synchronize()
    assert torch.equal(dx, dx2)
    assert np.array_equal(dpos, dpos2)


def _cal_loss_grad(plan, mf, cells, torch):
    """L = -sum of E at the reflector cells, and dL/dp from sonar_energyscape_vjp."""
    beam = plan.beamform(mf)
    E = plan.envelope(beam)
    f_i, d_i, q_i = cells
    L = -float(E[f_i, d_i, q_i].double().sum().item())
    dE = torch.zeros_like(E)
    dE[f_i, d_i, q_i] = -1.0
    _, _, dpos = plan.vjp(mf, beam, dE, want_dx=False)
    return L, dpos


def _cell_index(cells, torch):
    f_i = [f for f, fc in enumerate(cells) for _ in fc]
    d_i = [d for fc in cells for d, _ in fc]
    q_i = [q for fc in cells for _, q in fc]
    return tuple(torch.tensor(v, dtype=torch.long, device="cuda") for v in (f_i, d_i, q_i))


def _oracle_cal_grad(w, pos, P):
    """Oracle dL/dp of the calibration loss; dE vanishes outside the cells, so only the
    cells' directions and beam samples contribute."""
    R = w.decim
    h = O.default_lowpass(R)
    K = h.size
    g = np.zeros_like(pos)
    for f, fc in enumerate(w.cells):
        Y = O.matched_filter_spectrum(w.x[f].astype(np.float64), w.chirp, P, w.fs, w.band)
        for d, q in fc:
            u = w.dirs[d:d + 1]
            Dl = O.delays(pos, u, w.fs, w.c)
            n_idx = np.arange(q * R - (K - 1) // 2, q * R + (K - 1) // 2 + 1)
            b = O.das_fd(Y, Dl, n_idx)
            G_b = O.envelope_vjp(b, h, -np.ones((1, 1)), 1, R)
            _, dDl = O.das_fd_vjp(Y, Dl, n_idx, G_b)
            g += O.delays_vjp(dDl, u, w.fs, w.c)
    return g


def _geometry_error(pos, true_pos):
    d = pos - true_pos
    d = d - d.mean(axis=0)   # a common translation only shifts every beam in range
    n = np.linalg.norm(d, axis=1)
    return float(np.sqrt(np.mean(n * n))), float(n.max())


@pytest.mark.parametrize("mode", ["fd", "td", "cubic"])
def test_cells_match_oracle(gpu, torch_mod, mode):
    """sonar_energyscape_cells: E at chosen cells (edges of the range included, one cell
    repeated, one outside the plan) and dL/dp for random weights, against the oracle's
    energyscape and its whole derivative chain with dE scattered onto those cells."""
    torch = torch_mod
    w = synth.make_workload("c2", frames=2, n_samples=4096, n_dirs=37)
    _say(f"case cells {mode}: M=32 N=4096 D=37 F=2")
    plan = _plan(gpu, w, mode, max_frames=2)
    x = torch.from_numpy(w.x).cuda()
    mf = plan.matched_filter(x)
    rng = np.random.default_rng(np.random.SeedSequence([4, 1, 2, 3]))
    cells = [(0, 0, 0), (0, 36, plan.Q - 1), (1, 5, 17), (1, 5, 17), (0, 12, plan.Q // 2)]
    cells += [(int(rng.integers(2)), int(rng.integers(plan.D)), int(rng.integers(plan.Q))) for _ in range(11)]
    wts = rng.standard_normal(len(cells)).astype(np.float32)
    bad = (0, plan.D, 3)   # outside the plan: E = NaN, adds nothing
    ct = torch.tensor(cells + [bad], dtype=torch.int32, device="cuda")
    E, dpos = plan.cells(mf, ct, torch.from_numpy(np.append(wts, 5.0).astype(np.float32)).cuda())
    E = E.cpu().numpy()
    assert np.isnan(E[-1])
    dpos_o = np.zeros((plan.M, 3))
    E_o = np.zeros(len(cells))
    E_scale = 0.0
    for f in range(2):
        steps = _oracle_steps(w, f, plan, mode)
        R, h, Q = steps[:3]
        Eo = O.envelope(steps[6], h, Q, R)
        E_scale = max(E_scale, float(np.max(np.abs(Eo))))
        dEf = np.zeros((plan.D, Q))
        for i, (cf, cd, cq) in enumerate(cells):
            if cf == f:
                E_o[i] = Eo[cd, cq]
                dEf[cd, cq] += wts[i]
        G_b = O.envelope_vjp(steps[6], h, dEf, Q, R)
        dpos_o += _oracle_back(w, plan, mode, steps, G_b)[2]
    # E as the dense tests hold it: relative L2 over the cells, and every cell within 1e-5 of the
    # energyscape's largest value (a cell in the noise is a sum over the band whose terms cancel, so
    # its own relative error is larger)
    errE = rel_l2(E[:-1], E_o)
    errE_max = float(np.max(np.abs(E[:-1] - E_o))) / E_scale
    errP = rel_l2(dpos, dpos_o)
    _say(f"cells: E rel L2 {errE:.2e}, max err / max E {errE_max:.2e}, "
         f"max rel err per cell {float(np.max(np.abs(E[:-1] - E_o) / np.abs(E_o))):.2e}; dpos rel L2 {errP:.2e}")
    assert errE <= 1e-5
    assert errE_max <= 1e-5
    assert errP <= TOL_GRAD


def test_cells_errors(gpu, torch_mod):
    """Status codes of sonar_energyscape_cells: modes without a cells reading, TD_NEAREST's position
    derivative, more cells than the workspace holds."""
    torch = torch_mod
    w = synth.make_workload("c1", frames=1, n_dirs=7)
    x = torch.from_numpy(w.x).cuda()
    cells = torch.tensor([[0, 1, 2]], dtype=torch.int32, device="cuda")
    one = torch.ones(1, dtype=torch.float32, device="cuda")
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, w.x.shape[2], fs=w.fs, c=w.c, mode="td_bf16g")
    with pytest.raises(gpu.SonarError) as ei:
        plan.cells(plan.matched_filter(x), cells, one)
    assert ei.value.status == gpu.SONAR_E_UNSUPPORTED
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, w.x.shape[2], fs=w.fs, c=w.c, mode="td_nearest")
    mf = plan.matched_filter(x)
    E, _ = plan.cells(mf, cells, one, want_dpos=False)      # the energyscape cell alone is fine
    assert np.isfinite(E.cpu().numpy()).all()
    with pytest.raises(gpu.SonarError) as ei:
        plan.cells(mf, cells, one)
    assert ei.value.status == gpu.SONAR_E_UNSUPPORTED
    many = cells.repeat(plan.D + 1, 1).contiguous()         # above max_frames * D = 7
    with pytest.raises(gpu.SonarError) as ei:
        plan.cells(mf, many, torch.ones(many.shape[0], dtype=torch.float32, device="cuda"), want_dpos=False)
    assert ei.value.status == gpu.SONAR_E_INVALID


def test_cells_match_dense_calibration(gpu, torch_mod):
    """The calibration workload (32 mics, 16384 samples, 1500 directions, 10 frames of 5
    reflectors): the cells path gives the dense path's loss and gradient."""
    torch = torch_mod
    w = synth.make_calibration()
    F, M, N = w.x.shape
    _say(f"case cells vs dense: M={M} N={N} D={w.dirs.shape[0]} F={F}")
    plan = gpu.Plan(w.start_pos, w.chirp, w.dirs, N, fs=w.fs, c=w.c, band=w.band, decim=w.decim, mode="fd_fp32",
                    max_frames=F)
    x = torch.from_numpy(w.x).cuda()
    mf = plan.matched_filter(x)
    cells = _cell_index(w.cells, torch)
    L, g = _cal_loss_grad(plan, mf, cells, torch)
    ct = torch.stack(cells, dim=1).to(torch.int32).contiguous()
    E, g2 = plan.cells(mf, ct, torch.full((ct.shape[0],), -1.0, dtype=torch.float32, device="cuda"))
    L2 = -float(E.double().sum().item())
    _say(f"cells vs dense: loss {L2:.9e} vs {L:.9e}, dpos rel L2 {rel_l2(g2, g):.2e}")
    assert abs(L2 - L) <= 1e-5 * abs(L)
    assert rel_l2(g2, g) <= TOL_GRAD


def test_self_calibration_recovers_positions(gpu, torch_mod):
    torch = torch_mod
    from scipy.optimize import minimize

    w = synth.make_calibration()
    F, M, N = w.x.shape
    _say(f"case self-calibration: M={M} N={N} D={w.dirs.shape[0]} F={F} reflectors/frame={len(w.cells[0])}")
    plan = gpu.Plan(w.start_pos, w.chirp, w.dirs, N, fs=w.fs, c=w.c, band=w.band, decim=w.decim, mode="fd_fp32",
                    max_frames=F)
    x = torch.from_numpy(w.x).cuda()
    mf = plan.matched_filter(x)
    cells = _cell_index(w.cells, torch)

    # the gradient at the perturbed start against the oracle's (full size)
    L0, g0 = _cal_loss_grad(plan, mf, cells, torch)
    g0_o = _oracle_cal_grad(w, w.start_pos, plan.P)
    err = rel_l2(g0, g0_o)
    _say(f"calibration gradient at start: rel L2 vs oracle = {err:.2e}")
    assert err <= TOL_GRAD

    # central difference of the GPU forward pass along a seeded direction, h = 1e-6 m.  The
    # loss (~3e3) carries FP32 rounding of ~1e-4 per evaluation against a difference
    # Lp - Lm of ~3e-2, so the bar is 1e-2 relative.
    v = np.random.default_rng(np.random.SeedSequence([4, 0, 0, 7])).standard_normal(w.start_pos.shape)
    v /= np.linalg.norm(v)
    hstep = 1e-6
    plan.set_positions(w.start_pos + hstep * v)
    Lp, _ = _cal_loss_grad(plan, mf, cells, torch)
    plan.set_positions(w.start_pos - hstep * v)
    Lm, _ = _cal_loss_grad(plan, mf, cells, torch)
    fd = (Lp - Lm) / (2 * hstep)
    an = float(np.sum(g0 * v))
    _say(f"directional derivative: central difference {fd:.6e}, adjoint {an:.6e}")
    assert abs(fd - an) <= 1e-2 * abs(an)

    # quasi-Newton descent on the positions (millimetre units)
    evals = [0]

    def fun(z):
        pos = z.reshape(M, 3) * 1e-3
        plan.set_positions(pos)
        L, g = _cal_loss_grad(plan, mf, cells, torch)
        evals[0] += 1
        return L, g.ravel() * 1e-3

    e0 = _geometry_error(w.start_pos, w.true_pos)
    res = minimize(fun, w.start_pos.ravel() * 1e3, jac=True, method="L-BFGS-B",
                   options=dict(maxiter=80, gtol=1e-9, ftol=1e-15))
    pos = res.x.reshape(M, 3) * 1e-3
    e1 = _geometry_error(pos, w.true_pos)
    _say(f"self-calibration: {evals[0]} evaluations, loss {L0:.3f} -> {res.fun:.3f}; "
         f"rms/max position error {e0[0] * 1e3:.4f}/{e0[1] * 1e3:.4f} mm -> {e1[0] * 1e3:.5f}/{e1[1] * 1e3:.5f} mm")
    assert e1[0] < 0.05e-3
    assert e1[1] < 0.05e-3
