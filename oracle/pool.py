"""Process-pool driver of the FP64 oracle (TEST INFRASTRUCTURE ONLY).

The paper's processing node hands measurements to worker processes (§3) and
its CPU timings come from Python code whose numerical work is bound to one
interpreter at a time (§5).  This module runs ``sonar_oracle.energyscape`` the
same way: independent calls, one per (recording, mode, direction subset),
spread over worker processes.  It does no arithmetic of its own: every value
it returns is what ``energyscape`` returns for that call, and a result split
over direction subsets is the rows of the unsplit call (the oracle computes
each direction independently).

Like the rest of ``oracle/``, only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may use it.  Workers are started with the
``spawn`` method, so a parent that already holds a GPU context never forks it.
"""

from __future__ import annotations

import concurrent.futures as cf
import dataclasses
import multiprocessing as mp
import os
import time

import numpy as np

from . import sonar_oracle as _O


def default_workers(cap: int = 16) -> int:
    """Worker processes: the CPUs this process may run on, at most `cap`."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(cap, n))


@dataclasses.dataclass
class Job:
    """One oracle energyscape: x [M][N] (any float dtype; taken as float64), and the keyword
    arguments of sonar_oracle.energyscape."""
    x: np.ndarray
    chirp: np.ndarray
    mic_pos: np.ndarray
    dirs: np.ndarray
    fs: float
    c: float
    P: int
    R: int = 10
    band: tuple | None = None
    mode: str = "td"
    alpha_steps: int | None = None
    taps: np.ndarray | None = None
    dir_index: np.ndarray | None = None


def _run(args):
    """Worker: one energyscape call with BLAS and FFT on one thread; returns (E, stage seconds)."""
    i, job = args
    try:
        import threadpoolctl
        limit = threadpoolctl.threadpool_limits(1)
    except ImportError:   # pragma: no cover - threadpoolctl is installed here
        limit = None
    t = {}
    t0 = time.perf_counter()
    E = _O.energyscape(np.asarray(job.x, dtype=np.float64), job.chirp, job.mic_pos, job.dirs, fs=job.fs, c=job.c,
                       P=job.P, R=job.R, taps=job.taps, band=job.band, mode=job.mode, dir_index=job.dir_index,
                       alpha_steps=job.alpha_steps, timings=t)
    t["total"] = time.perf_counter() - t0
    if limit is not None:
        limit.unregister()
    return i, E, t


def split_directions(job: Job, pieces: int) -> list:
    """The job as `pieces` jobs over consecutive direction subsets (rows of the whole result)."""
    D = job.dirs.shape[0] if job.dir_index is None else len(job.dir_index)
    idx = np.arange(D) if job.dir_index is None else np.asarray(job.dir_index)
    out = []
    for part in np.array_split(idx, max(1, min(pieces, D))):
        if part.size:
            out.append(dataclasses.replace(job, dir_index=part))
    return out


def run(jobs, workers: int | None = None, split: int = 1):
    """Runs the jobs on a spawn pool; returns (list of E in job order, list of per-job stage seconds
    summed over its pieces, wall seconds).  With split > 1 each job is cut into that many direction
    subsets (for a few large jobs on many workers) and its rows are put back in order."""
    workers = default_workers() if workers is None else int(workers)
    pieces = []
    owner = []
    for j, job in enumerate(jobs):
        for sub in (split_directions(job, split) if split > 1 else [job]):
            pieces.append(sub)
            owner.append(j)
    t0 = time.perf_counter()
    if workers <= 1 or len(pieces) <= 1:
        res = [_run((i, p)) for i, p in enumerate(pieces)]
    else:
        # a worker that dies (or cannot start) breaks the executor with an error instead of being
        # replaced again and again
        with cf.ProcessPoolExecutor(max_workers=min(workers, len(pieces)), mp_context=mp.get_context("spawn")) as ex:
            res = list(ex.map(_run, list(enumerate(pieces))))
    wall = time.perf_counter() - t0
    res.sort(key=lambda r: r[0])
    Es = [[] for _ in jobs]
    times = [dict(matched_filter=0.0, beamform=0.0, envelope=0.0, total=0.0) for _ in jobs]
    for (i, E, t) in res:
        j = owner[i]
        Es[j].append(E)
        for k in times[j]:
            times[j][k] += t[k]
    return [np.concatenate(e, axis=0) for e in Es], times, wall
