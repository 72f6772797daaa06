"""Runs the FP64 oracle over many independent lines or rows on the host's cores, for parity
checks whose oracle work would take minutes on one core. The workers are started fresh
(spawn context: a new interpreter, never a fork of a process that holds GPU state) and
import only numpy, scipy and the oracle."""
from __future__ import annotations

import multiprocessing as mp
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np


def host_workers(cap: int = 16) -> int:
    """Worker count: the CPUs this process may run on, at most `cap`."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(cap, n))


def _one_thread():
    """Worker initializer: one BLAS/OpenMP thread per worker (the pool already fills the host's
    cores; a thread pool per worker, sized by OMP_NUM_THREADS, would oversubscribe them)."""
    os.environ["OMP_NUM_THREADS"] = "1"
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:
        pass


def pool(workers: int | None = None) -> ProcessPoolExecutor:
    return ProcessPoolExecutor(max_workers=workers or host_workers(), mp_context=mp.get_context("spawn"),
                               initializer=_one_thread)


def mapper(ex: ProcessPoolExecutor, chunksize: int = 16):
    """map_lines for the oracle's 2-D filters: fn over the lines on the pool, order kept."""
    return lambda fn, items: ex.map(fn, items, chunksize=chunksize)


def rel_l2(a, b) -> float:
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def row_errors(task):
    """One row of a batched transform: the oracle's forward of x_row with `plan` against the
    GPU's output row `got` (complex64). Returns (row id, rel-L2 over the row, over its first
    `edge` outputs, over its last `edge` outputs)."""
    from oracle import morlet_oracle as O
    rid, x_row, got, plan, edge = task
    got = np.asarray(got, dtype=np.complex128)
    want = O.forward(np.asarray(x_row, dtype=np.float64), plan)
    n = got.shape[0]
    e = min(edge, n)
    return (rid, rel_l2(got, want), rel_l2(got[:e], want[:e]), rel_l2(got[n - e:], want[n - e:]))


_SCALOGRAM_X = None


def scalogram_chunk_errors(task):
    """Rows of the ragged-scalogram workload: the worker regenerates the seeded input itself
    (workloads.ragged_scalogram, the same values the GPU read) and reads the GPU's output rows
    from the shared-memory block the parent filled. task = (block name, output length, rows
    [(row id, signal b, length, output offset)], oracle plan per row, edge length per row).
    Returns [(row id, rel-L2 row, first edge, last edge)]."""
    global _SCALOGRAM_X
    from multiprocessing import shared_memory
    import workloads
    from oracle import morlet_oracle as O
    if _SCALOGRAM_X is None:
        x, lengths, _, _ = workloads.ragged_scalogram()
        _SCALOGRAM_X = (x.astype(np.float64), np.concatenate([[0], np.cumsum(lengths)]))
    xd, offs = _SCALOGRAM_X
    name, total, rows, plans, edges = task
    shm = shared_memory.SharedMemory(name=name)
    try:
        W = np.ndarray((total,), dtype=np.complex64, buffer=shm.buf)
        out = []
        for (rid, b, n, o), plan, edge in zip(rows, plans, edges):
            want = O.forward(xd[offs[b]:offs[b] + n], plan)
            g = W[o:o + n].astype(np.complex128)
            e = min(edge, n)
            out.append((rid, rel_l2(g, want), rel_l2(g[:e], want[:e]), rel_l2(g[n - e:], want[n - e:])))
        del W
    finally:
        shm.close()
    return out
