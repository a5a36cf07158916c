"""Oracle rows assembled in parallel worker processes (test infrastructure).

The oracle stays single-threaded; large parity cases split their rows over
a pool of spawned processes (at most 16, one per available core), each of
which imports only the oracle and runs ``assemble_rows`` on its share."""
import os
from concurrent.futures import ProcessPoolExecutor
import multiprocessing as mp

import numpy as np


def _rows(args):
    import oracle as O
    spec, rows = args
    return O.Problem(spec).assemble_rows(rows)


def workers():
    return max(1, min(16, len(os.sched_getaffinity(0))))


def assemble_rows(spec, rows, nproc=None):
    """Rows `rows` of the oracle matrix of `spec` as a (len(rows), n) array."""
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    nproc = nproc or workers()
    parts = [p for p in np.array_split(rows, min(nproc, len(rows))) if len(p)]
    if len(parts) == 1:
        return _rows((spec, parts[0]))
    with ProcessPoolExecutor(max_workers=len(parts), mp_context=mp.get_context("spawn")) as ex:
        out = list(ex.map(_rows, [(spec, p) for p in parts]))
    return np.concatenate(out, axis=0)


def assemble(spec, nproc=None):
    """The full oracle matrix (column-major complex128), rows in parallel."""
    n = spec.order
    nproc = nproc or workers()
    # interleaved rows: both equation blocks in every share
    shares = [np.arange(s, n, nproc * 4, dtype=np.int32) for s in range(nproc * 4)]
    A = np.empty((n, n), dtype=np.complex128, order="F")
    rows_all = np.concatenate(shares)
    A[rows_all] = assemble_rows(spec, rows_all, nproc)
    return A
