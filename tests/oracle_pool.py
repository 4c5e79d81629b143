"""Oracle evaluations of many parameter points in parallel CPU processes.

Test infrastructure: the workers are fresh interpreters (spawn) that load
only the oracle and the events (memory-mapped from a file), never the GPU
library."""
import multiprocessing as mp
import os

import numpy as np

_state = {}


def _init(desc, xpath, wpath):
    import oracle
    _state["om"] = oracle.Model(desc)
    _state["x"] = np.load(xpath, mmap_mode="r")
    _state["w"] = None if wpath is None else np.load(wpath, mmap_mode="r")


def _eval(theta):
    om = _state["om"]
    nll, g, _, bad = om.nll(np.asarray(_state["x"]), np.asarray(theta), w=_state["w"], order=1)
    return nll, np.asarray(g)[om.free], bad


def workers():
    return max(1, min(16, os.cpu_count() or 1))


def oracle_points(desc, x64, thetas, tmpdir, w64=None):
    """[(nll, gradient over free parameters, bad count)] at each point."""
    xpath = os.path.join(str(tmpdir), "x.npy")
    np.save(xpath, np.ascontiguousarray(x64, dtype=np.float64))
    wpath = None
    if w64 is not None:
        wpath = os.path.join(str(tmpdir), "w.npy")
        np.save(wpath, np.ascontiguousarray(w64, dtype=np.float64))
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers(), initializer=_init, initargs=(desc, xpath, wpath)) as pool:
        return pool.map(_eval, [np.asarray(t, dtype=np.float64) for t in thetas], chunksize=1)
