"""The FP64 oracle's per-tile work of one problem on a pool of host
processes (tests only).  Each worker builds the problem once, from the
arguments it is started with; a call then carries only tile arguments:
Local-Solver runs (oracle.solver.local_solve) and network starts
(oracle.warm.network_start_tile).  Workers are spawned, not forked, so they
share nothing with a parent that has initialised the GPU."""
import multiprocessing as mp
import os

_STATE = {}


def _init(geom, model, psfs, y, W, prior, frame):
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)
    from oracle import operator as op
    from oracle.layout import make_layout
    from oracle.solver import Problem
    L = make_layout(*geom, model=model)
    operator = op.FFTOperator(L, psfs, frame) if frame else None
    _STATE["prob"] = Problem(L, psfs, y, W, operator=operator, **prior)


def _local(args):
    from oracle import solver
    return solver.local_solve(_STATE["prob"], *args)


def _network(args):
    from oracle import warm
    return warm.network_start_tile(_STATE["prob"], *args)


def workers():
    """Host CPUs this process may use, at most 16."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


class OraclePool:
    """geom = make_layout's (M, T, p, o, P, G); prior = Problem keywords;
    frame = the FFT backend's frame (None: direct convolution)."""

    def __init__(self, geom, psfs, y, W, prior, frame=None, model="interp", procs=None):
        self.pool = mp.get_context("spawn").Pool(procs or workers(), initializer=_init,
                                                 initargs=(geom, model, psfs, y, W, prior, frame))

    def local(self, jobs):
        return self.pool.map(_local, jobs, chunksize=1)

    def network(self, jobs):
        return self.pool.map(_network, jobs, chunksize=1)

    def close(self):
        self.pool.close()
        self.pool.join()
