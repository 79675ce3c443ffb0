"""Process pool for the oracle's column loop (test infrastructure).

The columns of the method are independent (the letter generates G column by
column, in parallel over j), so the oracle spreads them over host cores.  The
workers come from a fork server: a clean Python process started once, before
anything in the calling process touches a GPU, which then forks each worker.
A process whose GPU runtime is live is never forked (its runtime threads and
locks would be copied into the child in whatever state they were in), and a
worker that dies raises BrokenProcessPool in the caller instead of being
silently replaced.

start() must therefore run before the first GPU call of a process that wants
more than one oracle worker; executor() refuses otherwise.
"""
from __future__ import annotations

import concurrent.futures as cf
import multiprocessing as mp
import multiprocessing.forkserver as _fs
import os

_PRELOAD = ["numpy", "scipy.linalg", "oracle.solve"]
_started = False


def gpu_runtime_live() -> bool:
    """True when this process holds the kernel driver's compute device open
    (any HIP runtime initialisation does), or torch reports an initialised
    CUDA/HIP state."""
    try:
        for fd in os.listdir("/proc/self/fd"):
            try:
                if os.readlink(f"/proc/self/fd/{fd}") == "/dev/kfd":
                    return True
            except OSError:
                continue
    except OSError:
        pass
    import sys
    torch = sys.modules.get("torch")
    try:
        return bool(torch is not None and torch.cuda.is_initialized())
    except Exception:
        return False


def start() -> None:
    """Start the fork server (idempotent).  Call before any GPU work."""
    global _started
    if _started:
        return
    if gpu_runtime_live():
        raise RuntimeError("oracle.pool.start() after the GPU runtime was initialised in this "
                           "process; start the pool first")
    mp.set_forkserver_preload(_PRELOAD)
    _fs.ensure_running()
    _started = True


def default_workers() -> int:
    env = os.environ.get("ORACLE_WORKERS")
    if env:
        return max(1, int(env))
    return max(1, min(16, len(os.sched_getaffinity(0))))


def executor(workers: int, initializer=None, initargs=()) -> cf.ProcessPoolExecutor:
    """A ProcessPoolExecutor over fork-server workers.  Starts the server
    when no GPU runtime is live yet; refuses when one is and the server was
    not started before it."""
    if not _started:
        start()
    return cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("forkserver"),
                                  initializer=initializer, initargs=initargs)
