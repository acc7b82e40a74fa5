"""Oracle reference runs too long for the body of one test (minutes of CPU
time at the workloads' full sizes).  conftest.py starts the jobs that the
collected tests ask for (marker ``oracle_job("name")``) as background
processes when collection ends, so they run while the other GPU tests do;
a test then waits for its result with ``oracle_result``.

Each job calls the oracle only (no HIP library, no torch):
  * ``option_batch``: serial fine integration of each of the 512 options of
    the batched workload (process pool over the options).

Usage: python -m tests.oracle_jobs NAME OUT.npy
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import OPTION_BATCH, option_batch  # noqa: E402


def _one_option(o):
    return oracle.serial_fine(oracle.params_from(o), o["M"], o["N"], OPTION_BATCH["fine_steps"],
                              OPTION_BATCH["payoff_mode"]).ravel()


def option_batch_ref(workers: int = 8):
    """Serial fine solution of every option, packed option after option
    ((N_o+1) x M_o each, in option order)."""
    from multiprocessing import Pool
    opts = option_batch(OPTION_BATCH)
    # largest first, so the pool's tail is short
    order = sorted(range(len(opts)), key=lambda i: -opts[i]["N"] * opts[i]["M"])
    with Pool(workers) as pool:
        parts = pool.map(_one_option, [opts[i] for i in order], chunksize=1)
    out = [None] * len(opts)
    for i, a in zip(order, parts):
        out[i] = a
    return np.concatenate(out)


JOBS = {"option_batch": option_batch_ref}

# Started jobs of this test session: name -> (process, output path, start time)
_RUNNING = {}
_DIR = [None]


def start(names):
    """Start the named jobs as background processes (once per session)."""
    names = [n for n in names if n not in _RUNNING]
    if not names:
        return
    if _DIR[0] is None:
        _DIR[0] = tempfile.mkdtemp(prefix="bsp_oracle_jobs_")
    for name in names:
        out = os.path.join(_DIR[0], f"{name}.npy")
        log = open(os.path.join(_DIR[0], f"{name}.log"), "w")
        proc = subprocess.Popen([sys.executable, "-m", "tests.oracle_jobs", name, out], cwd=ROOT,
                                stdout=log, stderr=subprocess.STDOUT)
        _RUNNING[name] = (proc, out, time.time())


def stop_all():
    for proc, _, _ in _RUNNING.values():
        if proc.poll() is None:
            proc.kill()
            proc.wait()
    _RUNNING.clear()
    if _DIR[0]:
        shutil.rmtree(_DIR[0], ignore_errors=True)
        _DIR[0] = None


def oracle_result(name, timeout=900.0):
    """Wait for the background job `name` (started now if it was not) and load
    its result."""
    import pytest

    if name not in _RUNNING:
        start([name])
    proc, out, t0 = _RUNNING[name]
    last = time.time()
    while proc.poll() is None:
        if time.time() - t0 > timeout:
            proc.kill()
            pytest.fail(f"oracle job {name} took longer than {timeout:.0f} s")
        if time.time() - last > 20:
            print(f"[oracle job {name}] running for {time.time() - t0:.0f} s", flush=True)
            last = time.time()
        time.sleep(0.5)
    if proc.returncode != 0 or not os.path.exists(out):
        with open(os.path.join(_DIR[0], f"{name}.log")) as f:
            pytest.fail(f"oracle job {name} failed: {f.read()[-2000:]}")
    return np.load(out)


def main():
    name, path = sys.argv[1], sys.argv[2]
    t0 = time.time()
    res = JOBS[name]()
    tmp = path + ".tmp.npy"
    np.save(tmp, res)
    os.replace(tmp, path)
    print(f"oracle job {name}: {time.time() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    main()
