"""The CPU oracle on all host cores -- TEST INFRASTRUCTURE.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use this module.  Each worker thread makes one call of the
unchanged single-threaded oracle (``libsco.so``; a ctypes call releases the
Python lock) over its own contiguous range of photon indices or its own
list of pixels, and the results are merged in range order.  Photons and
camera paths draw counter-based random numbers (Philox), so every photon
and every pixel is computed exactly as in one sequential call.  The only
difference is the caustic map: each cell is the FP64 sum of its range
sums, added in range order, instead of one FP64 sum in photon order; the
two differ by reassociation only (relative ~1e-15), far below the single
rounding to FP32 that follows.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import OracleScene, render as _render, render_outputs, sincos2pi, trace_photons as _trace_photons


def host_threads(cap: int = 16) -> int:
    """Worker threads: the host's cores, at most `cap`."""
    return max(1, min(cap, os.cpu_count() or 1))


def _ranges(a: int, b: int, k: int):
    k = max(1, min(k, b - a)) if b > a else 1
    return [(a + (b - a) * i // k, a + (b - a) * (i + 1) // k) for i in range(k)]


def trace_photons(osc: OracleScene, n_photons: int, max_depth: int, wl, seed: int, p0: int = 0, p1=None,
                  threads: int | None = None):
    """The oracle's photon pass over [p0, p1) on `threads` threads.  Returns
    what oracle.trace_photons returns: (map f32, map FP64 sums, counts,
    stats)."""
    p1 = n_photons if p1 is None else p1
    threads = threads or host_threads()
    sincos2pi(0.0)   # the oracle's sin/cos table is filled once, before the threads
    parts = _ranges(p0, p1, threads)
    with ThreadPoolExecutor(len(parts)) as ex:
        res = list(ex.map(lambda r: _trace_photons(osc, n_photons, max_depth, wl, seed, p0=r[0], p1=r[1]), parts))
    msum = res[0][1]
    cnt = res[0][2]
    stats = dict(res[0][3])
    for _, ms, c, st in res[1:]:
        msum += ms
        cnt += c
        for k, v in st.items():
            stats[k] = v + stats[k] if k == "segments" else (stats[k][0] + v[0], stats[k][1] + v[1])
    return msum.astype(np.float32), msum, cnt, stats


def render(osc: OracleScene, cam, spp: int, max_depth: int, wl, seed: int, caustic_map=None, pixels=None,
           want_tie: bool = False, threads: int | None = None, chunks_per_thread: int = 4):
    """oracle.render over the listed pixels (all if None) on `threads`
    threads, each taking contiguous slices of the list in turn."""
    threads = threads or host_threads()
    sincos2pi(0.0)
    if pixels is None:
        pixels = np.arange(cam.w * cam.h, dtype=np.uint32)
    pixels = np.ascontiguousarray(pixels, dtype=np.uint32)
    out = render_outputs(cam, want_tie)
    cmap = None if caustic_map is None else np.ascontiguousarray(caustic_map, dtype=np.float32)
    parts = _ranges(0, len(pixels), threads * chunks_per_thread)

    def run(r):
        if r[1] <= r[0]:
            return 0
        return _render(osc, cam, spp, max_depth, wl, seed, caustic_map=cmap, pixels=pixels[r[0]:r[1]],
                       want_tie=want_tie, out=out)["segments"]

    with ThreadPoolExecutor(threads) as ex:
        segs = sum(ex.map(run, parts))
    out["segments"] = segs
    return out
