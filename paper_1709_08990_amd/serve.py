"""Serving loop driver over the library's native scheduler (svb_server_*).

The scheduler (C++ in the library) keeps the list pool in device memory, admits
queries by output memory and launches continuous batches; this module feeds it
queries on a clock and measures latency: a query's latency runs from its
(scheduled) arrival to the moment the host sees it complete.
"""
import time

import numpy as np

from . import (svb_server_create, svb_server_destroy, svb_server_poll, svb_server_release, svb_server_replay,
               svb_server_replay_poisson,
               svb_server_set_batching, svb_server_stats, svb_server_step, svb_server_submit)


class Server:
    """A native serving scheduler over a device-resident pool of streams.

    counts, in_off, in_bytes: device uint64 tensors (one entry per list); streams: device
    uint8 tensor holding all lists; starts: device int32 tensor of delta start values, or
    None for plainly coded lists."""

    def __init__(self, counts, in_off, in_bytes, streams, starts=None, arena_bytes=1 << 30, slots=4,
                 max_batch_lists=8192):
        self._keep = (counts, in_off, in_bytes, streams, starts)
        self.m = counts.numel()
        self.handle = svb_server_create(self.m, counts, in_off, in_bytes, streams, starts, arena_bytes, slots,
                                        max_batch_lists)

    def submit(self, query_id, list_ids):
        svb_server_submit(self.handle, query_id, list_ids)

    def step(self, block=False):
        return svb_server_step(self.handle, block)

    def poll(self):
        return svb_server_poll(self.handle)

    def release(self, query_id):
        svb_server_release(self.handle, query_id)

    def stats(self):
        return svb_server_stats(self.handle)

    def set_batching(self, min_lists, max_wait_us):
        """While a batch is on the device, hold the next one until min_lists lists are admitted
        or its oldest query has waited max_wait_us."""
        svb_server_set_batching(self.handle, min_lists, max_wait_us)

    def replay(self, picks, arrivals=None, outstanding=0):
        """Native load generator: open loop at ``arrivals`` or closed loop with ``outstanding``
        queries in flight; results are released unread.  Returns (latencies, wall seconds)."""
        return svb_server_replay(self.handle, picks, arrivals, outstanding)

    def replay_poisson(self, trace, qps, seconds, warmup_s=0.25, seed=0):
        """Native open loop with Poisson arrivals drawn in the call over a trace used cyclically;
        returns the figures (queries, ints, wall_s, p50_s, p99_s, mean_s, generated, batches)."""
        return svb_server_replay_poisson(self.handle, trace, qps, seconds, warmup_s, seed)

    def close(self):
        if self.handle:
            svb_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_open_loop(server, arrivals, picks, on_result=None):
    """Submits query i at time arrivals[i] (seconds from start) until all complete.
    on_result(query_id, arena_offset, ints) runs before each result is released.
    Returns (latencies in seconds, wall seconds)."""
    nq = len(picks)
    lat = np.zeros(nq)
    t0 = time.perf_counter()
    nxt = done = 0
    while done < nq:
        now = time.perf_counter() - t0
        while nxt < nq and arrivals[nxt] <= now:
            server.submit(nxt, picks[nxt])
            nxt += 1
        server.step(block=False)
        fin = server.poll()
        now = time.perf_counter() - t0
        for qid, off, n in fin:
            lat[qid] = now - arrivals[qid]
            if on_result is not None:
                on_result(qid, off, n)
            server.release(qid)
        done += len(fin)
    return lat, time.perf_counter() - t0


def run_closed_loop(server, picks, outstanding):
    """Keeps `outstanding` queries in the system until all of picks are served.
    Returns (latencies in seconds, wall seconds)."""
    nq = len(picks)
    lat = np.zeros(nq)
    sent = np.zeros(nq)
    t0 = time.perf_counter()
    nxt = done = 0
    while done < nq:
        while nxt < nq and nxt - done < outstanding:
            sent[nxt] = time.perf_counter() - t0
            server.submit(nxt, picks[nxt])
            nxt += 1
        server.step(block=True)
        fin = server.poll()
        now = time.perf_counter() - t0
        for qid, off, n in fin:
            lat[qid] = now - sent[qid]
            server.release(qid)
        done += len(fin)
    return lat, time.perf_counter() - t0
