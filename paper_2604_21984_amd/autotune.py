"""Autotuner for the batched persistent launch.

Picks the tile shape of the work items (16 x 16 or 32 x 8 pixels), the persistent grid
size (workgroups per compute unit) and the work assignment (contiguous runs of tiles per
workgroup, which keeps neighbouring tiles in one XCD's L2, or round robin) by timing
graph-replayed iterations of the actual batch, then the
propagation schedule: the candidate update period f (propagate every f-th iteration,
App. B.3), judged at equal wall time from the batch's current state (the start of the
encode when the tuner runs first): the first candidate period runs `window` iterations,
every other period runs for as long as that took, and the period with the lowest batch
loss at that time wins.  The schedule trials start where the encode starts because the
period changes the pass index, and with it the jump schedule and the cost of the
early, long-jump passes: trials from a warmed-up state re-run long jumps that the real
encode has behind it, and favoured f = 4, which loses at equal wall time over a whole
1000-iteration encode.  The launch-shape trials start from the state reached after
`warm` iterations past the current one (the first iterations of an encode cost many
times the steady state, so timing them would tune for the wrong regime).  The batch's
state is restored after the trials, so tuning does not change the encode.  Results are
cached per workload signature (image shapes, site counts, K) in memory and optionally
in a JSON file.
"""
import json
import os

import torch


def _signature(enc):
    return f"K{enc.K}|" + ";".join(f"{h}x{w}:{n}" for (h, w), n in zip(enc.shapes, enc.n_sites))


def candidates(n_items, n_cu):
    out = [(0, 0)]  # one workgroup per tile
    for per_cu in (2, 3, 4, 6, 8):
        g = per_cu * n_cu
        if g < n_items:
            out += [(g, 1), (g, 0)]
    return out


class Autotuner:
    def __init__(self, cache_path=None):
        self.cache_path = cache_path
        self.cache = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                self.cache = json.load(f)

    def tune(self, enc, pairs=3, reps=2, schedules=(1,), window=128, warm=12,
             tile_widths=(16, 32)):
        """Return (grid, chunked, timings) for a BatchEncoder and apply the best launch
        (its tile width is then enc.tile_w);
        with more than one candidate update period in `schedules` also pick and apply
        the period (reported under timings["prop_every"]).  `warm` (even) iterations
        are run first and every launch trial starts from the state they reach; the
        schedule trials start from the state the batch had on entry."""
        sig = (_signature(enc) + f"|f{','.join(map(str, schedules))}"
               f"|t{','.join(map(str, tile_widths))}")
        if sig in self.cache:
            grid, chunked, tw = self.cache[sig]["best"]
            enc.set_launch(grid, chunked, tw)
            if "prop_every" in self.cache[sig]:
                enc.set_prop_every(self.cache[sig]["prop_every"])
            return grid, chunked, self.cache[sig]["timings"]
        if enc.cur != 0:
            raise RuntimeError("tune after an even number of iterations (the trials record "
                               "graphs of iteration pairs)")
        n_cu = torch.cuda.get_device_properties(enc.device).multi_processor_count
        orig = enc.snapshot()
        for _ in range(2 * ((max(0, warm) + 1) // 2)):
            enc.step()
        snap = enc.snapshot()
        timings = {}
        for tw in tile_widths:
            enc.set_launch(0, 0, tw)
            for grid, chunked in candidates(enc.T_tot, n_cu):
                enc.restore(snap)
                enc.set_launch(grid, chunked, tw)
                enc.capture()
                enc.replay(1)
                torch.cuda.synchronize()
                best = float("inf")
                for _ in range(reps):
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record()
                    enc.replay(pairs)
                    e1.record()
                    torch.cuda.synchronize()
                    best = min(best, e0.elapsed_time(e1) / (2 * pairs))
                timings[f"{grid}/{chunked}/{tw}"] = best
        enc.restore(orig)
        key = min(timings, key=timings.get)
        grid, chunked, tw = (int(x) for x in key.split("/"))
        enc.set_launch(grid, chunked, tw)
        self.cache[sig] = {"best": [grid, chunked, tw], "timings": timings}
        if len(schedules) > 1:
            sched = {}

            def run(n_pairs):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                enc.replay(n_pairs)
                e1.record()
                torch.cuda.synchronize()
                return e0.elapsed_time(e1)

            chunk = 1           # pairs of iterations between two clock readings
            budget = None
            for f in schedules:
                enc.restore(orig)
                enc.set_prop_every(f)
                enc.capture()
                enc.replay(1)           # the graph's first replay, untimed
                torch.cuda.synchronize()
                enc.restore(orig)
                t, its, last = 0.0, 0, 0.0
                if budget is None:      # the first period sets the wall-time budget
                    while its < window:
                        t += run(chunk)
                        its += 2 * chunk
                    budget = t
                else:                   # others stop before they would exceed it
                    while its == 0 or t + last <= budget:
                        last = run(chunk)
                        t += last
                        its += 2 * chunk
                sched[f] = (t, its, sum(enc.losses()))
            best_f = min(schedules, key=lambda f: (sched[f][2], f))
            enc.restore(orig)
            enc.set_prop_every(best_f)
            timings["prop_every"] = {str(f): {"ms": v[0], "iterations": v[1], "loss": v[2]}
                                     for f, v in sched.items()}
            timings["prop_every_best"] = best_f
            self.cache[sig]["prop_every"] = best_f
        if self.cache_path:
            with open(self.cache_path, "w") as f:
                json.dump(self.cache, f, indent=1)
        return grid, chunked, timings
