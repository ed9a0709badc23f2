"""Autotuner for the launch configuration of the shifted solver.

Candidates are timed on the caller's own solver and operator (no extra device
memory): for each candidate the solver is re-initialised with the caller's
start vector and run for a few iterations, timed as whole iterations with HIP
events on the solver's stream (best of two starts), and the fastest wins.
Whole iterations are timed because a launch shape also changes what the
caches hold for the other kernels of the step.  The solver
is left freshly initialised with the winning configuration.  Choices are
cached in a JSON file keyed by device, method, storage, layout and the
power-of-two buckets of the dimension and shift count, so later solvers of
a similar size skip the search.

Knobs searched:
  whole-x mode:          steps per block of the update (blocked update), or
                         the per-step update's shift block and grid order, x
                         nontemporal streaming
  Heisenberg operators:  work-groups of the row product
The shift block, streaming and grid order change no result bit (each element
is computed by the same arithmetic whatever the launch shape); the steps per
block and the product's work-group count change rounding only (the order of
the x, p sums and of the r.Hr sum).
"""
import json
import math
import os

import torch

from . import komega as K

# whole-x candidates (steps per block, shift block, nontemporal, order): the
# blocked update at 32, 16 and 8 steps, and the per-step update in two shapes
SHIFT_CANDIDATES = ([(steps, 2, nt, 0) for steps in (32, 16, 8) for nt in (0, 1)]
                    + [(1, 2, 1, 0), (1, 8, 1, 1)])
HEIS_VARIANTS = (1,)   # the row kernel; the group kernel (2) lost at every size measured
SPMV_BLOCKS = (0, 1024, 1280, 1472, 1792)   # 0 = the library's automatic choice (one resident round)


def cache_path():
    return os.environ.get("KOMEGA_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "komega_hip", "tune.json"))


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, table):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _bucket(n):
    return 1 << max(0, round(math.log2(max(int(n), 1))))


def key(solver, op, what):
    dev = torch.cuda.get_device_name(torch.cuda.current_device()).replace("|", "/")
    layout = "batched" if solver.rows is not None else f"nrhs{solver.nrhs}"
    store = "c64" if solver.x32 else ("f64" if solver.method == K.CG_R else "c128")
    return "|".join([what, dev, str(solver.method), store, layout, op.kind,
                     f"M~{_bucket(solver.ndim)}", f"nz~{_bucket(solver.nz)}", f"nl{solver.nl}"])


def _time_iterations(solver, op, b, P, iters, warm, reps=2):
    """Mean time of one whole iteration (every kernel of the step, so that a
    launch shape's effect on the caches of the other kernels counts), timed
    with HIP events on the solver's stream; best of `reps` fresh starts."""
    st = solver._stream_obj
    best = None
    for _ in range(reps):
        solver.init(b, P=P, x=solver.x)
        solver.iterate(op, warm)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        solver.iterate(op, iters)
        e1.record(st)
        e1.synchronize()
        t = e0.elapsed_time(e1) / iters
        best = t if best is None else min(best, t)
    return best


def autotune(solver, op, b, P=None, iters=6, warm=2, use_cache=True, path=None):
    """Choose the fastest launch configuration for this solver and operator.
    b, P: the start vector and projection the solve will use (the solver is
    re-initialised with them at the end).  Returns the chosen settings and the
    per-candidate timings (empty when taken from the cache)."""
    path = path or cache_path()
    table = _load(path) if use_cache else {}
    chosen, timings = {}, {}
    if solver.nl == 0:
        k = key(solver, op, "shift")
        if k in table and "shift_steps" in table[k]:
            steps, sb, nt, order = (table[k]["shift_steps"], table[k]["shift_block"], table[k]["shift_nt"],
                                    table[k].get("shift_order", 0))
        else:
            best = None
            for steps, sb, nt, order in SHIFT_CANDIDATES:
                solver.set_tuning(K.T_SHIFT_STEPS, steps)
                solver.set_tuning(K.T_SHIFT_BLOCK, sb)
                solver.set_tuning(K.T_SHIFT_NT, nt)
                solver.set_tuning(K.T_SHIFT_ORDER, order)
                # whole blocks are timed (at least 32 steps), so every
                # candidate applies its blocks as a long solve does
                n = -(-max(iters, 32) // steps) * steps
                t = _time_iterations(solver, op, b, P, n, warm)
                timings[f"shift_steps={steps},shift_block={sb},nt={nt},order={order}"] = t
                if best is None or t < best[0]:
                    best = (t, steps, sb, nt, order)
            _, steps, sb, nt, order = best
            table[k] = {"shift_steps": steps, "shift_block": sb, "shift_nt": nt, "shift_order": order,
                        "ms": best[0]}
        solver.set_tuning(K.T_SHIFT_STEPS, steps)
        solver.set_tuning(K.T_SHIFT_BLOCK, sb)
        solver.set_tuning(K.T_SHIFT_NT, nt)
        solver.set_tuning(K.T_SHIFT_ORDER, order)
        chosen.update(shift_steps=steps, shift_block=sb, shift_nt=nt, shift_order=order)
    if op.kind == "heisenberg":
        k = key(solver, op, "heis")
        if k in table:
            v, nb = table[k]["variant"], table[k].get("spmv_blocks", 0)
        else:
            best = None
            for v in HEIS_VARIANTS:
                try:
                    op.set_variant(v)
                except K.KomegaError:
                    continue  # does not fit this operator
                for nb in SPMV_BLOCKS:
                    solver.set_tuning(K.T_SPMV_BLOCKS, nb)
                    t = _time_iterations(solver, op, b, P, iters, warm)
                    timings[f"heis_variant={v},spmv_blocks={nb}"] = t
                    if best is None or t < best[0]:
                        best = (t, v, nb)
            _, v, nb = best
            table[k] = {"variant": v, "spmv_blocks": nb, "ms": best[0]}
        op.set_variant(v)
        solver.set_tuning(K.T_SPMV_BLOCKS, nb)
        chosen.update(heis_variant=v, spmv_blocks=nb)
    if use_cache:
        _store(path, table)
    solver.init(b, P=P, x=solver.x)
    return chosen, timings
