"""Throughput of the shifted Krylov iteration on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
                    [--workload heis24|anderson64|anderson64csr|anderson16|batch64|batch64x32|j1j2grad]

A step is one full iteration of the solver: operator product fused with the
inner product r.Hr and alpha, three-term seed update fused with rho / ||r|| /
P r and the recurrences of every shift (pi, alpha^k, beta^k, y/u), seed
switch and convergence test, plus the whole-x shift update when x is kept.
W untimed steps follow the set-up (operator, basis, tables and start vector
are built and resident in HBM before timing); then K steps are timed between
two device synchronisations.

Prints one JSON line.  value = N_z * M * iterations / s (nominal N_z, summed
over right-hand sides).  The roofline object reports the dominant kernel:
algorithmic bytes per launch (algorithmic_bytes below) over its mean launch time,
measured with HIP events on the solver's stream during the timed region.
The K timed steps run in R windows (--repeats, default 5), each between two
device synchronisations; ms_per_step and value are the median window,
"windows" gives the spread.  cpu_baseline times the CPU oracle on a bounded
slice of the same workload (all host threads, median of 3, and one thread in
a child process started before the GPU is touched).

The default run (heis24) adds the metric's two other parts, measured in the
same process: "wholex" (the 64^3 contour workload with every x^(k) kept: the
whole-x update kernel's HBM rate, and the whole iteration's against its
algorithmic bytes) and "gradient" (the J1-J2 coupling gradient: forward +
adjoint time over the forward's, both to convergence).
"""
import argparse
import json
import os
import statistics
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "shifted-COCG N_z·M·iter/s + HBM GB/s on 1 GPU; fwd+adjoint vs fwd time"
UNIT = "N_z·M·iter/s"
HBM_PEAK_GBS = 8000.0
CLASS_NAMES = {0: "k_spmv", 1: "k_seed", 2: "k_shift", 3: "k_dot"}

# HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE runs (KiB per
# full dispatch), scaled by a 2 GiB copy (FETCH x2.00, WRITE x1.00); see
# profiles/hbm_counters.md.  Valid only for the kernel source they were taken
# at: any change to komega_kernels.hip or komega_internal.h turns the figure
# into null.
TRAFFIC_SOURCE_SHA16 = "477a452c5c730ff0"
TRAFFIC_BYTES = {
    ("heis24", "k_spmv"): (84052.9 * 2.0 + 48414.9) * 1024,
    ("heis24", "k_seed"): (84641.5 * 2.0 + 42380.6) * 1024,
    ("anderson64", "k_shift"): (3155757.8 * 2.0 + 4194640.9) * 1024,   # one launch = 32 composed steps
    ("anderson64", "k_seed"): (98626.1 * 2.0 + 65729.3) * 1024,
    ("anderson64", "k_spmv"): (58381.4 * 2.0 + 82164.0) * 1024,
    ("batch64", "k_shift"): (5547758.3 * 2.0 + 10111973.0) * 1024,   # one launch = 32 composed steps
    ("anderson64csr", "k_spmv"): (143636.0 * 2.0 + 70261.9) * 1024,
    ("anderson64csr", "k_shift"): (3155821.7 * 2.0 + 4194703.0) * 1024,   # one launch = 32 composed steps
}


def kernel_source_sha16():
    """sha256 prefix of the device code's sources: the kernels and the header
    of constants and layouts they include, concatenated."""
    import hashlib
    h = hashlib.sha256()
    for name in ("komega_kernels.hip", "komega_internal.h"):
        with open(os.path.join(ROOT, "paper_2001_08707_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ----------------------------------------------------------------- workloads
def make_workload(name):
    """Returns (operator description, solver arguments, start data) for the
    named workload; everything is generated from the seeded input module."""
    from paper_2001_08707_amd import inputs as I
    if name == "heis24":
        w = I.config2()
        return dict(name="heisenberg_ring_L24_Sz0_projected", kind="heis", w=w, L=24, nz=w.z.size, nl=1, nrhs=1,
                    M=w.M, tol=1e-10,
                    config={"workload": "heisenberg_ring_L24_Sz0_projected", "L": 24, "M": int(w.M),
                            "n_shifts": int(w.z.size), "shifts": "linspace(-1,8,1024)+0.02i", "method": "cocg",
                            "mode": "projected a^H x (M_left=1)", "b": "S^z(pi) v, v unit random (seed 2)",
                            "operator": "matrix-free Heisenberg, two-table index"})
    if name == "anderson64":
        w = I.config3()
        return dict(name="anderson_64cubed_16rhs_32contour_wholex", kind="stencil", w=w, L=64, nz=w.z.size, nl=0,
                    nrhs=w.b.shape[0], M=w.M, tol=1e-10,
                    config={"workload": "anderson_64cubed_16rhs_32contour_wholex", "L": 64, "M": int(w.M),
                            "W": 16.5, "n_rhs": int(w.b.shape[0]), "n_shifts": int(w.z.size),
                            "shifts": "0.5 exp(2 pi i (j+1/2)/32)", "method": "cocg", "mode": "whole x kept",
                            "operator": "3D periodic stencil"})
    if name == "anderson64csr":
        w = I.config3()
        return dict(name="anderson_64cubed_16rhs_32contour_wholex_csr", kind="csr", w=w, L=64, nz=w.z.size,
                    nl=0, nrhs=w.b.shape[0], M=w.M, tol=1e-10,
                    config={"workload": "anderson_64cubed_16rhs_32contour_wholex_csr", "L": 64, "M": int(w.M),
                            "W": 16.5, "n_rhs": int(w.b.shape[0]), "n_shifts": int(w.z.size),
                            "shifts": "0.5 exp(2 pi i (j+1/2)/32)", "method": "cocg", "mode": "whole x kept",
                            "operator": "CSR of the 3D periodic stencil: 7 real entries per row, int64 row "
                                        "pointers, int32 columns"})
    if name == "anderson16":
        w = I.config1()
        return dict(name="anderson_16cubed_64shifts_projected", kind="stencil", w=w, L=16, nz=w.z.size, nl=1,
                    nrhs=1, M=w.M, tol=1e-10,
                    config={"workload": "anderson_16cubed_64shifts_projected", "L": 16, "M": int(w.M), "W": 4.0,
                            "n_shifts": int(w.z.size), "method": "cocg", "mode": "projected a^H x",
                            "operator": "3D periodic stencil"})
    if name in ("batch64", "batch64x32"):
        w = I.config5()
        x32 = name == "batch64x32"
        rows = [int(i.M) for i in w.instances]
        Mtot = int(sum(rows))
        tag = "anderson_64instances_edges8to40_256shifts_wholex" + ("_complex64" if x32 else "")
        return dict(name=tag, kind="batch", w=w, nz=w.z.size, nl=0, nrhs=1, M=Mtot, tol=1e-10, x32=x32,
                    rows=rows,
                    config={"workload": tag, "instances": len(rows), "M_total": Mtot,
                            "edges": "rng(5).integers(8, 41, 64)", "W": "rng(5).uniform(2, 20, 64)",
                            "n_shifts": int(w.z.size), "shifts": "linspace(-10,10,256)+0.02i", "method": "cocg",
                            "mode": "whole x kept" + (" as complex64 (double arithmetic)" if x32 else ""),
                            "operator": "batched 3D periodic stencils, one launch per kernel class"})
    if name == "j1j2grad":
        w = I.config4()
        return dict(name="j1j2_ring_L20_gradient", kind="grad", w=w, L=20, nz=w.z.size, nl=0, nrhs=1, M=w.M,
                    tol=1e-10,
                    config={"workload": "j1j2_ring_L20_gradient", "L": 20, "M": int(w.M), "n_couplings": 40,
                            "n_shifts": int(w.z.size), "shifts": "linspace(-2,6,256)+0.05i", "method": "cocg",
                            "b": "S^z(pi/2) v, v unit random (seed 4)", "tol": 1e-10,
                            "loss": "sum_k (Im F_k - t_k)^2, t from couplings perturbed by 0.05 N(0,1) (seed 5)"})
    raise SystemExit(f"unknown workload {name}")


# Operator data per row, read once per product for all right-hand sides:
# the spin state (u32), the on-site energy (f64), or a CSR row of the 3D
# stencil (row pointer i64, 7 columns i32 and 7 values f64).
OP_BYTES_PER_ROW = {"heis": 4, "stencil": 8, "batch": 8, "csr": 8 + 7 * (4 + 8)}


def stencil_csr(L, eps, hop=1.0):
    """CSR arrays of the periodic L^3 stencil (diagonal eps_i, -hop on the six
    neighbours; site i = x + L y + L^2 z), columns ascending in each row."""
    import numpy as np
    i = np.arange(L ** 3, dtype=np.int64)
    x, y, z = i % L, (i // L) % L, i // (L * L)
    nb = [((x + dx) % L) + L * ((y + dy) % L) + L * L * ((z + dz) % L)
          for dx, dy, dz in ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1))]
    cols = np.stack([i] + nb, axis=1)
    vals = np.concatenate([np.asarray(eps, dtype=np.float64)[:, None], np.full((L ** 3, 6), -hop)], axis=1)
    order = np.argsort(cols, axis=1, kind="stable")
    cols = np.take_along_axis(cols, order, axis=1)
    vals = np.take_along_axis(vals, order, axis=1)
    rowptr = np.arange(0, 7 * L ** 3 + 1, 7, dtype=np.int64)
    return rowptr, cols.reshape(-1).astype(np.int32), vals.reshape(-1)


def algorithmic_bytes(wl, cls, steps=1):
    """Bytes one launch of kernel class `cls` must move at minimum
    (complex128 = 16 B per vector element).  A whole-x update launch that
    applies `steps` composed steps reads and writes x^k, p^k once and reads
    the residual of every step."""
    M, nrhs, nz, nl = wl["M"], wl["nrhs"], wl["nz"], wl["nl"]
    if cls == 0:   # operator product: operator data once + read r, write q per rhs
        op_bytes = OP_BYTES_PER_ROW[wl["kind"]] * M
        return op_bytes + nrhs * M * 32
    if cls == 1:   # seed: read r_n, q, r_{n-1}, write r_{n+1} (per rhs) + P rows once
        return nrhs * M * 64 + nl * M * 16
    if cls == 2:   # whole-x update: read+write x and p for every shift, read r once per step
        per = 32 if wl.get("x32") else 64
        return nrhs * nz * M * per + nrhs * M * 16 * steps
    return 0


def iteration_algorithmic_bytes(wl):
    """What one whole iteration must move at minimum, counted as in the
    method's own cost table (Table 2): the seed reads r_n, r_{n-1} and the
    projection row and writes r_{n+1} (4 x 16 B per row and right-hand side)
    plus the operator data (spin state 4 B or on-site energy 8 B per row); a
    kept solution adds a read and a write of x^k and p^k per shift and row
    (64 B, or 32 B as complex64).  Heisenberg L=24 projected: 68 B per row
    (184 MB); 64^3 contour workload: 8 + 16 x (64 + 32 x 64) B per row
    (8.86 GB; the on-site energies are read once for all right-hand sides)."""
    M, nrhs, nz = wl["M"], wl["nrhs"], wl["nz"]
    op_bytes = OP_BYTES_PER_ROW[wl["kind"]]
    per = 32 if wl.get("x32") else 64
    return M * (op_bytes + nrhs * 64) + (nrhs * nz * M * per if wl["nl"] == 0 else 0)


def blocked_bytes_per_step(wl, steps_blk):
    """Bytes one iteration moves at minimum with the blocked whole-x update:
    Table 2's seed and operator bytes, plus 1/steps_blk of one update launch
    (x^k, p^k read and written once per block, the residual of every step
    read once).  Table 2 counts the x^k, p^k traffic at every step, so its
    per-step bytes over the step time can exceed the HBM peak."""
    per = 32 if wl.get("x32") else 64
    xp_step = wl["nrhs"] * wl["nz"] * wl["M"] * per
    return algorithmic_bytes(wl, 2, steps_blk) / steps_blk + iteration_algorithmic_bytes(wl) - xp_step


def design_bytes_per_row(wl):
    """Bytes per row the two-launch design moves (projected Heisenberg: the
    product reads the state and r_n and writes q; the seed update reads r_n,
    q, r_{n-1} and the projection row and writes r_{n+1})."""
    return 4 + 32 + 80 if wl["kind"] == "heis" else None


# ------------------------------------------------------------- GPU pieces
def build_gpu(wl):
    import torch
    from paper_2001_08707_amd import komega as K
    w = wl["w"]
    if wl["kind"] == "batch":
        import numpy as np
        L = np.array([[i.L] * 3 for i in w.instances], dtype=np.int32)
        op = K.Operator.stencil3d_batch(L, [i.eps for i in w.instances])
        b = torch.as_tensor(np.concatenate([i.b[0] for i in w.instances]), device="cuda")
        s = K.Solver("cocg", w.z, rows=wl["rows"], tol=wl["tol"], itermax=10 ** 7, x32=wl["x32"])
        s.init(b)
        torch.cuda.synchronize()
        return K, op, s, b
    if wl["kind"] == "heis":
        op = K.Operator.heisenberg(wl["L"], wl["L"] // 2, w.bonds, w.J)
        op.set_variant(wl.get("variant", 0))
        b = op.szq(w.w, torch.as_tensor(w.v, device="cuda")).reshape(1, -1)
    elif wl["kind"] == "csr":
        op = K.Operator.csr(*stencil_csr(wl["L"], w.eps))
        b = torch.as_tensor(w.b, dtype=torch.complex128, device="cuda")
    else:
        L = wl["L"]
        op = K.Operator.stencil3d(L, L, L, w.eps)
        b = torch.as_tensor(w.b, dtype=torch.complex128, device="cuda")
    s = K.Solver("cocg", w.z, wl["M"], nl=wl["nl"], nrhs=wl["nrhs"], tol=wl["tol"], itermax=10 ** 7)
    P = torch.conj(b[0]).resolve_conj().reshape(1, -1) if wl["nl"] else None
    s.init(b, P=P)
    torch.cuda.synchronize()
    return K, op, s, b


def timed_windows(s, op, steps, repeats):
    """The K timed steps as `repeats` consecutive windows, each bracketed by
    device synchronisations.  Returns [(seconds, steps)]."""
    import torch
    repeats = max(1, min(repeats, steps))
    out = []
    for r in range(repeats):
        n = steps // repeats + (1 if r < steps % repeats else 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.iterate(op, n)
        torch.cuda.synchronize()
        out.append((time.perf_counter() - t0, n))
    return out


def window_stats(windows):
    ms = [1e3 * t / n for t, n in windows]
    return {"n": len(ms), "steps_each": [n for _, n in windows], "ms_per_step": ms,
            "median": statistics.median(ms), "min": min(ms), "max": max(ms),
            "mean_over_all_steps": 1e3 * sum(t for t, _ in windows) / sum(n for _, n in windows)}


def run_gpu(wl, steps, warmup, repeats=5, dom=None):
    """Set-up, W warm-up steps (timing every kernel class to find the
    dominant one, unless `dom` names it), then K steps in timed windows with
    the dominant class bracketed by HIP events on the solver's stream."""
    import torch
    K, op, s, b = build_gpu(wl)
    tuned = None
    if wl.get("tune"):
        from paper_2001_08707_amd import tune as T
        P = torch.conj(b.reshape(-1)[: wl["M"]]).resolve_conj().reshape(1, -1) if wl["nl"] else None
        chosen, timings = T.autotune(s, op, b, P=P, use_cache=False)
        tuned = {"chosen": chosen, "candidate_ms": timings}
    if wl.get("shift_block"):
        s.set_tuning(K.T_SHIFT_BLOCK, wl["shift_block"])
    if wl.get("shift_nt") is not None:
        s.set_tuning(K.T_SHIFT_NT, wl["shift_nt"])
    if wl.get("shift_order") is not None:
        s.set_tuning(K.T_SHIFT_ORDER, wl["shift_order"])
    if wl.get("spmv_blocks"):
        s.set_tuning(K.T_SPMV_BLOCKS, wl["spmv_blocks"])
    if wl.get("shift_steps"):
        s.set_tuning(K.T_SHIFT_STEPS, wl["shift_steps"])
    # calibration during warm-up: time every kernel class, pick the dominant
    s.set_timing(0xF)
    s.iterate(op, max(warmup, 1))
    torch.cuda.synchronize()
    per = {c: s.get_timing(c) for c in range(4)}
    if dom is None:
        dom = max(per, key=lambda c: per[c][0])
    s.set_timing(1 << dom)
    s.get_timing(dom, reset=True)
    windows = timed_windows(s, op, steps, repeats)
    ms_dom, n_dom = s.get_timing(dom)
    st = s.state()
    done = warmup if warmup >= 1 else 1
    for r in st:
        if r["status"] != K.OK or r["iter"] != done + steps:
            raise SystemExit(f"solver stopped inside the timed region: {r}")
    wall = sum(t for t, _ in windows)
    steps_blk = s.get_tuning(K.T_SHIFT_STEPS) if wl["nl"] == 0 else 1
    out = dict(wall=wall, windows=windows, dom=dom, ms_dom=ms_dom, n_dom=n_dom, tuned=tuned, steps_blk=steps_blk,
               shift_block=s.get_tuning(K.T_SHIFT_BLOCK), shift_nt=s.get_tuning(K.T_SHIFT_NT),
               shift_order=s.get_tuning(K.T_SHIFT_ORDER),
               warm_ms={CLASS_NAMES[c]: per[c][0] / max(per[c][1], 1) for c in per if per[c][1]},
               iters=st[0]["iter"], seed=st[0]["seed"], maxres=st[0]["maxres"])
    s.close()
    op.close()
    return out


def run_unbatched(wl, steps, warmup, chunk):
    """The same 64 systems as separate solvers (two launches per system and
    iteration, plus one whole-x update per system and block, instead of the
    batch's shared launches), for the batching comparison.  Each solver is
    advanced `chunk` steps per call, the batch's block length, so both sides
    compose the same number of steps per whole-x pass."""
    import numpy as np
    import torch
    from paper_2001_08707_amd import komega as K
    w = wl["w"]
    sys_ = []
    for i in w.instances:
        op = K.Operator.stencil3d(i.L, i.L, i.L, i.eps)
        s = K.Solver("cocg", w.z, op.M, tol=wl["tol"], itermax=10 ** 7, x32=wl["x32"])
        s.init(torch.as_tensor(i.b[0], device="cuda"))
        sys_.append((op, s))
    for op, s in sys_:
        s.iterate(op, max(warmup, 1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        n = min(chunk, steps - done)
        for op, s in sys_:
            s.iterate(op, n)
        done += n
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for op, s in sys_:
        s.close()
        op.close()
    return wall


def copy_calibration(nbytes=1 << 31, reps=5):
    """Plain device copy of a known size, for scaling the HBM byte counters."""
    import torch
    x = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": nbytes, "bytes_written": nbytes, "reps": reps}))


def bandwidth_probe(nbytes=1 << 30, reps=20):
    """Bandwidth the HBM sustains for streams like the whole-x update's: the
    library's probe kernels (16-byte nontemporal accesses) copy n bytes (read
    n + write n) and read 2n bytes, timed with HIP events on the current
    stream, best of `reps`."""
    import torch
    from paper_2001_08707_amd import komega as K
    src = torch.ones(2 * nbytes // 16, dtype=torch.complex128, device="cuda")
    dst = torch.empty(nbytes // 16, dtype=torch.complex128, device="cuda")
    part = torch.empty(K.stream_probe_groups(), dtype=torch.complex128, device="cuda")

    def best(fn, moved):
        for _ in range(3):
            fn()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for e0, e1 in ev:
            e0.record()
            fn()
            e1.record()
        torch.cuda.synchronize()
        return moved / (min(e0.elapsed_time(e1) for e0, e1 in ev) * 1e-3) / 1e9

    half = src[: nbytes // 16]
    copy = best(lambda: K.stream_probe(half, dst, 0), 2 * nbytes)
    read = best(lambda: K.stream_probe(src, part, 1), 2 * nbytes)
    del src, dst, part, half
    torch.cuda.empty_cache()
    return {"copy_GBs": copy, "read_GBs": read, "copy_bytes": nbytes, "read_bytes": 2 * nbytes, "reps": reps,
            "kind": "komega_stream_probe: 16-byte nontemporal accesses, best of reps"}


# ------------------------------------------------------------- CPU baseline
def host_cpu():
    """CPU model, sockets, cores and logical CPUs of the host (from
    /proc/cpuinfo), and the CPUs this process may run on (nproc)."""
    info = {"model": None, "sockets": None, "cores_per_socket": None, "logical_cpus": os.cpu_count(),
            "nproc": len(os.sched_getaffinity(0))}
    try:
        phys, cores = set(), None
        with open("/proc/cpuinfo") as f:
            for ln in f:
                k, _, v = ln.partition(":")
                k, v = k.strip(), v.strip()
                if k == "model name" and info["model"] is None:
                    info["model"] = v
                elif k == "physical id":
                    phys.add(v)
                elif k == "cpu cores" and cores is None:
                    cores = int(v)
        info["sockets"] = len(phys) or None
        info["cores_per_socket"] = cores
    except OSError:
        pass
    return info


def _oracle_problem(wl):
    """The oracle's operator, right-hand side and projection for a workload."""
    from oracle import oracle as O
    w = wl["w"]
    if wl["kind"] == "heis":
        oop = O.Operator.heisenberg(wl["L"], wl["L"] // 2, w.bonds, w.J)
        b = O.szq(oop.states, wl["L"], w.w, w.v)
    elif wl["kind"] == "csr":
        oop = O.Operator.csr(*stencil_csr(wl["L"], w.eps))
        b = w.b[0]
    else:
        L = wl["L"]
        oop = O.Operator.stencil3d(L, L, L, w.eps)
        b = w.b[0]
    return oop, b, (b.conj()[None, :] if wl["nl"] else None)


def cpu_slice(wl, n, instances=None, prob=None):
    """Runs the oracle for n iterations of the workload (batch: n iterations
    of each of the first `instances` systems); returns (seconds, N_z*M*iter
    done).  Set-up (operator, basis) is excluded from the time."""
    from oracle import oracle as O
    w = wl["w"]
    if wl["kind"] == "batch":
        t_all, work = 0.0, 0
        for i in w.instances[:instances]:
            oop = O.Operator.stencil3d(i.L, i.L, i.L, i.eps)
            t = time.perf_counter()
            O.solve(oop, i.b[0], w.z, tol=0.0, itermax=n)
            t_all += time.perf_counter() - t
            work += wl["nz"] * i.M * n
        return t_all, work
    oop, b, P = prob or _oracle_problem(wl)
    t = time.perf_counter()
    O.solve(oop, b, w.z, P=P, tol=0.0, itermax=n)
    return time.perf_counter() - t, wl["nz"] * wl["M"] * n


def cpu_baseline(wl, workload, budget_s=12.0):
    """The oracle as it stands, on the host cores: the same workload (one
    right-hand side) for a bounded number of iterations, set-up excluded,
    scaled to N_z*M*iter/s.  All threads: median of 3 runs.  One thread: one
    run in a child process (OMP_NUM_THREADS=1).  Called before the GPU is
    touched, so the child is started from a process without a GPU context."""
    from oracle import oracle as O
    w = wl["w"]
    if wl["kind"] == "batch":
        # instances in order until a third of the budget is spent, 20 iterations each
        n, used, t_used = 20, 0, 0.0
        while used < len(w.instances) and t_used <= budget_s / 3:
            t_used += cpu_slice_one(wl, n, used)
            used += 1
        runs = [cpu_slice(wl, n, instances=used) for _ in range(3)]
        what = f"{n} iterations of each of the first {used} instances (whole x, 256 shifts)"
        child_args = ["--cpu-iters", str(n), "--cpu-instances", str(used)]
    else:
        prob = _oracle_problem(wl)
        t2, _ = cpu_slice(wl, 2, prob=prob)
        n = int(max(2, min(200, budget_s / 3 / max(t2 / 2, 1e-6))))
        runs = [cpu_slice(wl, n, prob=prob) for _ in range(3)]
        what = f"{n} iterations on one right-hand side ({wl['M']} rows x {wl['nz']} shifts)"
        # one thread: about a third of the budget, from the all-threads time per iteration
        t_it = min(t for t, _ in runs) / n
        n1 = int(max(2, min(100 * n, budget_s / 3 / max(t_it * max(O.threads(), 1), 1e-9))))
        child_args = ["--cpu-iters", str(n1)]
    rates = [work / t for t, work in runs]
    out = {"value": statistics.median(rates), "unit": UNIT, "cores": O.threads(), "kind": "oracle",
           "sample": what + f", median of 3 runs ({', '.join(f'{t:.1f}' for t, _ in runs)} s), set-up excluded",
           "runs": rates, "host": host_cpu(),
           "oracle": "plain C99 FP64; OpenMP only over row loops that write disjoint outputs; every "
                     "reduction (inner products, projections) is sequential in index order on one thread"}
    env = dict(os.environ, OMP_NUM_THREADS="1")
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-child", workload] + child_args
    try:
        r = subprocess.run(cmd, env=env, capture_output=True, text=True, timeout=300, check=True)
        one = json.loads(r.stdout.strip().splitlines()[-1])
        out["one_thread"] = {"value": one["work"] / one["seconds"], "cores": one["threads"],
                             "seconds": one["seconds"], "iterations": one["iters"]}
    except (subprocess.SubprocessError, ValueError, KeyError, IndexError) as e:
        out["one_thread"] = {"error": str(e)[:200]}
    return out


def cpu_slice_one(wl, n, k):
    """Seconds for n oracle iterations of batched instance k alone."""
    from oracle import oracle as O
    i = wl["w"].instances[k]
    oop = O.Operator.stencil3d(i.L, i.L, i.L, i.eps)
    t = time.perf_counter()
    O.solve(oop, i.b[0], wl["w"].z, tol=0.0, itermax=n)
    return time.perf_counter() - t


def cpu_child(workload, n, instances):
    from oracle import oracle as O
    wl = make_workload(workload)
    t, work = cpu_slice(wl, n, instances=instances)
    print(json.dumps({"seconds": t, "work": work, "iters": n, "threads": O.threads()}), flush=True)


def run_grad(wl, reps=2):
    """The coupling gradient's cost, every solve to convergence:
      fwd        the forward an autograd function must run: F_k with every
                 x_k kept (N_z shifts), the vectors the backward contracts;
      fwd+adj    forward + adjoint + backward: whole x over {z_k} U {conj z_k}
                 (one Krylov sequence, a = b), F_k, the bond contraction and
                 the chain rule;
      projected  F_k alone (M_left = 1, no vector kept): the cheapest way to
                 get the spectrum without its gradient.
    Best of `reps` wall times each."""
    import torch
    from paper_2001_08707_amd import komega as K
    from paper_2001_08707_amd import grad as G
    w = wl["w"]
    op = K.Operator.heisenberg(wl["L"], wl["L"] // 2, w.bonds, w.J)
    b = op.szq(w.w, torch.as_tensor(w.v, device="cuda"))
    model = G.HeisenbergSpectrum(wl["L"], wl["L"] // 2, w.bonds, b, b, w.z, tol=wl["tol"], itermax=100000)
    J = torch.tensor(w.J, dtype=torch.float64, requires_grad=True)
    Jt = torch.tensor(w.J_target, dtype=torch.float64)
    with torch.no_grad():
        t = model(Jt).imag
    torch.cuda.synchronize()
    tf, ta, tp = [], [], []
    for _ in range(reps):
        t0 = time.perf_counter()
        Fp, stp = K.greens_function(op, b, b, w.z, tol=wl["tol"], itermax=100000)
        torch.cuda.synchronize()
        tp.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        F = model.forward_only(J.detach())
        torch.cuda.synchronize()
        tf.append(time.perf_counter() - t0)
        it_f = model.last["fwd_iters"]
        J.grad = None
        t0 = time.perf_counter()
        F = model(J)
        loss = ((F.imag - t) ** 2).sum()
        loss.backward()
        torch.cuda.synchronize()
        ta.append(time.perf_counter() - t0)
        it_a = model.last["iters"]
    op.close()
    return dict(t_fwd=min(tf), t_fwd_adj=min(ta), t_proj=min(tp), it_fwd=it_f, it_fwd_adj=it_a,
                it_proj=stp["iter"], loss=float(loss.detach()), grad_norm=float(J.grad.norm()))


def gradient_object(wl, g):
    return {"workload": wl["config"]["workload"], "M": int(wl["M"]), "n_shifts": int(wl["nz"]),
            "n_couplings": 40, "tol": wl["tol"],
            "t_fwd_s": g["t_fwd"], "t_fwd_adj_s": g["t_fwd_adj"], "t_projected_s": g["t_proj"],
            "ratio_fwd_adj_over_fwd": g["t_fwd_adj"] / g["t_fwd"],
            "ratio_fwd_adj_over_projected": g["t_fwd_adj"] / g["t_proj"],
            "iterations_fwd": g["it_fwd"], "iterations_fwd_adj": g["it_fwd_adj"],
            "iterations_projected": g["it_proj"], "loss": g["loss"], "grad_norm": g["grad_norm"],
            "fwd": "whole x kept over the 256 shifts (what the backward contracts), to convergence",
            "fwd_adj": "whole x over the 512 shifts {z, conj z} + a^H x + bond contraction + chain rule",
            "projected": "a^H x only (M_left = 1), no vector kept; information, not the target's denominator",
            "target": "fwd_adj <= 2.5 x fwd"}


def run_wholex(steps=64, warmup=32, repeats=2):
    """The 64^3 contour workload (16 right-hand sides x 32 nodes, whole x
    kept) on a short slice whose windows hold whole blocks of the blocked
    update: the update kernel's rate against the bytes one launch moves (x^k
    and p^k read and written once, the residual of every composed step read),
    and the whole iteration's against Table 2's per-step count (which the
    blocked update undercuts: its x^k, p^k traffic is spread over the steps
    of a block)."""
    wl = make_workload("anderson64")
    g = run_gpu(wl, steps, warmup, repeats=repeats, dom=2)
    ws = window_stats(g["windows"])
    t_shift = g["ms_dom"] / max(g["n_dom"], 1) / 1e3
    per_launch = min(g["steps_blk"], steps // repeats)
    b_shift = algorithmic_bytes(wl, 2, per_launch)
    ib = iteration_algorithmic_bytes(wl)
    t_step = ws["median"] / 1e3
    moved = blocked_bytes_per_step(wl, per_launch)
    return {"workload": wl["config"]["workload"], "M": int(wl["M"]), "n_rhs": int(wl["nrhs"]),
            "n_shifts": int(wl["nz"]), "steps": steps, "warmup": warmup, "windows": ws,
            "ms_per_step": ws["median"], "value": wl["nz"] * wl["M"] * wl["nrhs"] / t_step, "unit": UNIT,
            "k_shift": {"steps_per_launch": per_launch, "bytes_per_launch": b_shift, "mean_launch_us": 1e6 * t_shift,
                        "achieved_GBs": b_shift / t_shift / 1e9, "frac": b_shift / t_shift / 1e9 / HBM_PEAK_GBS},
            "iteration": {"table2_bytes": ib, "table2_GBs": ib / t_step / 1e9,
                          "bytes_moved_per_step": moved, "achieved_GBs": moved / t_step / 1e9,
                          "frac": moved / t_step / 1e9 / HBM_PEAK_GBS},
            "launch": {"shift_steps": g["steps_blk"], "shift_nontemporal": g["shift_nt"]}}


# -------------------------------------------------------------------- main
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--repeats", type=int, default=5, help="timed windows the K steps are split into")
    ap.add_argument("--workload", default="heis24",
                    choices=["heis24", "anderson64", "anderson64csr", "anderson16", "batch64", "batch64x32", "j1j2grad"])
    ap.add_argument("--compare-unbatched", action="store_true",
                    help="batch workloads: also time the systems as separate solvers")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true",
                    help="heis24: skip the whole-x and gradient parts of the metric")
    ap.add_argument("--heis-variant", type=int, default=0, help="Heisenberg product kernel (0 auto, 1 row, 2 group)")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--tune", action="store_true", help="run the autotuner before timing (no cache)")
    ap.add_argument("--shift-block", type=int, default=0, help="whole-x update: shifts per thread")
    ap.add_argument("--shift-nt", type=int, default=None, help="whole-x update: 1 = nontemporal streaming")
    ap.add_argument("--shift-order", type=int, default=None,
                    help="whole-x update grid: 0 = row tiles fastest, 1 = shift blocks fastest")
    ap.add_argument("--spmv-blocks", type=int, default=0, help="operator product work-groups (0 automatic)")
    ap.add_argument("--shift-steps", type=int, default=0, help="whole-x update: steps composed per block (0 default)")
    ap.add_argument("--cpu-child", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-iters", type=int, default=2, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-instances", type=int, default=None, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_child:
        cpu_child(args.cpu_child, args.cpu_iters, args.cpu_instances)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the solver has no multi-GPU path (independent "
              "right-hand sides or instances would be split across GPUs, one process each).", file=sys.stderr)
        sys.exit(2)
    wl = make_workload(args.workload)
    wl["variant"] = args.heis_variant
    wl["tune"] = args.tune
    wl["shift_block"] = args.shift_block
    wl["shift_nt"] = args.shift_nt
    wl["shift_order"] = args.shift_order
    wl["spmv_blocks"] = args.spmv_blocks
    wl["shift_steps"] = args.shift_steps
    # the CPU legs run first, before anything touches the GPU
    cpu = None
    if not args.no_cpu and not args.copy_calibration and wl["kind"] != "grad":
        log("cpu baseline ...")
        cpu = cpu_baseline(wl, args.workload)
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    if args.copy_calibration:
        copy_calibration()
        return
    if wl["kind"] == "grad":
        g = run_grad(wl)
        value = wl["nz"] * wl["M"] * g["it_fwd"] / g["t_fwd"]
        print(json.dumps({
            "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": g["it_fwd"], "warmup": 0,
            "ms_per_step": 1e3 * g["t_fwd"] / g["it_fwd"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic", "config": wl["config"],
            "gradient": gradient_object(wl, g)}), flush=True)
        return
    if wl["kind"] in ("stencil", "batch", "csr") and wl["nl"] == 0:
        # ms per step: keep the timed region short; every timed window holds
        # whole blocks of the blocked whole-x update (the library's default
        # block: 32 steps, 16 with complex64 x), so each launch of the update
        # applies the same number of steps
        blk = wl.get("shift_steps") or (16 if wl.get("x32") else 32)
        args.steps = max(blk * args.repeats, min(args.steps, 200) // (blk * args.repeats) * blk * args.repeats)
    log(f"{args.workload}: {args.warmup} warm-up + {args.steps} timed steps in {args.repeats} windows ...")
    g = run_gpu(wl, args.steps, args.warmup, repeats=args.repeats)
    K = args.steps
    ws = window_stats(g["windows"])
    ms_per_step = ws["median"]
    value = wl["nz"] * wl["M"] * wl["nrhs"] / (ms_per_step / 1e3)
    dom = g["dom"]
    bytes_dom = algorithmic_bytes(wl, dom, min(g["steps_blk"], K // args.repeats) if dom == 2 else 1)
    t_dom = g["ms_dom"] / max(g["n_dom"], 1) / 1e3
    achieved = bytes_dom / t_dom / 1e9
    iter_bytes = iteration_algorithmic_bytes(wl)
    traffic = None
    default_launch = not (wl.get("variant") or wl.get("tune") or wl.get("shift_block") or wl.get("spmv_blocks")
                          or wl.get("shift_steps")
                          or wl.get("shift_nt") is not None or wl.get("shift_order") is not None)
    if kernel_source_sha16() == TRAFFIC_SOURCE_SHA16 and default_launch:
        traffic = TRAFFIC_BYTES.get((args.workload, CLASS_NAMES[dom]))
    out = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if not wl.get("x32") else "f64 (x, p stored as c64)", "data": "synthetic",
        "config": wl["config"],
        "roofline": {"bound": "hbm", "kernel": CLASS_NAMES[dom], "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_unit": "bytes per launch", "bytes_per_launch": bytes_dom,
                     "mean_launch_us": t_dom * 1e6,
                     "traffic_over_algorithmic": (traffic / bytes_dom) if traffic else None},
        "windows": ws,
        "iteration": {"algorithmic_bytes": iter_bytes, "algorithmic_bytes_per_row": iter_bytes / wl["M"],
                      "algorithmic_GBs": iter_bytes / (ms_per_step / 1e3) / 1e9,
                      "frac": iter_bytes / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS},
        "kernel_mean_us_warmup": {k: v * 1e3 for k, v in g["warm_ms"].items()},
    }
    dbr = design_bytes_per_row(wl)
    if dbr:
        out["iteration"]["design_bytes_per_row"] = dbr
        out["iteration"]["design_GBs"] = dbr * wl["M"] / (ms_per_step / 1e3) / 1e9
    if wl["nl"] == 0 and g["steps_blk"] > 1:
        moved = blocked_bytes_per_step(wl, min(g["steps_blk"], K // args.repeats))
        out["iteration"].update({
            "note": "algorithmic_* count Table 2's per-step bytes; the blocked whole-x update moves x^k, p^k "
                    "once per block, so the step moves bytes_moved_per_step",
            "bytes_moved_per_step": moved, "moved_GBs": moved / (ms_per_step / 1e3) / 1e9,
            "moved_frac": moved / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS})
    if wl["nl"] == 0:
        out["launch"] = {"shift_steps": g["steps_blk"], "shift_block": g["shift_block"],
                         "shift_nontemporal": g["shift_nt"], "shift_order": g["shift_order"]}
    if g["tuned"]:
        out["autotune"] = g["tuned"]
    if wl["kind"] == "batch" and args.compare_unbatched:
        blk = max(g.get("steps_blk", 1), 1)
        t_sep = run_unbatched(wl, K, args.warmup, blk)
        out["unbatched"] = {"ms_per_step": 1e3 * t_sep / K, "speedup_of_batched": t_sep / g["wall"],
                            "steps_per_call": blk,
                            "launches_per_step": {"batched": 2 + 1 / blk,
                                                  "separate": len(wl["rows"]) * (2 + 1 / blk)}}
    if args.workload == "heis24" and not args.no_extra:
        log("whole-x slice (64^3 contour workload) ...")
        out["wholex"] = run_wholex()
        log("gradient (J1-J2 L=20) ...")
        out["gradient"] = gradient_object(make_workload("j1j2grad"), run_grad(make_workload("j1j2grad")))
    log("bandwidth probe ...")
    probe = bandwidth_probe()
    out["bandwidth_probe"] = probe
    out["roofline"]["frac_of_probe"] = out["roofline"]["achieved"] / max(probe["copy_GBs"], probe["read_GBs"])
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
