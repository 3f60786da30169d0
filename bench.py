"""Throughput benchmark of the thermal PEPS-VMC hot path on one MI355X.

Workload (default): 8x8 open-boundary spin-1/2 Heisenberg model, vectorised
PEPS with d^2 = 4, bond dimension D = 4, boundary dimension chi = 16,
1024 Markov chains x 200 sweeps per SR step, seeded random site tensors of
unit Frobenius norm.  One step = 200 Metropolis sweeps of every chain, each
followed by a measurement of the chain's configuration (log|psi|, E_loc, O
row), then the stochastic-reconfiguration solve by conjugate gradient on all
204,800 samples and the parameter update.  Metric: samples per second of
whole steps (one sample = one chain's sweep + measurement; the SR solve is
inside the timed region).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--budget-s T]

Warm-up: W one-sweep steps of each precision (sweep, measurement, SR on
those 1024 samples, update).  Timed: up to K full steps of the mixed path
(FP32 MFMA strip contractions, FP64 QR/SVD, reductions and SR), stopping
after the step that ends past the wall budget T; `steps` reports how many
were timed.  The plain FP64 path runs at most --fp64-steps full steps from
the same state for the comparison.  Energy error (the precision gate of
`value`): local energies of the same samples and parameters from both
precisions, on the random state after the timed steps and on a cooled state
(identity plus N(0, 0.05^2) noise, cooled through the package's cooling loop
with |rho| sampling up to beta_phys = 0.3 and |rho|^2 after it, to
beta_phys = 4): the mean, the 99th percentile and the largest per-sample
relative error must all lie within --tol on both.  `value` is the rate of the faster of the two paths among those
meeting the bar.

Prints one JSON line.  The CPU baseline is the FP64 oracle (tests only,
never the product path) timed on a bounded sample on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MI355X_HBM_GBS = 8000.0
MI355X_FP64_TFLOPS = 78.6
MI355X_FP32_MFMA_TFLOPS = 157.3


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# Algorithmic work model of one row compression (two-sweep QR/SVD truncation).
def _leg(L1, L2, D, r, c):
    return (1 if c == 0 else D, 1 if r == 0 else D, 1 if c == L2 - 1 else D, 1 if r == L1 - 1 else D)


def _compressed(shapes, chi):
    a = [s[0] for s in shapes]
    p = [s[1] for s in shapes]
    b = [s[2] for s in shapes]
    L = len(shapes)
    for c in range(L - 1):
        k = min(a[c] * p[c], b[c])
        b[c] = k
        a[c + 1] = k
    for c in range(L - 1, 0, -1):
        k = min(chi, a[c], p[c] * b[c])
        a[c] = k
        b[c - 1] = k
    return list(zip(a, p, b))


def _qr_flops(m, n):
    # Householder R plus explicit thin Q (Golub & Van Loan operation counts)
    if m >= n:
        return 2 * (2 * m * n * n - 2 * n ** 3 / 3)
    return 2 * (2 * n * m * m - 2 * m ** 3 / 3)


def _svd_flops(m, n):
    # R-SVD with U and V (Golub & Van Loan): 4 m^2 n + 8 m n^2 + 9 n^3, m >= n
    if m < n:
        m, n = n, m
    return 4 * m * m * n + 8 * m * n * n + 9 * n ** 3


def compression_flops(L1, L2, D, chi, direction, r, prev):
    """Flops of compressing one boundary row of one chain; returns (flops,
    new dims).  prev: dims (a, p, b) of the previous boundary row or None."""
    shapes, fl = [], 0.0
    for c in range(L2):
        Dl, Du, Dr, Dd = _leg(L1, L2, D, r, c)
        a, q, b = prev[c] if prev else (1, 1, 1)
        pp = Dd if direction == 0 else Du
        fl += 2.0 * a * Dl * pp * b * Dr * q                  # absorption
        shapes.append((a * Dl, pp, b * Dr))
    a = [s[0] for s in shapes]
    p = [s[1] for s in shapes]
    b = [s[2] for s in shapes]
    for c in range(L2 - 1):                                    # QR sweep
        m, n = a[c] * p[c], b[c]
        k = min(m, n)
        fl += _qr_flops(m, n)
        fl += 2.0 * k * n * p[c + 1] * b[c + 1] - k * k * p[c + 1] * b[c + 1]  # R B_{c+1}
        b[c] = k
        a[c + 1] = k
    for c in range(L2 - 1, 0, -1):                             # SVD sweep
        m, n = a[c], p[c] * b[c]
        k = min(chi, m, n)
        fl += _svd_flops(m, n)
        fl += 2.0 * a[c - 1] * p[c - 1] * m * k                # B_{c-1} U S
        a[c] = k
        b[c - 1] = k
    return fl, _compressed(shapes, chi)


def sweep_compression_flops(L1, L2, D, chi):
    """Compressions per step: top[0..L1-2] during the sweep and
    bot[L1-1..1] for the measurement (reused by the next sweep)."""
    total, n = 0.0, 0
    prev = None
    for r in range(L1 - 1):
        f, prev = compression_flops(L1, L2, D, chi, 0, r, prev)
        total += f
        n += 1
    prev = None
    for r in range(L1 - 1, 0, -1):
        f, prev = compression_flops(L1, L2, D, chi, 1, r, prev)
        total += f
        n += 1
    return total, n


def model_row_flops(L2, D, chi):
    """Work of one boundary-row compression in the per-sample model of the
    measurement plan: L2 [2 chi^2 D^4 (absorption) + 4 chi^3 D^4 (QR) +
    16 chi^3 D^3 (SVD and product)] flops per chain and row, every site
    counted at full bond dimensions."""
    return L2 * (2 * chi ** 2 * D ** 4 + 4 * chi ** 3 * D ** 4 + 16 * chi ** 3 * D ** 3)


# ---------------------------------------------------------------------------
def _oracle_worker(args):
    L1, L2, D, chi, seed_theta, ch, seed = args
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        import numpy as np
        import synth
        from oracle import measure, sampler
        from oracle.lattice import Lattice
        lat = Lattice(L1, L2, D=D, chi=chi)
        th = synth.theta_random_unit(L1, L2, D, 2, seed=seed_theta)
        S = synth.configs_diagonal(1, lat.N, 2, seed=1000 + ch)[0].astype(np.int64)
        t0 = time.perf_counter()
        res = sampler.sweep(lat, th, S, chi, seed, ch, 0)
        ev = measure.evaluate(lat, th, res["S"], chi, tops=res["tops"])
        return time.perf_counter() - t0, res["S"], ev["O"], ev["e_loc"]


def cpu_baseline(L1, L2, D, chi, seed_theta, seed, cg_iters, target_core_s=20.0):
    """Oracle samples/s on this host's cores (bounded sample)."""
    import concurrent.futures as cf

    import numpy as np
    cores = len(os.sched_getaffinity(0))
    workers = max(1, min(cores, 16))   # the box grants one GPU's share of 16 host cores
    # one probe sample sizes the bounded run
    t_probe, _, _, _ = _oracle_worker((L1, L2, D, chi, seed_theta, 0, seed))
    n_samples = int(max(workers, min(8 * workers, round(target_core_s / max(t_probe, 1e-3)))))
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        outs = list(ex.map(_oracle_worker, [(L1, L2, D, chi, seed_theta, ch, seed) for ch in range(n_samples)]))
    wall = time.perf_counter() - t0
    # oracle CG on the same samples (its cost is linear in the sample count)
    from threadpoolctl import threadpool_limits

    from oracle import sr
    from oracle.lattice import Lattice
    lat = Lattice(L1, L2, D=D, chi=chi)
    cfg = np.array([o[1] for o in outs])
    O = np.array([o[2] for o in outs])
    e = np.array([o[3] for o in outs])
    with threadpool_limits(workers):
        t1 = time.perf_counter()
        sr.sr_solve(lat, cfg, O, e, 0.02, 1e-4, cg_iters, 0.0)
        t_cg = time.perf_counter() - t1
    cpu_model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": n_samples / (wall + t_cg), "unit": "samples/s", "cores": workers, "kind": "oracle",
            "cores_visible": cores, "cpu_model": cpu_model,
            "sample": f"{n_samples} chains x 1 sweep + measurement of the same workload on {workers} processes "
                      f"({wall:.1f} s wall), then oracle CG with {cg_iters} iterations on those samples "
                      f"({t_cg:.1f} s); NumPy FP64, one BLAS thread per process during sampling"}




# ---------------------------------------------------------------------------
def measured_traffic(kernel, L, D, chi, chains):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy kernel), or None
    when the workload differs or the kernel's sources changed since the
    counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if [L, D, chi, chains] != rec.get("workload_key"):
        return None
    h = hashlib.sha256()
    for src in rec["sources"]:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec["sources_sha256"]:
        return None
    return rec["read_bytes_per_launch"] + rec["write_bytes_per_launch"]


class Path:
    """One precision's state and buffers for full steps (args.sweeps sweeps
    of every chain in one library call, a measurement after each, then one
    SR solve on all n * sweeps samples and the update)."""

    def __init__(self, p, torch, desc, theta0, configs0, args, seed):
        self.p, self.torch, self.desc, self.args, self.seed = p, torch, desc, args, seed
        dev = theta0.device
        n = configs0.shape[0]
        self.n = n
        self.theta = theta0.clone()
        self.configs = configs0.clone()
        self.nnz = p.peps_orow_count(desc)
        self.n_accept = torch.zeros((n, 3), dtype=torch.int32, device=dev)
        self.status = p.new_status(dev)
        self.gsweep = 0
        # room for every traced launch of one full step (about 8 L1 per sweep
        # and library call; one call per chunk of chains with --chunk)
        calls = -(-n // args.chunk) if args.chunk and args.chunk < n else 1
        self.trace = p.Trace(16 * desc.L1 * args.sweeps * calls + 64)
        if getattr(args, "progress", False):
            self.trace.on_progress(f"{desc.L1}x{desc.L2} D={desc.D} chi={desc.chi}")
        self.out = None

    def _buffers(self, S):
        t = self.torch
        dev = self.theta.device
        n = self.n
        if self.out is None or self.out["e_loc"].shape[0] != S:
            self.out = None
            self.out = {"log_abs": t.empty((S, n), dtype=t.float64, device=dev),
                        "sign": t.empty((S, n), dtype=t.int8, device=dev),
                        "e_loc": t.empty((S, n), dtype=t.float64, device=dev),
                        "O": t.empty((S, n, self.nnz), dtype=t.float64, device=dev),
                        "configs": t.empty((S, n, self.desc.N), dtype=t.uint8, device=dev)}
        return self.out

    def step(self, S, trace=None):
        p, a, n = self.p, self.args, self.n
        out = self._buffers(S)
        if a.chunk and a.chunk < n:
            # one library call per chunk of chains (one sweep each), a
            # progress line after each; each chunk draws from its own seed
            for c0 in range(0, n, a.chunk):
                c1 = min(n, c0 + a.chunk)
                sub = {k: v[:, c0:c1] for k, v in out.items()}
                p.peps_sample_sweep(self.desc, self.theta, self.configs[c0:c1], self.seed + c0, self.gsweep, S,
                                    n_accept=self.n_accept[c0:c1], status=self.status, out=sub, trace=trace)
                self.torch.cuda.synchronize()
                progress(f"chains {c0}..{c1 - 1} swept and measured")
        else:
            p.peps_sample_sweep(self.desc, self.theta, self.configs, self.seed, self.gsweep, S,
                                n_accept=self.n_accept, status=self.status, out=out, trace=trace)
        self.gsweep += S
        _, _, stats, _ = p.sr_cg_solve(self.desc, out["configs"].view(S * n, self.desc.N),
                                       out["O"].view(S * n, self.nnz), out["e_loc"].view(S * n), a.tau, a.eps,
                                       a.cg_iters, 1e-10, want_g=False, theta=self.theta, status=self.status,
                                       trace=trace)
        return stats

    def warmup(self, k):
        for _ in range(k):
            self.step(1)
        self.torch.cuda.synchronize()
        self.p.check(self.status, "warmup")

    def timed(self, max_steps, budget_s, label):
        """Up to max_steps full steps, stopping after the one that ends past
        budget_s of wall time; HIP events on torch's current stream (the
        library's stream) bracket the whole run."""
        t, p = self.torch, self.p
        S = self.args.sweeps
        self._buffers(S)
        self.n_accept.zero_()
        t.cuda.synchronize()
        p.check(self.status, "before timed steps")
        self.trace.read()
        ev0, ev1 = t.cuda.Event(enable_timing=True), t.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record()
        k, stats = 0, None
        prof = {}
        while k < max_steps:
            stats = self.step(S, trace=self.trace)
            k += 1
            t.cuda.synchronize()
            for c, (ms, cnt) in self.trace.read().items():
                a, b = prof.get(c, (0.0, 0))
                prof[c] = (a + ms, b + cnt)
            el = time.perf_counter() - t0
            progress(f"{label}: step {k} done, {el:.1f} s")
            if el >= budget_s:
                break
        ev1.record()
        t.cuda.synchronize()
        wall = time.perf_counter() - t0
        p.check(self.status, "timed steps")
        ms_per_step = ev0.elapsed_time(ev1) / k
        acc = (self.n_accept.sum(dim=0).to(t.float64) / float(self.n * S * k)).cpu().numpy()
        return {"steps": k, "ms_per_step": ms_per_step, "samples_per_s": self.n * S / (ms_per_step / 1e3),
                "wall": wall, "prof": prof, "stats": stats.cpu().numpy(), "accepted_per_sweep": acc}


def graph_rate(p, torch, desc, theta0, configs0, args, seed, k=3, warm=True):
    """A one-sweep step (sweep, measurement, SR on those n samples, update)
    run eagerly and, captured once in HIP graphs (caller-owned workspaces,
    device sweep counter), replayed: ms per step of both, k each.  With
    --chunk the sweep of each chunk of chains is a graph of its own and the
    SR solve another, replayed in order with a progress line after each."""
    dev = theta0.device
    n = configs0.shape[0]
    nnz = p.peps_orow_count(desc)
    theta = theta0.clone()
    configs = configs0.clone()
    ctr = torch.zeros(1, dtype=torch.int64, device=dev)
    n_accept = torch.zeros((n, 3), dtype=torch.int32, device=dev)
    status = p.new_status(dev)
    chunk = args.chunk if args.chunk and args.chunk < n else n
    bounds = [(c0, min(n, c0 + chunk)) for c0 in range(0, n, chunk)]
    ws = torch.empty(p.workspace_bytes(desc, chunk, "sweep"), dtype=torch.uint8, device=dev)
    ws_sr = torch.empty(p.workspace_bytes(desc, n, "sr"), dtype=torch.uint8, device=dev)
    out = {"log_abs": torch.empty((1, n), dtype=torch.float64, device=dev),
           "sign": torch.empty((1, n), dtype=torch.int8, device=dev),
           "e_loc": torch.empty((1, n), dtype=torch.float64, device=dev),
           "O": torch.empty((1, n, nnz), dtype=torch.float64, device=dev)}

    def sweep(c0, c1):
        sub = {key: v[:, c0:c1] for key, v in out.items()}
        p.peps_sample_sweep(desc, theta, configs[c0:c1], seed + c0, 0, 1, n_accept=n_accept[c0:c1], status=status,
                            out=sub, sweep_counter=ctr, ws=ws)

    def solve():
        p.sr_cg_solve(desc, configs, out["O"][0], out["e_loc"][0], args.tau, args.eps, args.cg_iters, 1e-10,
                      want_g=False, theta=theta, status=status, ws=ws_sr)

    pieces = [(lambda b=b: sweep(*b)) for b in bounds] + [solve]

    def run(fns, label):
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(k):
            for i, fn in enumerate(fns):
                fn()
                if len(fns) > 2:
                    torch.cuda.synchronize()
                    progress(f"{label}: piece {i + 1} of {len(fns)} done")
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / k

    if warm:
        for fn in pieces:
            fn()
        torch.cuda.synchronize()
    eager_ms = run(pieces, "eager step")
    graphs = []
    for fn in pieces:
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            fn()
        graphs.append(g)
    torch.cuda.synchronize()
    graph_ms = run([g.replay for g in graphs], "replayed step")
    p.check(status, "graph replays")
    del graphs
    return {"eager_ms_per_step": round(eager_ms, 3), "graph_ms_per_step": round(graph_ms, 3),
            "graph_samples_per_s": round(n / (graph_ms / 1e3), 2), "steps_each": k, "graphs_per_step": len(pieces),
            "sweeps_run": int(ctr.item())}


def simple_update_rate(p, torch, desc, steps=20, tau=0.01):
    """Device time of one simple-update step (every bond of the lattice once)
    from the identity plus noise, averaged over `steps` steps after two
    untimed ones; None where the model has no simple update."""
    import synth
    if desc.model != p.MODEL_HEISENBERG or desc.J2 != 0.0 or desc.D > 8:
        return None
    dev = torch.device("cuda:0")
    theta = torch.tensor(synth.theta_identity(desc.L1, desc.L2, desc.D, 2, noise=1e-2, seed=96), device=dev)
    lam = torch.ones((p.su_bond_count(desc), desc.D), dtype=torch.float64, device=dev)
    p.peps_simple_update(desc, theta, lam, tau, 2)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    st = p.peps_simple_update(desc, theta, lam, tau, steps)
    ev1.record()
    torch.cuda.synchronize()
    p.check(st, "simple update")
    return {"ms_per_step": round(ev0.elapsed_time(ev1) / steps, 3), "bonds": p.su_bond_count(desc), "steps": steps,
            "note": "one first-order Trotter step over every nearest-neighbour bond (FP64), for the highest "
                    "temperatures before SR"}


UNEVEN_SHAPES = [(6, 4, 16), (8, 6, 36), (10, 6, 36), (16, 8, 64)]   # L (square, OBC), D, chi


def uneven_batch(p, torch, args, seed):
    """The uneven batch of Heisenberg lattices 6x6 (D=4, chi=16), 8x8 and
    10x10 (D=6, chi=36) and 16x16 (D=8, chi=64), args.chains chains each,
    mixed precision: one step per lattice (one sweep with its measurement,
    then SR with args.cg_iters CG iterations and the update), the four step
    sequences enqueued at once on four HIP streams so that their kernels
    share the GPU.  Each lattice is timed by events on its own stream, the
    batch by the wall clock around all four; a progress line (the library's
    stderr printer) as each traced launch completes.  The largest lattice uses the smallest workspace
    layout (its full layout would not fit beside the others)."""
    import synth
    dev = torch.device("cuda:0")
    n = args.chains
    jobs = []
    for k, (L, D, chi) in enumerate(UNEVEN_SHAPES):
        if L > args.uneven_max_L:
            continue
        desc = p.Desc(L, L, D, chi, precision=p.PREC_MIXED)
        kind = "min" if chi * D > 256 else "sweep"
        job = {"L": L, "D": D, "chi": chi, "desc": desc,
               "theta": torch.tensor(synth.theta_random_unit(L, L, D, 2, seed=104 + k), device=dev),
               "configs": torch.tensor(synth.configs_diagonal(n, L * L, 2, seed=7 + k), device=dev),
               "ws": torch.empty(p.workspace_bytes(desc, n, kind), dtype=torch.uint8, device=dev),
               "ws_sr": torch.empty(p.workspace_bytes(desc, n, "sr"), dtype=torch.uint8, device=dev),
               "status": p.new_status(dev), "stream": torch.cuda.Stream(),
               "ev": (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)),
               "trace": p.Trace(64 * L + 64), "layout": kind}
        nnz = p.peps_orow_count(desc)
        job["out"] = {"log_abs": torch.empty((1, n), dtype=torch.float64, device=dev),
                      "sign": torch.empty((1, n), dtype=torch.int8, device=dev),
                      "e_loc": torch.empty((1, n), dtype=torch.float64, device=dev),
                      "O": torch.empty((1, n, nnz), dtype=torch.float64, device=dev),
                      "configs": torch.empty((1, n, L * L), dtype=torch.uint8, device=dev)}
        job["trace"].on_progress(f"uneven batch {L}x{L} D={D} chi={chi}")
        jobs.append(job)
    torch.cuda.synchronize()
    progress(f"uneven batch: {len(jobs)} lattices x {n} chains set up, "
             f"{torch.cuda.memory_allocated() / 2 ** 30:.1f} GiB allocated")
    t0 = time.perf_counter()
    for job in jobs:
        with torch.cuda.stream(job["stream"]):
            d, o = job["desc"], job["out"]
            job["ev"][0].record()
            p.peps_sample_sweep(d, job["theta"], job["configs"], seed, 0, 1, status=job["status"], out=o,
                                ws=job["ws"], trace=job["trace"])
            p.sr_cg_solve(d, o["configs"][0], o["O"][0], o["e_loc"][0], args.tau, args.eps, args.cg_iters, 1e-10,
                          want_g=False, theta=job["theta"], status=job["status"], ws=job["ws_sr"],
                          trace=job["trace"])
            job["ev"][1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rows = []
    for job in jobs:
        p.check(job["status"], f"uneven batch {job['L']}x{job['L']}")
        ms = job["ev"][0].elapsed_time(job["ev"][1])
        job["trace"].on_progress(None)
        prof = job["trace"].read()
        rows.append({"lattice": [job["L"], job["L"]], "D": job["D"], "chi": job["chi"], "chains": n,
                     "workspace_layout": "smallest" if job["layout"] == "min" else "full",
                     "ms": round(ms, 1), "samples_per_s": round(n / (ms / 1e3), 2),
                     "kernel_ms": {k: round(v[0], 1) for k, v in prof.items() if v[1]}})
        job["trace"].close()
    return {"lattices": rows, "wall_s": round(wall, 2),
            "total_samples_per_s": round(n * len(jobs) / wall, 2),
            "note": "one step per lattice (sweep + measurement + SR), four streams in flight at once; per-lattice "
                    "times by events on each stream"}


def direct_sampling_rate(p, torch, n=1024, draws=5, chi_dl=16):
    """Direct (autoregressive) sampling, reweighted (p_4, dynamic diagonal
    weight), at the 4x4 D = 2 chi = 4 shape of the small cooling workload:
    device time per draw of n chains after two untimed draws (the timed
    draws reuse their double layer, theta being unchanged), the kernel
    split (per-row draw kernel vs the top-boundary and double-layer
    compressions), and the rate of the importance weights' inputs: one
    peps_eval_batch of the drawn samples."""
    import synth
    dev = torch.device("cuda:0")
    desc = p.Desc(4, 4, 2, 4)
    theta = torch.tensor(synth.theta_identity(4, 4, 2, 2, noise=0.05, seed=98), device=dev)
    b = torch.tensor([1.0], dtype=torch.float64, device=dev)
    ws = torch.empty(p.peps_direct_workspace_bytes(desc, n, chi_dl), dtype=torch.uint8, device=dev)
    st = p.new_status(dev)
    for k in range(2):
        cfg, lp, _ = p.peps_direct_sample(desc, theta, n, chi_dl, 11, draw=k, reweight=True, b_diag=b, update_b=True,
                                          status=st, ws=ws)
    tr = p.Trace(64 * draws)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for k in range(draws):
        # theta is fixed across these draws, as within one cooling step: the
        # double layer of the untimed draws is reused
        cfg, lp, _ = p.peps_direct_sample(desc, theta, n, chi_dl, 11, draw=2 + k, reweight=True, b_diag=b,
                                          update_b=True, reuse_double_layer=True, status=st, ws=ws, trace=tr)
    ev1.record()
    torch.cuda.synchronize()
    p.check(st, "direct sampling")
    ms = ev0.elapsed_time(ev1) / draws
    prof = tr.read()
    tr.close()
    la, _, _, st2 = p.peps_eval_batch(desc, theta, cfg, want_e=False)
    w = p.peps_importance_weights(la, lp)
    torch.cuda.synchronize()
    p.check(st2, "direct sampling weights")
    wh = w.cpu().numpy()
    return {"workload": f"4x4 Heisenberg, D=2, chi=4, chi_dl={chi_dl}, {n} chains, p_4 with dynamic b",
            "ms_per_draw": round(ms, 3), "samples_per_s": round(n / (ms / 1e3), 1), "draws": draws,
            "kernel_ms_per_draw": {k: round(v[0] / draws, 3) for k, v in prof.items() if v[1]},
            "b_diag_after": round(float(b.item()), 4),
            "effective_sample_fraction": round(float(wh.sum() ** 2 / (wh ** 2).sum() / n), 4)}


def energy_error(p, torch, desc64, descmx, theta, configs):
    """Local energies of the same samples and parameters from both
    precisions: relative error of the mean energy, the same error in units
    of the Monte Carlo standard error, per-sample relative errors (scale
    max(|E_i|, mean |E|)), and the fraction of samples whose mixed local
    energy equals the FP64 one bit for bit (those whose every row strip the
    mixed path measured again in FP64, or whose FP32 rounding happened to
    cancel)."""
    import numpy as np
    _, _, e64, s1 = p.peps_eval_batch(desc64, theta, configs)
    _, _, emx, s2 = p.peps_eval_batch(descmx, theta, configs)
    torch.cuda.synchronize()
    p.check(s1, "fp64 eval")
    p.check(s2, "mixed eval")
    e64 = e64.cpu().numpy()
    emx = emx.cpu().numpy()
    dE = abs(emx.mean() - e64.mean())
    rel = np.abs(emx - e64) / np.maximum(np.abs(e64), np.abs(e64).mean())
    return {"n_samples": int(e64.size),
            "E_per_site_fp64": float(e64.mean() / (2 * desc64.N)),
            "mean_E_rel": float(dE / abs(e64.mean())),
            "dE_over_stderr": float(dE / max(e64.std() / np.sqrt(e64.size), 1e-300)),
            "sample_rel_median": float(np.median(rel)),
            "sample_rel_p99": float(np.quantile(rel, 0.99)),
            "sample_rel_max": float(rel.max()),
            "fp64_equal_fraction": float(np.mean(emx == e64))}


def cooled_state(p, torch, L1, L2, D, chi, n, steps, sweeps, tau, eps, cg_iters, seed):
    """theta and configurations after `steps` SR steps of the cooling loop
    (FP64) from the beta = 0 identity plus N(0, 0.05^2) noise: |rho|
    sampling with the Eq. A1 weights up to beta_phys = 0.3, |rho|^2 after it
    (beta_phys = 4 steps tau at the end).  Returns (theta, configs, last
    record)."""
    import synth
    dev = torch.device("cuda:0")
    desc = p.Desc(L1, L2, D, chi, alpha=1)
    theta = torch.tensor(synth.theta_identity(L1, L2, D, 2, noise=0.05, seed=101), device=dev)
    configs = torch.tensor(synth.configs_diagonal(n, L1 * L2, 2, seed=8), device=dev)
    recs = p.cool(desc, theta, configs, steps + 1, sweeps, tau, eps, seed, cg_iters=cg_iters, alpha_switch_beta=0.3)
    return theta, configs, recs[-1]


def eval_rate(p, torch, desc, theta, configs, reps=3):
    """peps_eval_batch samples/s on fixed configurations."""
    p.peps_eval_batch(desc, theta, configs)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        p.peps_eval_batch(desc, theta, configs)
    ev1.record()
    torch.cuda.synchronize()
    return configs.shape[0] * reps / (ev0.elapsed_time(ev1) / 1e3)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="most full SR steps timed (mixed path)")
    ap.add_argument("--warmup", type=int, default=2, help="one-sweep warm-up steps per precision")
    ap.add_argument("--budget-s", type=float, default=120.0,
                    help="wall-time budget of the timed mixed steps (the step that crosses it is the last)")
    ap.add_argument("--fp64-steps", type=int, default=2, help="most full FP64 steps for the comparison")
    ap.add_argument("--sweeps", type=int, default=200, help="sweeps (samples per chain) per SR step")
    ap.add_argument("--L", type=int, default=8)
    ap.add_argument("--D", type=int, default=4)
    ap.add_argument("--chi", type=int, default=16)
    ap.add_argument("--J2", type=float, default=0.0, help="next-nearest-neighbour coupling (J1 = 1)")
    ap.add_argument("--graph", action="store_true",
                    help="with --only: also time a one-sweep step eagerly and as a replayed HIP graph")
    ap.add_argument("--model", choices=["heisenberg", "hubbard"], default="heisenberg",
                    help="hubbard (with --only): t = 1, U = 8, mu = 4, d^2 = 16, random parity-even tensors")
    ap.add_argument("--chains", type=int, default=1024)
    ap.add_argument("--chunk", type=int, default=0,
                    help="with --only and --sweeps 1: sweep the chains in library calls of this many chains, with a "
                         "progress line after each (large lattices), each chunk from its own seed")
    ap.add_argument("--graph-steps", type=int, default=3, help="steps of each kind timed by --graph")
    ap.add_argument("--uneven", action="store_true",
                    help="only the uneven batch of lattices (6x6, 8x8, 10x10, 16x16; --chains each) on four streams")
    ap.add_argument("--direct", action="store_true",
                    help="only the direct-sampling rate (4x4, D=2, chi=4, chi_dl=16, --chains draws per call)")
    ap.add_argument("--uneven-max-L", type=int, default=16,
                    help="with --uneven: only the lattices of at most this side length")
    ap.add_argument("--progress", action="store_true",
                    help="a progress line as each traced launch completes (long calls on large lattices)")
    ap.add_argument("--cg-iters", type=int, default=200)
    ap.add_argument("--tau", type=float, default=0.02)
    ap.add_argument("--eps", type=float, default=1e-4)
    ap.add_argument("--tol", type=float, default=1e-4, help="energy error bar of the mixed path (relative)")
    ap.add_argument("--cool-steps", type=int, default=50,
                    help="SR steps of the cooled-state energy check (beta_phys = 4 * steps * tau = 4 by default)")
    ap.add_argument("--cool-sweeps", type=int, default=4, help="sweeps per SR step of the cooled-state check")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the graph replay, evaluation-only and simple-update figures")
    ap.add_argument("--only", choices=["both", "fp64", "mixed"], default="both",
                    help="run one precision only (profiling runs); the JSON line then carries that path")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run one elementwise kernel over 512 MiB (reads 512 MiB, writes 512 MiB) as the "
                         "reference for HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU sharding of this "
              "path is a design note, not an implemented mode", file=sys.stderr)
        sys.exit(2)
    t_start = time.perf_counter()

    import torch

    import paper_2409_05285_amd as p
    import synth

    dev = torch.device("cuda:0")
    L1 = L2 = args.L
    D, chi, n = args.D, args.chi, args.chains
    seed_theta, seed = 102, 20240905
    if args.model == "hubbard":
        if args.only == "both":
            print("--model hubbard needs --only fp64 or --only mixed", file=sys.stderr)
            sys.exit(2)
        hub = dict(d=4, model=p.MODEL_HUBBARD, t=1.0, U=8.0, mu=4.0, J2=args.J2)
        desc64 = p.Desc(L1, L2, D, chi, **hub)
        descmx = p.Desc(L1, L2, D, chi, precision=p.PREC_MIXED, **hub)
        theta0 = torch.tensor(synth.theta_random_parity_even(L1, L2, D, 4, seed=seed_theta), device=dev)
        configs0 = torch.tensor(synth.configs_diagonal(n, L1 * L2, 4, seed=7), device=dev)
    else:
        desc64 = p.Desc(L1, L2, D, chi, J2=args.J2)
        descmx = p.Desc(L1, L2, D, chi, J2=args.J2, precision=p.PREC_MIXED)
        theta0 = torch.tensor(synth.theta_random_unit(L1, L2, D, 2, seed=seed_theta), device=dev)
        configs0 = torch.tensor(synth.configs_diagonal(n, L1 * L2, 2, seed=7), device=dev)
    progress(f"setup done ({time.perf_counter() - t_start:.1f} s)")

    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    if args.direct:
        res = direct_sampling_rate(p, torch, n=args.chains)
        res["bench_wall_s"] = round(time.perf_counter() - t_start, 1)
        print(json.dumps(res), flush=True)
        return
    if args.uneven:
        res = uneven_batch(p, torch, args, seed)
        res["bench_wall_s"] = round(time.perf_counter() - t_start, 1)
        print(json.dumps(res), flush=True)
        return
    if args.chunk and args.sweeps != 1:
        print("--chunk needs --sweeps 1", file=sys.stderr)
        sys.exit(2)
    if args.only != "both":
        desc = desc64 if args.only == "fp64" else descmx
        path = Path(p, torch, desc, theta0, configs0, args, seed)
        path.warmup(args.warmup)
        r = path.timed(args.steps, args.budget_s, args.only)
        line = {"only": args.only, "model": args.model, "lattice": [L1, L2], "D": D, "chi": chi,
                "J2": args.J2, "chains": n, "chunk": args.chunk or n, "steps": r["steps"],
                "peak_device_GiB": round(torch.cuda.max_memory_allocated() / 2 ** 30, 2),
                "sweeps_per_step": args.sweeps, "samples_per_s": round(r["samples_per_s"], 2),
                "ms_per_step": round(r["ms_per_step"], 3),
                "kernel_ms_per_step": {k: round(v[0] / r["steps"], 3) for k, v in r["prof"].items()},
                "kernel_launches": {k: v[1] for k, v in r["prof"].items()}}
        if args.graph:
            progress("one-sweep step, eager and replayed graph")
            line["graph_replay"] = graph_rate(p, torch, desc, theta0, configs0, args, seed, k=args.graph_steps,
                                              warm=args.warmup > 0)
        print(json.dumps(line), flush=True)
        return

    pmx = Path(p, torch, descmx, theta0, configs0, args, seed)
    p64 = Path(p, torch, desc64, theta0, configs0, args, seed)
    pmx.warmup(args.warmup)
    p64.warmup(args.warmup)
    progress(f"warm-up done ({time.perf_counter() - t_start:.1f} s)")
    # both paths restart from the same state for the timed steps
    pmx = Path(p, torch, descmx, theta0, configs0, args, seed)
    rmx = pmx.timed(args.steps, args.budget_s, "mixed")
    progress(f"mixed path: {rmx['steps']} steps, {rmx['ms_per_step']:.1f} ms per step")
    p64 = Path(p, torch, desc64, theta0, configs0, args, seed)
    r64 = p64.timed(min(args.fp64_steps, args.steps), args.budget_s, "fp64")
    progress(f"fp64 path: {r64['steps']} steps, {r64['ms_per_step']:.1f} ms per step")

    # precision gate: the same samples and parameters through both paths, on
    # the random state after the FP64 steps and on a cooled state
    err_random = energy_error(p, torch, desc64, descmx, p64.theta, p64.configs)
    th_c, cfg_c, rec_c = cooled_state(p, torch, L1, L2, D, chi, n, args.cool_steps, args.cool_sweeps, args.tau,
                                      args.eps, args.cg_iters, seed)
    err_cooled = energy_error(p, torch, desc64, descmx, th_c, cfg_c)
    gate = {name: all(e[k] <= args.tol for k in ("mean_E_rel", "sample_rel_p99", "sample_rel_max"))
            for name, e in (("random", err_random), ("cooled", err_cooled))}
    mixed_ok = all(gate.values())
    progress(f"energy error checks done ({time.perf_counter() - t_start:.1f} s)")
    extras = {}
    if not args.no_extras:
        extras["graph_replay"] = {"fp64": graph_rate(p, torch, desc64, theta0, configs0, args, seed),
                                  "mixed": graph_rate(p, torch, descmx, theta0, configs0, args, seed),
                                  "note": "one-sweep step (1024 samples, SR on them) eager vs captured once as a "
                                          "HIP graph and replayed"}
        extras["simple_update"] = simple_update_rate(p, torch, desc64)
        extras["direct_sampling"] = direct_sampling_rate(p, torch)
        extras["eval_samples_per_s"] = {"fp64": round(eval_rate(p, torch, desc64, p64.theta, p64.configs), 1),
                                        "mixed": round(eval_rate(p, torch, descmx, p64.theta, p64.configs), 1)}
        progress(f"extras done ({time.perf_counter() - t_start:.1f} s)")
    # the rate reported is that of the faster path meeting the precision bar
    # (the FP64 path always does)
    best = rmx if (mixed_ok and rmx["samples_per_s"] >= r64["samples_per_s"]) else r64
    best_name = "mixed" if best is rmx else "fp64"
    prof = best["prof"]

    # dominant kernel class and its roofline: the row compression against the
    # FP64 peak, work per launch = model flops per chain and row x chains
    dom = max(prof, key=lambda k: prof[k][0])
    comp_flops, comp_n = sweep_compression_flops(L1, L2, D, chi)
    ms, launches = prof["compress"]
    avg_ms = ms / max(launches, 1)
    model_fl = model_row_flops(L2, D, chi) * n
    exact_fl = comp_flops / comp_n * n
    achieved = model_fl / (avg_ms / 1e3) / 1e12
    traffic = measured_traffic("k_compress2", L1, D, chi, n)
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": MI355X_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / MI355X_FP64_TFLOPS, 4), "traffic": traffic,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "kernel": "k_compress2", "kernel_class_share": round(ms / sum(v[0] for v in prof.values()), 4),
            "dominant_class": dom, "avg_launch_ms": round(avg_ms, 4), "launches": launches,
            "flops_per_launch": model_fl,
            "flops_model": "L2 (2 chi^2 D^4 + 4 chi^3 D^4 + 16 chi^3 D^3) per chain and row",
            "exact_dims_flops_per_launch": exact_fl,
            "exact_dims_achieved": round(exact_fl / (avg_ms / 1e3) / 1e12, 3),
            "exact_dims_frac": round(exact_fl / (avg_ms / 1e3) / 1e12 / MI355X_FP64_TFLOPS, 4)}

    # SR: O is read twice per CG iteration (O x, then O^T y), plus the
    # gradient pass
    nnz = p.peps_orow_count(desc64)
    sr_ms = prof["sr"][0] / best["steps"]
    cg_it = int(best["stats"][2])
    sr_bytes = (2 * cg_it + 1) * n * args.sweeps * nnz * 8
    sr_roof = {"bound": "hbm", "achieved": round(sr_bytes / (sr_ms / 1e3) / 1e9, 1), "peak": MI355X_HBM_GBS,
               "unit": "GB/s", "frac": round(sr_bytes / (sr_ms / 1e3) / 1e9 / MI355X_HBM_GBS, 4),
               "kernel": "sr_cg_solve", "ms_per_solve": round(sr_ms, 3), "cg_iters": cg_it}

    def summary(r):
        return {"steps": r["steps"], "samples_per_s": round(r["samples_per_s"], 2),
                "ms_per_step": round(r["ms_per_step"], 3),
                "kernel_ms_per_step": {k: round(v[0] / r["steps"], 3) for k, v in r["prof"].items()},
                "accepted_moves_per_chain_and_sweep": {"h": round(float(r["accepted_per_sweep"][0]), 3),
                                                       "site": round(float(r["accepted_per_sweep"][1]), 3),
                                                       "v": round(float(r["accepted_per_sweep"][2]), 3)},
                "E_per_site_last_step": float(r["stats"][0]) / (2 * L1 * L2),
                "cg_iters_last_step": int(r["stats"][2]), "cg_converged_last_step": bool(r["stats"][4] == 0.0)}

    line = {
        "metric": "PEPS-VMC samples/s (amp+O_k+E_loc) FP32-MFMA vs FP64 at stated energy error",
        "value": round(best["samples_per_s"], 2),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": best["steps"],
        "steps_requested": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(best["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if best_name == "mixed" else "f64",
        "value_path": best_name,
        "data": "synthetic",
        "config": {"workload": f"{L1}x{L2} Heisenberg OBC, d^2=4, D={D}, chi={chi}, {n} chains x "
                               f"{args.sweeps} sweeps per SR step, random unit-Frobenius tensors; step = "
                               f"{args.sweeps} sweeps each followed by a measurement + SR CG on all "
                               f"{n * args.sweeps} samples ({args.cg_iters} it max) + update",
                   "lattice": [L1, L2], "D": D, "chi": chi, "chains": n, "sweeps_per_step": args.sweeps,
                   "cg_iters": args.cg_iters,
                   "precision": "mixed (FP32 MFMA strips, FP64 QR/SVD/SR)" if best_name == "mixed" else "fp64"},
        "roofline": roof,
        "roofline_sr": sr_roof,
        "sr_steps_per_s": round(1e3 / best["ms_per_step"], 4),
        "fp64": summary(r64),
        "mixed": summary(rmx),
        "mixed_vs_fp64": round(rmx["samples_per_s"] / r64["samples_per_s"], 4),
        "energy_error": {"tol": args.tol, "within_tol": mixed_ok, "gate": gate,
                         "cooled": dict(err_cooled, beta_phys=rec_c["beta_phys"],
                                        E_per_site_cooling=rec_c["E_per_site"],
                                        E_stderr_cooling=rec_c["E_stderr"],
                                        state=f"identity + N(0, 0.05^2) noise after {args.cool_steps} SR steps "
                                              f"of {n} chains x {args.cool_sweeps} sweeps (alpha 1 below "
                                              f"beta_phys 0.3, then 2)"),
                         "random": dict(err_random, state="random unit-Frobenius tensors after the FP64 steps")},
        "host_wall_ms_per_step": round(best["wall"] * 1e3 / best["steps"], 3),
    }
    line.update(extras)
    if not args.no_cpu_baseline:
        progress(f"CPU oracle baseline ({time.perf_counter() - t_start:.1f} s)")
        line["cpu_baseline"] = cpu_baseline(L1, L2, D, chi, seed_theta, seed, args.cg_iters)
    line["bench_wall_s"] = round(time.perf_counter() - t_start, 1)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
