"""Benchmark: forward + adjoint of a batch of 512 Toeplitz operators.

Workload (seeded, synthetic): 512 square Toeplitz operators, sizes
log-uniform in [256, 65536], first row/column CN(0,1) in complex64, each with
1..32 CN(0,1) columns. One step applies every operator forward, y_i = T_i x_i,
and then adjoint, z_i = T_i^H y_i. Inputs are resident in HBM before timing.

Throughput = algorithmic bytes / time, where the algorithmic bytes of one
direction of operator i are: read x (N_i n_i 8 B) + write y (M_i n_i 8 B) +
read the spectrum once (L_i 8 B).

Prints one JSON line. ``--gpus N`` with N > 1 exits: the benchmark measures
one GPU.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
STAGE_SOURCES = ("batch.hip", "batch.h", "epi.h", "xform.h", "mixed.h", "kernels.h", "common.h")
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "stage_kernel_toeplitz512_fwd_adj.md")


def stage_source_hash():
    """sha256 (16 hex digits) over the sources of the batched stage kernel."""
    import hashlib

    h = hashlib.sha256()
    for f in STAGE_SOURCES:
        with open(os.path.join(ROOT, "paper_1710_09578_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per direction from the committed FETCH_SIZE / WRITE_SIZE
    summary, or None when the kernel sources changed since it was taken."""
    try:
        with open(TRAFFIC_PROFILE) as fh:
            kv = dict(line.split(": ", 1) for line in fh.read().splitlines() if ": " in line)
    except OSError:
        return None
    if kv.get("source_hash", "").strip() != stage_source_hash():
        return None
    return int(kv["traffic_bytes_per_direction"])


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def setup_toeplitz(nops, device):
    import torch

    import paper_1710_09578_amd as fm
    from workloads import toeplitz_batch

    t0 = time.time()
    data = toeplitz_batch(nops=nops)
    log(f"generated inputs for {nops} operators in {time.time() - t0:.1f}s")
    ops, xs, ys, zs = [], [], [], []
    for i in range(nops):
        d = data["ops"][i]
        ops.append(fm.Toeplitz(torch.from_numpy(d["col"]).to(device),
                               torch.from_numpy(d["row"]).to(device)))
        x = torch.from_numpy(d["x"]).to(device)
        xs.append(x)
        ys.append(torch.empty_like(x))
        zs.append(torch.empty_like(x))
    torch.cuda.synchronize()
    sizes = data["sizes"]
    ncols = data["ncols"]
    Ls = np.array([op.transform_length for op in ops])
    alg_bytes = int(np.sum(2 * (2 * sizes * ncols * 8) + 2 * Ls * 8))
    return {"ops": ops, "xs": xs, "ys": ys, "zs": zs, "sizes": sizes, "ncols": ncols,
            "Ls": Ls, "alg_bytes": alg_bytes, "data": data}


def plain_step_factory(w):
    """One fm_apply per operator and direction on the current stream."""
    import torch

    from paper_1710_09578_amd import capi

    lib = capi.load()
    stream = torch.cuda.current_stream().cuda_stream
    calls = []
    wsmax = 0
    for op, x in zip(w["ops"], w["xs"]):
        for d in (capi.FM_FWD, capi.FM_ADJ):
            wsmax = max(wsmax, capi.fm_workspace_size(op.handle, d, x.shape[0]))
    ws = torch.empty(max(wsmax, 1), dtype=torch.uint8, device="cuda")
    for op, x, y, z in zip(w["ops"], w["xs"], w["ys"], w["zs"]):
        n = x.shape[1]
        nc = x.shape[0]
        calls.append((op.handle, capi.FM_FWD, nc, x.data_ptr(), n, y.data_ptr(), n))
        calls.append((op.handle, capi.FM_ADJ, nc, y.data_ptr(), n, z.data_ptr(), n))
    f = lib.fm_apply
    wsp, wsb = ws.data_ptr(), ws.numel()

    def step():
        for h, d, nc, xp, ldx, yp, ldy in calls:
            st = f(h, d, nc, xp, ldx, yp, ldy, wsp, wsb, stream)
            if st != 0:
                raise RuntimeError(capi.fm_last_error())

    return step, ws


def batched_step_factory(w):
    """The whole batch as one pipelined sequence of stage launches per direction."""
    import paper_1710_09578_amd as fm
    from paper_1710_09578_amd import capi

    batch = fm.Batch(w["ops"], [int(v) for v in w["ncols"]])
    lib = capi.load()
    import ctypes as C
    import torch

    n = len(w["ops"])
    P = C.c_void_p * n
    I = C.c_int64 * n
    args = {
        capi.FM_FWD: (P(*[x.data_ptr() for x in w["xs"]]), I(*[x.shape[1] for x in w["xs"]]),
                      P(*[y.data_ptr() for y in w["ys"]]), I(*[y.shape[1] for y in w["ys"]])),
        capi.FM_ADJ: (P(*[y.data_ptr() for y in w["ys"]]), I(*[y.shape[1] for y in w["ys"]]),
                      P(*[z.data_ptr() for z in w["zs"]]), I(*[z.shape[1] for z in w["zs"]])),
    }
    stream = torch.cuda.current_stream().cuda_stream
    f = lib.fm_batch_apply

    def launch(d):
        st = f(batch._h, d, *args[d], stream)
        if st != 0:
            raise RuntimeError(capi.fm_last_error())

    def step():
        launch(capi.FM_FWD)
        launch(capi.FM_ADJ)

    return step, launch, batch


def warm_up(step, min_steps, min_s=0.0):
    """Untimed repetitions of ``step``: at least ``min_steps``, and with
    ``min_s`` > 0 as many more as fill ``min_s`` seconds of wall time. After
    an idle period (data generated on the host) the device needs ~0.1-0.2 s
    of sustained work before its clocks settle: the wide circulant took
    0.494 ms per step after 5 warm-up steps and 0.427 ms after 400."""
    import torch

    t0 = time.perf_counter()
    n = 0
    while n < min_steps or time.perf_counter() - t0 < min_s:
        step()
        n += 1
        if min_s > 0 and n % 8 == 0:
            torch.cuda.synchronize()  # the host clock follows the device
    torch.cuda.synchronize()
    return n


# warm-up time of the secondary legs (the headline keeps exactly --warmup steps)
LEG_WARM_S = 0.5


def time_steps(step, steps, warmup, warm_s=0.0):
    import torch

    warm_up(step, warmup, warm_s)
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    t0 = time.time()
    start.record()
    for _ in range(steps):
        step()
    end.record()
    torch.cuda.synchronize()
    wall = time.time() - t0
    gpu_ms = start.elapsed_time(end) / steps
    return max(wall * 1e3 / steps, gpu_ms), gpu_ms


def fista_solves(w, iters=100, stop_tol=1e-5, tune=True, reps=3):
    """FISTA for every column of every operator: batched (fm_batch_fista) and
    plain (one fm_fista per operator). Measurements b = T x_true + noise are
    formed on the GPU by the library's batched forward apply. Each form is
    timed ``reps`` times after a warm-up (the plain warm-up solves every
    operator once, so its workspaces and tables exist); the median is
    reported. A seeded sample of operators is checked: batched and plain x
    must be equal bit for bit."""
    import torch

    import paper_1710_09578_amd as fm
    from workloads import toeplitz_batch

    data = toeplitz_batch(nops=len(w["ops"]), with_fista=True)
    ncols = [int(v) for v in w["ncols"]]
    batch = fm.Batch(w["ops"], ncols)
    xt = [torch.from_numpy(data["ops"][i]["x_true"]).cuda() for i in range(len(ncols))]
    if tune:
        # the fold limit stays the per-operator path's (the batch's initial
        # schedule), so batched and plain x can be compared bit for bit; the
        # slot region is tuned
        fold = batch.schedule()["max_fuse"]
        sc = batch.tune(xt, reps=2)
        if sc["max_fuse"] != fold:
            batch.set_schedule(fold, sc["region_mib"])
    bs = batch.apply(xt)
    for i in range(len(ncols)):
        bs[i].add_(torch.from_numpy(data["ops"][i]["noise"]).cuda())
    torch.cuda.synchronize()
    total = sum(ncols)
    batch.fista(bs, iters=2, lam_rel=0.05)  # warm-up (state allocation, bounds)
    torch.cuda.synchronize()
    tbs = []
    for _ in range(reps):
        t0 = time.time()
        xb, st = batch.fista(bs, iters=iters, lam_rel=0.05, stop_tol=stop_tol)
        torch.cuda.synchronize()
        tbs.append(time.time() - t0)
    tb = float(np.median(tbs))
    counts = np.array([s["iters"] for s in st])
    Ls = []
    gi = 0
    for i in range(len(ncols)):
        Ls.append(st[gi]["L"] if ncols[i] else 1.0)
        gi += ncols[i]

    def plain():
        out = []
        for i, op in enumerate(w["ops"]):
            out.append(fm.fista(op, bs[i], iters=iters, lam_rel=0.05, L=Ls[i], stop_tol=stop_tol)[0]
                       if ncols[i] else None)
        return out

    for i, op in enumerate(w["ops"]):  # warm-up: every operator once
        if ncols[i]:
            fm.fista(op, bs[i], iters=2, lam_rel=0.05, L=Ls[i])
    torch.cuda.synchronize()
    tps = []
    for _ in range(reps):
        t0 = time.time()
        xp = plain()
        torch.cuda.synchronize()
        tps.append(time.time() - t0)
    tp = float(np.median(tps))
    rng = np.random.default_rng(0)
    sample = sorted(rng.choice(len(ncols), 32, replace=False).tolist())
    same = all(torch.equal(xb[i], xp[i]) for i in sample if ncols[i])
    log(f"FISTA {iters} it, stop {stop_tol}: batched {tb:.3f} s, plain {tp:.3f} s for {total} problems "
        f"(median of {reps}); iterations used: mean {counts.mean():.1f}, min {counts.min()}, max {counts.max()}; "
        f"batched == plain bit for bit on {len(sample)} sampled operators: {same}")
    if not same:
        raise RuntimeError("batched and plain FISTA solutions differ")
    return {"problems": total, "iters": iters, "stop_tol": stop_tol, "batched_s": round(tb, 4),
            "plain_s": round(tp, 4), "batched_solves_per_s": round(total / tb, 1),
            "plain_solves_per_s": round(total / tp, 1), "batched_over_plain": round(tp / tb, 2),
            "mean_iters": round(float(counts.mean()), 2), "reps": reps, "statistic": "median",
            "batched_equals_plain_sampled_ops": len(sample)}


GRAPH_STEPS = 50


def circulant_1024_latency(ncols=16, steps=2000, warmup=50):
    """Forward + adjoint of the 1024-point circulant on 16 columns (complex64,
    128 KiB per block; cache-resident and launch-bound): microseconds per
    fwd+adj, as two fm_apply calls per step and as GRAPH_STEPS such steps
    captured once in a graph and replayed (time per step). The replay is
    checked against the eager result bit for bit."""
    import torch

    from paper_1710_09578_amd import capi
    import paper_1710_09578_amd as fm
    from workloads import circulant_1024

    dev = torch.device("cuda:0")
    c, x = circulant_1024(ncols=ncols)
    C = fm.Circulant(torch.from_numpy(c).to(dev))
    X = torch.from_numpy(x).to(dev)
    Y = torch.empty_like(X)
    Z = torch.empty_like(X)
    n = c.size
    h = C.handle

    def step():
        st = torch.cuda.current_stream().cuda_stream
        capi.fm_apply(h, capi.FM_FWD, ncols, X, n, Y, n, None, 0, st)
        capi.fm_apply(h, capi.FM_ADJ, ncols, Y, n, Z, n, None, 0, st)

    ms_plain, ev_plain = time_steps(step, steps, warmup, LEG_WARM_S)
    z_eager = Z.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    # GRAPH_STEPS steps per graph, so that one replay's host cost is spread
    # over many launches (a replay of one step costs the host more than the
    # two direct launches it replaces)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(GRAPH_STEPS):
            step()
    Z.zero_()
    ms_graph, ev_graph = time_steps(g.replay, max(1, steps // GRAPH_STEPS), 1, LEG_WARM_S)
    ms_graph /= GRAPH_STEPS
    ev_graph /= GRAPH_STEPS
    same = torch.equal(Z, z_eager)
    alg = 2 * (2 * X.numel() * 8 + n * 8)
    log(f"circulant 1024 x {ncols}: {ev_plain * 1e3:.2f} us per fwd+adj (two fm_apply calls, events), "
        f"{ev_graph * 1e3:.2f} us replayed from a graph; replay == eager: {same}")
    if not same:
        raise RuntimeError("graph replay of the circulant differs from the eager result")
    return {"workload": f"Circulant N=1024, {ncols} CN(0,1) columns, complex64, fwd+adj",
            "us_per_fwd_adj_plain": round(ev_plain * 1e3, 3), "us_per_fwd_adj_graph": round(ev_graph * 1e3, 3),
            "us_per_fwd_adj_plain_wall": round(ms_plain * 1e3, 3), "us_per_fwd_adj_graph_wall": round(ms_graph * 1e3, 3),
            "alg_bytes_per_step": int(alg), "steps": steps, "steps_per_graph": GRAPH_STEPS}


def compressed_sensing_fista(iters=200, reps=7):
    """FISTA on the row-selected Rademacher circulant (N = 65536, M = 4096
    rows, 64-sparse truth, noise 1e-3, lam = 0.05 ||A^H b||_inf, 200
    iterations), in complex64 and complex128: solves per second (median of
    ``reps``), with the FP64 power iteration for L timed on its own."""
    import torch

    import paper_1710_09578_amd as fm
    from workloads import compressed_sensing_65536

    dev = torch.device("cuda:0")
    w = compressed_sensing_65536()
    n = w["c"].size
    out = {"workload": "FISTA 200 it on S C(c): N=65536 Rademacher circulant, M=4096 rows, K=64, noise 1e-3, "
                       "lam = 0.05 ||A^H b||_inf, one problem"}
    for name, dt in (("c64", torch.complex64), ("c128", torch.complex128)):
        rows = torch.from_numpy(w["rows"]).to(dev)
        A = fm.Product(fm.SelectRows(n, rows, dt), fm.Circulant(torch.from_numpy(w["c"]).to(dev).to(dt)))
        b = A.apply(torch.from_numpy(w["x_true"]).to(dev).to(dt)) + torch.from_numpy(w["noise"]).to(dev).to(dt)
        warm_up(lambda: fm.power_iteration(A), 1, LEG_WARM_S)
        tp = []
        for _ in range(3):
            t0 = time.perf_counter()
            L, pit = fm.power_iteration(A)
            torch.cuda.synchronize()
            tp.append(time.perf_counter() - t0)
        t_pow = float(np.median(tp))
        warm_up(lambda: fm.fista(A, b, iters=iters, lam_rel=0.05, L=L), 1, LEG_WARM_S)
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            x, st = fm.fista(A, b, iters=iters, lam_rel=0.05, L=L)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        t = float(np.median(ts))
        log(f"compressed sensing FISTA {iters} it ({name}): {t * 1e3:.3f} ms per solve, {1 / t:.1f} solves/s "
            f"(median of {reps}); power iteration {t_pow * 1e3:.2f} ms (median of 3; {pit} it, L = {L:.6g})")
        out[name] = {"ms_per_solve": round(t * 1e3, 4), "solves_per_s": round(1 / t, 2),
                     "power_iteration_ms": round(t_pow * 1e3, 3), "power_iterations": int(pit),
                     "us_per_iteration": round(t / iters * 1e6, 2)}
    return out


def learn_circulant_steps(steps=5, warmup=2, iters=20, checkpoint=5):
    """Training steps/s of learning a circulant generator through unrolled
    FISTA (N = 16384, M = 2048 selected rows, 256 pairs of 32-sparse vectors,
    20 steps): the checkpointed unrolled solver (autograd.unrolled_fista)
    against plain autograd over per-step operator applications with every
    intermediate saved. One training step = forward, backward, Adam update of c."""
    import torch

    import paper_1710_09578_amd as fm
    from paper_1710_09578_amd import autograd as ag
    from workloads import learn_circulant

    d = learn_circulant()
    dev = torch.device("cuda:0")
    c_true = torch.from_numpy(d["c_true"]).to(dev)
    rows = torch.from_numpy(d["rows"]).to(dev)
    x = torch.from_numpy(d["x"]).to(dev)
    n = c_true.numel()
    A_true = fm.Product(fm.SelectRows(n, rows), fm.Circulant(c_true))
    b = A_true.apply(x)
    b.add_(torch.from_numpy(d["noise"]).to(dev))
    g = A_true.apply(b, adjoint=True)
    lam = 0.05 * g.abs().amax(dim=1).double()
    S = fm.SelectRows(n, rows)

    def soft(z, s):
        a = z.abs()
        keep = a > s
        a_safe = torch.where(keep, a, torch.ones_like(a))
        return torch.where(keep, z * (1 - s / a_safe), torch.zeros_like(z))

    def run(kind):
        c = torch.from_numpy(d["c_init"]).to(dev).requires_grad_(True)
        opt = torch.optim.Adam([c], lr=1e-3)
        betas = [fm.capi.fm_fista_momentum(k) for k in range(iters)]

        def one():
            opt.zero_grad(set_to_none=True)
            Cc = fm.Circulant(c.detach())
            L = fm.capi.fm_op_norm_bound(Cc.handle, 0)
            if kind == "checkpointed":
                xk = ag.unrolled_fista(c, b, rows, lam, L=L, iters=iters, checkpoint=checkpoint)
            else:
                s = (lam / L).reshape(-1, 1).to(torch.float32)
                xp = torch.zeros_like(x)
                y = xp
                for k in range(iters):
                    r = ag.apply(S, ag.circulant_apply(c, y)) - b
                    gk = ag.circulant_apply(c, ag.apply(S, r, adjoint=True), adjoint=True)
                    xk = soft(y - gk / L, s)
                    y = xk + betas[k] * (xk - xp)
                    xp = xk
                xk = xp
            loss = (xk - x).abs().pow(2).mean()
            loss.backward()
            opt.step()
            return float(loss.detach())

        warm_up(lambda: A_true.apply(b, adjoint=True), 1, LEG_WARM_S)  # stateless: training starts after it
        for _ in range(warmup):
            one()
        torch.cuda.synchronize()
        torch.cuda.reset_peak_memory_stats()
        t0 = time.time()
        losses = [one() for _ in range(steps)]
        torch.cuda.synchronize()
        dt = (time.time() - t0) / steps
        return dt, torch.cuda.max_memory_allocated() / 2**30, losses

    out = {}
    for kind in ("checkpointed", "plain"):
        dt, mem, losses = run(kind)
        log(f"learn-circulant {kind}: {dt * 1e3:.1f} ms/step, peak {mem:.2f} GiB, loss {losses[0]:.4e} -> {losses[-1]:.4e}")
        out[kind] = {"ms_per_step": round(dt * 1e3, 2), "steps_per_s": round(1 / dt, 2), "peak_gib": round(mem, 3)}
    out["speedup"] = round(out["plain"]["ms_per_step"] / out["checkpointed"]["ms_per_step"], 2)
    out["workload"] = "N=16384, M=2048, 256 pairs, 20 unrolled FISTA steps, checkpoints every 5, Adam"
    return out


def kron_hfg_bandwidth(steps=5, warmup=2):
    """Forward + adjoint of Kron(H_1024, F_256, G_32) on 64 columns of
    8,388,608 rows (complex64, 4 GiB per block). Algorithmic bytes per
    direction: read the block + write the block (+ the 8 KiB factor)."""
    import torch

    import paper_1710_09578_amd as fm
    from workloads import kron_hfg

    dev = torch.device("cuda:0")
    g, X = kron_hfg(device=dev)
    K = fm.Kron(fm.Hadamard(1024), fm.Fourier(256), fm.Dense(torch.from_numpy(g).to(dev)))
    Y = torch.empty_like(X)
    Z = torch.empty_like(X)
    from paper_1710_09578_amd import capi

    ws = torch.empty(max(capi.fm_workspace_size(K.handle, capi.FM_FWD, X.shape[0]),
                         capi.fm_workspace_size(K.handle, capi.FM_ADJ, X.shape[0]), 1),
                     dtype=torch.uint8, device=dev)

    def step():
        K.apply(X, out=Y, workspace=ws)
        K.apply(Y, adjoint=True, out=Z, workspace=ws)

    ms, _ = time_steps(step, steps, warmup, LEG_WARM_S)
    alg = 2 * (2 * X.numel() * 8 + g.size * 8)
    gbs = alg / (ms * 1e-3) / 1e9
    log(f"kron H1024 x F256 x G32, 64 columns: {ms:.3f} ms per fwd+adj, {gbs:.1f} GB/s")
    del X, Y, Z, ws
    torch.cuda.empty_cache()
    return {"workload": "Kron(H_1024, F_256, G_32 real N(0,1/32)), 64 columns of 8388608, complex64, fwd+adj",
            "ms_per_step": round(ms, 4), "gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
            "alg_bytes_per_step": int(alg)}


def circulant_wide_bandwidth(steps=40, warmup=5):
    """Forward + adjoint of the 1024-point circulant on 65,536 columns
    (complex64, 512 MiB per block): one single-pass convolution launch per
    direction. Algorithmic bytes per direction: read the block + write the
    block (+ the 8 KiB spectrum)."""
    import torch

    import paper_1710_09578_amd as fm
    from workloads import many_columns

    dev = torch.device("cuda:0")
    c, X = many_columns(device=dev)
    C = fm.Circulant(torch.from_numpy(c).to(dev))
    Y = torch.empty_like(X)
    Z = torch.empty_like(X)

    def step():
        C.apply(X, out=Y)
        C.apply(Y, adjoint=True, out=Z)

    ms, _ = time_steps(step, steps, warmup, LEG_WARM_S)
    alg = 2 * (2 * X.numel() * 8 + c.size * 8)
    gbs = alg / (ms * 1e-3) / 1e9
    log(f"circulant 1024 x 65536 columns: {ms:.3f} ms per fwd+adj, {gbs:.1f} GB/s")
    del X, Y, Z
    torch.cuda.empty_cache()
    return {"workload": "Circulant N=1024, 65536 CN(0,1) columns, complex64, fwd+adj",
            "ms_per_step": round(ms, 4), "gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
            "alg_bytes_per_step": int(alg)}


def ultrasound_model(steps=5, warmup=2):
    """The compressed ultrasound model b = Psi H x on synthetic generators:
    H = 32 x 32 blocks of 2-level Toeplitz (levels 32, 512; embedding
    64 x 1024), x of 524288 entries, Psi keeps one Fourier coefficient per
    A-scan (1024 measurements). Times H fwd+adj (spectral mixing; and block by
    block for comparison), Psi H fwd+adj and a 20-step FISTA solve.
    Algorithmic bytes of one H direction: every block spectrum read once
    (1024 x 65536 complex64) + x read + y written."""
    import torch

    import paper_1710_09578_amd as fm
    from workloads import ultrasound

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    w = ultrasound()
    n1, n2, n3, nf = w["shape"]
    t = torch.from_numpy(w["t"]).to(dev)
    H, Psi, PH = fm.compressed_ultrasound(t, w["psi_rows"])
    del t
    torch.cuda.synchronize()
    log(f"ultrasound model built in {time.perf_counter() - t0:.1f} s")
    n = n1 * n2 * n3
    total = (2 * n2) * (2 * n3)
    x = torch.from_numpy(w["x_true"]).to(dev)
    y = torch.empty_like(x)
    z = torch.empty_like(x)

    def h_step(op):
        def step():
            op.apply(x, out=y)
            op.apply(y, adjoint=True, out=z)
        return step

    ms_h, _ = time_steps(h_step(H), steps, warmup, LEG_WARM_S)
    alg_dir = n1 * n1 * total * 8 + 2 * n * 8
    gbs_h = 2 * alg_dir / (ms_h * 1e-3) / 1e9
    log(f"ultrasound H fwd+adj (spectral mixing): {ms_h:.3f} ms, {gbs_h:.1f} GB/s")
    blocks = H._keep
    Hg = fm.Blocks([[fm.Product(blocks[0])] + list(blocks[1:n1])] +
                   [list(blocks[i * n1:(i + 1) * n1]) for i in range(1, n1)])
    ms_g, _ = time_steps(h_step(Hg), 1, 1)
    log(f"ultrasound H fwd+adj (block by block): {ms_g:.3f} ms")
    del Hg
    m = PH.shape[0]
    b = PH.apply(x) + torch.from_numpy(w["noise"]).to(dev)
    v = torch.empty((1, m), dtype=x.dtype, device=dev)

    def ph_step():
        PH.apply(x, out=v)
        PH.apply(v, adjoint=True, out=z)

    ms_ph, _ = time_steps(ph_step, steps, warmup, LEG_WARM_S)
    log(f"ultrasound Psi H fwd+adj: {ms_ph:.3f} ms")
    L, _ = fm.power_iteration(PH)
    torch.cuda.synchronize()
    warm_up(lambda: fm.fista(PH, b, iters=20, lam_rel=0.05, L=L), 1, LEG_WARM_S)
    ts = []
    for _ in range(5):
        t1 = time.perf_counter()
        xr, st = fm.fista(PH, b, iters=20, lam_rel=0.05, L=L)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t1)
    fista_ms = float(np.median(ts)) * 1e3
    log(f"ultrasound FISTA 20 steps on Psi H: {fista_ms:.2f} ms per solve (L = {L:.4g})")
    del x, y, z, b, v, H, Psi, PH
    torch.cuda.empty_cache()
    return {"workload": "compressed ultrasound model: H = 32 x 32 blocks of 2-level Toeplitz (32 x 512), "
                        "Psi = 1 Fourier coefficient per A-scan, complex64",
            "h_ms_fwd_adj": round(ms_h, 4), "h_gbs": round(gbs_h, 1), "h_hbm_frac": round(gbs_h / HBM_PEAK_GBS, 4),
            "h_block_by_block_ms": round(ms_g, 3), "mix_speedup": round(ms_g / ms_h, 1),
            "psi_h_ms_fwd_adj": round(ms_ph, 4), "fista20_ms": round(fista_ms, 3),
            "alg_bytes_per_direction": int(alg_dir)}


def omp_solves(ncols=64, k=64, reps=7):
    """OMP with 64 atoms on the row-selected Rademacher circulant (N = 65536,
    M = 4096, 64-sparse truths, noise 1e-3): one problem per call, and 64
    problems (columns) per call; median of ``reps`` calls."""
    import torch

    import paper_1710_09578_amd as fm
    from workloads import compressed_sensing_65536

    dev = torch.device("cuda:0")
    w = compressed_sensing_65536(ncols=ncols)
    n = w["c"].size
    A = fm.Product(fm.SelectRows(n, torch.from_numpy(w["rows"]).to(dev)), fm.Circulant(torch.from_numpy(w["c"]).to(dev)))
    b = A.apply(torch.from_numpy(w["x_true"]).to(dev)) + torch.from_numpy(w["noise"]).to(dev)
    out = {}
    for cols in (1, ncols):
        bb = b[:cols].contiguous()
        warm_up(lambda: fm.omp(A, bb, k), 1, LEG_WARM_S)
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            x, sup, st = fm.omp(A, bb, k)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        dt = float(np.median(ts))
        out[f"ncols_{cols}"] = {"ms_per_call": round(dt * 1e3, 3), "solves_per_s": round(cols / dt, 1), "reps": reps,
                                "statistic": "median"}
        log(f"OMP k={k} on N=65536 M=4096, {cols} problem(s) per call: {dt * 1e3:.2f} ms, {cols / dt:.1f} solves/s")
    out["workload"] = "OMP, 64 atoms, row-selected Rademacher circulant N=65536 M=4096, complex64"
    return out


def calibration_small(ncols=65536):
    """Run-time path choice for small operators: the device's calibration
    model (structured vs dense, the dense product of complex64 on the matrix
    cores) measured once over its grid, where the dense path wins, and the
    per-handle timing of three examples on many columns."""
    import torch

    import paper_1710_09578_amd as fm

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    table = fm.calibration_build()
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    names = {0: "circulant", 1: "toeplitz", 2: "fourier"}
    dense_wins = {}
    for e in table:
        if e["ms_dense"] < e["ms_fast"]:
            key = f"{names[e['cls']]}_{'c64' if e['dt'] == 1 else 'c128'}"
            dense_wins.setdefault(key, []).append([e["n"], e["ncols"], round(e["ms_fast"] / e["ms_dense"], 2)])
    log(f"calibration model: {len(table)} grid points in {build_s:.2f} s; dense wins (n, ncols, speedup): {dense_wins}")
    at_max = {f"{names[e['cls']]}_{'c64' if e['dt'] == 1 else 'c128'}_n{e['n']}":
              {"structured_ms": round(e["ms_fast"], 4), "dense_ms": round(e["ms_dense"], 4)}
              for e in table if e["ncols"] == 65536}
    gen = torch.Generator(device=dev)
    gen.manual_seed(11)
    out = {"model_points": len(table), "model_build_s": round(build_s, 3), "dense_wins": dense_wins,
           "grid_at_65536_columns": at_max}
    for name, mk in (("circulant16", lambda: fm.Circulant(torch.randn(16, dtype=torch.complex64, device=dev,
                                                                          generator=gen))),
                     ("fourier32", lambda: fm.Fourier(32)),
                     ("toeplitz48", lambda: fm.Toeplitz(torch.randn(48, dtype=torch.complex64, device=dev, generator=gen),
                                                        torch.randn(48, dtype=torch.complex64, device=dev,
                                                                    generator=gen)))):
        op = mk()
        info = op.calibrate(ncols)
        out[name] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in info.items()}
        out[name]["model_choice"] = op.choose_path(ncols)
        log(f"calibration {name} x {ncols} columns: structured {info['ms_structured']:.4f} ms, "
            f"dense {info['ms_dense']:.4f} ms -> {info['path']} (model: {out[name]['model_choice']})")
    return out


def copy_bandwidth(nbytes=1 << 30, reps=10):
    """Device-to-device copy rate (read + write bytes per second): the
    practical ceiling of a streaming kernel on this device."""
    import torch

    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    gbs = 2 * nbytes * reps / (a.elapsed_time(b) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def cpu_baseline_toeplitz(w, budget_s=15.0):
    """The oracle's dense-free Toeplitz product (row blocks generated from the
    definition, BLAS products) on a bounded sample of the same operators."""
    from oracle import structured

    cores = len(os.sched_getaffinity(0))
    data = w["data"]
    order = list(range(len(w["ops"])))
    done_bytes = 0
    t0 = time.time()
    used = 0
    for i in order:
        d = data["ops"][i]
        n = int(w["sizes"][i])
        if n > 8192:
            continue  # keep the sample bounded: dense row blocks are O(N^2)
        y = structured.toeplitz_apply_blocks(d["col"], d["row"], d["x"])
        structured.toeplitz_apply_blocks(d["col"], d["row"], y, adjoint_dir=True)
        done_bytes += 2 * (2 * n * int(w["ncols"][i]) * 8) + 2 * int(w["Ls"][i]) * 8
        used += 1
        if time.time() - t0 > budget_s:
            break
    dt = time.time() - t0
    return {"value": done_bytes / dt / 1e9, "unit": "GB/s", "cores": cores, "kind": "oracle",
            "sample": f"{used} of the 512 operators with N <= 8192 (all their columns), fwd+adj by "
                      f"dense-definition row blocks x BLAS in {dt:.1f} s"}


def host_info():
    """CPU model, core count available to this process and the BLAS NumPy uses."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = "unknown"
    try:
        cfg = np.show_config(mode="dicts")
        bl = cfg.get("Build Dependencies", {}).get("blas", {})
        blas = f"{bl.get('name', '?')} {bl.get('version', '')}".strip()
    except Exception:
        pass
    return {"cpu_model": model, "cores": len(os.sched_getaffinity(0)), "blas": blas}


def cpu_structured_toeplitz(w, budget_s=15.0):
    """The same fast algorithm on the host: every sampled operator's
    fwd + adj as zero-padded FFT convolutions (scipy.fft, complex64, all
    cores), over the operators in order until the time budget is spent; the
    stand-in for the paper's matrix-free CPU evaluation."""
    import scipy.fft as sf

    cores = len(os.sched_getaffinity(0))
    data = w["data"]
    done_bytes, used = 0, 0
    t0 = time.time()
    for i in range(len(w["ops"])):
        d = data["ops"][i]
        n = int(w["sizes"][i])
        L = sf.next_fast_len(2 * n - 1)
        g = np.zeros(L, np.complex64)
        g[:n] = d["col"]
        g[L - n + 1:] = d["row"][1:][::-1]
        gh = sf.fft(g, workers=cores)
        xp = np.zeros((d["x"].shape[0], L), np.complex64)
        xp[:, :n] = d["x"]
        y = sf.ifft(sf.fft(xp, axis=1, workers=cores) * gh, axis=1, workers=cores)[:, :n]
        xp[:, :n] = y
        xp[:, n:] = 0
        sf.ifft(sf.fft(xp, axis=1, workers=cores) * np.conj(gh), axis=1, workers=cores)
        done_bytes += 2 * (2 * n * int(w["ncols"][i]) * 8) + 2 * int(w["Ls"][i]) * 8
        used += 1
        if time.time() - t0 > budget_s:
            break
    dt = time.time() - t0
    return {"value": done_bytes / dt / 1e9, "unit": "GB/s", "cores": cores, "kind": "structured (scipy.fft c64)",
            "sample": f"{used} of the 512 operators in order, fwd+adj by zero-padded FFT convolution in {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--nops", type=int, default=512)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fista", action="store_true")
    ap.add_argument("--no-learn", action="store_true")
    ap.add_argument("--no-kron", action="store_true")
    ap.add_argument("--no-wide", action="store_true", help="skip the 1024-point circulant on 65536 columns")
    ap.add_argument("--no-ultrasound", action="store_true", help="skip the compressed ultrasound model")
    ap.add_argument("--no-omp", action="store_true", help="skip the OMP solves")
    ap.add_argument("--no-calib", action="store_true", help="skip the small-operator path calibration")
    ap.add_argument("--no-c1", action="store_true", help="skip the 1024-point circulant on 16 columns")
    ap.add_argument("--no-cs", action="store_true", help="skip the compressed-sensing FISTA solves")
    ap.add_argument("--no-tune", action="store_true", help="keep the default batch schedule")
    ap.add_argument("--schedule", default="", help="MAX_FUSE,REGION_MIB: fixed batch schedule (no tuning)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 512 MiB device to device (reference for traffic counters)")
    ap.add_argument("--only", default="", choices=["", "wide", "kron", "c1", "cs", "fista", "learn", "ultrasound",
                                                    "omp", "calib"],
                    help="run one leg alone (for profiling) and print its result")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the path would shard over independent columns and operators, one process per GPU)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1710_09578_amd as fm

    fm.load()
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        src = torch.empty(512 << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.only:
        legs = {"wide": circulant_wide_bandwidth, "kron": kron_hfg_bandwidth, "c1": circulant_1024_latency,
                "cs": compressed_sensing_fista, "learn": learn_circulant_steps, "ultrasound": ultrasound_model,
                "omp": omp_solves, "calib": calibration_small}
        if args.only == "fista":
            res = fista_solves(setup_toeplitz(args.nops, dev), tune=not args.no_tune)
        else:
            res = legs[args.only]()
        print(json.dumps({"only": args.only, "result": res}), flush=True)
        return
    w = setup_toeplitz(args.nops, dev)
    alg = w["alg_bytes"]
    log(f"algorithmic bytes per fwd+adj step: {alg / 1e9:.3f} GB ({alg} B)")

    plain_step, _ws = plain_step_factory(w)
    plain_ms, _ = time_steps(plain_step, max(2, args.steps // 4), 1, LEG_WARM_S)
    plain_gbs = alg / (plain_ms * 1e-3) / 1e9
    log(f"plain (one fm_apply per operator and direction): {plain_ms:.3f} ms/step, {plain_gbs:.1f} GB/s")

    step, launch, _batch = batched_step_factory(w)
    sched = _batch.schedule()
    if args.schedule:
        mf, rg = (int(v) for v in args.schedule.split(","))
        _batch.set_schedule(mf, rg)
        sched = _batch.schedule()
        log(f"fixed schedule: {sched}")
    elif not args.no_tune:
        sched = _batch.tune(w["xs"], outs=w["ys"], reps=2)
        log(f"tuned schedule: {sched}")
    ms, gpu_ms = time_steps(step, args.steps, args.warmup)
    gbs = alg / (ms * 1e-3) / 1e9
    log(f"batched: {ms:.3f} ms/step wall, {gpu_ms:.3f} ms/step events, {gbs:.1f} GB/s")

    # dominant kernel: stage_kernel; events on the launch stream bracket the
    # stage launches of each direction
    import torch

    from paper_1710_09578_amd import capi

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(2 * args.steps)]
    k = 0
    for _ in range(args.steps):
        for d in (capi.FM_FWD, capi.FM_ADJ):
            ev[k][0].record()
            launch(d)
            ev[k][1].record()
            k += 1
    torch.cuda.synchronize()
    launch_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    per_launch = alg / 2  # one direction
    achieved = per_launch / (launch_ms * 1e-3) / 1e9
    log(f"one direction (all its stage launches): {launch_ms:.3f} ms avg, {achieved:.1f} GB/s")
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(),
            "kernel": "stage_kernel: all stage launches of one direction (fm_batch_apply)",
            "alg_bytes_per_launch": int(per_launch), "launch_ms": round(launch_ms, 4)}
    fres = None if args.no_fista else fista_solves(w, tune=not args.no_tune)
    c1 = None if args.no_c1 else circulant_1024_latency()
    cs = None if args.no_cs else compressed_sensing_fista()
    learn = None if args.no_learn else learn_circulant_steps()
    kron = None if args.no_kron else kron_hfg_bandwidth()
    wide = None if args.no_wide else circulant_wide_bandwidth()
    us = None if args.no_ultrasound else ultrasound_model()
    ompr = None if args.no_omp else omp_solves()
    calib = None if args.no_calib else calibration_small()
    copy_gbs = copy_bandwidth()
    log(f"device copy: {copy_gbs:.1f} GB/s")
    roof["copy_gbs"] = round(copy_gbs, 1)
    roof["copy_frac"] = round(achieved / copy_gbs, 4)
    cpu = cpu_struct = None
    host = host_info()
    log(f"host: {host}")
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_toeplitz(w)
        cpu.update({"cpu_model": host["cpu_model"], "blas": host["blas"]})
        log(f"cpu oracle baseline: {cpu['value']:.3f} GB/s on {cpu['cores']} cores")
        cpu_struct = cpu_structured_toeplitz(w)
        cpu_struct.update({"cpu_model": host["cpu_model"]})
        log(f"cpu structured baseline: {cpu_struct['value']:.3f} GB/s on {cpu_struct['cores']} cores "
            f"({cpu_struct['sample']})")
    out = {
        "metric": "batched fwd+adj operator GB/s (% HBM peak); FISTA solves/s, batched vs plain",
        "value": round(gbs, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": "512 Toeplitz operators, N log-uniform in [256, 65536], 1-32 "
                               "columns each, complex64, fwd+adj",
                   "path": "batched (fm_batch_apply: software-pipelined stage launches replayed from a HIP graph, schedule from fm_batch_tune)",
                   "alg_bytes_per_step": w["alg_bytes"],
                   "schedule": sched,
                   "plain_gbs": round(plain_gbs, 2),
                   "batched_over_plain": round(gbs / plain_gbs, 2),
                   "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)},
        "roofline": roof,
        "fista": fres,
        "circulant_1024x16": c1,
        "compressed_sensing": cs,
        "learn_circulant": learn,
        "kron": kron,
        "wide_circulant": wide,
        "ultrasound": us,
        "omp": ompr,
        "calibration": calib,
        "cpu_baseline": cpu,
        "cpu_structured": cpu_struct,
        "host": host,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
