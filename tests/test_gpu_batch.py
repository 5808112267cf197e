"""GPU parity of the batched stage launches (fm_batch_apply, fm_batch_fista).

The batched launch runs the same per-transform code, splits, spectra and
twiddles as one fm_apply per operator, so its results must equal the plain
path bit for bit; both are also compared with the FP64 oracle.
"""

import numpy as np
import pytest

from oracle import structured
from tests.gpu_util import TOL, crandn, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu


def build_batch(gpu, sizes, ncols, seed, square=True):
    rng = np.random.default_rng(seed)
    ops, data = [], []
    for n, nc in zip(sizes, ncols):
        m = n if square else max(1, int(n * 0.75))
        col, row = crandn(rng, m), crandn(rng, n)
        x = crandn(rng, (nc, n))
        u = crandn(rng, (nc, m))
        ops.append(gpu.Toeplitz(to_dev(col), to_dev(row)))
        data.append((col, row, x, u))
    return ops, data


@pytest.mark.parametrize("square", [True, False])
def test_batch_equals_plain_and_oracle(gpu, square):
    # lengths on both sides of the single-pass limit (embedding 2^12 vs 2^13+),
    # ragged column counts, including a zero-column operator
    sizes = [3, 100, 1000, 2047, 2049, 3000, 5000, 17000, 40000, 65536, 300, 9000]
    ncols = [1, 5, 3, 2, 4, 0, 2, 3, 1, 2, 17, 6]
    ops, data = build_batch(gpu, sizes, ncols, seed=1, square=square)
    batch = gpu.Batch(ops, ncols)
    xs = [to_dev(d[2]) for d in data]
    us = [to_dev(d[3]) for d in data]
    ys = batch.apply(xs)
    zs = batch.apply(us, adjoint=True)
    for i, (op, (col, row, x, u)) in enumerate(zip(ops, data)):
        if ncols[i] == 0:
            continue
        y_plain = to_host(op @ xs[i])
        z_plain = to_host(op.H @ us[i])
        y_b, z_b = to_host(ys[i]), to_host(zs[i])
        assert np.array_equal(y_b, y_plain), f"op {i}: batched forward differs from plain"
        assert np.array_equal(z_b, z_plain), f"op {i}: batched adjoint differs from plain"
        assert rel_err(y_b, structured.toeplitz_apply_fft64(col, row, x)) <= TOL["c64"]
        assert rel_err(z_b, structured.toeplitz_apply_fft64(col, row, u, True)) <= TOL["c64"]


def test_batch_repeated_calls_and_pointer_tables(gpu):
    """Alternating pointer tables (more than the cached copies) and repeated
    launches give the same bits every time."""
    import torch

    sizes = [700, 6000, 33000]
    ncols = [3, 2, 2]
    ops, data = build_batch(gpu, sizes, ncols, seed=2)
    batch = gpu.Batch(ops, ncols)
    xs = [to_dev(d[2]) for d in data]
    ref = [to_host(y) for y in batch.apply(xs)]
    outs = [[torch.empty_like(x) for x in xs] for _ in range(6)]
    for rep in range(3):
        for k in range(6):
            batch.apply(xs, outs=outs[k])
        for k in range(6):
            for i in range(3):
                assert np.array_equal(to_host(outs[k][i]), ref[i])


def test_batch_circulant_ops(gpu):
    rng = np.random.default_rng(4)
    cs = [crandn(rng, n) for n in (1024, 16384, 131072)]
    ops = [gpu.Circulant(to_dev(c)) for c in cs]
    ncols = [4, 3, 2]
    xs = [to_dev(crandn(rng, (nc, c.size))) for nc, c in zip(ncols, cs)]
    batch = gpu.Batch(ops, ncols)
    for adj in (False, True):
        ys = batch.apply(xs, adjoint=adj)
        for c, x, y in zip(cs, xs, ys):
            assert rel_err(to_host(y), structured.circulant_apply_fft64(c, to_host(x), adj)) <= TOL["c64"]


def test_batch_toeplitz_workload_sample(gpu):
    """The 512-operator Toeplitz workload in one launch; a seeded sample of
    operators (all small ones and a few large) is checked against the oracle."""
    from workloads import toeplitz_batch

    full = toeplitz_batch()
    sizes, ncols = full["sizes"], full["ncols"]
    ops, xs = [], []
    for i in range(len(sizes)):
        d = full["ops"][i]
        ops.append(gpu.Toeplitz(to_dev(d["col"]), to_dev(d["row"])))
        xs.append(to_dev(d["x"]))
    batch = gpu.Batch(ops, list(ncols))
    ys = batch.apply(xs)
    zs = batch.apply(ys, adjoint=True)
    rng = np.random.default_rng(0)
    small = [i for i in range(len(sizes)) if sizes[i] <= 1024]
    large = list(rng.choice([i for i in range(len(sizes)) if sizes[i] > 1024], 12, replace=False))
    for i in small[:40] + large:
        d = full["ops"][i]
        y = to_host(ys[i])
        assert rel_err(y, structured.toeplitz_apply_fft64(d["col"], d["row"], d["x"])) <= TOL["c64"]
        z = to_host(zs[i])
        assert rel_err(z, structured.toeplitz_apply_fft64(d["col"], d["row"], y, True)) <= TOL["c64"]


def fista_batch_problem(gpu, sizes, ncols, seed):
    rng = np.random.default_rng(seed)
    ops, data = [], []
    for n, nc in zip(sizes, ncols):
        col, row = crandn(rng, n), crandn(rng, n)
        xt = np.zeros((nc, n), np.complex128)
        for j in range(nc):
            k = max(n // 256, 1)
            xt[j, rng.choice(n, k, replace=False)] = rng.standard_normal(k)
        b = (structured.toeplitz_apply_fft64(col, row, xt) + 1e-3 * crandn(rng, (nc, n), np.complex128))
        ops.append(gpu.Toeplitz(to_dev(col), to_dev(row)))
        data.append((col, row, b.astype(np.complex64)))
    return ops, data


def embedding_length(need):
    """The documented Toeplitz embedding: the smallest L >= need among the
    powers of two and, above 4096, 4096 * n2 for n2 in 3, 5, 6, 9, 10, 12,
    20, 24, 30."""
    cands = [1 << int(np.ceil(np.log2(need)))]
    if need > 4096:
        cands += [4096 * n2 for n2 in (3, 5, 6, 9, 10, 12, 20, 24, 30) if 4096 * n2 >= need]
    return min(cands)


def test_batch_fista_equals_plain_and_oracle(gpu):
    sizes = [300, 1000, 3000, 5000, 20000]
    ncols = [3, 2, 0, 2, 2]
    ops, data = fista_batch_problem(gpu, sizes, ncols, seed=11)
    batch = gpu.Batch(ops, ncols)
    bs = [to_dev(d[2]) for d in data]
    xs, st = batch.fista(bs, iters=30, lam_rel=0.05)
    gi = 0
    for i, (op, (col, row, b)) in enumerate(zip(ops, data)):
        if ncols[i] == 0:
            continue
        L = st[gi]["L"]
        lam = np.array([st[gi + j]["lam"] for j in range(ncols[i])])
        # the bound max |DFT(g)|^2 is at least ||T||^2 (here compared to the
        # spectrum of the embedding computed by the oracle)
        m = col.size
        Lemb = embedding_length(m + row.size - 1)
        g = np.zeros(Lemb, np.complex128)
        g[:m] = col
        g[Lemb - row.size + 1:] = row[1:][::-1]
        assert abs(L - np.max(np.abs(np.fft.fft(g))) ** 2) <= 1e-12 * L
        x_plain, _ = gpu.fista(op, bs[i], iters=30, lam_rel=0.05, L=L)
        assert np.array_equal(to_host(xs[i]), to_host(x_plain)), f"op {i}: batched solve differs from plain"
        x_ref, _ = structured.toeplitz_fista_fft64(col, row, b, lam, L, 30)
        assert rel_err(to_host(xs[i]), x_ref) <= TOL["c64"]
        gi += ncols[i]


def test_batch_fista_stopping(gpu):
    sizes = [500, 2500, 9000]
    ncols = [4, 3, 2]
    ops, data = fista_batch_problem(gpu, sizes, ncols, seed=12)
    batch = gpu.Batch(ops, ncols)
    bs = [to_dev(d[2]) for d in data]
    xs, st = batch.fista(bs, iters=150, lam_rel=0.05, stop_tol=1e-4)
    counts = [s["iters"] for s in st]
    assert min(counts) < 150
    gi = 0
    for i, (col, row, b) in enumerate(data):
        L = st[gi]["L"]
        lam = np.array([st[gi + j]["lam"] for j in range(ncols[i])])
        x_ref, done = structured.toeplitz_fista_fft64(col, row, b, lam, L, 150, stop_tol=1e-4)
        got = np.array(counts[gi:gi + ncols[i]])
        assert np.all(np.abs(got - done) <= 1)
        # each column equals the oracle run stopped at the GPU's own count
        for j in range(ncols[i]):
            xj, _ = structured.toeplitz_fista_fft64(col, row, b[j:j + 1], lam[j], L, int(got[j]))
            assert rel_err(to_host(xs[i])[j:j + 1], xj) <= TOL["c64"]
        gi += ncols[i]


def test_batch_graph_replays_match_eager(gpu):
    """The stage sequence is captured once and replayed: every replay, with
    other library and torch work and synchronisations in between, equals the
    per-operator (eager) path bit for bit."""
    import torch

    sizes = [500, 3000, 9000, 40000]
    ncols = [4, 3, 2, 2]
    ops, data = build_batch(gpu, sizes, ncols, seed=5)
    batch = gpu.Batch(ops, ncols)
    xs = [to_dev(d[2]) for d in data]
    ref = [to_host(op @ x) for op, x in zip(ops, xs)]
    ref_h = [to_host(op.H @ x) for op, x in zip(ops, xs)]
    ys = [torch.empty_like(x) for x in xs]
    zs = [torch.empty_like(x) for x in xs]
    other = gpu.Circulant(to_dev(crandn(np.random.default_rng(9), 1024)))
    w = to_dev(crandn(np.random.default_rng(10), (3, 1024)))
    for rep in range(4):
        for y in ys:
            y.fill_(float("nan"))
        batch.apply(xs, outs=ys)
        batch.apply(xs, adjoint=True, outs=zs)
        _ = other @ w  # eager work between the replays
        torch.cuda.synchronize()
        for i in range(len(ops)):
            assert np.array_equal(to_host(ys[i]), ref[i]), f"replay {rep}, op {i}"
            assert np.array_equal(to_host(zs[i]), ref_h[i]), f"replay {rep}, op {i} (adjoint)"
    assert batch.schedule()["graphs"] == 1


def test_batch_tune(gpu):
    sizes = [300, 2500, 7000, 20000, 65536]
    ncols = [3, 2, 4, 2, 1]
    ops, data = build_batch(gpu, sizes, ncols, seed=6)
    batch = gpu.Batch(ops, ncols)
    xs = [to_dev(d[2]) for d in data]
    ys = [to_dev(np.zeros_like(d[2])) for d in data]
    sc = batch.tune(xs, outs=ys, reps=2)
    assert 0 <= sc["max_fuse"] <= 5 and sc["region_mib"] in (24, 48, 96) and sc["ms"] > 0
    assert batch.schedule() == sc and sc["stages"] >= 1
    zs = batch.apply(xs, adjoint=True)
    for i, (col, row, x, u) in enumerate(data):
        assert rel_err(to_host(ys[i]), structured.toeplitz_apply_fft64(col, row, x)) <= TOL["c64"]
        assert rel_err(to_host(zs[i]), structured.toeplitz_apply_fft64(col, row, x, True)) <= TOL["c64"]


def test_batch_every_mixed_factor(gpu):
    """One operator per strided factor n2 of the mixed embedding (N = 2048 n2,
    so L = 4096 n2 exactly), under fold limits 2^0 (every factor through the
    separate strided passes), 2^3 (the default: n2 <= 8 folded) and 2^5 (all
    folded): forward and adjoint against the FP64 oracle, and at the default
    limit bit-identical to the plain path."""
    n2s = (3, 5, 6, 9, 10, 12, 20, 24, 30)
    sizes = [2048 * n2 for n2 in n2s]
    ncols = [1, 2, 1, 2, 1, 2, 1, 2, 1]
    ops, data = build_batch(gpu, sizes, ncols, seed=21)
    assert [op.transform_length for op in ops] == [4096 * n2 for n2 in n2s]
    batch = gpu.Batch(ops, ncols)
    xs = [to_dev(d[2]) for d in data]
    for mf in (0, 3, 5):
        batch.set_schedule(mf, 48)
        ys = batch.apply(xs)
        zs = batch.apply(xs, adjoint=True)
        for i, (op, (col, row, x, u)) in enumerate(zip(ops, data)):
            y_b, z_b = to_host(ys[i]), to_host(zs[i])
            assert rel_err(y_b, structured.toeplitz_apply_fft64(col, row, x)) <= TOL["c64"], (mf, n2s[i])
            assert rel_err(z_b, structured.toeplitz_apply_fft64(col, row, x, True)) <= TOL["c64"], (mf, n2s[i])
            if mf == 3:
                assert np.array_equal(y_b, to_host(op @ xs[i])), n2s[i]
                assert np.array_equal(z_b, to_host(op.H @ xs[i])), n2s[i]


def test_batch_set_schedule(gpu):
    from paper_1710_09578_amd import capi

    sizes = [1500, 9000, 40000]
    ncols = [2, 3, 2]
    ops, data = build_batch(gpu, sizes, ncols, seed=7)
    batch = gpu.Batch(ops, ncols)
    xs = [to_dev(d[2]) for d in data]
    for mf, rg in ((0, 24), (5, 96), (2, 16)):
        batch.set_schedule(mf, rg)
        sc = batch.schedule()
        assert sc["max_fuse"] == mf and sc["region_mib"] == rg
        ys = batch.apply(xs)
        for i, (col, row, x, u) in enumerate(data):
            assert rel_err(to_host(ys[i]), structured.toeplitz_apply_fft64(col, row, x)) <= TOL["c64"]
    with pytest.raises(capi.FmError):
        batch.set_schedule(6, 48)


def _pow2_at_least(v):
    return 1 << int(np.ceil(np.log2(v)))


def test_batch_fista_full_workload(gpu):
    """The batched-FISTA workload itself: 512 Toeplitz operators (N
    log-uniform in [256, 65536], 1-32 columns each), K = N/256-sparse truths,
    noise 1e-3, 100 iterations, lam = 0.05 ||T^H b||_inf per column, stop
    1e-5. Measurements b = T x_true + noise come from the oracle. Checked
    against the FP64 oracle (its own L and lam, FFT64 products): a seeded
    pair of columns of every operator with N <= 4096, and of one operator per
    embedding length above 4096, so that every FISTA form of the stage kernel
    (every strided factor of the four-step split) meets the oracle.

    Each column must equal the oracle's iterate at the GPU's own iteration
    count. The count itself is a decision taken on complex64 iterates: the
    relative change ||x_k - x_{k-1}|| / ||x_k|| is compared with 1e-5, about
    80 float32 ulps, so rounding moves the crossing by several iterations
    where the change flattens out near the tolerance. The count is therefore
    checked against the oracle's window: not before the first k whose FP64
    relative change is <= 1e-5 (1 + s), not after the first k whose change is
    <= 1e-5 (1 - s), s = 0.5 (the change carries the difference of two
    iterate errors, up to ~2.5e-6 of ||x_k||). The per-length operators are
    also solved by the plain fm_fista and must give the same bits and
    counts."""
    from workloads import toeplitz_batch

    iters, tol, rel, band = 100, 1e-5, 0.05, 0.5
    full = toeplitz_batch(with_fista=True)
    sizes, ncols = full["sizes"], full["ncols"]
    nops = len(sizes)
    ops, bs = [], []
    for i in range(nops):
        d = full["ops"][i]
        n = int(sizes[i])
        b = structured.toeplitz_apply_fft64(d["col"], d["row"], d["x_true"], L=_pow2_at_least(2 * n - 1))
        bs.append((b + d["noise"]).astype(np.complex64))
        ops.append(gpu.Toeplitz(to_dev(d["col"]), to_dev(d["row"])))
    bd = [to_dev(b) for b in bs]
    batch = gpu.Batch(ops, list(ncols))
    xs, st = batch.fista(bd, iters=iters, lam_rel=rel, stop_tol=tol)
    first = np.concatenate([[0], np.cumsum(ncols)[:-1]])
    # the checked columns
    rng = np.random.default_rng(77)
    lengths = {}
    for i in range(nops):
        lengths.setdefault(embedding_length(2 * int(sizes[i]) - 1), []).append(i)
    chosen = [i for i in range(nops) if sizes[i] <= 4096]
    per_length = [min(v, key=lambda i: (ncols[i], i)) for L, v in sorted(lengths.items()) if L > 4096]
    worst = {"x": 0.0, "lam": 0.0, "L": 0.0}
    stopped = same_count = 0
    for i in chosen + per_length:
        d = full["ops"][i]
        n = int(sizes[i])
        cols = np.sort(rng.choice(int(ncols[i]), min(2, int(ncols[i])), replace=False))
        Lemb = embedding_length(2 * n - 1)
        g = np.zeros(Lemb, np.complex128)
        g[:n] = d["col"]
        g[Lemb - n + 1:] = d["row"][1:][::-1]
        L_o = float(np.max(np.abs(np.fft.fft(g))) ** 2)
        emb = _pow2_at_least(2 * n - 1)
        b = bs[i][cols]
        lam_o = rel * np.max(np.abs(structured.toeplitz_apply_fft64(d["col"], d["row"], b, True, L=emb)), axis=1)
        _, _, hist = structured.toeplitz_fista_fft64(d["col"], d["row"], b, lam_o, L_o, iters, embed=emb,
                                                     history=True)
        H = np.stack([np.zeros_like(hist[0])] + hist)           # x_0 .. x_iters
        change = np.linalg.norm(H[1:] - H[:-1], axis=2) / np.maximum(np.linalg.norm(H[1:], axis=2), 1e-30)
        got_x = to_host(xs[i])[cols]
        for jj, j in enumerate(cols):
            s = st[first[i] + j]
            worst["L"] = max(worst["L"], abs(s["L"] - L_o) / L_o)
            worst["lam"] = max(worst["lam"], abs(s["lam"] - lam_o[jj]) / lam_o[jj])
            k = int(s["iters"])
            r = change[:, jj]                                  # r[k-1]: change of iteration k
            lo = np.flatnonzero(r <= tol * (1 + band))
            hi = np.flatnonzero(r <= tol * (1 - band))
            k_lo = int(lo[0]) + 1 if lo.size else iters
            k_hi = int(hi[0]) + 1 if hi.size else iters
            assert k_lo <= k <= k_hi, f"op {i} column {j}: stopped at {k}, oracle window [{k_lo}, {k_hi}]"
            stopped += k < iters
            same_count += k == (int(np.flatnonzero(r <= tol)[0]) + 1 if np.any(r <= tol) else iters)
            e = rel_err(got_x[jj:jj + 1], H[k, jj:jj + 1])
            worst["x"] = max(worst["x"], e)
            assert e <= TOL["c64"], f"op {i} (N={n}, L={Lemb}) column {j} at iteration {k}: {e:.3e}"
    assert worst["L"] <= 1e-12 and worst["lam"] <= TOL["c64"], worst
    print(f"batched FISTA workload: {len(chosen) + len(per_length)} operators checked, worst {worst}, "
          f"{stopped} columns stopped early, {same_count} at the oracle's own count")
    # plain solver on the same operators: same bits, same counts
    for i in per_length:
        x_p, st_p = gpu.fista(ops[i], bd[i], iters=iters, lam_rel=rel, L=st[first[i]]["L"], stop_tol=tol)
        assert np.array_equal(to_host(x_p), to_host(xs[i])), f"op {i}: batched solve differs from plain"
        assert [s["iters"] for s in st_p] == [st[first[i] + j]["iters"] for j in range(int(ncols[i]))]
