"""GPU parity of block matrices (fm_op_create_blocks), block-diagonal runs,
row / column restriction and the compressed ultrasound model Psi H against
the FP64 oracle.

Small cases compare whole outputs with the dense oracle matrix. The model at
its benchmark size (n1 = n2 = 32, n3 = 512: H has 524288 columns) is checked
on sampled output rows, each built from the definition of its 32 blocks.
"""

import numpy as np
import pytest

from oracle import dense, fista
from tests.gpu_util import TOL, crandn, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

NP = {"c64": np.complex64, "c128": np.complex128}


def tdt(prec):
    import torch

    return {"c64": torch.complex64, "c128": torch.complex128}[prec]


def check_both(op, a, rng, prec, ncols=3):
    m, n = a.shape
    x = crandn(rng, (ncols, n), NP[prec])
    y = crandn(rng, (ncols, m), NP[prec])
    ey = rel_err(to_host(op @ to_dev(x)), dense.apply(a, x))
    ez = rel_err(to_host(op.H @ to_dev(y)), dense.apply(a, y, True))
    assert ey <= TOL[prec] and ez <= TOL[prec], (ey, ez)


@pytest.mark.parametrize("prec", ["c64", "c128"])
@pytest.mark.parametrize("grid,levels", [((3, 3), (4, 16)), ((2, 5), (8, 32)), ((4, 1), (3, 20)),
                                         ((1, 1), (16, 64)), ((5, 4), (2, 5))])
def test_blocks_of_ml_toeplitz_mix_path(gpu, prec, grid, levels):
    """Every block a 2-level Toeplitz of one geometry: transforms once per
    slice, mixing per frequency bin (also non-square grids, one block)."""
    rng = np.random.default_rng(sum(grid) * 7 + levels[0])
    nbr, nbc = grid
    n2, n3 = levels
    ts = [[crandn(rng, (2 * n2 - 1, 2 * n3 - 1), NP[prec]) for _ in range(nbc)] for _ in range(nbr)]
    op = gpu.Blocks([[gpu.MLToeplitz([n2, n3], to_dev(t)) for t in r] for r in ts])
    a = dense.blocks([[dense.ml_toeplitz([n2, n3], t) for t in r] for r in ts])
    check_both(op, a, rng, prec)


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_blocks_general_path_uneven(gpu, prec):
    """Mixed block kinds and uneven block sizes, a repeated handle, and the
    accumulate path (a Blocks inside a Sum)."""
    rng = np.random.default_rng(5)
    dt = tdt(prec)
    c = crandn(rng, 8, NP[prec])
    col, row = crandn(rng, 8, NP[prec]), crandn(rng, 9, NP[prec])
    d1, d2 = crandn(rng, (8, 4), NP[prec]), crandn(rng, (5, 9), NP[prec])
    dg = crandn(rng, 4, NP[prec])
    C = gpu.Circulant(to_dev(c))
    T = gpu.Toeplitz(to_dev(col), to_dev(row))
    D1, D2 = gpu.Dense(to_dev(d1)), gpu.Dense(to_dev(d2))
    Dg = gpu.Diag(to_dev(dg))
    F = gpu.Fourier(8, dt)
    P = gpu.Product(D1, Dg)  # 8 x 4
    e1, e2 = crandn(rng, (5, 8), NP[prec]), crandn(rng, (5, 4), NP[prec])
    grid = [[C, P, T], [gpu.Dense(to_dev(e1)), gpu.Dense(to_dev(e2)), D2], [F, P, T]]
    op = gpu.Blocks(grid)
    dC, dT, dP, dF = dense.circulant(c), dense.toeplitz(col, row), dense.product(d1, dense.diag(dg)), dense.fourier(8)
    a = dense.blocks([[dC, dP, dT], [e1, e2, d2], [dF, dP, dT]])
    check_both(op, a, rng, prec)
    S = gpu.Sum(op, op)
    check_both(S, 2 * a, rng, prec)


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_blocks_mix_equals_general(gpu, prec):
    """The mixing path and the block-by-block path agree: the same grid once
    as multilevel Toeplitz blocks (mixed) and once with one block wrapped in a
    one-term product (general path)."""
    rng = np.random.default_rng(11)
    n2, n3 = 8, 24
    ts = [[crandn(rng, (2 * n2 - 1, 2 * n3 - 1), NP[prec]) for _ in range(3)] for _ in range(2)]
    blocks = [[gpu.MLToeplitz([n2, n3], to_dev(t)) for t in r] for r in ts]
    mixed = gpu.Blocks(blocks)
    general = gpu.Blocks([[gpu.Product(blocks[0][0])] + blocks[0][1:], blocks[1]])
    x = crandn(rng, (2, 3 * n2 * n3), NP[prec])
    y = crandn(rng, (2, 2 * n2 * n3), NP[prec])
    assert rel_err(to_host(mixed @ to_dev(x)), to_host(general @ to_dev(x))) <= TOL[prec]
    assert rel_err(to_host(mixed.H @ to_dev(y)), to_host(general.H @ to_dev(y))) <= TOL[prec]


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_blkdiag_runs_of_one_block(gpu, prec):
    """Runs of a repeated block next to distinct blocks (one call per block),
    and whole-operator runs (one call batched over the run), including a
    four-step transform."""
    rng = np.random.default_rng(13)
    dt = tdt(prec)
    F = gpu.Fourier(16, dt)
    F2 = gpu.Fourier(8192, dt)
    d = crandn(rng, 5, NP[prec])
    D = gpu.Diag(to_dev(d))
    op = gpu.BlkDiag(F, F, F, D, F, F2, F2)
    a = dense.blkdiag(*([dense.fourier(16)] * 3 + [dense.diag(d), dense.fourier(16)] + [dense.fourier(8192)] * 2))
    check_both(op, a, rng, prec, ncols=2)
    check_both(gpu.BlkDiag(F, F, F), dense.blkdiag(*[dense.fourier(16)] * 3), rng, prec, ncols=2)
    check_both(gpu.BlkDiag(F2, F2, F2), dense.blkdiag(*[dense.fourier(8192)] * 3), rng, prec, ncols=2)


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_partial_rows_and_columns(gpu, prec):
    rng = np.random.default_rng(17)
    col, row = crandn(rng, 40, NP[prec]), crandn(rng, 30, NP[prec])
    T = gpu.Toeplitz(to_dev(col), to_dev(row))
    rows = np.array([0, 3, 7, 20, 39], np.int32)
    cols = np.array([1, 2, 5, 11, 29, 17], np.int32)
    t = dense.toeplitz(col, row)
    check_both(gpu.Partial(T, rows=to_dev(rows), cols=to_dev(cols)), t[rows][:, cols], rng, prec)
    check_both(gpu.Partial(T, cols=to_dev(cols)), t[:, cols], rng, prec)
    check_both(gpu.Partial(T, rows=to_dev(rows)), t[rows], rng, prec)


def small_model(gpu, prec, n1=3, n2=4, n3=16, nf=2, k=6, seed=21):
    from workloads import ultrasound

    w = ultrasound(n1, n2, n3, nf, k=k, seed=seed)
    t = w["t"].astype(NP[prec])
    H, Psi, PH = gpu.compressed_ultrasound(to_dev(t), w["psi_rows"])
    h = dense.blocks([[dense.ml_toeplitz([n2, n3], t[i, j]) for j in range(n1)] for i in range(n1)])
    psi = dense.blkdiag(*[dense.fourier_rows(n3, r) for r in w["psi_rows"]])
    return w, (H, Psi, PH), (h, psi, psi @ h)


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_compressed_ultrasound_small(gpu, prec):
    rng = np.random.default_rng(23)
    _, ops, mats = small_model(gpu, prec)
    for op, a in zip(ops, mats):
        check_both(op, a, rng, prec, ncols=2)


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_compressed_ultrasound_fista_20(gpu, prec):
    """20 FISTA steps on Psi H (the reconstruction run of the compressed
    model) against the oracle's iteration with the same L and lambda."""
    w, (_, _, PH), (_, _, a) = small_model(gpu, prec, n1=4, n2=4, n3=32, nf=4, k=8)
    b = (dense.apply(a, w["x_true"]) + w["noise"]).astype(NP[prec])
    L = fista.spectral_norm_sq(a)
    lam = fista.lambda_rule(a, b, 0.05)
    x_ref, _ = fista.fista(a, b, lam, L, 20)
    x, st = gpu.fista(PH, to_dev(b), iters=20, lam=float(lam[0]), L=L)
    assert st[0]["iters"] == 20 and st[0]["status"] == 0
    assert rel_err(to_host(x), x_ref) <= TOL[prec]


def test_compressed_ultrasound_full_size_sampled_rows(gpu):
    """n1 = n2 = 32, n3 = 512, nf = 1 (H: 524288 x 524288 in 1024 blocks of
    2-level Toeplitz), complex64, the launch configuration the benchmark
    times: sampled rows of H x and of H^H y, each from the definition of the
    32 blocks involved, and every row of Psi H x against Psi's definition
    applied to the library's H x."""
    import torch

    from workloads import ultrasound

    w = ultrasound()
    n1, n2, n3, nf = w["shape"]
    nb = n2 * n3
    t = w["t"]
    H, Psi, PH = gpu.compressed_ultrasound(torch.from_numpy(t).cuda(), w["psi_rows"])
    rng = np.random.default_rng(29)
    x = crandn(rng, (1, n1 * nb))
    yv = crandn(rng, (1, n1 * nb))
    Hx = to_host(H @ to_dev(x))[0]
    Hty = to_host(H.H @ to_dev(yv))[0]
    PHx = to_host(PH @ to_dev(x))[0]
    rows = np.sort(rng.choice(n1 * nb, 24, replace=False))
    ref_f, ref_a = [], []
    for r in rows:
        i, rl = divmod(int(r), nb)
        ref_f.append(sum(dense.ml_toeplitz_rows([n2, n3], t[i, j], [rl])[0] @ x[0, j * nb:(j + 1) * nb]
                         for j in range(n1)))
        # row r of H^H = conj of column r of H: column rl of block column i
        ref_a.append(sum(np.conj(dense.ml_toeplitz_rows([n2, n3], t[j, i][::-1, ::-1], [rl])[0])
                         @ yv[0, j * nb:(j + 1) * nb] for j in range(n1)))
    ef = np.linalg.norm(Hx[rows] - np.array(ref_f)) / np.linalg.norm(ref_f)
    ea = np.linalg.norm(Hty[rows] - np.array(ref_a)) / np.linalg.norm(ref_a)
    # Psi H x = Psi (H x): Psi from its definition on every A-scan of the
    # library's H x (whose rows are checked above)
    hx = Hx.astype(np.complex128).reshape(n1 * n2, n3)
    ref_p = np.concatenate([dense.fourier_rows(n3, w["psi_rows"][a_]) @ hx[a_] for a_ in range(n1 * n2)])
    ep = np.linalg.norm(PHx - ref_p) / np.linalg.norm(ref_p)
    print(f"ultrasound full size: H {ef:.2e} H^H {ea:.2e} Psi H {ep:.2e}")
    assert ef <= TOL["c64"] and ea <= TOL["c64"] and ep <= TOL["c64"]
