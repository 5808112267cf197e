"""Operator objects in the paper's notation over the C ABI.

``A @ x`` is the forward transform y = A x (eq. (3)) and ``A.H @ y`` the
backward transform A^H y (eq. (4)); composites are built with ``Product``
(also ``A @ B`` for two operators), ``Sum``, ``Kron`` and ``BlkDiag``. Blocks of
vectors are torch tensors of shape (ncols, rows) on the GPU (a 1-D tensor is
one vector). Torch provides the device memory and the current stream; every
operation itself runs in the HIP library.
"""

from __future__ import annotations

import torch

from . import capi

_DT = {
    torch.complex64: capi.FM_C64,
    torch.complex128: capi.FM_C128,
    torch.int32: capi.FM_I32,
    torch.int64: capi.FM_I64,
}
_TORCH = {v: k for k, v in _DT.items()}


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _dt(dtype) -> int:
    try:
        return _DT[dtype]
    except KeyError:
        raise TypeError(f"unsupported dtype {dtype}") from None


def _dev(t: torch.Tensor, dtype=None) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError("parameter arrays must be GPU tensors")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    return t.contiguous()


class Operator:
    """An immutable structured linear operator (a handle of the library)."""

    def __init__(self, handle, keep=()):
        self._h = handle
        self._keep = keep  # Python objects that must outlive the handle
        m, n, dt = capi.fm_op_shape(handle)
        self.shape = (m, n)
        self.dtype = _TORCH[dt]

    @property
    def handle(self):
        return self._h

    @property
    def transform_length(self):
        """Cyclic length of the operator's transforms (the embedding length
        for Toeplitz), 0 for kinds without one."""
        return capi.fm_op_transform_length(self._h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None:
            try:
                capi.fm_op_release(h)
            except Exception:
                pass
            self._h = None

    # ------------------------------------------------------------ views
    @property
    def H(self) -> "Operator":
        """Hermitian transpose (shares storage)."""
        return Operator(capi.fm_op_adjoint(self._h), keep=(self,))

    @property
    def conj(self) -> "Operator":
        """Complex conjugate conj(A) (shares storage)."""
        return Operator(capi.fm_op_conj(self._h), keep=(self,))

    @property
    def T(self) -> "Operator":
        """Transpose A^T = conj(A)^H (shares storage)."""
        c = self.conj
        return Operator(capi.fm_op_adjoint(c.handle), keep=(c,))

    @property
    def gram(self) -> "Operator":
        """Gramian A^H A, fused from the structure where one exists."""
        return Operator(capi.fm_op_gram(self._h), keep=(self,))

    def calibrate(self, ncols: int) -> dict:
        """Time the structured and the dense evaluation on ncols columns and
        keep the faster (operators up to 64 x 64)."""
        choice, tf, td = capi.fm_op_calibrate(self._h, int(ncols), _stream())
        return {"path": "dense" if choice else "structured", "ms_structured": tf, "ms_dense": td}

    def set_path(self, path: str):
        """Force the evaluation path: "structured" or "dense"."""
        capi.fm_op_set_path(self._h, 1 if path == "dense" else 0)

    def choose_path(self, ncols: int) -> str:
        """Set the evaluation path from the device's calibration model
        (calibration_build / calibration_load) without timing this handle."""
        return "dense" if capi.fm_op_choose_path(self._h, int(ncols)) else "structured"

    @property
    def inverse(self) -> "Operator":
        """Structured inverse A^-1 (Circulant, Diag, Fourier, Hadamard,
        permutations and their Kron / BlkDiag / Product / views)."""
        return Operator(capi.fm_op_inverse(self._h), keep=(self,))

    # ------------------------------------------------------------ application
    def _block(self, x: torch.Tensor, rows: int):
        if x.dtype != self.dtype:
            raise TypeError(f"operator is {self.dtype}, input is {x.dtype}")
        if not x.is_cuda:
            raise ValueError("input must be a GPU tensor")
        vec = x.dim() == 1
        xb = x.unsqueeze(0) if vec else x
        if xb.dim() != 2 or xb.shape[1] != rows:
            raise ValueError(f"expected a block of shape (ncols, {rows}), got {tuple(x.shape)}")
        if xb.stride(1) != 1:
            xb = xb.contiguous()
        return xb, vec

    def apply(self, x: torch.Tensor, adjoint: bool = False, out: torch.Tensor | None = None,
              workspace: torch.Tensor | None = None) -> torch.Tensor:
        m, n = self.shape
        rin, rout = (m, n) if adjoint else (n, m)
        xb, vec = self._block(x, rin)
        ncols = xb.shape[0]
        if out is None:
            y = torch.empty((ncols, rout), dtype=self.dtype, device=xb.device)
        else:
            y = out.unsqueeze(0) if out.dim() == 1 else out
            if y.shape != (ncols, rout) or y.stride(1) != 1 or y.dtype != self.dtype:
                raise ValueError("out has the wrong shape, layout or dtype")
        d = capi.FM_ADJ if adjoint else capi.FM_FWD
        need = capi.fm_workspace_size(self._h, d, ncols)
        if workspace is None and need:
            workspace = torch.empty(need, dtype=torch.uint8, device=xb.device)
        wsb = 0 if workspace is None else workspace.numel()
        capi.fm_apply(self._h, d, ncols, xb, max(xb.stride(0), rin), y, max(y.stride(0), rout),
                      workspace, wsb, _stream())
        return y.squeeze(0) if vec and out is None else (out if out is not None else y)

    def forward(self, x):
        return self.apply(x, False)

    def backward(self, x):
        return self.apply(x, True)

    def __matmul__(self, other):
        if isinstance(other, Operator):
            return Product(self, other)
        return self.apply(other, False)

    def __add__(self, other):
        return Sum(self, other)

    def __repr__(self):
        return f"<Operator {self.shape[0]}x{self.shape[1]} {self.dtype}>"


# ---------------------------------------------------------------- elementary
def Fourier(n: int, dtype=torch.complex64) -> Operator:
    return Operator(capi.fm_op_create_fourier(n, _dt(dtype)))


def Hadamard(n: int, dtype=torch.complex64) -> Operator:
    return Operator(capi.fm_op_create_hadamard(n, _dt(dtype)))


def Diag(d: torch.Tensor) -> Operator:
    d = _dev(d)
    return Operator(capi.fm_op_create_diag(d.numel(), d, _dt(d.dtype), _stream()))


def Dense(a: torch.Tensor) -> Operator:
    """Dense (m, n) matrix given as a torch tensor indexed [row, col]."""
    a = _dev(a)
    m, n = a.shape
    colmajor = a.t().contiguous()  # element (i, j) at i + j*m
    return Operator(capi.fm_op_create_dense(m, n, colmajor, m, _dt(a.dtype), _stream()))


def Circulant(c: torch.Tensor) -> Operator:
    c = _dev(c)
    return Operator(capi.fm_op_create_circulant(c.numel(), c, _dt(c.dtype), _stream()))


def LFSRCirculant(order: int, taps: int, state: int = 1, dtype=torch.complex64) -> Operator:
    """Circulant of size 2^order - 1 whose first column is the +-1 output of a
    linear feedback shift register (taps / state bit masks)."""
    return Operator(capi.fm_op_create_lfsr_circulant(int(order), int(taps), int(state), _dt(dtype), _stream()))


def Toeplitz(col: torch.Tensor, row: torch.Tensor) -> Operator:
    col, row = _dev(col), _dev(row, col.dtype)
    return Operator(capi.fm_op_create_toeplitz(col.numel(), row.numel(), col, row, _dt(col.dtype),
                                               _stream()))


def MLToeplitz(n_levels, t: torch.Tensor) -> Operator:
    t = _dev(t)
    return Operator(capi.fm_op_create_mltoeplitz(len(n_levels), list(n_levels), t, _dt(t.dtype),
                                                 _stream()))


def SelectRows(n_in: int, rows: torch.Tensor, dtype=torch.complex64) -> Operator:
    rows = _dev(rows, torch.int32)
    return Operator(capi.fm_op_create_select_rows(n_in, rows.numel(), rows, _dt(dtype), _stream()))


# ---------------------------------------------------------------- composites
def _compose(kind, ops):
    ops = list(ops)
    return Operator(capi.fm_op_compose(kind, [o.handle for o in ops]), keep=tuple(ops))


def Product(*ops) -> Operator:
    return _compose(capi.FM_PRODUCT, ops)


def Sum(*ops) -> Operator:
    return _compose(capi.FM_SUM, ops)


def Kron(*ops) -> Operator:
    return _compose(capi.FM_KRON, ops)


def BlkDiag(*ops) -> Operator:
    return _compose(capi.FM_BLKDIAG, ops)


def Blocks(grid) -> Operator:
    """Block matrix [[A_00, A_01, ...], [A_10, ...], ...] (a list of block rows).
    Blocks of one block row share their row count, blocks of one block column
    their column count."""
    rows = [list(r) for r in grid]
    if not rows or not rows[0] or any(len(r) != len(rows[0]) for r in rows):
        raise ValueError("Blocks needs a non-empty rectangular grid")
    flat = [a for r in rows for a in r]
    return Operator(capi.fm_op_create_blocks(len(rows), len(rows[0]), [a.handle for a in flat]), keep=tuple(flat))


def Partial(A: Operator, rows=None, cols=None) -> Operator:
    """A restricted to the selected rows and / or columns: S_rows A S_cols^H
    (x of length len(cols) is placed at the selected columns, zeros
    elsewhere)."""
    terms = []
    if rows is not None:
        terms.append(SelectRows(A.shape[0], rows, A.dtype))
    terms.append(A)
    if cols is not None:
        terms.append(SelectRows(A.shape[1], cols, A.dtype).H)
    return terms[0] if len(terms) == 1 else Product(*terms)


def compressed_ultrasound(t: torch.Tensor, psi_rows):
    """The compressed ultrasound model b = Psi H x (eq. (9) with the block
    structure of eq. (6)/(7)). t: (n1, n1, 2 n2 - 1, 2 n3 - 1) generators of
    the 2-level Toeplitz blocks H_ij (levels n2, n3); psi_rows: (n1 n2, nf)
    Fourier rows kept per A-scan of n3 samples. Psi = BlkDiag of the row
    selections S_a F_n3, applied as one batched DFT of all A-scans followed by
    one gather. Returns (H, Psi, Psi H)."""
    t = _dev(t)
    n1, n2, n3 = t.shape[0], (t.shape[2] + 1) // 2, (t.shape[3] + 1) // 2
    if t.shape[1] != n1:
        raise ValueError("t must hold an n1 x n1 grid of generators")
    H = Blocks([[MLToeplitz([n2, n3], t[i, j].contiguous()) for j in range(n1)] for i in range(n1)])
    rows = torch.as_tensor(psi_rows, dtype=torch.int64)
    glob = (rows + n3 * torch.arange(rows.shape[0], dtype=torch.int64)[:, None]).reshape(-1)
    F = Fourier(n3, t.dtype)
    Psi = Product(SelectRows(n1 * n2 * n3, glob.to(device=t.device, dtype=torch.int32), t.dtype),
                  BlkDiag(*([F] * (n1 * n2))))
    return H, Psi, Product(Psi, H)


# ---------------------------------------------------------------- solver
def calibration_build():
    """Measure the device's calibration model (structured vs dense times of
    circulant, Toeplitz and Fourier operators over sizes 8..64 and 1..65536
    columns); returns its table."""
    capi.fm_calibration_build(_stream())
    return capi.fm_calibration_entries()


def calibration_table():
    """The current device's calibration model as a list of dicts (empty when
    none was built or loaded)."""
    return capi.fm_calibration_entries()


def calibration_load(table):
    """Install a saved calibration model on the current device."""
    capi.fm_calibration_load(list(table))


def fista_options(iters=200, momentum=True, lam=None, lam_rel=None, L=None, stop_tol=0.0,
                  x0_given=False, power_iters=500, power_tol=1e-13, seed=0):
    o = capi.fm_fista_opts()
    o.max_iters = int(iters)
    o.momentum = 1 if momentum else 0
    o.x0_given = 1 if x0_given else 0
    o.power_max_iters = int(power_iters)
    o.lambda_abs = float(lam) if lam is not None else 0.0
    o.lambda_rel = float(lam_rel) if lam_rel is not None else 0.0
    o.L = float(L) if L is not None else 0.0
    o.stop_tol = float(stop_tol)
    o.power_tol = float(power_tol)
    o.seed = int(seed)
    return o


def fista(A: Operator, b: torch.Tensor, iters=200, momentum=True, lam=None, lam_rel=None, L=None,
          stop_tol=0.0, x0=None, power_iters=500, power_tol=1e-13, seed=0):
    """FISTA (momentum=True) or ISTA for min 1/2||A x - b||^2 + lam ||x||_1 per
    column of b (shape (ncols, m)); lam absolute, or lam_rel * ||A^H b||_inf.
    Returns (x, stats) with stats a list of dicts per column."""
    import ctypes as C

    m, n = A.shape
    bb = b.unsqueeze(0) if b.dim() == 1 else b
    if bb.stride(1) != 1:
        bb = bb.contiguous()
    ncols = bb.shape[0]
    if x0 is not None:
        x = (x0.unsqueeze(0) if x0.dim() == 1 else x0).clone().contiguous()
    else:
        x = torch.empty((ncols, n), dtype=A.dtype, device=bb.device)
    o = fista_options(iters, momentum, lam, lam_rel, L, stop_tol, x0 is not None, power_iters, power_tol, seed)
    need = capi.fm_fista_workspace_size(A.handle, ncols, o)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=bb.device)
    stats = (capi.fm_fista_stat * max(ncols, 1))()
    capi.fm_fista(A.handle, ncols, bb, max(bb.stride(0), m), x, n, o, stats, ws, ws.numel(), _stream())
    st = [{"iters": stats[j].iters_done, "status": stats[j].status, "L": stats[j].L_used,
           "lam": stats[j].lambda_used} for j in range(ncols)]
    return (x.squeeze(0) if b.dim() == 1 else x), st


def omp(A: Operator, b: torch.Tensor, k: int, tol: float = 0.0):
    """Orthogonal matching pursuit with at most k atoms per column of b (shape
    (ncols, m)), stopping a column once ||b - A x|| <= tol ||b||. Returns
    (x, support, stats): support (ncols, k) int32 on the device in selection
    order (-1 after the last atom), stats a list of dicts per column."""
    m, n = A.shape
    bb = b.unsqueeze(0) if b.dim() == 1 else b
    if bb.stride(1) != 1:
        bb = bb.contiguous()
    ncols = bb.shape[0]
    x = torch.empty((ncols, n), dtype=A.dtype, device=bb.device)
    sup = torch.empty((ncols, k), dtype=torch.int32, device=bb.device)
    need = capi.fm_omp_workspace_size(A.handle, ncols, k)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=bb.device)
    stats = (capi.fm_omp_stat * max(ncols, 1))()
    capi.fm_omp(A.handle, ncols, bb, max(bb.stride(0), m), int(k), float(tol), x, n, sup, stats, ws, ws.numel(),
                _stream())
    st = [{"atoms": stats[j].atoms, "status": stats[j].status, "res_norm": stats[j].res_norm} for j in range(ncols)]
    if b.dim() == 1:
        return x.squeeze(0), sup.squeeze(0), st
    return x, sup, st


def power_iteration(A: Operator, v0: torch.Tensor | None = None, seed=0, max_iters=500, tol=1e-13):
    """L = ||A||_2^2 in FP64; v0: complex128 GPU start vector (default:
    SplitMix64 vector of ``seed``). Returns (L, iterations)."""
    if v0 is not None:
        v0 = _dev(v0, torch.complex128)
    return capi.fm_power_iteration(A.handle, v0, seed, max_iters, tol, _stream())


# ---------------------------------------------------------------- batching
class Batch:
    """Many circulant / Toeplitz operators applied together in pipelined stage launches.

    ``ncols[i]`` is the number of columns operator i is applied to; blocks are
    passed per call as lists of tensors of shape (ncols[i], rows).
    """

    def __init__(self, ops, ncols):
        self.ops = list(ops)
        self.ncols = [int(v) for v in ncols]
        if len(self.ops) != len(self.ncols):
            raise ValueError("one column count per operator")
        self._h = capi.fm_batch_create([o.handle for o in self.ops], self.ncols)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None:
            try:
                capi.fm_batch_release(h)
            except Exception:
                pass
            self._h = None

    def apply(self, xs, adjoint: bool = False, outs=None):
        if len(xs) != len(self.ops):
            raise ValueError("one block per operator")
        if outs is None:
            outs = []
            for op, x, nc in zip(self.ops, xs, self.ncols):
                m, n = op.shape
                outs.append(torch.empty((nc, n if adjoint else m), dtype=op.dtype, device=x.device))
        ldx = [max(x.stride(0), 1) if x.dim() == 2 else x.shape[-1] for x in xs]
        ldy = [max(y.stride(0), 1) if y.dim() == 2 else y.shape[-1] for y in outs]
        capi.fm_batch_apply(self._h, capi.FM_ADJ if adjoint else capi.FM_FWD, xs, ldx, outs, ldy,
                            _stream())
        return outs

    def tune(self, xs, adjoint: bool = False, outs=None, reps: int = 3):
        """Times every candidate schedule on these blocks and keeps the
        fastest (fm_batch_tune); returns the chosen schedule as a dict."""
        if outs is None:
            outs = [torch.empty((nc, op.shape[1] if adjoint else op.shape[0]), dtype=op.dtype, device=x.device)
                    for op, x, nc in zip(self.ops, xs, self.ncols)]
        ldx = [max(x.stride(0), 1) if x.dim() == 2 else x.shape[-1] for x in xs]
        ldy = [max(y.stride(0), 1) if y.dim() == 2 else y.shape[-1] for y in outs]
        return capi.fm_batch_tune(self._h, capi.FM_ADJ if adjoint else capi.FM_FWD, xs, ldx, outs, ldy, reps,
                                  _stream())

    def schedule(self):
        return capi.fm_batch_get_schedule(self._h)

    def set_schedule(self, max_fuse: int, region_mib: int):
        capi.fm_batch_set_schedule(self._h, max_fuse, region_mib)

    def fista(self, bs, iters=100, momentum=True, lam=None, lam_rel=None, L=None, stop_tol=0.0, x0s=None):
        """FISTA for every column of every operator; bs[i] has shape
        (ncols[i], m_i). Returns (xs, stats) with stats per batch column."""
        xs = []
        for op, b, nc in zip(self.ops, bs, self.ncols):
            xs.append(torch.empty((nc, op.shape[1]), dtype=op.dtype, device=b.device))
        if x0s is not None:
            for x, x0 in zip(xs, x0s):
                x.copy_(x0)
        o = fista_options(iters, momentum, lam, lam_rel, L, stop_tol, x0s is not None)
        total = sum(self.ncols)
        stats = (capi.fm_fista_stat * max(total, 1))()
        ldb = [max(b.stride(0), 1) if b.dim() == 2 else b.shape[-1] for b in bs]
        ldx = [op.shape[1] for op in self.ops]
        capi.fm_batch_fista(self._h, bs, ldb, xs, ldx, o, stats, _stream())
        st = [{"iters": stats[j].iters_done, "status": stats[j].status, "L": stats[j].L_used,
               "lam": stats[j].lambda_used} for j in range(total)]
        return xs, st
