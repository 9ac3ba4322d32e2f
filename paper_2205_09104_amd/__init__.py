"""MI355X coarsest-level solver: Python binding of libdcsolve.so.

Thin argument marshalling over the C ABI (include/dcsolve.h): PyTorch supplies
device memory and the current HIP stream; every step of the solve runs in the
library's HIP kernels.  Tensors are complex128 (FP64 paths) or complex64
(reduced-precision applies) on the current CUDA/HIP device, shaped [V, n] for
vectors, [V, n, n] for self blocks and [V, 4, n, n] for forward hop blocks.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib
from ._lib import (DC_PREC_F16S, DC_PREC_F32, DC_PREC_F64, DC_STORE_F16S, DC_STORE_F32,
                   DC_STORE_F64, DcError, check, load)

PREC = {"f64": DC_PREC_F64, "f32": DC_PREC_F32, "f16s": DC_PREC_F16S}
STORE = {"f64": DC_STORE_F64, "f32": DC_STORE_F32, "f16s": DC_STORE_F16S}


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor):
    return C.c_void_p(t.data_ptr())


def _vec_dtype(prec: str):
    return torch.complex128 if prec == "f64" else torch.complex64


@dataclass
class Opts:
    """Solver options (mirror of dc_solve_opts)."""
    m: int = 30
    k: int = 0
    d: int = 0
    u: int = 10
    max_cycles: int = 100000
    block_jacobi: int = 0
    prec: str = "f64"
    outer: int = 0
    m_outer: int = 10
    max_outer: int = 50
    inner_tol: float = 1e-4
    seed: int = 0
    v0: torch.Tensor | None = field(default=None, repr=False)
    schur: int = 0      # 1: odd-even reduced system (even extents only)
    ortho: int = 0      # 1: single-sync Arnoldi (one reduction per step)
    x_ref: torch.Tensor | None = field(default=None, repr=False)   # [R, V, n] complex128
    graphs: int = 0     # 1: replay whole Arnoldi cycles as captured HIP graphs

    def to_c(self) -> _lib.SolveOpts:
        o = _lib.SolveOpts()
        o.m, o.k, o.d, o.u = self.m, self.k, self.d, self.u
        o.max_cycles, o.block_jacobi = self.max_cycles, self.block_jacobi
        o.prec = PREC[self.prec]
        o.outer, o.m_outer, o.max_outer = self.outer, self.m_outer, self.max_outer
        o.inner_tol, o.seed = float(self.inner_tol), int(self.seed)
        o.schur = int(self.schur)
        o.ortho = int(self.ortho)
        o.graphs = int(self.graphs)
        if self.v0 is not None:
            assert self.v0.dtype == torch.complex128 and self.v0.is_cuda
            o.v0 = self.v0.data_ptr()
        if self.x_ref is not None:
            assert self.x_ref.dtype == torch.complex128 and self.x_ref.is_cuda
            assert self.x_ref.is_contiguous()
            o.x_ref = self.x_ref.data_ptr()
        return o


def _desc(dims, n_tv, store, mu, on_device):
    desc = _lib.OpDesc()
    for i in range(4):
        desc.dims[i] = int(dims[i])
    desc.n_tv = int(n_tv)
    desc.store = sum(STORE[s] for s in set(store) | {"f64"})
    desc.where = _lib.DC_WHERE_DEVICE if on_device else _lib.DC_WHERE_HOST
    desc.mu = float(mu)
    return desc


def workspace_bytes(dims, n_tv, store=("f64",), mu=0.0, opts: "Opts | None" = None,
                    max_rhs=0, on_device=True):
    """(persistent, scratch) device bytes of a handle built on caller memory
    (dc_workspace_bytes)."""
    pb, sb = C.c_size_t(), C.c_size_t()
    o = (opts or Opts()).to_c()
    check(load().dc_workspace_bytes(C.byref(_desc(dims, n_tv, store, mu, on_device)), C.byref(o),
                                    int(max_rhs), C.byref(pb), C.byref(sb)))
    return pb.value, sb.value


def device_allocations():
    """(count, bytes held) of the library's own hipMalloc allocations."""
    c, b = C.c_int64(), C.c_int64()
    check(load().dc_device_allocations(C.byref(c), C.byref(b)))
    return c.value, b.value


class CoarseOp:
    """Handle of the coarse operator D_c (build_coarse_op)."""

    def __init__(self, self_blocks: torch.Tensor, hop_blocks: torch.Tensor, dims, mu=0.0,
                 store=("f64",), stream=None, workspace=None):
        """workspace: optional (persistent, scratch) pair of CUDA uint8 tensors
        sized by workspace_bytes(); the handle then takes all its device
        memory from them (build_coarse_op_ws) and keeps them alive."""
        lib = load()
        assert self_blocks.dtype == torch.complex128 and hop_blocks.dtype == torch.complex128
        V, n, n2 = self_blocks.shape
        assert n == n2 and n % 2 == 0 and hop_blocks.shape == (V, 4, n, n)
        self.dims = tuple(int(d) for d in dims)
        assert int(np.prod(self.dims)) == V
        self.V, self.n, self.mu = V, n, float(mu)
        self.store = tuple(store)
        desc = _lib.OpDesc()
        for i in range(4):
            desc.dims[i] = self.dims[i]
        desc.n_tv = n // 2
        desc.store = sum(STORE[s] for s in set(store) | {"f64"})
        on_dev = self_blocks.is_cuda
        assert hop_blocks.is_cuda == on_dev
        desc.where = _lib.DC_WHERE_DEVICE if on_dev else _lib.DC_WHERE_HOST
        desc.mu = self.mu
        sb = self_blocks.contiguous()
        hb = hop_blocks.contiguous()
        h = C.c_void_p()
        st = _stream_ptr(stream) if on_dev or torch.cuda.is_available() else None
        self._ws = workspace
        if workspace is None:
            check(lib.build_coarse_op(C.byref(desc), _ptr(sb), _ptr(hb), st, C.byref(h)))
        else:
            pw, sw = workspace
            assert pw.dtype == torch.uint8 and sw.dtype == torch.uint8
            assert pw.is_cuda and sw.is_cuda and pw.is_contiguous() and sw.is_contiguous()
            check(lib.build_coarse_op_ws(C.byref(desc), _ptr(sb), _ptr(hb), _ptr(pw),
                                         pw.numel(), _ptr(sw), sw.numel(), st, C.byref(h)))
        self._h = h

    def graph_stats(self):
        """(captured, launched) Arnoldi-cycle graphs of this handle."""
        c, l = C.c_int64(), C.c_int64()
        check(load().dc_graph_stats(self._h, C.byref(c), C.byref(l)))
        return c.value, l.value

    def workspace_used(self):
        """Peak (persistent, scratch) bytes used of the caller's workspaces."""
        pb, sb = C.c_size_t(), C.c_size_t()
        check(load().dc_workspace_used(self._h, C.byref(pb), C.byref(sb)))
        return pb.value, sb.value

    # -- lifetime
    def close(self):
        if getattr(self, "_h", None):
            load().destroy_coarse_op(self._h)
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def update(self, self_blocks, hop_blocks, stream=None):
        check(load().update_coarse_op(self._h, _ptr(self_blocks.contiguous()),
                                      _ptr(hop_blocks.contiguous()), _stream_ptr(stream)))

    # -- operator
    def empty(self, prec="f64", batch=None):
        shape = (self.V, self.n) if batch is None else (batch, self.V, self.n)
        return torch.empty(shape, dtype=_vec_dtype(prec), device="cuda")

    def apply(self, x: torch.Tensor, prec="f64", adjoint=False, out=None, stream=None):
        x = x.contiguous()
        assert x.dtype == _vec_dtype(prec) and x.shape == (self.V, self.n)
        out = self.empty(prec) if out is None else out
        check(load().dc_apply(self._h, PREC[prec], int(adjoint), _ptr(x), _ptr(out),
                              _stream_ptr(stream)))
        return out

    def apply_reduced(self, x: torch.Tensor, prec="f64", adjoint=False, out=None, stream=None,
                      block_jacobi=False):
        """Odd-even reduced operator on a compressed even-site vector [V/2, n];
        block_jacobi: D_ee^{-1} S (adjoint not available)."""
        x = x.contiguous()
        assert x.dtype == _vec_dtype(prec) and x.shape == (self.V // 2, self.n)
        out = torch.empty_like(x) if out is None else out
        if block_jacobi:
            assert not adjoint
            check(load().dc_apply_reduced_bj(self._h, PREC[prec], _ptr(x), _ptr(out),
                                             _stream_ptr(stream)))
        else:
            check(load().dc_apply_reduced(self._h, PREC[prec], int(adjoint), _ptr(x),
                                          _ptr(out), _stream_ptr(stream)))
        return out

    def apply_multi(self, X: torch.Tensor, prec="f64", adjoint=False, out=None, stream=None):
        """Y[r] = D X[r] for X of shape [R, V, n] (one MFMA launch)."""
        X = X.contiguous()
        assert X.dtype == _vec_dtype(prec) and X.shape[1:] == (self.V, self.n)
        out = torch.empty_like(X) if out is None else out
        check(load().dc_apply_multi(self._h, PREC[prec], int(adjoint), X.shape[0], _ptr(X),
                                    _ptr(out), _stream_ptr(stream)))
        return out

    def grad_hops(self, lam: torch.Tensor, x: torch.Tensor, tied=True, stream=None):
        g = torch.empty((self.V, 4 if tied else 8, self.n, self.n), dtype=torch.complex128,
                        device="cuda")
        check(load().dc_grad_hops(self._h, _ptr(lam.contiguous()), _ptr(x.contiguous()),
                                  _ptr(g), int(tied), _stream_ptr(stream)))
        return g

    def neighbours(self) -> np.ndarray:
        out = np.empty((8, self.V), dtype=np.int32)
        check(load().dc_neighbours(self._h, out.ctypes.data_as(C.POINTER(C.c_int32))))
        return out

    def export_f16(self):
        codes = np.empty((self.V, 5, self.n, self.n, 2), dtype=np.uint16)
        scales = np.empty((self.V, 5), dtype=np.float32)
        check(load().dc_export_f16(self._h, codes.ctypes.data_as(C.POINTER(C.c_uint16)),
                                   scales.ctypes.data_as(C.POINTER(C.c_float))))
        return codes, scales

    # -- polynomial / Arnoldi
    def poly_setup(self, opts: Opts, stream=None) -> np.ndarray:
        th = np.zeros(2 * max(opts.d, 1), dtype=np.float64)
        du = C.c_int32()
        o = opts.to_c()
        check(load().dc_poly_setup(self._h, C.byref(o), _stream_ptr(stream),
                                   th.ctypes.data_as(C.POINTER(C.c_double)), C.byref(du)))
        return (th[0::2] + 1j * th[1::2])[:du.value]

    def poly_set(self, theta, opts: Opts):
        """Install the polynomial roots theta (complex, in chain order) for the
        variant of opts (opts.d == len(theta))."""
        th = np.asarray(theta, dtype=np.complex128)
        buf = np.empty(2 * th.size, dtype=np.float64)
        buf[0::2], buf[1::2] = th.real, th.imag
        o = opts.to_c()
        check(load().dc_poly_set(self._h, C.byref(o), buf.ctypes.data_as(C.POINTER(C.c_double)),
                                 int(th.size)))

    def poly_apply(self, x: torch.Tensor, opts: Opts, stream=None):
        x = x.contiguous()
        out = torch.empty_like(x)
        o = opts.to_c()
        check(load().dc_poly_apply(self._h, C.byref(o), _ptr(x), _ptr(out), _stream_ptr(stream)))
        return out

    def arnoldi(self, v: torch.Tensor, steps: int, opts: Opts, stream=None):
        hb = np.zeros(2 * (steps + 1) * steps, dtype=np.float64)
        sd = C.c_int32()
        o = opts.to_c()
        check(load().dc_arnoldi(self._h, C.byref(o), _ptr(v.contiguous()), int(steps),
                                _stream_ptr(stream), hb.ctypes.data_as(C.POINTER(C.c_double)),
                                C.byref(sd)))
        H = (hb[0::2] + 1j * hb[1::2]).reshape(steps, steps + 1).T
        return H[:sd.value + 1, :sd.value], sd.value

    # -- solves
    def solve(self, b: torch.Tensor, tol, opts: Opts | None = None, x0=None, adjoint=False,
              stream=None):
        """Solve D_c x = b (or D_c^H x = b).  b: [V, n] or [R, V, n] complex128.
        Returns (x, [stats dict per right-hand side], return code)."""
        opts = opts or Opts()
        single = b.dim() == 2
        bb = (b[None] if single else b).contiguous()
        R = bb.shape[0]
        assert bb.dtype == torch.complex128 and bb.shape[1:] == (self.V, self.n)
        if x0 is not None:
            x = (x0[None] if single else x0).clone().contiguous()
        else:
            x = torch.empty_like(bb)
        tols = np.broadcast_to(np.asarray(tol, dtype=np.float64), (R,)).copy()
        stats = (_lib.SolveStats * R)()
        o = opts.to_c()
        fn = load().solve_coarse_adjoint if adjoint else load().solve_coarse
        rc = check(fn(self._h, C.byref(o), R, _ptr(bb), _ptr(x),
                      tols.ctypes.data_as(C.POINTER(C.c_double)), int(x0 is not None),
                      _stream_ptr(stream), stats))
        st = [stats[i].as_dict() for i in range(R)]
        return (x[0] if single else x), st, rc

    def solve_batch(self, b: torch.Tensor, tol, opts: Opts | None = None, x0=None,
                    adjoint=False, stream=None):
        """Batched lockstep solve of R systems, b: [R, V, n] complex128; tol scalar or [R]."""
        opts = opts or Opts()
        bb = b.contiguous()
        R = bb.shape[0]
        assert bb.dtype == torch.complex128 and bb.shape[1:] == (self.V, self.n)
        x = x0.clone().contiguous() if x0 is not None else torch.empty_like(bb)
        tols = np.broadcast_to(np.asarray(tol, dtype=np.float64), (R,)).copy()
        stats = (_lib.SolveStats * R)()
        o = opts.to_c()
        rc = check(load().solve_coarse_batch(self._h, C.byref(o), int(adjoint), R, _ptr(bb),
                                             _ptr(x), tols.ctypes.data_as(C.POINTER(C.c_double)),
                                             int(x0 is not None), _stream_ptr(stream), stats))
        return x, [stats[i].as_dict() for i in range(R)], rc

    def solve_block(self, b: torch.Tensor, tol, opts: Opts | None = None, x0=None, stream=None):
        """Block GMRES with one shared Krylov space over R systems, b: [R, V, n]
        complex128; tol scalar or [R]; x0 an optional start ([R, V, n])."""
        opts = opts or Opts()
        bb = b.contiguous()
        R = bb.shape[0]
        assert bb.dtype == torch.complex128 and bb.shape[1:] == (self.V, self.n)
        x = x0.clone().contiguous() if x0 is not None else torch.empty_like(bb)
        tols = np.broadcast_to(np.asarray(tol, dtype=np.float64), (R,)).copy()
        stats = (_lib.SolveStats * R)()
        o = opts.to_c()
        rc = check(load().solve_coarse_block(self._h, C.byref(o), R, _ptr(bb), _ptr(x),
                                             tols.ctypes.data_as(C.POINTER(C.c_double)),
                                             int(x0 is not None), _stream_ptr(stream), stats))
        return x, [stats[i].as_dict() for i in range(R)], rc

    @staticmethod
    def solve_multi(ops, bs, tols, opts: "Opts | None" = None, adjoint=False, stream=None):
        """Mixed batch of lattices: ops[i] solves bs[i] ([R_i, V_i, n] complex128)
        to tolerances tols[i] (scalar or [R_i]), all in lockstep with one
        multi-apply launch per step over every operator's sites.
        Returns ([x_i], [[stats per right-hand side] per operator], rc)."""
        opts = opts or Opts()
        G = len(ops)
        assert G == len(bs) == len(tols) and G >= 1
        bb = [b.contiguous() for b in bs]
        xs = [torch.empty_like(b) for b in bb]
        R = [b.shape[0] for b in bb]
        for op, b in zip(ops, bb):
            assert b.dtype == torch.complex128 and b.shape[1:] == (op.V, op.n)
        tl = [np.broadcast_to(np.asarray(t, dtype=np.float64), (r,)).copy() for t, r in zip(tols, R)]
        stats = [(_lib.SolveStats * max(r, 1))() for r in R]
        hs = (C.c_void_p * G)(*[op._h for op in ops])
        nr = (C.c_int32 * G)(*R)
        bp = (C.c_void_p * G)(*[b.data_ptr() for b in bb])
        xp = (C.c_void_p * G)(*[x.data_ptr() for x in xs])
        tp = (C.POINTER(C.c_double) * G)(*[t.ctypes.data_as(C.POINTER(C.c_double)) for t in tl])
        sp = (C.POINTER(_lib.SolveStats) * G)(*[C.cast(s, C.POINTER(_lib.SolveStats)) for s in stats])
        o = opts.to_c()
        rc = check(load().solve_coarse_multi(hs, G, C.byref(o), int(adjoint), nr, bp, xp, tp, 0,
                                             _stream_ptr(stream), sp))
        return xs, [[stats[g][i].as_dict() for i in range(R[g])] for g in range(G)], rc

    # -- diagnostics
    def profile_apply(self, every: int = 1):
        """Start (clearing the totals) HIP-event timing of one in `every`
        launches of the apply's block kernel; every = 0 (or False) stops."""
        check(load().dc_profile_apply(self._h, int(every)))

    def profile_apply_read(self, prec: str, include_noops: bool = False, kernel: int = 0):
        """(launches, total ms) of a block kernel in precision prec since the
        last profile_apply: kernel 0 the full lattice's, 1 / 2 the reduced
        operator's A_o^{-1} D_oe / A_e - D_eo kernel; launches that did work, or with
        include_noops every launch (no-op launches of finished cycles too)."""
        n, ms, na, msa = C.c_int64(), C.c_double(), C.c_int64(), C.c_double()
        check(load().dc_profile_apply_read(self._h, PREC[prec], int(kernel), C.byref(n),
                                           C.byref(ms), C.byref(na), C.byref(msa)))
        return (na.value, msa.value) if include_noops else (n.value, ms.value)

    def profile_apply_passes(self, prec: str, kernel: int = 0) -> int:
        """Vector passes (distinct vectors read plus vectors written, each over
        the kernel's rows) summed over the launches profile_apply_read counts
        as having done work."""
        v = C.c_int64()
        check(load().dc_profile_apply_passes(self._h, PREC[prec], int(kernel), C.byref(v)))
        return v.value

    def export_recycle(self, opts: Opts, adjoint=False, stream=None):
        k = max(opts.k, 1)
        rows = self.V // 2 if opts.schur else self.V
        U = torch.zeros((k, rows, self.n), dtype=torch.complex128, device="cuda")
        Cm = torch.zeros_like(U)
        kk = C.c_int32()
        o = opts.to_c()
        check(load().dc_export_recycle(self._h, C.byref(o), int(adjoint), _ptr(U), _ptr(Cm),
                                       C.byref(kk), _stream_ptr(stream)))
        return U[:kk.value], Cm[:kk.value]


class CoarseSolve(torch.autograd.Function):
    """x = D_c^{-1} b with gradients for b and the (tied) forward hop blocks.

    backward: lambda = D_c^{-H} g (adjoint solve through Gamma5), grad_b = lambda,
    grad_B[x, mu] = -lambda_x x_{x+mu}^H - Gamma5 x_x lambda_{x+mu}^H Gamma5.
    `hops` must be the tensor the handle `op` was built from.
    """

    @staticmethod
    def forward(ctx, b, hops, op: CoarseOp, opts: Opts, tol: float):
        x, st, rc = op.solve(b.detach(), tol, opts)
        if rc != 0:
            raise DcError(rc, f"forward solve did not converge: {st}")
        ctx.op, ctx.opts, ctx.tol = op, opts, tol
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, g):
        (x,) = ctx.saved_tensors
        lam, st, rc = ctx.op.solve(g.contiguous(), ctx.tol, ctx.opts, adjoint=True)
        if rc != 0:
            raise DcError(rc, f"adjoint solve did not converge: {st}")
        grad_hops = ctx.op.grad_hops(lam, x, tied=True) if ctx.needs_input_grad[1] else None
        return lam, grad_hops, None, None, None


# host-only dense helpers (no device needed)
def multi_tile(prec: str, n: int, n_rhs: int, sites: int) -> int:
    """Right-hand-side tile the multi-apply autotuner chose for a shape (0: not yet)."""
    return int(load().dc_multi_tile(PREC[prec], n, n_rhs, sites))


def set_multi_tile_mode(mode: int):
    """0: autotune (and forget earlier choices); 16 / 32 / 64: force that tile."""
    check(load().dc_set_multi_tile_mode(int(mode)))


def set_reduced_kernels(mode: int):
    """Reduced operator's kernel form (process-wide): 0 the single-read pair
    where it applies (FP32 / FP16 blocks, n a multiple of 8), 1 always the
    two-kernel form; equal results."""
    check(load().dc_set_reduced_kernels(int(mode)))


def set_batch_launches(batched: int):
    """Lockstep batched solves: 1 (default) one launch per Gram-Schmidt pass for
    up to 16 columns and per chain step for up to 8 operators, 0 launches per
    column and per operator; equal results."""
    check(load().dc_set_batch_launches(int(batched)))


def dense_eig(A: np.ndarray, vectors=False):
    lib = load()
    n = A.shape[0]
    a = _colmajor(A)
    w = np.zeros(2 * n)
    Z = np.zeros(2 * n * n) if vectors else None
    check(lib.dc_dense_eig(n, a.ctypes.data_as(C.POINTER(C.c_double)),
                           w.ctypes.data_as(C.POINTER(C.c_double)),
                           Z.ctypes.data_as(C.POINTER(C.c_double)) if vectors else None))
    ev = w[0::2] + 1j * w[1::2]
    if not vectors:
        return ev
    Zc = (Z[0::2] + 1j * Z[1::2]).reshape(n, n).T
    return ev, Zc


def _colmajor(A):
    return np.ascontiguousarray(np.asarray(A, dtype=np.complex128).T).view(np.float64).ravel()


def dense_solve(A: np.ndarray, B: np.ndarray):
    """X with A X = B (host LU with partial pivoting of the library)."""
    lib = load()
    n = A.shape[0]
    B2 = np.asarray(B, dtype=np.complex128).reshape(n, -1)
    a = _colmajor(A)
    b = _colmajor(B2).copy()      # written in place: never the caller's array
    check(lib.dc_dense_solve(n, a.ctypes.data_as(C.POINTER(C.c_double)), B2.shape[1],
                             b.ctypes.data_as(C.POINTER(C.c_double))))
    return (b[0::2] + 1j * b[1::2]).reshape(B2.shape[1], n).T


def dense_lstsq(A: np.ndarray, b: np.ndarray):
    lib = load()
    rows, cols = A.shape
    a = _colmajor(A)
    bb = np.ascontiguousarray(np.asarray(b, dtype=np.complex128)).view(np.float64)
    x = np.zeros(2 * cols)
    rn = C.c_double()
    check(lib.dc_dense_lstsq(rows, cols, a.ctypes.data_as(C.POINTER(C.c_double)),
                             bb.ctypes.data_as(C.POINTER(C.c_double)),
                             x.ctypes.data_as(C.POINTER(C.c_double)), C.byref(rn)))
    return x[0::2] + 1j * x[1::2], rn.value


def harmonic_ritz(Hbar: np.ndarray):
    lib = load()
    d = Hbar.shape[1]
    h = _colmajor(Hbar)
    th = np.zeros(2 * d)
    check(lib.dc_harmonic_ritz(d, h.ctypes.data_as(C.POINTER(C.c_double)),
                               th.ctypes.data_as(C.POINTER(C.c_double))))
    return th[0::2] + 1j * th[1::2]


def leja_order(theta: np.ndarray):
    lib = load()
    t = np.ascontiguousarray(np.asarray(theta, dtype=np.complex128)).view(np.float64)
    out = np.zeros_like(t)
    check(lib.dc_leja_order(len(theta), t.ctypes.data_as(C.POINTER(C.c_double)),
                            out.ctypes.data_as(C.POINTER(C.c_double))))
    return out[0::2] + 1j * out[1::2]
