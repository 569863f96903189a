"""ctypes binding of libhqdwh.so (same names as the C ABI in include/hq.h)."""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "libhqdwh.so")

c_d = ctypes.c_double
c_i32 = ctypes.c_int32
c_i64 = ctypes.c_int64
c_vp = ctypes.c_void_p
P = ctypes.POINTER


class LibraryMissing(RuntimeError):
    pass


class HQError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"hq status {status}: {msg}")
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [("leaf", c_i32), ("tol", c_d), ("delta", c_d), ("max_rank", c_i32), ("max_iter", c_i32),
                ("record_ranks", c_i32), ("predictor", c_vp), ("precision", c_i32), ("c_fp32_max", c_d),
                ("graph", c_i32), ("method", c_i32), ("zolo_r", c_i32)]


class Tuning(ctypes.Structure):
    _fields_ = [("qr_tile_rows", c_i32), ("split_min_k", c_i32), ("split_chunk", c_i32), ("split_max", c_i32),
                ("schur_keep", c_i32), ("gemm_small_tiles", c_i32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


def tuning() -> dict:
    """The tile shapes and thresholds in use (the autotuner's table, or the defaults)."""
    t = Tuning()
    _check(lib().hq_tuning_get(ctypes.byref(t)))
    d = t.as_dict()
    d["source"] = lib().hq_tuning_source().decode()
    return d


def set_tuning(**kw) -> dict:
    """Replace entries of the table for the rest of the process; returns the previous values."""
    t = Tuning()
    _check(lib().hq_tuning_get(ctypes.byref(t)))
    old = t.as_dict()
    for k, v in kw.items():
        if k not in old:
            raise KeyError(k)
        setattr(t, k, int(v))
    _check(lib().hq_tuning_set(ctypes.byref(t)))
    return old


class Info(ctypes.Structure):
    _fields_ = [("iters", c_i32), ("alpha", c_d), ("l0", c_d), ("a", c_d * 16), ("b", c_d * 16), ("c", c_d * 16),
                ("max_rank_iter", c_i32 * 16), ("max_rank", c_i32), ("redo_count", c_i32), ("bytes", c_i64),
                ("peak_bytes", c_i64), ("launches", c_i64), ("seconds", c_d), ("setup_seconds", c_d),
                ("givens_seconds", c_d), ("levels", c_i32), ("level_ranks", c_i32 * (16 * 4 * 24)),
                ("capacity_columns", c_i64), ("fp32_iter", c_i32 * 16), ("graphs", c_i32), ("graph_nodes", c_i64),
                ("graph_build_seconds", c_d), ("zolo_r", c_i32), ("iter_seconds", c_d * 16)]

    def as_dict(self) -> dict:
        K = self.iters
        return {"iters": K, "alpha": self.alpha, "l0": self.l0, "a": list(self.a[:K]), "b": list(self.b[:K]),
                "c": list(self.c[:K]), "max_rank_iter": list(self.max_rank_iter[:K]), "max_rank": self.max_rank,
                "redo_count": self.redo_count, "bytes": self.bytes, "peak_bytes": self.peak_bytes,
                "launches": self.launches, "seconds": self.seconds, "setup_seconds": self.setup_seconds,
                "givens_seconds": self.givens_seconds, "levels": self.levels,
                "capacity_columns": self.capacity_columns, "fp32_iter": list(self.fp32_iter[:K]),
                "graphs": self.graphs, "graph_nodes": self.graph_nodes,
                "graph_build_seconds": self.graph_build_seconds, "zolo_r": self.zolo_r,
                "iter_seconds": list(self.iter_seconds[:K])}

    def level_ranks_array(self) -> np.ndarray:
        """[k][o][l]: o = 0 X_{k+1}, 1 Z_k, 2 L_k^{-1}, 3 Y_k (filled with opts record_ranks)."""
        return np.ctypeslib.as_array(self.level_ranks).reshape(16, 4, 24)[: self.iters, :, : self.levels].copy()


def iteration_records(info: dict, **tags) -> list:
    """One record per iteration (Zolo-pd: per step) of a solve's info, for a JSON-lines log: k, the
    weights (a, b, c), whether it ran in FP32, the largest off-diagonal rank of X_{k+1}, its wall time,
    plus the given tags."""
    out = []
    for k in range(info["iters"]):
        rec = dict(tags)
        rec.update({"k": k, "a": info["a"][k], "b": info["b"][k], "c": info["c"][k],
                    "fp32": bool(info["fp32_iter"][k]), "max_rank": info["max_rank_iter"][k],
                    "seconds": info["iter_seconds"][k]})
        out.append(rec)
    return out


_lib = None

_SIGS = {
    "hq_default_opts": (c_i32, [P(Opts)]),
    "hodlr_build": (c_i32, [c_vp, c_i64, c_i32, c_i64, c_d, c_d, P(Opts), c_vp, P(c_vp)]),
    "hodlr_cholesky_solve": (c_i32, [c_vp, c_vp, c_i64, c_i32, c_vp, c_i64, c_d, c_i32, c_i32, c_vp, P(c_d)]),
    "qdwh_sign": (c_i32, [c_vp, c_i64, c_i32, c_i64, c_d, P(Opts), c_vp, P(c_vp), P(Info)]),
    "spectral_projector": (c_i32, [c_vp, c_i64, c_i32, c_i64, c_d, P(Opts), c_vp, P(c_vp), P(Info)]),
    "spectral_projector_batched": (c_i32, [c_i32, P(c_vp), P(c_i64), P(c_i32), P(c_i64), P(c_d), P(Opts), c_vp,
                                           P(c_vp), P(Info)]),
    "apply_projector": (c_i32, [c_vp, c_vp, c_i64, c_i32, c_vp, c_i64, c_vp]),
    "apply_projector_noalloc": (c_i32, [c_vp, c_vp, c_i64, c_i32, c_vp, c_i64, c_vp]),
    "apply_projector_noalloc_max_bytes": (ctypes.c_size_t, []),
    "hq_tuning_get": (c_i32, [c_vp]),
    "hq_tuning_set": (c_i32, [c_vp]),
    "hq_tuning_source": (ctypes.c_char_p, []),
    "hodlr_to_dense": (c_i32, [c_vp, c_vp, c_i64, c_vp]),
    "hodlr_shape": (c_i32, [c_vp, P(c_i64), P(c_i32), P(c_i32), P(c_i32)]),
    "hodlr_get_leaf": (c_i32, [c_vp, c_i32, c_vp, c_i64, P(c_i64), P(c_i64)]),
    "hodlr_get_block": (c_i32, [c_vp, c_i32, c_i32, c_vp, c_vp, c_i64, P(c_i32), P(c_i64), P(c_i64), P(c_i64)]),
    "hq_shift_for_count": (c_i32, [c_vp, c_i64, c_i32, c_i64, c_i64, P(c_d), P(c_d)]),
    "hodlr_destroy": (None, [c_vp]),
    "hodlr_to_hmatrix": (c_i32, [c_vp, c_d, c_vp, P(c_vp)]),
    "hmatrix_shape": (c_i32, [c_vp, P(c_i64), P(c_i64), P(c_i64), P(c_i64), P(c_i64), P(c_i32)]),
    "hmatrix_get_block": (c_i32, [c_vp, c_i64, P(c_i64), P(c_i64), P(c_i64), P(c_i64), P(c_i32), c_vp, c_vp, c_i64]),
    "hmatrix_destroy": (None, [c_vp]),
    "hq_status_string": (ctypes.c_char_p, [c_i32]),
    "hq_last_error": (ctypes.c_char_p, []),
    "hq_test_gemm": (c_i32, [c_vp, c_vp, c_vp, c_i32, c_i32, c_i32, c_i32, c_i32, c_i32, c_i32, c_i32, c_d, c_d, c_i32,
                             c_vp]),
    "hq_test_qr_r": (c_i32, [c_vp, c_i32, c_i32, c_i32, c_vp, c_i32, c_vp]),
    "hq_test_recompress": (c_i32, [c_vp, c_i32, c_vp, c_i32, c_i32, c_d, c_i32, c_vp, c_vp, P(c_i32), c_i32, c_vp]),
    "hq_test_from_dense": (c_i32, [c_vp, c_i64, c_i64, P(Opts), c_i32, c_vp, P(c_vp)]),
    "hq_test_product": (c_i32, [c_vp, c_i32, c_vp, c_i32, c_d, c_vp, c_i32, c_d, c_i32, c_i32, c_d, c_vp, P(c_vp)]),
    "hq_test_cholesky_inverse": (c_i32, [c_vp, c_i32, c_d, c_vp, P(c_vp)]),
    "hq_test_q_factors": (c_i32, [c_vp, c_i64, c_i32, c_i64, c_d, c_d, c_i32, c_vp, P(c_vp), P(c_vp), P(c_i64)]),
    "hq_test_q_dense_host": (c_i32, [c_vp, c_i64, c_i32, c_i64, c_d, c_d, c_i32, c_vp, c_vp, P(c_i64)]),
    "hq_test_schedule": (c_i32, [c_d, c_d, c_i32, c_vp, c_vp, c_vp, c_vp, P(c_i32)]),
    "hq_test_zolo": (c_i32, [c_d, c_i32, c_vp, c_vp, P(c_d), P(c_d)]),
    "hq_profile_enable": (c_i32, [c_i32]),
    "hq_profile_select": (c_i32, [c_i32]),
    "hq_profile_read": (c_i32, [c_vp, c_i32]),
    "hq_profile_svd": (c_i32, [c_vp]),
    "hq_profile_mfma": (c_i32, [c_vp, c_i32]),
    "hq_predictor_create": (c_i32, [ctypes.c_uint64, P(c_vp)]),
    "hq_predictor_nparams": (c_i64, []),
    "hq_predictor_get_params": (c_i32, [c_vp, c_vp]),
    "hq_predictor_set_params": (c_i32, [c_vp, c_vp]),
    "hq_predictor_forward": (c_i32, [c_vp, c_vp, c_i64, c_vp, c_vp]),
    "hq_predictor_set_margin": (c_i32, [c_vp, c_vp]),
    "hq_predictor_get_margin": (c_i32, [c_vp, c_vp]),
    "hq_predictor_loss_grad": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_i64, P(ctypes.c_float), c_vp, c_vp]),
    "hq_predictor_train": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_i64, c_i32, ctypes.c_float, c_vp,
                                   P(ctypes.c_float)]),
    "hq_predictor_rows": (c_i32, [P(Info), c_i64, c_i32, P(Opts), c_vp, c_vp, c_vp, P(c_i32)]),
    "hq_predictor_destroy": (None, [c_vp]),
}

KCLASSES = ("gemm", "tsqr", "core_svd", "leaf_cholesky", "leaf_inverse", "stack", "leaf_elementwise", "other")


class KStat(ctypes.Structure):
    _fields_ = [("launches", c_i64), ("ms", c_d), ("flops", c_d), ("bytes", c_d)]


def profile(on: bool, classes=None):
    """Enable/disable the library's kernel timers (and clear them when enabling); `classes` (names
    from KCLASSES) restricts the timers to those kernel classes, None times all of them."""
    if on:
        profile_read(reset=True)
        profile_mfma(reset=True)
        mask = -1 if classes is None else sum(1 << KCLASSES.index(c) for c in classes)
        _check(lib().hq_profile_select(mask))
    _check(lib().hq_profile_enable(1 if on else 0))


def profile_svd() -> dict:
    a = (c_i64 * 8)()
    _check(lib().hq_profile_svd(ctypes.cast(a, c_vp)))
    n = max(a[6], 1)
    return {"cores": a[6], "qr_us": a[0] / 100.0, "jacobi_us": a[1] / 100.0, "out_us": a[2] / 100.0,
            "mean_r": a[3] / n, "mean_t": a[4] / n, "mean_sweeps": a[5] / n}


def profile_mfma(reset: bool = True) -> dict:
    """Flops issued to the matrix cores since the last reset (FP64, FP32)."""
    a = (c_d * 2)()
    _check(lib().hq_profile_mfma(ctypes.cast(a, c_vp), 1 if reset else 0))
    return {"fp64": a[0], "fp32": a[1]}


def profile_read(reset: bool = True) -> dict:
    arr = (KStat * 8)()
    _check(lib().hq_profile_read(ctypes.cast(arr, c_vp), 1 if reset else 0))
    return {KCLASSES[i]: {"launches": arr[i].launches, "ms": arr[i].ms, "flops": arr[i].flops,
                          "bytes": arr[i].bytes} for i in range(8)}

EXPORTED = tuple(_SIGS)


def lib():
    """Load libhqdwh.so; raise LibraryMissing if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise LibraryMissing(f"{LIBPATH} not found: run __graft_entry__.build() or "
                                 "python paper_1608_01164_amd/build.py")
        # PyTorch wheels carry their own HIP runtime.  Importing torch first makes the library bind to
        # that same runtime (one runtime per process), so that torch's device pointers and streams are
        # valid in the library whichever side touches the device first.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIBPATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status: int):
    if status != 0:
        L = lib()
        raise HQError(status, f"{L.hq_status_string(status).decode()}: {L.hq_last_error().decode()}")


def _opts(leaf=256, tol=1e-10, delta=1e-15, max_rank=512, max_iter=10, record_ranks=False, predictor=None,
          precision="fp64", c_fp32_max=16.0, graph=False, method="qdwh", zolo_r=0) -> Opts:
    o = Opts()
    _check(lib().hq_default_opts(ctypes.byref(o)))
    o.leaf, o.tol, o.delta, o.max_rank, o.max_iter = int(leaf), float(tol), float(delta), int(max_rank), int(max_iter)
    o.record_ranks = 1 if record_ranks else 0
    o.predictor = predictor._h if predictor is not None else None
    if precision not in ("fp64", "mixed"):
        raise ValueError("precision must be 'fp64' or 'mixed'")
    o.precision = 1 if precision == "mixed" else 0
    o.c_fp32_max = float(c_fp32_max)
    o.graph = 1 if graph else 0
    if method not in ("qdwh", "zolo"):
        raise ValueError("method must be 'qdwh' or 'zolo'")
    o.method = 1 if method == "zolo" else 0
    o.zolo_r = int(zolo_r)
    return o


def _stream(stream):
    if stream is None:
        import torch
        return c_vp(torch.cuda.current_stream().cuda_stream)
    return c_vp(int(stream))


def _dev_f64(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError(f"{name} must be a float64 CUDA/HIP tensor")
    return t


def _band_args(band):
    band = _dev_f64(band, "band")
    if band.dim() != 2 or not band.is_contiguous():
        raise ValueError("band must be a contiguous (n, ld) tensor in lower band storage")
    n, ld = band.shape
    return c_vp(band.data_ptr()), n, ld


class HODLR:
    """A HODLR matrix owned by the library (handle)."""

    def __init__(self, handle: c_vp):
        self._h = handle
        n = c_i64()
        lv = c_i32()
        nl = c_i32()
        _check(lib().hodlr_shape(self._h, ctypes.byref(n), ctypes.byref(lv), ctypes.byref(nl), None))
        self.n, self.levels, self.nleaves = n.value, lv.value, nl.value

    @property
    def handle(self):
        return self._h

    def max_rank(self) -> int:
        r = c_i32()
        _check(lib().hodlr_shape(self._h, None, None, None, ctypes.byref(r)))
        return r.value

    def apply(self, X, out=None, stream=None):
        """Y = H X for a device tensor X of shape (n,) or (n, k) (float64)."""
        import torch
        X = _dev_f64(X, "X")
        vec = X.dim() == 1
        Xm = X.reshape(self.n, -1)
        # column-major n x k view: use the transpose of a contiguous (k, n) tensor
        Xc = Xm.t().contiguous()
        Y = torch.empty_like(Xc) if out is None else out
        k = Xc.shape[0]
        _check(lib().apply_projector(self._h, c_vp(Xc.data_ptr()), self.n, k, c_vp(Y.data_ptr()), self.n,
                                     _stream(stream)))
        Y = Y.t()
        return Y.reshape(self.n) if vec else Y

    def apply_noalloc(self, Xt, Yt, stream=None):
        """Y = H X through apply_projector_noalloc, which allocates nothing.  Xt, Yt: contiguous (k, n)
        float64 device tensors holding X and Y column-major (row j of Xt is column j of X)."""
        _dev_f64(Xt, "Xt")
        _dev_f64(Yt, "Yt")
        if Xt.dim() != 2 or Xt.shape[1] != self.n or tuple(Yt.shape) != tuple(Xt.shape) or \
                not (Xt.is_contiguous() and Yt.is_contiguous()):
            raise ValueError("Xt and Yt must be contiguous (k, n) tensors")
        _check(lib().apply_projector_noalloc(self._h, c_vp(Xt.data_ptr()), self.n, Xt.shape[0], c_vp(Yt.data_ptr()),
                                             self.n, _stream(stream)))
        return Yt

    def to_dense(self, stream=None):
        import torch
        out = torch.empty((self.n, self.n), dtype=torch.float64, device="cuda")
        _check(lib().hodlr_to_dense(self._h, c_vp(out.data_ptr()), self.n, _stream(stream)))
        return out.t()  # column-major buffer -> row-major view

    def export(self) -> dict:
        """Host copy in the oracle's plain format {n, leaves, blocks}."""
        L = lib()
        leaves, blocks = [], []
        for i in range(self.nleaves):
            lo, m = c_i64(), c_i64()
            _check(L.hodlr_get_leaf(self._h, i, None, 0, ctypes.byref(lo), ctypes.byref(m)))
            buf = np.zeros((m.value, m.value))  # column-major fill through the transpose
            bt = np.zeros((m.value, m.value), order="F")
            _check(L.hodlr_get_leaf(self._h, i, bt.ctypes.data_as(c_vp), m.value, None, None))
            buf[:] = bt
            leaves.append((lo.value, lo.value + m.value, buf))
        nint = (1 << self.levels) - 1
        for p in range(nint):
            fac = []
            for s in (0, 1):
                r, lo, mid, hi = c_i32(), c_i64(), c_i64(), c_i64()
                _check(L.hodlr_get_block(self._h, p, s, None, None, 0, ctypes.byref(r), ctypes.byref(lo),
                                         ctypes.byref(mid), ctypes.byref(hi)))
                ld = max(mid.value - lo.value, hi.value - mid.value)
                U = np.zeros((ld, max(r.value, 1)), order="F")
                V = np.zeros((ld, max(r.value, 1)), order="F")
                _check(L.hodlr_get_block(self._h, p, s, U.ctypes.data_as(c_vp), V.ctypes.data_as(c_vp), ld,
                                         ctypes.byref(r), None, None, None))
                ma, mb = mid.value - lo.value, hi.value - mid.value
                ru, rv = (ma, mb) if s == 0 else (mb, ma)
                fac += [np.ascontiguousarray(U[:ru, : r.value]), np.ascontiguousarray(V[:rv, : r.value])]
            blocks.append((lo.value, mid.value, hi.value, *fac))
        return {"n": self.n, "leaves": leaves, "blocks": blocks}

    def close(self):
        if self._h is not None and self._h.value:
            lib().hodlr_destroy(self._h)
        self._h = c_vp(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class HMatrix:
    """An H-matrix made from a HODLR matrix (standard admissibility, Sec. 3.1.2); see hq.h."""

    def __init__(self, handle: c_vp, source):
        self._h = handle
        self._src = source  # keeps the HODLR matrix whose diagonal blocks it shares alive

    def shape(self) -> dict:
        n, nlr, nd, by, hb = (c_i64() for _ in range(5))
        mr = c_i32()
        _check(lib().hmatrix_shape(self._h, ctypes.byref(n), ctypes.byref(nlr), ctypes.byref(nd), ctypes.byref(by),
                                   ctypes.byref(hb), ctypes.byref(mr)))
        return {"n": n.value, "low_rank_blocks": nlr.value, "dense_blocks": nd.value, "bytes": by.value,
                "hodlr_bytes": hb.value, "max_rank": mr.value}

    def blocks(self):
        """[(row0, col0, U, V)] for low-rank blocks and [(row0, col0, D)] for dense ones (host arrays)."""
        sh = self.shape()
        r0, c0, m, nc = (c_i64() for _ in range(4))
        rk = c_i32()
        lr, dn = [], []
        for i in range(sh["low_rank_blocks"] + sh["dense_blocks"]):
            args = (ctypes.byref(r0), ctypes.byref(c0), ctypes.byref(m), ctypes.byref(nc), ctypes.byref(rk))
            _check(lib().hmatrix_get_block(self._h, i, *args, None, None, 0))  # sizes
            ld = max(m.value, nc.value, 1)
            if rk.value >= 0:
                k = rk.value
                U = np.zeros((ld, max(k, 1)), order="F")
                V = np.zeros((ld, max(k, 1)), order="F")
                _check(lib().hmatrix_get_block(self._h, i, *args, U.ctypes.data_as(c_vp), V.ctypes.data_as(c_vp), ld))
                lr.append((r0.value, c0.value, U[: m.value, :k].copy(), V[: nc.value, :k].copy()))
            else:
                D = np.zeros((ld, ld), order="F")
                _check(lib().hmatrix_get_block(self._h, i, *args, D.ctypes.data_as(c_vp), None, ld))
                dn.append((r0.value, c0.value, D[: m.value, : nc.value].copy()))
        return lr, dn

    def close(self):
        if self._h:
            lib().hmatrix_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hodlr_to_hmatrix(P, tol: float = 1e-10, stream=None) -> HMatrix:
    h = c_vp()
    _check(lib().hodlr_to_hmatrix(P.handle, float(tol), _stream(stream), ctypes.byref(h)))
    return HMatrix(h, P)


def hodlr_build(band, b: int, shift: float, scale: float, leaf: int = 256, stream=None) -> HODLR:
    p, n, ld = _band_args(band)
    h = c_vp()
    _check(lib().hodlr_build(p, n, int(b), ld, float(shift), float(scale), ctypes.byref(_opts(leaf=leaf)),
                             _stream(stream), ctypes.byref(h)))
    return HODLR(h)


def cholesky_solve(H, B, X, tol: float = 1e-12, cap: int = 0, method: str = "substitution", stream=None):
    """X = H^{-1} B for a symmetric positive definite HODLR handle H (device tensors, B and X of shape
    (ncols, n) row-major = n x ncols column-major).  method "substitution": HODLR triangular solves with
    the H-Cholesky factor; "inverse": products with the L^{-1} it forms.  Returns the seconds of the
    factorisation and of the solve."""
    m = {"substitution": 0, "inverse": 1}[method]
    ncols, n = B.shape
    sec = (c_d * 2)()
    _check(lib().hodlr_cholesky_solve(H.handle, c_vp(B.data_ptr()), n, ncols, c_vp(X.data_ptr()), X.shape[1],
                                      float(tol), int(cap), m, _stream(stream), sec))
    return sec[0], sec[1]


def _solve(fn, band, b, mu, stream, raw_info=False, **kw):
    p, n, ld = _band_args(band)
    h = c_vp()
    info = Info()
    _check(getattr(lib(), fn)(p, n, int(b), ld, float(mu), ctypes.byref(_opts(**kw)), _stream(stream),
                              ctypes.byref(h), ctypes.byref(info)))
    return HODLR(h), (info if raw_info else info.as_dict())


def spectral_projector(band, b: int, mu: float, stream=None, **opts):
    """(P, info): P ~ Pi_{<mu}(A) in HODLR format.  opts: leaf, tol, delta, max_rank, max_iter."""
    return _solve("spectral_projector", band, b, mu, stream, **opts)


def spectral_projector_batched(bands, bs, mus, stream=None, **opts):
    """([P_i], [info_i], status) for independent problems advanced together (one launch per step
    for all members).  bands: device band tensors.  A failed member gives None and its status is
    returned (the first failure); the call raises only for argument errors."""
    cnt = len(bands)
    ptrs = (c_vp * cnt)()
    ns = (c_i64 * cnt)()
    lds = (c_i64 * cnt)()
    bb = (c_i32 * cnt)(*[int(x) for x in bs])
    mm = (c_d * cnt)(*[float(x) for x in mus])
    for i, band in enumerate(bands):
        p, n, ld = _band_args(band)
        ptrs[i] = p.value
        ns[i] = n
        lds[i] = ld
    hs = (c_vp * cnt)()
    infos = (Info * cnt)()
    st = lib().spectral_projector_batched(cnt, ptrs, ns, bb, lds, mm, ctypes.byref(_opts(**opts)), _stream(stream),
                                          hs, infos)
    if st < 0:
        _check(st)
    return [HODLR(c_vp(h)) if h else None for h in hs], [i.as_dict() for i in infos], st


def qdwh_sign(band, b: int, mu: float, stream=None, **opts):
    return _solve("qdwh_sign", band, b, mu, stream, **opts)


def shift_for_count(band_host: np.ndarray, b: int, nu: int):
    """(mu, gap) with mu the midpoint of lambda_nu and lambda_{nu+1} (library's own inertia bisection)."""
    ab = np.ascontiguousarray(band_host, dtype=np.float64)
    n, ld = ab.shape
    mu, gap = c_d(), c_d()
    _check(lib().hq_shift_for_count(ab.ctypes.data_as(c_vp), n, int(b), ld, int(nu), ctypes.byref(mu),
                                    ctypes.byref(gap)))
    return mu.value, gap.value


# ---- test hooks ---------------------------------------------------------------------------------
def test_gemm(A, B, C, m, n, k, lda, ldb, ldc, opA, opB, alpha, beta, stream=None, fp32=False):
    _check(lib().hq_test_gemm(c_vp(A.data_ptr()), c_vp(B.data_ptr()), c_vp(C.data_ptr()), m, n, k, lda, ldb, ldc,
                              opA, opB, alpha, beta, 1 if fp32 else 0, _stream(stream)))


def test_qr_r(M, rows, r, ldm, R, stream=None, fp32=False):
    _check(lib().hq_test_qr_r(c_vp(M.data_ptr()), rows, r, ldm, c_vp(R.data_ptr()), 1 if fp32 else 0,
                              _stream(stream)))


def test_recompress(Us, m, Vs, n, r, tol, kcap, U, V, stream=None, fp32=False) -> int:
    k = c_i32()
    _check(lib().hq_test_recompress(c_vp(Us.data_ptr()), m, c_vp(Vs.data_ptr()), n, r, tol, kcap,
                                    c_vp(U.data_ptr()), c_vp(V.data_ptr()), ctypes.byref(k), 1 if fp32 else 0,
                                    _stream(stream)))
    return k.value


def test_from_dense(dense_colmajor, n, leaf, tol, cap, stream=None) -> HODLR:
    h = c_vp()
    _check(lib().hq_test_from_dense(c_vp(dense_colmajor.data_ptr()), n, n, ctypes.byref(_opts(leaf=leaf, tol=tol)),
                                    cap, _stream(stream), ctypes.byref(h)))
    return HODLR(h)


def test_product(A: HODLR, tA, B: HODLR, tB, alpha, D: HODLR | None, d_identity, delta, lower_only, cap, tol,
                 stream=None) -> HODLR:
    h = c_vp()
    _check(lib().hq_test_product(A.handle, tA, B.handle, tB, alpha, D.handle if D else None, d_identity, delta,
                                 lower_only, cap, tol, _stream(stream), ctypes.byref(h)))
    return HODLR(h)


def test_cholesky_inverse(Z: HODLR, cap, tol, stream=None) -> HODLR:
    h = c_vp()
    _check(lib().hq_test_cholesky_inverse(Z.handle, cap, tol, _stream(stream), ctypes.byref(h)))
    return HODLR(h)


def test_q_factors(band_host: np.ndarray, b, shift, scale, leaf, stream=None):
    ab = np.ascontiguousarray(band_host, dtype=np.float64)
    n, ld = ab.shape
    h1, h2, nr = c_vp(), c_vp(), c_i64()
    _check(lib().hq_test_q_factors(ab.ctypes.data_as(c_vp), n, b, ld, shift, scale, leaf, _stream(stream),
                                   ctypes.byref(h1), ctypes.byref(h2), ctypes.byref(nr)))
    return HODLR(h1), HODLR(h2), nr.value


def test_q_dense_host(band_host: np.ndarray, b, shift, scale, leaf):
    ab = np.ascontiguousarray(band_host, dtype=np.float64)
    n, ld = ab.shape
    Q1 = np.zeros((n, n), order="F")
    Q2 = np.zeros((n, n), order="F")
    nr = c_i64()
    _check(lib().hq_test_q_dense_host(ab.ctypes.data_as(c_vp), n, b, ld, shift, scale, leaf,
                                      Q1.ctypes.data_as(c_vp), Q2.ctypes.data_as(c_vp), ctypes.byref(nr)))
    return Q1, Q2, nr.value


def test_schedule(l0: float, delta: float = 1e-15, max_iter: int = 16):
    """The library's weight schedule (host only): arrays a, b, c (K entries) and l (K + 1 entries)."""
    a, b, c, l = (np.zeros(17) for _ in range(4))
    K = c_i32()
    _check(lib().hq_test_schedule(l0, delta, max_iter, a.ctypes.data_as(c_vp), b.ctypes.data_as(c_vp),
                                  c.ctypes.data_as(c_vp), l.ctypes.data_as(c_vp), ctypes.byref(K)))
    k = K.value
    return a[:k].copy(), b[:k].copy(), c[:k].copy(), l[: k + 1].copy()


def test_zolo(l: float, r: int):
    """The library's Zolo-pd coefficients of one step (host only): c (2r + 1 entries, c[0] = 0),
    a (r + 1 entries, a[0] = 0), mhat, l_next."""
    c, a = np.zeros(2 * r + 1), np.zeros(r + 1)
    m, ln = c_d(), c_d()
    _check(lib().hq_test_zolo(float(l), int(r), c.ctypes.data_as(c_vp), a.ctypes.data_as(c_vp), ctypes.byref(m),
                              ctypes.byref(ln)))
    return c, a, m.value, ln.value


# ---- rank predictor --------------------------------------------------------------------------
NFEAT, NOUT = 10, 4


class Predictor:
    """The library's rank predictor network (device parameters); see hq.h."""

    def __init__(self, seed: int = 0):
        self._h = c_vp()
        _check(lib().hq_predictor_create(ctypes.c_uint64(seed), ctypes.byref(self._h)))

    @staticmethod
    def nparams() -> int:
        return int(lib().hq_predictor_nparams())

    def params(self) -> np.ndarray:
        out = np.zeros(self.nparams(), dtype=np.float32)
        _check(lib().hq_predictor_get_params(self._h, out.ctypes.data_as(c_vp)))
        return out

    def set_params(self, p) -> None:
        p = np.ascontiguousarray(p, dtype=np.float32)
        if p.size != self.nparams():
            raise ValueError("wrong number of parameters")
        _check(lib().hq_predictor_set_params(self._h, p.ctypes.data_as(c_vp)))

    def margin(self) -> np.ndarray:
        out = np.zeros(NOUT, dtype=np.float32)
        _check(lib().hq_predictor_get_margin(self._h, out.ctypes.data_as(c_vp)))
        return out

    def set_margin(self, m) -> None:
        m = np.ascontiguousarray(m, dtype=np.float32)
        _check(lib().hq_predictor_set_margin(self._h, m.ctypes.data_as(c_vp)))

    def forward(self, X, Y, stream=None) -> None:
        """Y (rows x 4) = net(X (rows x 10)); device float32 tensors."""
        _check(lib().hq_predictor_forward(self._h, c_vp(X.data_ptr()), X.shape[0], c_vp(Y.data_ptr()),
                                          _stream(stream)))

    def loss_grad(self, X, T, W, grad, stream=None) -> float:
        loss = ctypes.c_float()
        _check(lib().hq_predictor_loss_grad(self._h, c_vp(X.data_ptr()), c_vp(T.data_ptr()), c_vp(W.data_ptr()),
                                            X.shape[0], ctypes.byref(loss), c_vp(grad.data_ptr()), _stream(stream)))
        return loss.value

    def train(self, X, T, W, epochs: int, lr: float, stream=None) -> float:
        loss = ctypes.c_float()
        _check(lib().hq_predictor_train(self._h, c_vp(X.data_ptr()), c_vp(T.data_ptr()), c_vp(W.data_ptr()),
                                        X.shape[0], int(epochs), ctypes.c_float(lr), _stream(stream),
                                        ctypes.byref(loss)))
        return loss.value

    def close(self):
        if self._h is not None and self._h.value:
            lib().hq_predictor_destroy(self._h)
        self._h = c_vp(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def predictor_rows(info: Info, n: int, b: int, **opts):
    """(X, T, W) float32 host arrays: training rows of one solve run with record_ranks=True."""
    cap = 16 * 24
    X = np.zeros((cap, NFEAT), dtype=np.float32)
    T = np.zeros((cap, NOUT), dtype=np.float32)
    W = np.zeros((cap, NOUT), dtype=np.float32)
    rows = c_i32()
    _check(lib().hq_predictor_rows(ctypes.byref(info), int(n), int(b), ctypes.byref(_opts(**opts)),
                                   X.ctypes.data_as(c_vp), T.ctypes.data_as(c_vp), W.ctypes.data_as(c_vp),
                                   ctypes.byref(rows)))
    r = rows.value
    return X[:r], T[:r], W[:r]
