"""Python binding of the C ABI in include/hh.h (ctypes).

Argument marshalling only: every step of the build and of the products runs in
the native library. PyTorch provides device memory and the current stream. The
library must be built (``paper_2604_09147_amd/build_lib.py``); importing works
without it, but any call raises if ``lib/libhhmat.so`` is missing."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libhhmat.so")

HH_OK, HH_EINVAL, HH_ENOMEM, HH_EHIP, HH_ENOTSUP, HH_EINTERNAL = range(6)
LOG, INV_R, INV_R2, GAUSS, MATERN, DOUBLE_LAYER = 1, 2, 3, 4, 5, 6
FMT_FP64, FMT_FP32, FMT_FP16, FMT_BF16, FMT_CONT, FMT_Q43 = 0, 1, 2, 3, 4, 5
IO_F64, IO_F32 = 0, 1
BLK_FAR, BLK_NEAR, BLK_WEAK, BLK_DIAG, BLK_DENSE_NEAR = range(5)

# Exported functions, in the order include/hh.h declares them.
EXPORTS = ["hh_build", "hh_derive", "hh_switch_level_search", "hh_matvec", "hh_matvec_t",
           "hh_matvec_timed", "hh_matvec_batch", "hh_matvec_noalloc", "hh_solve", "hh_autotune",
           "hh_reserve",
           "hh_get_stats", "hh_block_count", "hh_get_block", "hh_get_block_factors",
           "hh_get_perm", "hh_io_dtype", "hh_size", "hh_free", "hh_plan_create", "hh_plan_info",
           "hh_plan_blocks", "hh_plan_perm", "hh_plan_free", "hh_quantize", "hh_quantize_cont",
           "hh_last_error"]


class HHError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"hh status {status}: {msg}")
        self.status = status


class Kernel(C.Structure):
    _fields_ = [("type", C.c_int), ("scale", C.c_double), ("h", C.c_double),
                ("normals", C.POINTER(C.c_double))]


class Options(C.Structure):
    _fields_ = [("precision_mask", C.c_uint32), ("uniform_fp64", C.c_int), ("io_dtype", C.c_int),
                ("seed", C.c_uint64), ("continuum", C.c_int), ("unit_bytes", C.c_int64),
                ("dot_task_elems", C.c_int64)]


class Stats(C.Structure):
    _fields_ = [("n", C.c_int32), ("d", C.c_int32), ("L", C.c_int32), ("ell", C.c_int32),
                ("leaf_size", C.c_int32), ("max_rank", C.c_int32),
                ("n_blocks_lowrank", C.c_int64), ("n_blocks_rank0", C.c_int64),
                ("n_blocks_dense", C.c_int64), ("blocks_by_format", C.c_int64 * 6),
                ("factor_bytes_by_format", C.c_int64 * 6), ("dense_bytes", C.c_int64),
                ("lowrank_entries", C.c_int64), ("dense_entries", C.c_int64),
                ("total_columns", C.c_int64), ("storage_words", C.c_double),
                ("storage_words_fp64", C.c_double), ("matvec_bytes", C.c_double),
                ("norm2_total", C.c_double), ("build_seconds", C.c_double),
                ("phase_bytes", C.c_double * 3)]

    def to_dict(self) -> dict:
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if isinstance(v, C.Array) else v
        return out


class Tuning(C.Structure):
    _fields_ = [("unit_bytes", C.c_int64), ("dot_task_elems", C.c_int64), ("ms", C.c_double)]


class BlockInfo(C.Structure):
    _fields_ = [("level", C.c_int32), ("kind", C.c_int32), ("rank", C.c_int32),
                ("format", C.c_int32), ("box_i", C.c_int64), ("box_j", C.c_int64),
                ("row_begin", C.c_int64), ("row_end", C.c_int64), ("col_begin", C.c_int64),
                ("col_end", C.c_int64), ("exp_u", C.c_int32), ("exp_v", C.c_int32),
                ("lowrank", C.c_int32), ("frac_bits", C.c_int32), ("norm2", C.c_double),
                ("entry_norm2", C.c_double),
                ("tail_prev", C.c_double), ("tail", C.c_double)]


_lib = None
_P = C.c_void_p
_I64P = C.POINTER(C.c_int64)
_I32P = C.POINTER(C.c_int32)
_DP = C.POINTER(C.c_double)


def lib() -> C.CDLL:
    """The loaded native library (raises when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2604_09147_amd/build_lib.py "
                           "(or __graft_entry__.build()); there is no fallback path")
    L = C.CDLL(LIB_PATH)
    sig = {
        "hh_build": ([_DP, C.c_int64, C.c_int, C.POINTER(Kernel), C.c_double, C.c_double, C.c_int,
                      C.c_int, C.POINTER(Options), C.POINTER(_P)], C.c_int),
        "hh_derive": ([_P, C.POINTER(Options), C.POINTER(_P)], C.c_int),
        "hh_switch_level_search": ([_DP, C.c_int64, C.c_int, C.POINTER(Kernel), C.c_double,
                                    C.c_double, C.c_int, C.POINTER(Options), _I32P, _DP, _DP,
                                    C.c_int32], C.c_int),
        "hh_matvec": ([_P, _P, _P, C.c_int64, _P], C.c_int),
        "hh_matvec_t": ([_P, _P, _P, C.c_int64, _P], C.c_int),
        "hh_matvec_timed": ([_P, _P, _P, C.c_int64, _P, C.c_int, _DP], C.c_int),
        "hh_matvec_batch": ([C.POINTER(_P), C.c_int, C.POINTER(_P), C.POINTER(_P), C.c_int64, _P],
                            C.c_int),
        "hh_matvec_noalloc": ([_P, _P, _P, C.c_int64, C.c_int, _P], C.c_int),
        "hh_solve": ([_P, _P, _P, C.c_double, C.c_double, C.c_int, C.c_int, C.c_int, _I32P, _DP, _P],
                     C.c_int),
        "hh_autotune": ([_P, _P, C.POINTER(Tuning), C.POINTER(Tuning), C.c_int32, _I32P], C.c_int),
        "hh_reserve": ([_P, C.c_int64], C.c_int),
        "hh_get_stats": ([_P, C.POINTER(Stats)], C.c_int),
        "hh_block_count": ([_P, _I64P], C.c_int),
        "hh_get_block": ([_P, C.c_int64, C.POINTER(BlockInfo)], C.c_int),
        "hh_get_block_factors": ([_P, C.c_int64, _DP, _DP], C.c_int),
        "hh_get_perm": ([_P, _I64P], C.c_int),
        "hh_io_dtype": ([_P], C.c_int),
        "hh_size": ([_P], C.c_int64),
        "hh_free": ([_P], None),
        "hh_plan_create": ([_DP, C.c_int64, C.c_int, C.c_double, C.c_int, C.c_int, C.POINTER(_P)],
                           C.c_int),
        "hh_plan_info": ([_P, _I32P, _I32P, _I64P], C.c_int),
        "hh_plan_blocks": ([_P, _I32P, _I32P, _I64P, _I64P, _I64P, _I64P, _I64P, _I64P], C.c_int),
        "hh_plan_perm": ([_P, _I64P], C.c_int),
        "hh_plan_free": ([_P], None),
        "hh_quantize": ([_DP, C.c_int64, C.c_int, C.c_int, _DP], C.c_int),
        "hh_quantize_cont": ([_DP, C.c_int64, C.c_int, _DP], C.c_int),
        "hh_last_error": ([], C.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(status: int) -> None:
    if status != HH_OK:
        msg = lib().hh_last_error().decode(errors="replace")
        raise HHError(status, msg)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_DP)


def _iptr(a: np.ndarray):
    return a.ctypes.data_as(_I64P)


# ----------------------------------------------------------------- host plan
def plan(points, eta: float, switch_level: int, leaf_size: int) -> dict:
    """Tree and block partition computed by the library on the host."""
    pts = np.ascontiguousarray(points, dtype=np.float64)
    n, d = pts.shape
    h = _P()
    _check(lib().hh_plan_create(_dptr(pts), n, d, eta, switch_level, leaf_size, C.byref(h)))
    try:
        L = C.c_int32()
        ell = C.c_int32()
        nb = C.c_int64()
        _check(lib().hh_plan_info(h, C.byref(L), C.byref(ell), C.byref(nb)))
        k = nb.value
        arrs = {"level": np.zeros(k, np.int32), "kind": np.zeros(k, np.int32),
                "i": np.zeros(k, np.int64), "j": np.zeros(k, np.int64),
                "ib": np.zeros(k, np.int64), "ie": np.zeros(k, np.int64),
                "jb": np.zeros(k, np.int64), "je": np.zeros(k, np.int64)}
        _check(lib().hh_plan_blocks(h, arrs["level"].ctypes.data_as(_I32P),
                                    arrs["kind"].ctypes.data_as(_I32P), _iptr(arrs["i"]),
                                    _iptr(arrs["j"]), _iptr(arrs["ib"]), _iptr(arrs["ie"]),
                                    _iptr(arrs["jb"]), _iptr(arrs["je"])))
        perm = np.zeros(n, np.int64)
        _check(lib().hh_plan_perm(h, _iptr(perm)))
        arrs.update({"L": L.value, "ell": ell.value, "perm": perm})
        return arrs
    finally:
        lib().hh_plan_free(h)


def quantize_cont(values, t: int) -> np.ndarray:
    """The library's continuum rounding (t fraction bits, RNE from float64)."""
    v = np.ascontiguousarray(values, dtype=np.float64).ravel()
    out = np.empty_like(v)
    _check(lib().hh_quantize_cont(_dptr(v), v.size, int(t), _dptr(out)))
    return out.reshape(np.shape(values))


def quantize(values, fmt: int, e: int = 0) -> np.ndarray:
    """The library's storage rounding (RNE from float64, scale 2^-e), decoded."""
    v = np.ascontiguousarray(values, dtype=np.float64).ravel()
    out = np.empty_like(v)
    _check(lib().hh_quantize(_dptr(v), v.size, fmt, e, _dptr(out)))
    return out.reshape(np.shape(values))


# ------------------------------------------------------------------ handles
def _kernel_options(kernel, scale, h, normals, mask, uniform_fp64, io_dtype, seed, continuum=False,
                    unit_bytes=0, dot_task_elems=0):
    """hh_kernel and hh_options structs (and the normals array they point to)."""
    nrm = None
    k = Kernel(int(kernel), float(scale), float(h), None)
    if normals is not None:
        nrm = np.ascontiguousarray(normals, dtype=np.float64)
        k.normals = _dptr(nrm)
    o = Options(int(mask), int(bool(uniform_fp64)), IO_F32 if io_dtype == "f32" else IO_F64,
                int(seed), int(continuum), int(unit_bytes), int(dot_task_elems))
    return k, o, nrm


def switch_level_search(points, kernel: int, tol: float, eta: float, leaf_size: int,
                        scale: float = 1.0, h: float = 1.0, normals=None, mask: int = 0xF,
                        uniform_fp64: bool = False, seed: int = 0) -> dict:
    """Switching level chosen by the walk of Alg. 2 over the storage gains
    S1(ell) - S2(ell) (hh_switch_level_search): {"ell", "L", "s1", "s2"}, with
    s2 NaN at the levels the walk did not build."""
    pts = np.ascontiguousarray(points, dtype=np.float64)
    n, d = pts.shape
    k, o, _nrm = _kernel_options(kernel, scale, h, normals, mask, uniform_fp64, "f64", seed)
    L = plan(pts, eta, -1, leaf_size)["L"]
    s1 = np.empty(L + 1)
    s2 = np.empty(L + 1)
    ell = C.c_int32()
    _torch_context()
    _check(lib().hh_switch_level_search(_dptr(pts), n, d, C.byref(k), float(tol), float(eta),
                                        int(leaf_size), C.byref(o), C.byref(ell), _dptr(s1),
                                        _dptr(s2), L + 1))
    return {"ell": ell.value, "L": L, "s1": s1, "s2": s2}


def _torch_context() -> None:
    """Let torch create its device context before the library's first HIP call
    (both then share the one initialised runtime)."""
    try:
        import torch
    except ImportError:
        return
    if torch.cuda.is_available():
        torch.cuda.init()

def _stream_ptr(stream=None, tensors=()):
    """Raw handle of the stream the library launches on. For a stream other
    than the current one, that stream first waits for the current stream (which
    produced the inputs and any contiguous copy of them) and the tensors are
    recorded as in use on it, so the caching allocator does not hand their
    memory out before the library's kernels have read or written it."""
    import torch
    cur = torch.cuda.current_stream()
    if stream is None or stream == cur:
        return C.c_void_p(cur.cuda_stream)
    stream.wait_stream(cur)
    for t in tensors:
        t.record_stream(stream)
    return C.c_void_p(stream.cuda_stream)


class HMatrix:
    """An H_h matrix built on the current GPU (wraps hh_build / hh_free).

    mask: bit f enables storage format f for the format rule (FMT_FP64,
    FMT_FP32, FMT_FP16, FMT_BF16, FMT_Q43; 0xF = the four fixed formats),
    as hh_options.precision_mask in include/hh.h."""

    def __init__(self, points, kernel: int, tol: float, eta: float, switch_level: int,
                 leaf_size: int, scale: float = 1.0, h: float = 1.0, normals=None,
                 mask: int = 0xF, uniform_fp64: bool = False, io_dtype: str = "f64",
                 seed: int = 0, continuum: int = 0, unit_bytes: int = 0,
                 dot_task_elems: int = 0, _handle=None):
        self._h = None
        if _handle is not None:
            self._h = _handle
        else:
            pts = np.ascontiguousarray(points, dtype=np.float64)
            n, d = pts.shape
            k, o, self._normals = _kernel_options(kernel, scale, h, normals, mask, uniform_fp64,
                                                  io_dtype, seed, continuum, unit_bytes,
                                                  dot_task_elems)
            _torch_context()
            hp = _P()
            _check(lib().hh_build(_dptr(pts), n, d, C.byref(k), float(tol), float(eta),
                                  int(switch_level), int(leaf_size), C.byref(o), C.byref(hp)))
            self._h = hp
        self.n = int(lib().hh_size(self._h))
        self.io_dtype = "f32" if lib().hh_io_dtype(self._h) == IO_F32 else "f64"

    # -- products
    def _prep(self, x, out):
        import torch
        if not x.is_cuda:
            raise ValueError("x must be a device tensor")
        dt = torch.float32 if self.io_dtype == "f32" else torch.float64
        if x.dtype != dt:
            raise TypeError(f"x must be {dt} for this handle")
        if x.dim() not in (1, 2) or x.shape[0] != self.n:
            raise ValueError(f"x must have shape ({self.n},) or ({self.n}, nrhs)")
        xc = x.contiguous()
        nrhs = 1 if x.dim() == 1 else x.shape[1]
        y = torch.empty_like(xc) if out is None else out
        if not y.is_cuda or y.shape != xc.shape or y.dtype != dt or not y.is_contiguous():
            raise ValueError("out must be a contiguous device tensor shaped like x")
        return xc, y, nrhs

    def matvec(self, x, out=None, stream=None):
        """y = H^ x on the current stream (Alg. 4)."""
        xc, y, nrhs = self._prep(x, out)
        _check(lib().hh_matvec(self._h, C.c_void_p(xc.data_ptr()), C.c_void_p(y.data_ptr()),
                               nrhs, _stream_ptr(stream, (xc, y))))
        return y

    def matvec_t(self, x, out=None, stream=None):
        """y = H^^T x on the current stream."""
        xc, y, nrhs = self._prep(x, out)
        _check(lib().hh_matvec_t(self._h, C.c_void_p(xc.data_ptr()), C.c_void_p(y.data_ptr()),
                                 nrhs, _stream_ptr(stream, (xc, y))))
        return y

    def matvec_timed(self, x, out=None, stream=None, trans=False):
        """One product with HIP events around its kernels: (y, [gather, dot, axpy] ms)."""
        xc, y, nrhs = self._prep(x, out)
        ms = np.zeros(3)
        _check(lib().hh_matvec_timed(self._h, C.c_void_p(xc.data_ptr()), C.c_void_p(y.data_ptr()),
                                     nrhs, _stream_ptr(stream, (xc, y)), int(bool(trans)), _dptr(ms)))
        return y, ms

    def solve(self, b, x0=None, shift: float = 0.0, rtol: float = 1e-10, restart: int = 30,
              max_iter: int = 300, trans: bool = False, stream=None):
        """Restarted GMRES for (H^ + shift I) x = b (hh_solve): (x, iterations,
        relative residual)."""
        import torch
        if self.io_dtype != "f64":
            raise TypeError("the solver works on handles with fp64 io")
        if not b.is_cuda or b.dtype != torch.float64 or b.shape != (self.n,):
            raise ValueError(f"b must be a float64 device vector of length {self.n}")
        bc = b.contiguous()
        x = torch.zeros_like(bc) if x0 is None else x0.detach().clone().contiguous()
        if x.shape != bc.shape or x.dtype != bc.dtype or not x.is_cuda:
            raise ValueError("x0 must be shaped like b")
        it = C.c_int32()
        rr = C.c_double()
        _check(lib().hh_solve(self._h, C.c_void_p(bc.data_ptr()), C.c_void_p(x.data_ptr()),
                              float(shift), float(rtol), int(restart), int(max_iter), int(bool(trans)),
                              C.byref(it), C.byref(rr), _stream_ptr(stream, (bc, x))))
        return x, it.value, rr.value

    def autotune(self, stream=None) -> dict:
        """Task-table sizes picked by measurement (hh_autotune); the handle keeps them."""
        best = Tuning()
        tried = (Tuning * 32)()
        nt = C.c_int32()
        _check(lib().hh_autotune(self._h, _stream_ptr(stream), C.byref(best), tried, 32, C.byref(nt)))
        return {"best": {"unit_bytes": best.unit_bytes, "dot_task_elems": best.dot_task_elems,
                         "ms": best.ms},
                "tried": [{"unit_bytes": t.unit_bytes, "dot_task_elems": t.dot_task_elems, "ms": t.ms}
                          for t in tried[:nt.value]]}

    def reserve(self, max_nrhs: int) -> None:
        _check(lib().hh_reserve(self._h, int(max_nrhs)))

    def derive(self, mask: int = 0xF, uniform_fp64: bool = False, io_dtype: str | None = None,
               seed: int = 0, continuum: int = 0) -> "HMatrix":
        io = self.io_dtype if io_dtype is None else io_dtype
        o = Options(int(mask), int(bool(uniform_fp64)), IO_F32 if io == "f32" else IO_F64, int(seed),
                    int(continuum))
        hp = _P()
        _check(lib().hh_derive(self._h, C.byref(o), C.byref(hp)))
        return HMatrix(None, 0, 0, 0, 0, 0, _handle=hp)

    # -- inspection
    def stats(self) -> dict:
        s = Stats()
        _check(lib().hh_get_stats(self._h, C.byref(s)))
        return s.to_dict()

    def block_count(self) -> int:
        c = C.c_int64()
        _check(lib().hh_block_count(self._h, C.byref(c)))
        return c.value

    def blocks(self) -> dict:
        """Per-block arrays in canonical order (level, i, j)."""
        k = self.block_count()
        names = [f for f, _ in BlockInfo._fields_]
        out = {nm: [] for nm in names}
        bi = BlockInfo()
        for i in range(k):
            _check(lib().hh_get_block(self._h, i, C.byref(bi)))
            for nm in names:
                out[nm].append(getattr(bi, nm))
        return {nm: np.array(v) for nm, v in out.items()}

    def block_factors(self, index: int):
        bi = BlockInfo()
        _check(lib().hh_get_block(self._h, index, C.byref(bi)))
        m = bi.row_end - bi.row_begin
        n = bi.col_end - bi.col_begin
        if bi.lowrank:
            U = np.zeros((bi.rank, m))
            V = np.zeros((bi.rank, n))
            if bi.rank:
                _check(lib().hh_get_block_factors(self._h, index, _dptr(U), _dptr(V)))
            return U.T.copy(), V.T.copy()
        D = np.zeros((n, m))
        _check(lib().hh_get_block_factors(self._h, index, _dptr(D), None))
        return D.T.copy(), None

    def perm(self) -> np.ndarray:
        p = np.zeros(self.n, np.int64)
        _check(lib().hh_get_perm(self._h, _iptr(p)))
        return p

    def free(self) -> None:
        if self._h is not None and _lib is not None:
            _lib.hh_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def matvec_batch(mats, xs, ys=None, stream=None):
    """y_t = H_t^ x_t for every handle in one pass of the kernels. Every x_t
    (and y_t, if given) is checked against its handle as in HMatrix.matvec,
    and all must carry the same number of right-hand sides."""
    count = len(mats)
    if count == 0 or len(xs) != count or (ys is not None and len(ys) != count):
        raise ValueError("matvec_batch needs one x (and one y, if given) per handle")
    prepped = [m._prep(x, None if ys is None else y)
               for m, x, y in zip(mats, xs, ys if ys is not None else [None] * count)]
    nrhs = prepped[0][2]
    if any(p[2] != nrhs or p[0].dim() != prepped[0][0].dim() for p in prepped):
        raise ValueError("every x of a batch must have the same number of right-hand sides")
    xcs = [p[0] for p in prepped]        # contiguous inputs, alive for the call
    outs = [p[1] for p in prepped]
    hs = (_P * count)(*[m._h for m in mats])
    xp = (_P * count)(*[C.c_void_p(x.data_ptr()) for x in xcs])
    yp = (_P * count)(*[C.c_void_p(y.data_ptr()) for y in outs])
    _check(lib().hh_matvec_batch(hs, count, xp, yp, nrhs, _stream_ptr(stream, xcs + outs)))
    return outs
