"""Python binding of libsympix (SymPix local-operator sampling on gfx950).

Argument marshalling only: every step of the computation runs in the C++ host
library and its HIP kernels.  Device buffers are passed as torch CUDA tensors
(or raw integer addresses) and streams as torch streams (or raw handles).
Importing this package fails loudly if the shared library has not been built.

Precision modes: FP64, FP32, BF16X3, BF16X6 (see include/sympix.h).
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsympix.so")
if not os.path.exists(_LIB_PATH):
    raise ImportError(f"{_LIB_PATH} is missing: build it with paper_1504_04653_amd.build.build() "
                      "(or __graft_entry__.build()); there is no fallback path")

# torch is imported before the library is loaded so that the library binds to
# the HIP runtime torch already carries: two HIP / HSA runtimes in one process
# do not share the device (the second one finds none).
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(_LIB_PATH)

FP64, FP32, BF16X3, BF16X6 = 0, 1, 2, 3
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3, "bf16x6": BF16X6}
PATTERN_ONE_HOP, PATTERN_TWO_HOP = 0, 1
PATTERNS = {"one_hop": PATTERN_ONE_HOP, "two_hop": PATTERN_TWO_HOP}

_STATUS = {0: "OK", -1: "EINVAL", -2: "EINFEASIBLE", -3: "ENOMEM", -4: "EHIP", -5: "ESIZE",
           -6: "EUNSUPPORTED"}


class SympixError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status
        self.code = _STATUS.get(status, str(status))


class Dims(ctypes.Structure):
    _fields_ = [("lmax", ctypes.c_int32), ("k", ctypes.c_int32), ("nrings", ctypes.c_int32),
                ("nbands_hemi", ctypes.c_int32), ("npix", ctypes.c_int64), ("ntiles", ctypes.c_int64),
                ("nadjacency", ctypes.c_int64), ("nblocks", ctypes.c_int64), ("nterms", ctypes.c_int64),
                ("nunique", ctypes.c_int64), ("polar_margin", ctypes.c_double),
                ("y_pattern_max", ctypes.c_double)]


_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_f64 = ctypes.c_double


def _sig(name, args, res=ctypes.c_int):
    fn = getattr(_lib, name)
    fn.argtypes = args
    fn.restype = res
    return fn


_grid_create = _sig("sympix_grid_create", [_i32, _i32, _f64, ctypes.POINTER(_vp)])
_grid_destroy = _sig("sympix_grid_destroy", [_vp], None)
_grid_dims = _sig("sympix_grid_dims", [_vp, ctypes.POINTER(Dims)])
_grid_rings = _sig("sympix_grid_rings", [_vp, _vp, _vp, _vp, _vp])
_grid_bands = _sig("sympix_grid_bands", [_vp, _vp, _vp, _vp])
_grid_pixels = _sig("sympix_grid_pixels", [_vp, _vp, _vp])
_grid_neighbours = _sig("sympix_grid_neighbours", [_vp, _vp, _vp])
_grid_blocks = _sig("sympix_grid_blocks", [_vp, _vp, _vp])
_grid_pattern_blocks = _sig("sympix_grid_pattern_blocks", [_vp, _i32, ctypes.POINTER(_i64), ctypes.POINTER(_i64),
                                                           _vp, _vp])
_grid_unique = _sig("sympix_grid_unique", [_vp, _vp, _vp, _vp, _vp])
_kernel_tabulate = _sig("sympix_kernel_tabulate", [_vp, _vp, _i32, _f64, _i32, _vp, ctypes.POINTER(_vp)])
_kernel_destroy = _sig("sympix_kernel_destroy", [_vp], None)
_kernel_eval = _sig("sympix_kernel_eval", [_vp, _vp, _vp, _i64, _vp])
_sample_D = _sig("sympix_sample_D", [_vp, _vp, _vp, _i64, _vp])
_sample_BtNB = _sig("sympix_sample_BtNB", [_vp, _vp, _vp, _i64, _i32, _vp, _i64, _vp])
_sample_BtNB_noalloc = _sig("sympix_sample_BtNB_noalloc", [_vp, _vp, _vp, _i64, _i32, _vp, _i64, _vp])
_sample_BtNB_pattern = _sig("sympix_sample_BtNB_pattern", [_vp, _vp, _vp, _i64, _i32, _i32, _vp, _i64, _vp])
_sample_D_BtNB = _sig("sympix_sample_D_BtNB", [_vp, _vp, _vp, _vp, _i64, _i32, _vp, _i64, _vp, _i64, _vp])
_convolve = _sig("sympix_convolve", [_vp, _vp, _vp, _i64, _vp, _i64, _vp])
_factor_diag = _sig("sympix_factor_diag", [_vp, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp])
_solve_diag = _sig("sympix_solve_diag", [_vp, _vp, _i64, _vp, _i64, _vp, _i64, _vp])
_last_error = _sig("sympix_last_error", [], ctypes.c_char_p)


class CrossSizes(ctypes.Structure):
    _fields_ = [("lmax_eff", ctypes.c_int32), ("max_terms", ctypes.c_int32), ("nadjacency", ctypes.c_int64),
                ("nunique", ctypes.c_int64), ("nblocks", ctypes.c_int64), ("nterms", ctypes.c_int64),
                ("y_pattern_max", ctypes.c_double)]


_cross_create = _sig("sympix_cross_create", [_vp, _vp, ctypes.POINTER(_vp)])
_cross_destroy = _sig("sympix_cross_destroy", [_vp], None)
_cross_dims = _sig("sympix_cross_dims", [_vp, ctypes.POINTER(CrossSizes)])
_cross_neighbours = _sig("sympix_cross_neighbours", [_vp, _vp, _vp, _vp, _vp])
_cross_unique = _sig("sympix_cross_unique", [_vp, _vp, _vp, _vp])
_kernel_tabulate_cross = _sig("sympix_kernel_tabulate_cross", [_vp, _vp, _i32, _f64, _i32, _vp, ctypes.POINTER(_vp)])
_sample_B_cross = _sig("sympix_sample_B_cross", [_vp, _vp, _vp, _i64, _vp])
_sample_BtNB_cross = _sig("sympix_sample_BtNB_cross", [_vp, _vp, _vp, _i64, _i32, _vp, _i64, _vp])

_sht_create = _sig("sympix_sht_create", [_vp, _i32, ctypes.POINTER(_vp)])
_sht_destroy = _sig("sympix_sht_destroy", [_vp], None)
_sht_synthesis = _sig("sympix_sht_synthesis", [_vp, _vp, _i64, _vp, _i64, _vp])
_sht_adjoint = _sig("sympix_sht_adjoint", [_vp, _vp, _i64, _vp, _i64, _vp])
_sht_analysis = _sig("sympix_sht_analysis", [_vp, _vp, _i64, _vp, _i64, _vp])
_sht_degrade = _sig("sympix_sht_degrade", [_vp, _vp, _vp, _i64, _vp, _i64, _vp])


class Problem(ctypes.Structure):
    _fields_ = [("g", _vp), ("b", _vp), ("ninv_dev", _vp), ("ninv_len", _i64), ("out_dev", _vp),
                ("out_len", _i64)]


_batch_create = _sig("sympix_batch_create", [ctypes.POINTER(Problem), _i32, _i32, _vp, ctypes.POINTER(_vp)])
_batch_set_schedule = _sig("sympix_batch_set_schedule", [_vp, _i32])
_batch_set_tiling = _sig("sympix_batch_set_tiling", [_vp, _i32])
_batch_tune = _sig("sympix_batch_tune", [_vp, _vp, ctypes.POINTER(_i32), ctypes.POINTER(_f64)])
_batch_launch = _sig("sympix_batch_launch", [_vp, _vp])
_batch_plan = _sig("sympix_batch_plan", [_vp, ctypes.POINTER(_i32)])
_batch_destroy = _sig("sympix_batch_destroy", [_vp], None)

SCHED_XCD_QUEUES, SCHED_GLOBAL_LPT, SCHED_PER_PROBLEM = 0, 1, 2
SCHEDULES = {"xcd_queues": SCHED_XCD_QUEUES, "global_lpt": SCHED_GLOBAL_LPT, "per_problem": SCHED_PER_PROBLEM}
TILES_64, TILES_32 = 0, 1
TILINGS = {"tiles64": TILES_64, "tiles32": TILES_32}


def plan_name(plan):
    """'schedule/tiling' of a tuner plan (schedule + len(SCHEDULES) * tiling)."""
    sched = {v: k for k, v in SCHEDULES.items()}[plan % len(SCHEDULES)]
    tiling = {v: k for k, v in TILINGS.items()}[plan // len(SCHEDULES)]
    return f"{sched}/{tiling}"

EXPORTED = ("sympix_grid_create", "sympix_grid_destroy", "sympix_grid_dims", "sympix_grid_rings",
            "sympix_grid_bands", "sympix_grid_pixels", "sympix_grid_neighbours", "sympix_grid_blocks", "sympix_grid_pattern_blocks", "sympix_grid_unique",
            "sympix_kernel_tabulate", "sympix_kernel_destroy", "sympix_kernel_eval", "sympix_sample_D",
            "sympix_sample_BtNB", "sympix_sample_BtNB_noalloc", "sympix_sample_BtNB_pattern", "sympix_sample_D_BtNB", "sympix_convolve", "sympix_factor_diag", "sympix_solve_diag", "sympix_batch_create", "sympix_batch_set_schedule", "sympix_batch_set_tiling", "sympix_batch_tune",
            "sympix_batch_launch", "sympix_batch_plan", "sympix_batch_destroy", "sympix_last_error",
            "sympix_cross_create", "sympix_cross_destroy", "sympix_cross_dims", "sympix_cross_neighbours",
            "sympix_cross_unique", "sympix_kernel_tabulate_cross", "sympix_sample_B_cross", "sympix_sample_BtNB_cross",
            "sympix_sht_create", "sympix_sht_destroy", "sympix_sht_synthesis", "sympix_sht_adjoint",
            "sympix_sht_analysis", "sympix_sht_degrade")


def _check(status):
    if status != 0:
        raise SympixError(status, (_last_error() or b"").decode())


def _ptr(x):
    """Device/host address of a torch tensor, numpy array or integer."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    raise TypeError(f"cannot take the address of {type(x)}")


def _stream(s):
    if s is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(s, int):
        return s
    return s.cuda_stream


def _numel(x):
    if hasattr(x, "numel"):
        return int(x.numel())
    return int(np.asarray(x).size)


def _require_f64_device(t, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")


class Grid:
    """SymPix grid (host object; device tables are created on first use)."""

    def __init__(self, lmax: int, k: int = 8, polar_margin: float | None = None):
        h = _vp()
        _check(_grid_create(int(lmax), int(k), math.nan if polar_margin is None else float(polar_margin),
                            ctypes.byref(h)))
        self._h = h
        d = Dims()
        _check(_grid_dims(self._h, ctypes.byref(d)))
        self.dims = d
        for f, _ in Dims._fields_:
            setattr(self, f, getattr(d, f))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _grid_destroy is not None:   # None at interpreter exit
            _grid_destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def rings(self):
        n = self.nrings
        theta = np.zeros(n)
        weight = np.zeros(n)
        npix = np.zeros(n, dtype=np.int32)
        first = np.zeros(n, dtype=np.int64)
        _check(_grid_rings(self._h, _ptr(theta), _ptr(weight), _ptr(npix), _ptr(first)))
        return theta, weight, npix, first

    def bands(self):
        nb = 2 * self.nbands_hemi
        tiles = np.zeros(nb, dtype=np.int32)
        alpha = np.zeros(nb, dtype=np.int32)
        ring0 = np.zeros(nb, dtype=np.int32)
        _check(_grid_bands(self._h, _ptr(tiles), _ptr(alpha), _ptr(ring0)))
        return tiles, alpha, ring0

    def neighbours(self):
        rp = np.zeros(self.ntiles + 1, dtype=np.int64)
        col = np.zeros(self.nadjacency, dtype=np.int32)
        _check(_grid_neighbours(self._h, _ptr(rp), _ptr(col)))
        return rp, col

    def blocks(self):
        rp = np.zeros(self.ntiles + 1, dtype=np.int64)
        col = np.zeros(self.nblocks, dtype=np.int32)
        _check(_grid_blocks(self._h, _ptr(rp), _ptr(col)))
        return rp, col

    def pattern_size(self, pattern=PATTERN_ONE_HOP):
        """(blocks, contraction terms) of a stored-block pattern."""
        if isinstance(pattern, str):
            pattern = PATTERNS[pattern]
        n, t = _i64(0), _i64(0)
        _check(_grid_pattern_blocks(self._h, int(pattern), ctypes.byref(n), ctypes.byref(t), None, None))
        return n.value, t.value

    def pattern_blocks(self, pattern=PATTERN_ONE_HOP):
        """(row_ptr, col) of a stored-block pattern (PATTERN_ONE_HOP / TWO_HOP)."""
        if isinstance(pattern, str):
            pattern = PATTERNS[pattern]
        n, _ = self.pattern_size(pattern)
        rp = np.zeros(self.ntiles + 1, dtype=np.int64)
        col = np.zeros(n, dtype=np.int32)
        _check(_grid_pattern_blocks(self._h, int(pattern), None, None, _ptr(rp), _ptr(col)))
        return rp, col

    def unique(self):
        uid = np.zeros(self.nadjacency, dtype=np.int32)
        bi = np.zeros(self.nunique, dtype=np.int32)
        bj = np.zeros(self.nunique, dtype=np.int32)
        de = np.zeros(self.nunique, dtype=np.int64)
        _check(_grid_unique(self._h, _ptr(uid), _ptr(bi), _ptr(bj), _ptr(de)))
        return uid, bi, bj, de

    def pixel_theta_phi(self):
        """Colatitude and longitude of every pixel in pixel order (host arrays)."""
        th = np.empty(self.npix)
        ph = np.empty(self.npix)
        _check(_grid_pixels(self._h, _ptr(th), _ptr(ph)))
        return th, ph

    @property
    def out_len(self):
        return self.nblocks * self.k ** 4


class Kernel:
    """Tabulated Eq. 10 kernel plus all unique local blocks of a grid."""

    def __init__(self, grid: Grid, coef_l, radius: float = 0.0, n_nodes: int = 65536, stream=None):
        coef = np.ascontiguousarray(coef_l, dtype=np.float64)
        h = _vp()
        self.grid = grid
        _check(_kernel_tabulate(grid.handle, _ptr(coef), int(coef.size), float(radius), int(n_nodes),
                                _stream(stream), ctypes.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _kernel_destroy is not None:
            _kernel_destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def eval(self, y, out, stream=None):
        _require_f64_device(y, "y")
        _require_f64_device(out, "out")
        if _numel(out) != _numel(y):
            raise ValueError("y and out differ in length")
        _check(_kernel_eval(self._h, _ptr(y), _ptr(out), _numel(y), _stream(stream)))
        return out


def sample_D(grid: Grid, kernel: Kernel, out, stream=None):
    _require_f64_device(out, "out")
    _check(_sample_D(grid.handle, kernel.handle, _ptr(out), _numel(out), _stream(stream)))
    return out


def sample_BtNB(grid: Grid, kernel: Kernel, ninv, out, prec=FP64, stream=None):
    if isinstance(prec, str):
        prec = PRECISIONS[prec]
    _require_f64_device(ninv, "ninv")
    _require_f64_device(out, "out")
    _check(_sample_BtNB(grid.handle, kernel.handle, _ptr(ninv), _numel(ninv), int(prec), _ptr(out),
                        _numel(out), _stream(stream)))
    return out


def sample_BtNB_noalloc(grid: Grid, kernel: Kernel, ninv, out, prec=FP64, stream=None):
    """sample_BtNB without any device allocation (static N^-1 scratch of the
    library; at most 2^24 pixels outside FP64; overlapping calls on one device
    race)."""
    if isinstance(prec, str):
        prec = PRECISIONS[prec]
    _require_f64_device(ninv, "ninv")
    _require_f64_device(out, "out")
    _check(_sample_BtNB_noalloc(grid.handle, kernel.handle, _ptr(ninv), _numel(ninv), int(prec), _ptr(out),
                                _numel(out), _stream(stream)))
    return out


def sample_BtNB_pattern(grid: Grid, kernel: Kernel, ninv, out, prec=FP64, pattern=PATTERN_ONE_HOP, stream=None):
    """B-hat^T N^-1 B-hat on the blocks of a stored-block pattern (out holds
    that pattern's nblocks k^4 values, in the order of grid.pattern_blocks)."""
    if isinstance(prec, str):
        prec = PRECISIONS[prec]
    if isinstance(pattern, str):
        pattern = PATTERNS[pattern]
    _require_f64_device(ninv, "ninv")
    _require_f64_device(out, "out")
    _check(_sample_BtNB_pattern(grid.handle, kernel.handle, _ptr(ninv), _numel(ninv), int(prec), int(pattern),
                                _ptr(out), _numel(out), _stream(stream)))
    return out


def sample_D_BtNB(grid: Grid, kd: Kernel, kb: Kernel, ninv, out_D, out_C, prec=FP64, stream=None):
    """D-hat blocks of kd into out_D and B-hat^T N^-1 B-hat blocks of kb into
    out_C in one call and one launch."""
    if isinstance(prec, str):
        prec = PRECISIONS[prec]
    _require_f64_device(ninv, "ninv")
    _require_f64_device(out_D, "out_D")
    _require_f64_device(out_C, "out_C")
    _check(_sample_D_BtNB(grid.handle, kd.handle, kb.handle, _ptr(ninv), _numel(ninv), int(prec), _ptr(out_D),
                          _numel(out_D), _ptr(out_C), _numel(out_C), _stream(stream)))
    return out_D, out_C


def convolve(grid: Grid, kernel: Kernel, f, out, stream=None):
    """out = B-hat f, the pixel-domain convolution with the kernel's local blocks."""
    _require_f64_device(f, "f")
    _require_f64_device(out, "out")
    _check(_convolve(grid.handle, kernel.handle, _ptr(f), _numel(f), _ptr(out), _numel(out), _stream(stream)))
    return out


def factor_diag(grid: Grid, D, C, U, info, stream=None):
    """U_J with U_J^T U_J = D_JJ + C_JJ for every tile J (C None: D_JJ alone),
    into U (ntiles k^4 float64) and info (ntiles int32: 0, or the failing
    pivot row + 1)."""
    import torch
    _require_f64_device(D, "D")
    if C is not None:
        _require_f64_device(C, "C")
    _require_f64_device(U, "U")
    if not (isinstance(info, torch.Tensor) and info.is_cuda and info.dtype == torch.int32 and info.is_contiguous()):
        raise TypeError("info must be a contiguous int32 CUDA tensor")
    _check(_factor_diag(grid.handle, _ptr(D), _numel(D), None if C is None else _ptr(C), 0 if C is None else _numel(C),
                        _ptr(U), _numel(U), _ptr(info), _numel(info), _stream(stream)))
    return U, info


def solve_diag(grid: Grid, U, r, x, stream=None):
    """x_J = (U_J^T U_J)^-1 r_J for every tile (x may be r)."""
    _require_f64_device(U, "U")
    _require_f64_device(r, "r")
    _require_f64_device(x, "x")
    _check(_solve_diag(grid.handle, _ptr(U), _numel(U), _ptr(r), _numel(r), _ptr(x), _numel(x), _stream(stream)))
    return x


class Cross:
    """The pair of grids (g2 = Y_2 auxiliary, g1 = Y_1) of B-hat = Y_2 B Y_1^T."""

    def __init__(self, g2: Grid, g1: Grid):
        h = _vp()
        _check(_cross_create(g2.handle, g1.handle, ctypes.byref(h)))
        self._h = h
        self.g2, self.g1 = g2, g1          # the pair refers to both grids
        d = CrossSizes()
        _check(_cross_dims(self._h, ctypes.byref(d)))
        for f, _ in CrossSizes._fields_:
            setattr(self, f, getattr(d, f))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _cross_destroy is not None:
            _cross_destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def neighbours(self):
        """(container[ntiles_2], row_ptr, col, uid) of the tile relation."""
        cont = np.zeros(self.g2.ntiles, dtype=np.int32)
        rp = np.zeros(self.g2.ntiles + 1, dtype=np.int64)
        col = np.zeros(self.nadjacency, dtype=np.int32)
        uid = np.zeros(self.nadjacency, dtype=np.int32)
        _check(_cross_neighbours(self._h, _ptr(cont), _ptr(rp), _ptr(col), _ptr(uid)))
        return cont, rp, col, uid

    def unique(self):
        bi = np.zeros(self.nunique, dtype=np.int32)
        bj = np.zeros(self.nunique, dtype=np.int32)
        de = np.zeros(self.nunique, dtype=np.int64)
        _check(_cross_unique(self._h, _ptr(bi), _ptr(bj), _ptr(de)))
        return bi, bj, de

    @property
    def out_len(self):
        return self.nblocks * self.g1.k ** 4

    @property
    def b_len(self):
        return self.nadjacency * self.g1.k ** 4


class CrossKernel(Kernel):
    """Eq. 10 kernel tabulated for a pair of grids, with every unique block of
    B-hat = Y_2 B Y_1^T."""

    def __init__(self, cross: Cross, coef_l, radius: float = 0.0, n_nodes: int = 65536, stream=None):
        coef = np.ascontiguousarray(coef_l, dtype=np.float64)
        h = _vp()
        self.grid = None
        self.cross = cross
        _check(_kernel_tabulate_cross(cross.handle, _ptr(coef), int(coef.size), float(radius), int(n_nodes),
                                      _stream(stream), ctypes.byref(h)))
        self._h = h


def sample_B_cross(cross: Cross, kernel: CrossKernel, out, stream=None):
    """The kept blocks of B-hat = Y_2 B Y_1^T in the relation's CSR order."""
    _require_f64_device(out, "out")
    _check(_sample_B_cross(cross.handle, kernel.handle, _ptr(out), _numel(out), _stream(stream)))
    return out


def sample_BtNB_cross(cross: Cross, kernel: CrossKernel, ninv2, out, prec=FP64, stream=None):
    """B-hat^T N_2^-1 B-hat on the stored blocks of Y_1, N_2^-1 on Y_2."""
    if isinstance(prec, str):
        prec = PRECISIONS[prec]
    _require_f64_device(ninv2, "ninv2")
    _require_f64_device(out, "out")
    _check(_sample_BtNB_cross(cross.handle, kernel.handle, _ptr(ninv2), _numel(ninv2), int(prec), _ptr(out),
                              _numel(out), _stream(stream)))
    return out


def raw_call(name):
    """The ctypes function of an exported symbol (for ABI-level tests)."""
    return getattr(_lib, name)


class Batch:
    """Many B-hat^T N^-1 B-hat problems (any precision mode) in one captured graph.

    problems: sequence of (grid, kernel, ninv, out) with ninv / out contiguous
    float64 CUDA tensors.  The batch keeps references to all of them."""

    def __init__(self, problems, prec=FP32, stream=None):
        if isinstance(prec, str):
            prec = PRECISIONS[prec]
        self._keep = list(problems)
        arr = (Problem * len(self._keep))()
        for i, (grid, kernel, ninv, out) in enumerate(self._keep):
            _require_f64_device(ninv, "ninv")
            _require_f64_device(out, "out")
            arr[i] = Problem(grid.handle, kernel.handle, _ptr(ninv), _numel(ninv), _ptr(out), _numel(out))
        h = _vp()
        _check(_batch_create(arr, len(self._keep), int(prec), _stream(stream), ctypes.byref(h)))
        self._h = h

    def __del__(self):
        self.close()

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _batch_destroy is not None:
            _batch_destroy(h)
            self._h = None

    def set_schedule(self, schedule):
        if isinstance(schedule, str):
            schedule = SCHEDULES[schedule]
        _check(_batch_set_schedule(self._h, int(schedule)))

    def set_tiling(self, tiling):
        if isinstance(tiling, str):
            tiling = TILINGS[tiling]
        _check(_batch_set_tiling(self._h, int(tiling)))

    def tune(self, stream=None):
        """Time every plan (schedule, tile shape) once, keep the fastest; returns
        (chosen plan, ms per plan), plan = schedule + len(SCHEDULES) * tiling."""
        chosen = _i32(-1)
        ms = (_f64 * (len(SCHEDULES) * len(TILINGS)))()
        _check(_batch_tune(self._h, _stream(stream), ctypes.byref(chosen), ms))
        return chosen.value, list(ms)

    def launch(self, stream=None):
        _check(_batch_launch(self._h, _stream(stream)))

    def plan(self):
        """The plan (schedule + len(SCHEDULES) * tiling) the graph was captured with."""
        p = _i32(-1)
        _check(_batch_plan(self._h, ctypes.byref(p)))
        return p.value


class Sht:
    """Transform plan of band limit lmax on a grid (the current device):
    synthesis Y a, transpose Y^T f and analysis Y^T W f in the real
    orthonormal basis, coefficients at l^2 + l + m (see include/sympix.h)."""

    def __init__(self, g: Grid, lmax: int):
        h = _vp()
        _check(_sht_create(g.handle, int(lmax), ctypes.byref(h)))
        self._h = h
        self.g = g                          # the plan refers to the grid
        self.lmax = int(lmax)
        self.nalm = (self.lmax + 1) ** 2

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _sht_destroy is not None:
            _sht_destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def synthesis(self, alm, out, stream=None):
        _require_f64_device(alm, "alm")
        _require_f64_device(out, "out")
        _check(_sht_synthesis(self._h, _ptr(alm), _numel(alm), _ptr(out), _numel(out), _stream(stream)))

    def adjoint(self, f, out, stream=None):
        _require_f64_device(f, "f")
        _require_f64_device(out, "out")
        _check(_sht_adjoint(self._h, _ptr(f), _numel(f), _ptr(out), _numel(out), _stream(stream)))

    def analysis(self, f, out, stream=None):
        _require_f64_device(f, "f")
        _require_f64_device(out, "out")
        _check(_sht_analysis(self._h, _ptr(f), _numel(f), _ptr(out), _numel(out), _stream(stream)))


def degrade(obs: Sht, target: Sht, theta_obs, out, stream=None):
    """theta_2 = W_2 Y_2 Y_obs^T theta_obs (Eq. 14) onto the target plan's grid."""
    _require_f64_device(theta_obs, "theta_obs")
    _require_f64_device(out, "out")
    _check(_sht_degrade(obs.handle, target.handle, _ptr(theta_obs), _numel(theta_obs), _ptr(out), _numel(out),
                        _stream(stream)))
