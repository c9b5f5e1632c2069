"""Python binding of libgcqbem (the C ABI declared in include/gcqbem.h).

Argument marshalling only: every step of the computation runs in the library's
HIP kernels.  Device arrays are torch tensors on the context's GPU (PyTorch is
used for device memory and streams); host arrays are numpy arrays.  Method
names follow the C entry points without their ``gcq_`` prefix.

The library must have been built (``python paper_2505_00715_amd/build.py``);
importing this module without it raises immediately -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgcqbem.so")

C128, C64, C64_SPLIT_BF16 = 0, 1, 2
PER_FREQUENCY, WEIGHTED_SUM, PLAIN_H = 0, 1, 2
FLAG_RECOMPRESS, FLAG_USE_PREDICTOR, FLAG_PER_FREQ_LAUNCH, FLAG_DOUBLE_LAYER = 1, 2, 4, 8
OK, NOT_CONVERGED, RANK_CAPPED = 0, 1, 2
N_MODEL_PARAMS = 4609


class TreeInfo(C.Structure):
    _fields_ = [("n_clusters", C.c_int32), ("n_leaves", C.c_int32), ("depth", C.c_int32),
                ("n_blocks", C.c_int32), ("n_far", C.c_int32), ("n_near", C.c_int32),
                ("far_dims", C.c_int64), ("near_entries", C.c_int64)]


class AcaStats(C.Structure):
    _fields_ = [("n_pairs", C.c_int64), ("aca_rank_sum", C.c_int64), ("rank_sum", C.c_int64),
                ("rank_max", C.c_int32), ("n_capped", C.c_int32), ("n_overflow", C.c_int64),
                ("entries", C.c_int64), ("storage_bytes", C.c_int64), ("device_ms", C.c_double)]


class Aca3dStats(C.Structure):
    _fields_ = [("n_blocks", C.c_int32), ("rank_min", C.c_int32), ("rank_max", C.c_int32),
                ("rank_mean", C.c_double), ("n_capped", C.c_int32),
                ("slice_rank_sum", C.c_int64), ("storage_bytes", C.c_int64),
                ("compression_rate", C.c_double), ("device_ms", C.c_double),
                ("far_entries", C.c_int64), ("far_flops", C.c_double), ("far_ms", C.c_double)]


class Fmm3dStats(C.Structure):
    _fields_ = [("n_far", C.c_int32), ("rank_max", C.c_int32), ("rank_mean", C.c_double),
                ("n_capped", C.c_int32), ("storage_bytes", C.c_int64), ("device_ms", C.c_double),
                ("m2l_ms", C.c_double)]


class SolveStats(C.Structure):
    _fields_ = [("n_systems", C.c_int32), ("n_converged", C.c_int32), ("iters_max", C.c_int32),
                ("resid_max", C.c_double), ("device_ms", C.c_double)]


class Tuning(C.Structure):
    _fields_ = [("aca3d_waves", C.c_int32 * 4), ("aca3d_stack_slices", C.c_int32),
                ("aca_waves", C.c_int32), ("product_graph", C.c_int32),
                ("product_cols_per_wave", C.c_int32)]


class TrainCfg(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float),
                ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("seed", C.c_uint64)]


class TrainStats(C.Structure):
    _fields_ = [("loss_first", C.c_float), ("loss_last", C.c_float), ("device_ms", C.c_double)]


class GcqError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"gcqbem error {code}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python paper_2505_00715_amd/build.py` (there is no CPU fallback)")
    # torch first: its bundled HIP runtime (soname libamdhip64.so.7) then also
    # serves this library, so that one HIP runtime drives the process
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    P, I32, I64, D, U32 = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_uint32
    sig = {
        "gcq_create": [C.c_int, P, C.POINTER(P)],
        "gcq_destroy": [P],
        "gcq_kernel_ms": [P, C.c_char_p],
        "gcq_set_tuning": [P, P],
        "gcq_get_tuning": [P, P],
        "gcq_upload_mesh": [P, P, I64, P, I64, D],
        "gcq_set_frequencies": [P, P, I32, I32],
        "gcq_contour": [I32, D, D, D, P, P],
        "gcq_contour_points": [I32, I32, P],
        "gcq_contour_steps": [P, I32, D, D, P],
        "gcq_gcq_convolve": [P, P, I32, P, I32, I32, P, I32, P, P],
        "gcq_gcq_solve": [P, P, I32, P, I32, I32, P, I32, P, P, D, I32, I32, P],
        "gcq_build_cluster_tree": [P, I32, D, P],
        "gcq_get_tree": [P, P, P],
        "gcq_trim": [P, I32],
        "gcq_upload_cluster_tree": [P, P, I32, P, P, P, I32, P, P, P, P],
        "gcq_assemble_slices": [P, P, I64, P, I64, P, I32, I32, P],
        "gcq_assemble_dlp_slices": [P, P, I64, P, I64, P, I32, I32, P],
        "gcq_assemble_slices_noalloc": [P, P, I64, P, I64, P, I32, I32, P],
        "gcq_aca_blocks": [P, P, I32, D, I32, I32, U32, P],
        "gcq_get_block_factors": [P, I32, I32, P, P, I32, P],
        "gcq_aca_ranks": [P, P, I64],
        "gcq_aca3d": [P, D, D, I32, I32, U32, P],
        "gcq_get_aca3d_block": [P, I32, I32, P, P, P, P],
        "gcq_aca3d_ranks": [P, P, P, I64],
        "gcq_fmm3d": [P, I32, D, I32, I32, P],
        "gcq_fmm3d_matvec": [P, P, P],
        "gcq_get_fmm3d_block": [P, I32, I32, P, P, P, P],
        "gcq_compressed_matvec": [P, I32, I32, P, P, I32],
        "gcq_sample_rows": [P, P, I32, I32, P],
        "gcq_solve": [P, P, P, D, I32, I32, I32, P],
        "gcq_rank_features": [P, P, I32, P],
        "gcq_rank_model_train": [P, P, P, I64, P, P],
        "gcq_rank_model_grad": [P, P, P, I64, P, P],
        "gcq_rank_model_predict": [P, P, I64, P],
        "gcq_rank_model_get": [P, P, P, P],
        "gcq_rank_model_set": [P, P, P, P],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int
    lib.gcq_kernel_ms.restype = C.c_double
    lib.gcq_last_error.argtypes = []
    lib.gcq_last_error.restype = C.c_char_p
    return lib


_lib = _load()
lib = _lib


def _check(code):
    if code < 0:
        raise GcqError(code, _lib.gcq_last_error().decode())
    return code


def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(C.c_void_p)


def _dev(t, dtype, numel=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a torch tensor on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


def contour(n_points: int, dt_min: float, dt_max: float, stage_ratio: float = 1.0):
    """Points s (n_points,) and weights w of the gCQ contour quadrature (gcq_contour)."""
    s = np.zeros(int(n_points), np.complex128)
    w = np.zeros(int(n_points), np.complex128)
    _check(_lib.gcq_contour(int(n_points), float(dt_min), float(dt_max), float(stage_ratio),
                            s.ctypes.data_as(C.c_void_p), w.ctypes.data_as(C.c_void_p)))
    return s, w


def contour_steps(A, dt_min: float, dt_max: float):
    """(dt_min', dt_max', stage_ratio) of the contour for Butcher matrix A (gcq_contour_steps)."""
    Ah, pa = _host(np.atleast_2d(np.asarray(A, np.float64)), np.float64)
    if Ah.shape[0] != Ah.shape[1]:
        raise ValueError("A must be square")
    out = np.zeros(3, np.float64)
    _check(_lib.gcq_contour_steps(pa, int(Ah.shape[0]), float(dt_min), float(dt_max),
                                  out.ctypes.data_as(C.c_void_p)))
    return float(out[0]), float(out[1]), float(out[2])


def contour_points(n_steps: int, stages: int = 2) -> int:
    """Number of contour points for n_steps steps (gcq_contour_points)."""
    n = C.c_int32(0)
    _check(_lib.gcq_contour_points(int(n_steps), int(stages), C.byref(n)))
    return n.value


class Context:
    """One library context on one GPU, enqueuing on torch's current stream of
    that device at creation time."""

    def __init__(self, device: int = 0, stream=None):
        """device = -1 gives a host-only context (geometry, trees, features)."""
        h = C.c_void_p()
        self.device = device
        if device < 0:
            _check(_lib.gcq_create(-1, None, C.byref(h)))
        else:
            import torch
            if stream is None:
                stream = torch.cuda.current_stream(device)
            self._stream = stream
            _check(_lib.gcq_create(device, C.c_void_p(stream.cuda_stream), C.byref(h)))
        self._h = h
        self.n = 0
        self.L = 0

    def destroy(self):
        if getattr(self, "_h", None):
            _lib.gcq_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def kernel_ms(self, name: str) -> float:
        return _lib.gcq_kernel_ms(self._h, name.encode())

    def set_tuning(self, aca3d_waves=None, aca3d_stack_slices=None, aca_waves=None,
                   product_graph=None, product_cols_per_wave=None):
        """aca3d_waves: 4 group sizes (waves per block) of the 3D-ACA size classes;
        aca3d_stack_slices: initial stack reservation of a far block (slices);
        aca_waves: waves per pair of aca_blocks; product_graph: replay the
        per-frequency product as a captured graph; product_cols_per_wave:
        frequency columns per wave of the split-bf16 product (32 or 64)."""
        t = self.get_tuning()
        if product_cols_per_wave is not None:
            t.product_cols_per_wave = int(product_cols_per_wave)
        if aca_waves is not None:
            t.aca_waves = int(aca_waves)
        if product_graph is not None:
            t.product_graph = int(product_graph)
        if aca3d_waves is not None:
            for c, w in enumerate(aca3d_waves):
                t.aca3d_waves[c] = int(w)
        if aca3d_stack_slices is not None:
            t.aca3d_stack_slices = int(aca3d_stack_slices)
        _check(_lib.gcq_set_tuning(self._h, C.byref(t)))

    def get_tuning(self) -> Tuning:
        t = Tuning()
        _check(_lib.gcq_get_tuning(self._h, C.byref(t)))
        return t

    # ---- geometry, frequencies, tree
    def upload_mesh(self, xyz, tri, wave_speed: float):
        xyz, px = _host(xyz, np.float64)
        tri, pt = _host(tri, np.int32)
        _check(_lib.gcq_upload_mesh(self._h, px, len(xyz), pt, len(tri), float(wave_speed)))
        self.n = len(tri)

    def set_frequencies(self, s, use_conjugate_symmetry: bool = True):
        s = np.ascontiguousarray(s, dtype=np.complex128)
        _check(_lib.gcq_set_frequencies(self._h, s.ctypes.data_as(C.c_void_p), len(s),
                                        int(bool(use_conjugate_symmetry))))
        self.L = len(s)

    def build_cluster_tree(self, leaf_size: int, eta: float) -> TreeInfo:
        info = TreeInfo()
        _check(_lib.gcq_build_cluster_tree(self._h, leaf_size, float(eta), C.byref(info)))
        self.tree_info = info
        return info

    def upload_cluster_tree(self, perm, cl_begin, cl_end, cl_son, blk_row, blk_col,
                            blk_admissible) -> TreeInfo:
        """Use a caller-made partition (gcq_upload_cluster_tree): perm (n),
        cl_begin, cl_end (n_clusters), cl_son (n_clusters x 2, -1 for leaves),
        blk_row, blk_col, blk_admissible (n_blocks)."""
        pp, p0 = _host(perm, np.int32)
        cb, p1 = _host(cl_begin, np.int32)
        ce, p2 = _host(cl_end, np.int32)
        cs, p3 = _host(np.asarray(cl_son).reshape(-1), np.int32)
        br, p4 = _host(blk_row, np.int32)
        bc, p5 = _host(blk_col, np.int32)
        ba, p6 = _host(blk_admissible, np.uint8)
        if len(ce) != len(cb) or len(cs) != 2 * len(cb) or len(bc) != len(br) or len(ba) != len(br):
            raise ValueError("tree arrays of inconsistent lengths")
        info = TreeInfo()
        _check(_lib.gcq_upload_cluster_tree(self._h, p0, len(cb), p1, p2, p3, len(br), p4, p5, p6,
                                            C.byref(info)))
        self.tree_info = info
        return info

    def trim(self, release_faces: bool = True):
        """Release the context's working buffers (and the per-frequency
        H-matrices) -- gcq_trim."""
        _check(_lib.gcq_trim(self._h, int(bool(release_faces))))

    def get_tree(self):
        nb = self.tree_info.n_blocks
        perm = np.zeros(self.n, np.int32)
        blocks = np.zeros((nb, 5), np.int32)
        _check(_lib.gcq_get_tree(self._h, perm.ctypes.data_as(C.c_void_p),
                                 blocks.ctypes.data_as(C.c_void_p)))
        return perm, blocks

    # ---- entries
    def assemble_slices(self, rows, cols, freq_idx, precision, out):
        import torch
        rows, pr = _host(rows, np.int32)
        cols, pc = _host(cols, np.int32)
        fi, pf = _host(freq_idx, np.int32)
        dt = torch.complex128 if precision == C128 else torch.complex64
        po = _dev(out, dt, len(fi) * len(cols) * len(rows), "out")
        _check(_lib.gcq_assemble_slices(self._h, pr, len(rows), pc, len(cols), pf, len(fi),
                                        precision, po))
        return out

    def assemble_slices_noalloc(self, rows, cols, freq_idx, precision, out):
        """gcq_assemble_slices_noalloc: as assemble_slices, staged in the
        device's fixed array (no device allocation, no synchronisation)."""
        import torch
        rows, pr = _host(rows, np.int32)
        cols, pc = _host(cols, np.int32)
        fi, pf = _host(freq_idx, np.int32)
        dt = torch.complex128 if precision == C128 else torch.complex64
        po = _dev(out, dt, len(fi) * len(cols) * len(rows), "out")
        _check(_lib.gcq_assemble_slices_noalloc(self._h, pr, len(rows), pc, len(cols), pf, len(fi),
                                                precision, po))
        return out

    def assemble_dlp_slices(self, rows, cols, freq_idx, precision, out):
        """Dense double-layer entries (gcq_assemble_dlp_slices), layout as assemble_slices."""
        import torch
        rows, pr = _host(rows, np.int32)
        cols, pc = _host(cols, np.int32)
        fi, pf = _host(freq_idx, np.int32)
        dt = torch.complex128 if precision == C128 else torch.complex64
        po = _dev(out, dt, len(fi) * len(cols) * len(rows), "out")
        _check(_lib.gcq_assemble_dlp_slices(self._h, pr, len(rows), pc, len(cols), pf, len(fi),
                                            precision, po))
        return out

    # ---- per-frequency H-matrices
    def aca_blocks(self, tol: float, max_rank: int, precision: int, flags: int = FLAG_RECOMPRESS,
                   freq_idx=None) -> AcaStats:
        st = AcaStats()
        if freq_idx is None:
            pf, nf = None, 0
        else:
            fi, pf = _host(freq_idx, np.int32)
            nf = len(fi)
        code = _check(_lib.gcq_aca_blocks(self._h, pf, nf, float(tol), int(max_rank), precision,
                                          flags, C.byref(st)))
        st.status = code
        return st

    def get_block_factors(self, block: int, freq: int, cap: int = 256):
        m = self.n  # upper bound on block dimensions
        _, blocks = self.get_tree() if not hasattr(self, "_blocks") else (None, self._blocks)
        self._blocks = blocks
        rb, re, cb, ce, _ = blocks[block]
        U = np.zeros((cap, re - rb), np.complex128)
        V = np.zeros((cap, ce - cb), np.complex128)
        r = C.c_int32()
        _check(_lib.gcq_get_block_factors(self._h, block, freq, U.ctypes.data_as(C.c_void_p),
                                          V.ctypes.data_as(C.c_void_p), cap, C.byref(r)))
        k = r.value
        return U[:k].T.copy(), V[:k].T.copy()

    # ---- 3D-ACA
    def aca_ranks(self, n_slots: int):
        """Ranks of the last aca_blocks call, (n_far, n_slots) int32."""
        nfar = self.tree_info.n_far
        out = np.zeros((nfar, n_slots), np.int32)
        _check(_lib.gcq_aca_ranks(self._h, out.ctypes.data_as(C.c_void_p), int(nfar * n_slots)))
        return out

    def aca3d(self, tol_aca: float, tol: float, max_freq_rank: int, precision: int,
              flags: int = 0) -> Aca3dStats:
        st = Aca3dStats()
        code = _check(_lib.gcq_aca3d(self._h, float(tol_aca), float(tol), int(max_freq_rank),
                                     precision, flags, C.byref(st)))
        self.F_precision = precision
        st.status = code
        return st

    def aca3d_ranks(self):
        """Per block of the partition: the number of 3D-ACA terms and, for an
        admissible block, the sum of its slices' ranks; two int32 arrays."""
        nb = int(self.get_tree()[1].shape[0])
        terms = np.zeros(nb, np.int32)
        cols = np.zeros(nb, np.int32)
        _check(_lib.gcq_aca3d_ranks(self._h, terms.ctypes.data_as(C.c_void_p),
                                    cols.ctypes.data_as(C.c_void_p), nb))
        return terms, cols

    def get_aca3d_block(self, block: int, nK: int, cap: int = 64):
        if not hasattr(self, "_blocks"):
            self._blocks = self.get_tree()[1]
        rb, re, cb, ce, _ = self._blocks[block]
        m, n = re - rb, ce - cb
        rank = C.c_int32()
        freqs = np.zeros(cap, np.int32)
        fib = np.zeros((cap, nK), np.complex128)
        sl = np.zeros((cap, n, m), np.complex128)
        _check(_lib.gcq_get_aca3d_block(self._h, block, cap, C.byref(rank),
                                        freqs.ctypes.data_as(C.c_void_p),
                                        fib.ctypes.data_as(C.c_void_p),
                                        sl.ctypes.data_as(C.c_void_p)))
        r = rank.value
        # slices: (r, m, n) row-major view of the column-major storage
        return freqs[:r].copy(), fib[:r].copy(), np.transpose(sl[:r], (0, 2, 1)).copy()

    # ---- FMM-based 3D-ACA
    def fmm3d(self, order: int, tol: float, max_freq_rank: int, precision: int) -> Fmm3dStats:
        """Chebyshev interpolation of `order` nodes per dimension on the far
        blocks, their M2L operators compressed over the frequencies (Alg. 1)."""
        st = Fmm3dStats()
        _check(_lib.gcq_fmm3d(self._h, int(order), float(tol), int(max_freq_rank), precision, C.byref(st)))
        self.fmm_order = int(order)
        self.fmm_precision = precision
        return st

    def fmm3d_matvec(self, X, Y):
        """Y[k] = V~(s_k) X[k] with the FMM-based operator (device tensors of
        L x n complex values in the precision of fmm3d)."""
        import torch
        dt = torch.complex128 if getattr(self, "fmm_precision", C64) == C128 else torch.complex64
        px = _dev(X, dt, self.L * self.n, "X")
        py = _dev(Y, dt, self.L * self.n, "Y")
        _check(_lib.gcq_fmm3d_matvec(self._h, px, py))
        return Y

    def get_fmm3d_block(self, block: int, nK: int, cap: int = 64):
        """(freqs, fibers (r, |K|), slices (r, p^3, p^3) row-major) of a far
        block's M2L 3D-ACA."""
        np3 = self.fmm_order ** 3
        rank = C.c_int32()
        freqs = np.zeros(cap, np.int32)
        fib = np.zeros((cap, nK), np.complex128)
        sl = np.zeros((cap, np3, np3), np.complex128)
        _check(_lib.gcq_get_fmm3d_block(self._h, int(block), cap, C.byref(rank),
                                        freqs.ctypes.data_as(C.c_void_p),
                                        fib.ctypes.data_as(C.c_void_p),
                                        sl.ctypes.data_as(C.c_void_p)))
        r = rank.value
        # column-major p^3 x p^3 slices: the stored array is the transpose
        return freqs[:r].copy(), fib[:r].copy(), np.transpose(sl[:r], (0, 2, 1)).copy()

    # ---- products and solve
    def sample_rows(self, rows, freq: int, out):
        """Rows of the compressed operator at frequency ``freq`` into ``out``
        (device tensor of len(rows) x n complex values, the operator's
        precision) -- gcq_sample_rows."""
        import torch
        rh, pr = _host(rows, np.int32)
        dt = torch.complex128 if self.F_precision == C128 else torch.complex64
        po = _dev(out, dt, len(rh) * self.n, "out")
        _check(_lib.gcq_sample_rows(self._h, pr, len(rh), int(freq), po))
        return out

    def compressed_matvec(self, mode: int, precision: int, X, Y):
        import torch
        dt = torch.complex128 if precision == C128 else torch.complex64
        px = _dev(X, dt, self.L * self.n, "X")
        py = _dev(Y, dt, (self.n if mode == WEIGHTED_SUM else self.L * self.n), "Y")
        _check(_lib.gcq_compressed_matvec(self._h, mode, precision, px, py, self.L))
        return Y

    def gcq_convolve(self, dt, w, Q, F, precision: int = C128, n_step_points: int = 1, A=None):
        """Forward gCQ convolution (gcq_gcq_convolve): dt the step sizes (a
        number for constant steps), A the Butcher matrix (None: implicit
        Euler), Q, F device float64 tensors of n_steps x m x n, w the contour
        weights (host)."""
        import torch
        Ah, pa, m = self._butcher(A)
        n_steps = Q.numel() // (m * self.n)
        dth, pd = _host(np.broadcast_to(np.asarray(dt, np.float64), (n_steps,)), np.float64)
        wh, pw = self._weights(w, n_step_points)
        pq = _dev(Q, torch.float64, n_steps * m * self.n, "Q")
        pf = _dev(F, torch.float64, n_steps * m * self.n, "F")
        _check(_lib.gcq_gcq_convolve(self._h, pa, m, pd, int(n_steps), int(n_step_points), pw, precision,
                                     pq, pf))
        return F

    def gcq_solve(self, dt, w, F, Q, precision: int = C128, rtol: float = 1e-8,
                  max_iter: int = 300, restart: int = 50, n_step_points: int = 1, A=None) -> int:
        """Densities of the gCQ scheme for given f (gcq_gcq_solve): F, Q device
        float64 tensors of n_steps x m x n; returns the largest GMRES count.
        The call's status is kept in ``last_status`` (NOT_CONVERGED, with a
        RuntimeWarning, when some step's solve ended above rtol)."""
        import torch
        Ah, pa, m = self._butcher(A)
        n_steps = F.numel() // (m * self.n)
        dth, pd = _host(np.broadcast_to(np.asarray(dt, np.float64), (n_steps,)), np.float64)
        wh, pw = self._weights(w, n_step_points)
        pf = _dev(F, torch.float64, n_steps * m * self.n, "F")
        pq = _dev(Q, torch.float64, n_steps * m * self.n, "Q")
        it = C.c_int32(0)
        code = _check(_lib.gcq_gcq_solve(self._h, pa, m, pd, int(n_steps), int(n_step_points), pw,
                                         precision, pf, pq, float(rtol), int(max_iter), int(restart),
                                         C.byref(it)))
        self.last_status = code
        if code == NOT_CONVERGED:
            import warnings
            warnings.warn("gcq_gcq_solve: the solve of some step ended above rtol", RuntimeWarning)
        return it.value

    def _weights(self, w, n_step_points):
        # one contour weight per frequency after the step points
        wh, pw = _host(np.asarray(w).reshape(-1), np.complex128)
        if wh.size != self.L - int(n_step_points):
            raise ValueError(f"w holds {wh.size} weights; the set has {self.L - int(n_step_points)} "
                             f"contour points after {int(n_step_points)} step points")
        return wh, pw

    @staticmethod
    def _butcher(A):
        A = np.ones((1, 1)) if A is None else np.asarray(A, np.float64)
        if A.ndim != 2 or A.shape[0] != A.shape[1]:
            raise ValueError("A must be a square Butcher matrix")
        Ah, pa = _host(A, np.float64)
        return Ah, pa, int(A.shape[0])

    def solve(self, B, X, rtol: float = 1e-6, max_iter: int = 500, restart: int = 50,
              precision: int = C64) -> SolveStats:
        import torch
        pb = _dev(B, torch.complex128, self.L * self.n, "B")
        px = _dev(X, torch.complex128, self.L * self.n, "X")
        st = SolveStats()
        code = _check(_lib.gcq_solve(self._h, pb, px, float(rtol), int(max_iter), int(restart),
                                     precision, C.byref(st)))
        st.status = code
        return st

    # ---- rank model
    def rank_features(self, freq_idx, n_far: int):
        fi, pf = _host(freq_idx, np.int32)
        out = np.zeros((n_far, len(fi), 5), np.float32)
        _check(_lib.gcq_rank_features(self._h, pf, len(fi), out.ctypes.data_as(C.c_void_p)))
        return out

    def rank_model_train(self, feat, target, epochs=30, batch=1024, lr=1e-3, beta1=0.9,
                         beta2=0.999, eps=1e-8, seed=0) -> TrainStats:
        feat, pfe = _host(feat, np.float32)
        target, pt = _host(target, np.float32)
        cfg = TrainCfg(epochs, batch, lr, beta1, beta2, eps, seed)
        st = TrainStats()
        _check(_lib.gcq_rank_model_train(self._h, pfe, pt, len(target), C.byref(cfg),
                                         C.byref(st)))
        return st

    def rank_model_grad(self, feat_std, target):
        feat_std, pfe = _host(feat_std, np.float32)
        target, pt = _host(target, np.float32)
        loss = np.zeros(1, np.float32)
        grad = np.zeros(N_MODEL_PARAMS, np.float32)
        _check(_lib.gcq_rank_model_grad(self._h, pfe, pt, len(target),
                                        loss.ctypes.data_as(C.c_void_p),
                                        grad.ctypes.data_as(C.c_void_p)))
        return float(loss[0]), grad

    def rank_model_predict(self, feat):
        feat, pfe = _host(feat, np.float32)
        out = np.zeros(len(feat), np.float32)
        _check(_lib.gcq_rank_model_predict(self._h, pfe, len(feat),
                                           out.ctypes.data_as(C.c_void_p)))
        return out

    def rank_model_get(self):
        p = np.zeros(N_MODEL_PARAMS, np.float32)
        mu = np.zeros(5, np.float32)
        sd = np.zeros(5, np.float32)
        _check(_lib.gcq_rank_model_get(self._h, p.ctypes.data_as(C.c_void_p),
                                       mu.ctypes.data_as(C.c_void_p),
                                       sd.ctypes.data_as(C.c_void_p)))
        return p, mu, sd

    def rank_model_set(self, params, mean=None, std=None):
        params, pp = _host(params, np.float32)
        pm = _host(mean, np.float32)[1] if mean is not None else None
        ps = _host(std, np.float32)[1] if std is not None else None
        _check(_lib.gcq_rank_model_set(self._h, pp, pm, ps))
