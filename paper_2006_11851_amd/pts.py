"""Python binding of libpts (the C ABI in include/pts.h).

Argument marshalling only: every step of the search, blend and energy runs
in the HIP kernels of libpts.so.  The functions keep the C names
(``pts_estep`` ...); ``Context`` wraps them for torch tensors, passing
``data_ptr()`` and the current torch stream.  There is no fallback: if the
library is missing or the device is not a gfx950, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpts.so")

PTS_OK = 0
PTS_ERR_ARG = -1
PTS_ERR_STATE = -2
PTS_ERR_OOM = -3
PTS_ERR_HIP = -4
PTS_ERR_UNSUPPORTED = -5

MODE_EXACT_FULL = 0
MODE_EXACT_PCA = 1
MODE_TREE = 2
MODE_BRUTE_BF16 = 3
MODE_LEARNED = 4
MODE_LEARNED_BF16 = 5
MODE_LEARNED_BF16_CLASS = 6
MODES = {
    "exact_full": MODE_EXACT_FULL,
    "exact_pca": MODE_EXACT_PCA,
    "tree": MODE_TREE,
    "brute_bf16": MODE_BRUTE_BF16,
    "learned": MODE_LEARNED,
    "learned_bf16": MODE_LEARNED_BF16,
    "learned_bf16_class": MODE_LEARNED_BF16_CLASS,
}


class PtsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libpts error {code}: {msg}")
        self.code = code


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)


class pts_alloc(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("release", RELEASE_FN), ("user", C.c_void_p)]


class TorchAllocator:
    """Serves the library's device memory (exemplar copy, pyramid, index,
    MLP, scratch) from PyTorch's caching allocator on the context's stream.
    ``budget`` (bytes, optional) makes it refuse requests that would exceed
    it, as a full device would: the library then returns PTS_ERR_OOM."""

    def __init__(self, device: int = 0, budget: int | None = None):
        self.device = device
        self.budget = budget
        self.in_use = 0
        self.sizes = {}
        self.refused = 0
        self.calls = 0  # allocation requests received
        self._alloc = ALLOC_FN(self._on_alloc)
        self._release = RELEASE_FN(self._on_release)

    def _on_alloc(self, user, nbytes, stream):
        import torch

        self.calls += 1
        if self.budget is not None and self.in_use + nbytes > self.budget:
            self.refused += 1
            return None
        try:
            ptr = torch.cuda.caching_allocator_alloc(int(nbytes), self.device, stream or None)
        except RuntimeError:
            self.refused += 1
            return None
        self.sizes[ptr] = int(nbytes)
        self.in_use += int(nbytes)
        return ptr

    def _on_release(self, user, ptr, nbytes, stream):
        import torch

        if ptr:
            self.in_use -= self.sizes.pop(ptr, 0)
            torch.cuda.caching_allocator_delete(ptr)

    def struct(self):
        return pts_alloc(self._alloc, self._release, None)


class pts_index_params(C.Structure):
    _fields_ = [
        ("w", C.c_int),
        ("pca_dims", C.c_int),
        ("variance_target", C.c_double),
        ("branching", C.c_int),
        ("depth", C.c_int),
        ("kmeans_max_iter", C.c_int),
        ("seed", C.c_uint64),
        ("make_bf16", C.c_int),
    ]


class pts_index_info(C.Structure):
    _fields_ = [
        ("N", C.c_int64),
        ("D", C.c_int),
        ("d", C.c_int),
        ("retained_variance", C.c_double),
        ("n_nodes", C.c_int),
        ("n_leaves", C.c_int),
        ("leaf_min", C.c_int64),
        ("leaf_max", C.c_int64),
        ("leaf_mean", C.c_double),
        ("build_ms", C.c_double),
    ]


class pts_index_host(C.Structure):
    _fields_ = [
        ("w", C.c_int),
        ("D", C.c_int),
        ("d", C.c_int),
        ("n_nodes", C.c_int),
        ("n_leaves", C.c_int),
        ("N", C.c_int64),
        ("mu", C.POINTER(C.c_double)),
        ("basis", C.POINTER(C.c_double)),
        ("eigenvalues", C.POINTER(C.c_double)),
        ("centroids", C.POINTER(C.c_double)),
        ("first_child", C.POINTER(C.c_int32)),
        ("n_children", C.POINTER(C.c_int32)),
        ("leaf_of_node", C.POINTER(C.c_int32)),
        ("leaf_off", C.POINTER(C.c_int64)),
        ("perm", C.POINTER(C.c_int32)),
    ]


class pts_estep_params(C.Structure):
    _fields_ = [
        ("mode", C.c_int),
        ("w", C.c_int),
        ("stride", C.c_int),
        ("topk", C.c_int),
        ("rerank_full", C.c_int),
        ("n_proposals", C.c_int),
        ("margin", C.c_float),
        ("residual", C.c_int),
        ("scan_slots", C.c_int),
    ]


class pts_estep_stats(C.Structure):
    _fields_ = [("nq", C.c_int64), ("fallbacks", C.c_int64), ("scan_overflows", C.c_int64),
                ("scan_rows", C.c_int64), ("collect_rows", C.c_int64), ("ms", C.c_double)]


class pts_mstep_params(C.Structure):
    _fields_ = [
        ("w", C.c_int),
        ("stride", C.c_int),
        ("r", C.c_float),
        ("delta", C.c_float),
        ("patch_offset", C.c_int),
        ("hist_bins", C.c_int),
    ]


class pts_level_params(C.Structure):
    _fields_ = [
        ("w", C.c_int),
        ("stride", C.c_int),
        ("iters", C.c_int),
        ("pca_dims", C.c_int),
        ("branching", C.c_int),
        ("depth", C.c_int),
    ]


class pts_solve_params(C.Structure):
    _fields_ = [
        ("levels", C.c_int),
        ("level", C.POINTER(pts_level_params)),
        ("mode", C.c_int),
        ("coarse_mode", C.c_int),
        ("topk", C.c_int),
        ("rerank_full", C.c_int),
        ("n_proposals", C.c_int),
        ("margin", C.c_float),
        ("residual", C.c_int),
        ("r", C.c_float),
        ("delta", C.c_float),
        ("patch_offset", C.c_int),
        ("guidance_weight", C.c_float),
        ("seed", C.c_uint64),
        ("kmeans_max_iter", C.c_int),
        ("reuse_finest_index", C.c_int),
        ("hist_bins", C.c_int),
        ("final_hist_match", C.c_int),
        ("scale_map", C.c_int),
        ("slant", C.c_double),
        ("tilt", C.c_double),
    ]


class pts_solve_trace(C.Structure):
    _fields_ = [
        ("capacity", C.c_int),
        ("count", C.c_int),
        ("level", C.POINTER(C.c_int32)),
        ("E", C.POINTER(C.c_double)),
        ("E2", C.POINTER(C.c_double)),
        ("ms", C.POINTER(C.c_double)),
        ("nq", C.POINTER(C.c_int64)),
        ("changes", C.POINTER(C.c_int64)),
        ("fallbacks", C.POINTER(C.c_int64)),
    ]


class pts_train_params(C.Structure):
    _fields_ = [
        ("steps", C.c_int64),
        ("batch", C.c_int),
        ("lr", C.c_float),
        ("beta1", C.c_float),
        ("beta2", C.c_float),
        ("eps", C.c_float),
        ("seed", C.c_uint64),
        ("bf16", C.c_int),
        ("log_every", C.c_int),
    ]


_P = C.c_void_p
_I = C.c_int
_I64 = C.c_int64
_F = C.c_float
_D = C.c_double

# name -> (restype, argtypes)
SIGNATURES = {
    "pts_create": (_I, [C.POINTER(_P), _I, _P, C.POINTER(pts_alloc)]),
    "pts_destroy": (None, [_P]),
    "pts_last_error": (C.c_char_p, [_P]),
    "pts_set_stream": (_I, [_P, _P]),
    "pts_set_exemplar": (_I, [_P, _P, _I, _I]),
    "pts_set_exemplar_u8": (_I, [_P, _P, _I, _I, _F]),
    "pts_fill_guidance": (_I, [_P, _P, _I, _I, _F]),
    "pts_rgbs_from_u8": (_I, [_P, _P, _I, _I, _F, _P]),
    "pts_build_index": (_I, [_P, C.POINTER(pts_index_params), C.POINTER(pts_index_info)]),
    "pts_export_index": (_I, [_P, C.POINTER(pts_index_host)]),
    "pts_import_index": (_I, [_P, C.POINTER(pts_index_host), _I]),
    "pts_estep": (_I, [_P, _P, _I, _I, C.POINTER(pts_estep_params), _P, _P, C.POINTER(pts_estep_stats)]),
    "pts_exact_search": (_I, [_P, _P, _I, _I, _I, _I, _P, _I64, _P, _P]),
    "pts_project": (_I, [_P, _P, _I, _I, _I, _P]),
    "pts_exemplar_projection": (_I, [_P, _P]),
    "pts_leaf_of": (_I, [_P, _P, _I64, _P]),
    "pts_descend": (_I, [_P, _P, _I64, _P]),
    "pts_mstep": (_I, [_P, _P, _P, _P, _I, _I, C.POINTER(pts_mstep_params)]),
    "pts_irls_weights": (_I, [_P, _P, _P, _P, _I, _I, C.POINTER(pts_mstep_params), _P]),
    "pts_histogram_match": (_I, [_P, _P, _I, _I]),
    "pts_scale_guidance": (_I, [_P, _P, _I, _I, _I, _I, _D, _D, _F]),
    "pts_scale_init": (_I, [_P, _P, _I, _I, _P, _I, _I, _I, _P, _D, _D, _F]),
    "pts_energy": (_I, [_P, _P, _I64, _F, _F, C.POINTER(_D), C.POINTER(_D)]),
    "pts_energy_device": (_I, [_P, _P, _I64, _F, _F, _P]),
    "pts_energy_device_noalloc": (_I, [_P, _P, _I64, _F, _F, _P]),
    "pts_solve": (_I, [_P, C.POINTER(pts_solve_params), _P, _I, _I, _P, _I, _I, C.POINTER(pts_solve_trace)]),
    "pts_exemplar_pyramid_level": (_I, [_P, _I, _I, _F, _P]),
    "pts_upsample2": (_I, [_P, _P, _I, _I, _F, _P]),
    "pts_mlp_init": (_I, [_P, _I, _I, _I, C.c_uint64]),
    "pts_mlp_n_params": (_I, [_P, C.POINTER(_I64)]),
    "pts_mlp_get_weights": (_I, [_P, _P]),
    "pts_mlp_set_weights": (_I, [_P, _P]),
    "pts_mlp_set_input_scale": (_I, [_P, _P]),
    "pts_mlp_forward": (_I, [_P, _P, _I64, _I, _P]),
    "pts_mlp_loss_grad": (_I, [_P, _P, _P, _I64, _I, _P, C.POINTER(_F)]),
    "pts_mlp_train": (_I, [_P, _P, _P, _I64, C.POINTER(pts_train_params), _P]),
    "pts_mlp_propose": (_I, [_P, _P, _I64, _I, _P, _P]),
    "pts_eig_sym_top": (_I, [_P, _I, _I, _P, _P, _I]),
    "pts_profile_enable": (_I, [_P, _I]),
    "pts_profile_count": (_I, [_P, C.POINTER(_I)]),
    "pts_profile_read": (_I, [_P, _I, C.c_char_p, _I, C.POINTER(_D), C.POINTER(_I64)]),
}

_lib = None


def lib():
    """Load libpts.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc, ctx=None):
    if rc != PTS_OK:
        msg = lib().pts_last_error(ctx)
        raise PtsError(rc, msg.decode() if msg else "")
    return rc


def _ptr(t):
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        if not t.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return C.c_void_p(t.data_ptr())
    if isinstance(t, np.ndarray):
        if not t.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be C-contiguous")
        return t.ctypes.data_as(C.c_void_p)
    return t


def eig_sym_top(Cm: np.ndarray, d: int, nthreads: int = 0):
    """Host FP64 eigensolve of the library (no device needed)."""
    Cm = np.ascontiguousarray(Cm, dtype=np.float64)
    n = Cm.shape[0]
    ev = np.empty(d, dtype=np.float64)
    vec = np.empty((n, d), dtype=np.float64)
    _check(lib().pts_eig_sym_top(_ptr(Cm), n, d, _ptr(ev), _ptr(vec), nthreads))
    return ev, vec


class Context:
    """One libpts context on a torch device, ordered on the current stream."""

    def __init__(self, device: int = 0, allocator: "TorchAllocator | None" = None):
        """allocator: None = the library's own (hipMalloc); a TorchAllocator
        serves the library's memory from PyTorch's caching allocator."""
        import torch

        self.torch = torch
        self.device = torch.device("cuda", device)
        self._h = C.c_void_p()
        self.allocator = allocator  # kept alive as long as the context
        stream = torch.cuda.current_stream(self.device).cuda_stream
        self._alloc_struct = allocator.struct() if allocator is not None else None
        _check(lib().pts_create(C.byref(self._h), device, C.c_void_p(stream),
                                C.byref(self._alloc_struct) if self._alloc_struct is not None else None), None)
        self.index_info = None

    # -- plumbing
    def close(self):
        if self._h:
            lib().pts_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ok(self, rc):
        return _check(rc, self._h)

    def sync_stream(self):
        self._ok(lib().pts_set_stream(self._h, C.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)))

    def _f32(self, shape):
        return self.torch.empty(shape, dtype=self.torch.float32, device=self.device)

    def _i32(self, shape):
        return self.torch.empty(shape, dtype=self.torch.int32, device=self.device)

    # -- exemplar and images
    def set_exemplar(self, rgbs):
        Hz, Wz = rgbs.shape[:2]
        self._ok(lib().pts_set_exemplar(self._h, _ptr(rgbs), Hz, Wz))
        self.Hz, self.Wz = Hz, Wz

    def set_exemplar_u8(self, u8: np.ndarray, guidance_weight: float = 0.5):
        u8 = np.ascontiguousarray(u8, dtype=np.uint8)
        Hz, Wz = u8.shape[:2]
        self._ok(lib().pts_set_exemplar_u8(self._h, _ptr(u8), Hz, Wz, guidance_weight))
        self.Hz, self.Wz = Hz, Wz

    def rgbs_from_u8(self, u8: np.ndarray, guidance_weight: float = 0.5):
        u8 = np.ascontiguousarray(u8, dtype=np.uint8)
        H, W = u8.shape[:2]
        out = self._f32((H, W, 4))
        self._ok(lib().pts_rgbs_from_u8(self._h, _ptr(u8), H, W, guidance_weight, _ptr(out)))
        return out

    def fill_guidance(self, x, guidance_weight: float = 0.5):
        self._ok(lib().pts_fill_guidance(self._h, _ptr(x), x.shape[0], x.shape[1], guidance_weight))

    # -- index
    def build_index(self, w, pca_dims, branching, depth, seed=0, kmeans_max_iter=50, make_bf16=True,
                    variance_target=0.95):
        p = pts_index_params(w, pca_dims, variance_target, branching, depth, kmeans_max_iter, seed, int(make_bf16))
        info = pts_index_info()
        self._ok(lib().pts_build_index(self._h, C.byref(p), C.byref(info)))
        self.index_info = info
        return info

    def export_index(self) -> dict:
        ix = pts_index_host()
        self._ok(lib().pts_export_index(self._h, C.byref(ix)))
        D, d, nn, nl, N = ix.D, ix.d, ix.n_nodes, ix.n_leaves, ix.N
        out = {
            "w": ix.w, "D": D, "d": d, "N": N, "n_nodes": nn, "n_leaves": nl,
            "mu": np.empty(D), "basis": np.empty((D, d)), "eigenvalues": np.empty(d),
            "centroids": np.empty((nn, d)), "first_child": np.empty(nn, np.int32),
            "n_children": np.empty(nn, np.int32), "leaf_of_node": np.empty(nn, np.int32),
            "leaf_off": np.empty(nl + 1, np.int64), "perm": np.empty(N, np.int32),
        }
        self._fill_host(ix, out)
        self._ok(lib().pts_export_index(self._h, C.byref(ix)))
        return out

    @staticmethod
    def _fill_host(ix, a):
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        ix.mu = a["mu"].ctypes.data_as(dp)
        ix.basis = a["basis"].ctypes.data_as(dp)
        ix.eigenvalues = a["eigenvalues"].ctypes.data_as(dp) if a.get("eigenvalues") is not None else None
        ix.centroids = a["centroids"].ctypes.data_as(dp)
        ix.first_child = a["first_child"].ctypes.data_as(ip)
        ix.n_children = a["n_children"].ctypes.data_as(ip)
        ix.leaf_of_node = a["leaf_of_node"].ctypes.data_as(ip)
        ix.leaf_off = a["leaf_off"].ctypes.data_as(C.POINTER(C.c_int64))
        ix.perm = a["perm"].ctypes.data_as(ip)

    def import_index(self, a: dict, make_bf16=True):
        a = {
            "mu": np.ascontiguousarray(a["mu"], np.float64),
            "basis": np.ascontiguousarray(a["basis"], np.float64),
            "eigenvalues": np.ascontiguousarray(a.get("eigenvalues", np.zeros(np.shape(a["basis"])[1])), np.float64),
            "centroids": np.ascontiguousarray(a["centroids"], np.float64),
            "first_child": np.ascontiguousarray(a["first_child"], np.int32),
            "n_children": np.ascontiguousarray(a["n_children"], np.int32),
            "leaf_of_node": np.ascontiguousarray(a["leaf_of_node"], np.int32),
            "leaf_off": np.ascontiguousarray(a["leaf_off"], np.int64),
            "perm": np.ascontiguousarray(a["perm"], np.int32),
            "w": int(a["w"]),
            "N": int(a["N"]),
        }
        ix = pts_index_host()
        ix.w = a["w"]
        ix.D = a["mu"].size
        ix.d = a["basis"].shape[1]
        ix.n_nodes = a["first_child"].size
        ix.n_leaves = a["leaf_off"].size - 1
        ix.N = a["N"]
        self._fill_host(ix, a)
        self._ok(lib().pts_import_index(self._h, C.byref(ix), int(make_bf16)))

    # -- search / blend / energy
    def nq(self, H, W, w, s):
        return ((H - w) // s + 1) * (W // s)

    def estep(self, x, w, stride, mode="tree", topk=8, rerank_full=0, n_proposals=4, margin=0.2, residual=0,
              stats=False, nn=None, dist=None, scan_slots=0):
        H, W = x.shape[:2]
        nq = self.nq(H, W, w, stride)
        nn = self._i32(nq) if nn is None else nn
        dist = self._f32(nq) if dist is None else dist
        p = pts_estep_params(MODES[mode] if isinstance(mode, str) else mode, w, stride, topk, rerank_full,
                             n_proposals, margin, int(residual), int(scan_slots))
        st = pts_estep_stats()
        self._ok(lib().pts_estep(self._h, _ptr(x), H, W, C.byref(p), _ptr(nn), _ptr(dist),
                                 C.byref(st) if stats else None))
        if stats:
            return nn, dist, st
        return nn, dist

    def exact_search(self, x, w, stride, qids):
        """Exhaustive full-D search of the listed output windows (int32 tensor)."""
        n = qids.numel()
        nn = self._i32(n)
        dist = self._f32(n)
        self._ok(lib().pts_exact_search(self._h, _ptr(x), x.shape[0], x.shape[1], w, stride, _ptr(qids), n, _ptr(nn),
                                        _ptr(dist)))
        return nn, dist

    def project(self, x, stride):
        H, W = x.shape[:2]
        info = self.index_info
        w = self._index_w
        nq = self.nq(H, W, w, stride)
        out = self._f32((nq, self._index_d))
        self._ok(lib().pts_project(self._h, _ptr(x), H, W, stride, _ptr(out)))
        return out

    @property
    def _index_w(self):
        ix = pts_index_host()
        self._ok(lib().pts_export_index(self._h, C.byref(ix)))
        return ix.w

    @property
    def _index_d(self):
        ix = pts_index_host()
        self._ok(lib().pts_export_index(self._h, C.byref(ix)))
        return ix.d

    def exemplar_projection(self):
        ix = pts_index_host()
        self._ok(lib().pts_export_index(self._h, C.byref(ix)))
        out = self._f32((ix.N, ix.d))
        self._ok(lib().pts_exemplar_projection(self._h, _ptr(out)))
        return out

    def leaf_of(self, nn):
        out = self._i32(nn.numel())
        self._ok(lib().pts_leaf_of(self._h, _ptr(nn), nn.numel(), _ptr(out)))
        return out

    def descend(self, qproj):
        out = self._i32(qproj.shape[0])
        self._ok(lib().pts_descend(self._h, _ptr(qproj), qproj.shape[0], _ptr(out)))
        return out

    def mstep(self, nn, dist, x, w, stride, r=0.8, delta=1e-3, patch_offset=0, hist_bins=0):
        p = pts_mstep_params(w, stride, r, delta, patch_offset, hist_bins)
        self._ok(lib().pts_mstep(self._h, _ptr(nn), _ptr(dist), _ptr(x), x.shape[0], x.shape[1], C.byref(p)))

    def irls_weights(self, nn, dist, x, w, stride, r=0.8, delta=1e-3, hist_bins=0):
        p = pts_mstep_params(w, stride, r, delta, 0, hist_bins)
        out = self._f32(nn.numel())
        self._ok(lib().pts_irls_weights(self._h, _ptr(nn), _ptr(dist), _ptr(x), x.shape[0], x.shape[1], C.byref(p),
                                        _ptr(out)))
        return out

    def histogram_match(self, x):
        self._ok(lib().pts_histogram_match(self._h, _ptr(x), x.shape[0], x.shape[1]))

    # -- perspective scale map
    def scale_guidance(self, x, slant, tilt, weight=0.5, ref=None):
        """x's guidance channel = weight * the normalised scale map of an
        image of size ref (default: x's own) resampled to x's size."""
        H, W = x.shape[:2]
        rh, rw = (H, W) if ref is None else ref
        self._ok(lib().pts_scale_guidance(self._h, _ptr(x), H, W, rh, rw, float(slant), float(tilt), weight))
        return x

    def scale_init(self, ex_rgbs, H, W, tile, rnd, slant, tilt, weight=0.5):
        """Scale-matched initial output [H][W][4] from the device exemplar
        ex_rgbs; rnd: device uint32 draws [tiles][2] (int32 storage)."""
        torch = self.torch
        Hz, Wz = ex_rgbs.shape[:2]
        nt = (-(-H // tile)) * (-(-W // tile))
        if rnd.numel() != 2 * nt or rnd.dtype not in (torch.int32, torch.uint32) or not rnd.is_contiguous():
            raise ValueError(f"rnd must hold {nt} x 2 contiguous 32-bit integers")
        out = self._f32((H, W, 4))
        self._ok(lib().pts_scale_init(self._h, _ptr(ex_rgbs), Hz, Wz, _ptr(out), H, W, tile, _ptr(rnd),
                                      float(slant), float(tilt), weight))
        return out

    def energy(self, dist, r=0.8, delta=1e-3):
        E = C.c_double()
        E2 = C.c_double()
        self._ok(lib().pts_energy(self._h, _ptr(dist), dist.numel(), r, delta, C.byref(E), C.byref(E2)))
        return E.value, E2.value

    def energy_device(self, dist, out=None, r=0.8, delta=1e-3):
        """(E, E2) as a float32 device tensor [2], without waiting for it."""
        if out is None:
            out = self._f32((2,))
        self._ok(lib().pts_energy_device(self._h, _ptr(dist), dist.numel(), r, delta, _ptr(out)))
        return out

    def energy_device_noalloc(self, dist, out, r=0.8, delta=1e-3):
        """energy_device without any device allocation: out is the caller's
        float32 device tensor [2]; the partial sums use the library's fixed
        per-device array, so overlapping calls on one device race."""
        self._ok(lib().pts_energy_device_noalloc(self._h, _ptr(dist), dist.numel(), r, delta, _ptr(out)))
        return out

    # -- multiscale
    def pyramid_level(self, levels, level, guidance_weight=0.5):
        h, w = self.Hz >> (levels - 1 - level), self.Wz >> (levels - 1 - level)
        out = self._f32((h, w, 4))
        self._ok(lib().pts_exemplar_pyramid_level(self._h, levels, level, guidance_weight, _ptr(out)))
        return out

    def upsample2(self, x, guidance_weight=0.5):
        H, W = x.shape[:2]
        out = self._f32((2 * H, 2 * W, 4))
        self._ok(lib().pts_upsample2(self._h, _ptr(x), H, W, guidance_weight, _ptr(out)))
        return out

    def solve(self, x0, levels, mode="tree", coarse_mode="tree", topk=8, rerank_full=0, n_proposals=4,
              margin=0.2, residual=0, r=0.8, delta=1e-3, patch_offset=0, guidance_weight=0.5, seed=0,
              kmeans_max_iter=50, reuse_finest_index=False, trace=True, hist_bins=0, final_hist_match=False,
              scale=None):
        """levels: list of dicts with w, stride, iters, pca_dims, branching, depth (coarse to fine);
        scale = (slant, tilt) in radians selects the scale-map guidance."""
        L = len(levels)
        lv = (pts_level_params * L)(*[
            pts_level_params(l["w"], l["stride"], l["iters"], l.get("pca_dims", 0), l.get("branching", 4),
                             l.get("depth", 0)) for l in levels])
        p = pts_solve_params(L, lv, MODES[mode] if isinstance(mode, str) else mode,
                             MODES[coarse_mode] if isinstance(coarse_mode, str) else coarse_mode, topk, rerank_full,
                             n_proposals, margin, int(residual), r, delta, patch_offset, guidance_weight, seed,
                             kmeans_max_iter, int(reuse_finest_index), int(hist_bins), int(final_hist_match),
                             int(scale is not None), *(map(float, scale) if scale is not None else (0.0, 0.0)))
        H0, W0 = x0.shape[:2]
        H, W = H0 << (L - 1), W0 << (L - 1)
        out = self._f32((H, W, 4))
        cap = sum(l["iters"] for l in levels)
        tr = None
        arrs = None
        if trace:
            arrs = {
                "level": np.zeros(cap, np.int32), "E": np.zeros(cap), "E2": np.zeros(cap), "ms": np.zeros(cap),
                "nq": np.zeros(cap, np.int64), "changes": np.zeros(cap, np.int64), "fallbacks": np.zeros(cap, np.int64),
            }
            tr = pts_solve_trace(cap, 0, *[arrs[k].ctypes.data_as(C.POINTER(
                {np.dtype(np.int32): C.c_int32, np.dtype(np.float64): C.c_double,
                 np.dtype(np.int64): C.c_int64}[arrs[k].dtype])) for k in
                ("level", "E", "E2", "ms", "nq", "changes", "fallbacks")])
        self._ok(lib().pts_solve(self._h, C.byref(p), _ptr(x0), H0, W0, _ptr(out), H, W,
                                 C.byref(tr) if tr is not None else None))
        if trace:
            n = tr.count
            return out, {k: v[:n] for k, v in arrs.items()}
        return out, None

    # -- learned proposal
    def mlp_init(self, n_in, hidden, n_out, seed=0):
        self._ok(lib().pts_mlp_init(self._h, n_in, hidden, n_out, seed))

    def mlp_n_params(self):
        n = C.c_int64()
        self._ok(lib().pts_mlp_n_params(self._h, C.byref(n)))
        return n.value

    def mlp_get_weights(self):
        out = np.empty(self.mlp_n_params(), np.float32)
        self._ok(lib().pts_mlp_get_weights(self._h, _ptr(out)))
        return out

    def mlp_set_weights(self, theta):
        theta = np.ascontiguousarray(theta, np.float32)
        self._ok(lib().pts_mlp_set_weights(self._h, _ptr(theta)))

    def mlp_set_input_scale(self, scale):
        scale = np.ascontiguousarray(scale, np.float32)
        self._ok(lib().pts_mlp_set_input_scale(self._h, _ptr(scale)))

    def mlp_forward(self, q, n_out, bf16=False):
        out = self._f32((q.shape[0], n_out))
        self._ok(lib().pts_mlp_forward(self._h, _ptr(q), q.shape[0], int(bf16), _ptr(out)))
        return out

    def mlp_loss_grad(self, q, labels, bf16=False):
        g = self._f32(self.mlp_n_params())
        loss = C.c_float()
        self._ok(lib().pts_mlp_loss_grad(self._h, _ptr(q), _ptr(labels), q.shape[0], int(bf16), _ptr(g),
                                         C.byref(loss)))
        return loss.value, g

    def mlp_train(self, q, labels, steps, batch=4096, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, seed=0,
                  bf16=True, log_every=100):
        p = pts_train_params(steps, batch, lr, beta1, beta2, eps, seed, int(bf16), log_every)
        log = np.zeros(max(1, steps // max(1, log_every)), np.float32)
        self._ok(lib().pts_mlp_train(self._h, _ptr(q), _ptr(labels), q.shape[0], C.byref(p), _ptr(log)))
        return log

    def mlp_propose(self, q, k=4):
        n = q.shape[0]
        leaves = self._i32((n, k))
        margin = self._f32(n)
        self._ok(lib().pts_mlp_propose(self._h, _ptr(q), n, k, _ptr(leaves), _ptr(margin)))
        return leaves, margin

    # -- profiling
    def profile_enable(self, on=True):
        self._ok(lib().pts_profile_enable(self._h, int(on)))

    def profile_read(self) -> dict:
        n = C.c_int()
        self._ok(lib().pts_profile_count(self._h, C.byref(n)))
        out = {}
        buf = C.create_string_buffer(128)
        for i in range(n.value):
            ms = C.c_double()
            cnt = C.c_int64()
            self._ok(lib().pts_profile_read(self._h, i, buf, 128, C.byref(ms), C.byref(cnt)))
            out[buf.value.decode()] = (ms.value, cnt.value)
        return out
