"""Python binding of libspnet (the C ABI in include/spnet.h): argument
marshalling only. Every step of the solve runs in the library's HIP kernels;
torch is used only for device memory and streams.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# SPNET_LIB selects another build of the library (the sanitizer build of build.py)
LIB_PATH = os.environ.get("SPNET_LIB") or os.path.join(_HERE, "libspnet.so")

SN_OK, SN_EINVAL, SN_ENOMEM, SN_EDEVICE, SN_ESINGULAR, SN_ENOTSPD, SN_ENOCONV, SN_EBUSY = 0, -1, -2, -3, -4, -5, -6, -7
MODEL_HEAT, MODEL_TRUSS, MODEL_BEAM = 0, 1, 2
STARS_ALL, STARS_FREE = 0, 1
FP64, FP32_STARS, FP32_STARS_COARSE = 0, 1, 2

_P = C.c_void_p
_i64, _i32, _dbl = C.c_int64, C.c_int32, C.c_double


class SolveOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("max_iter", C.c_int64), ("fixed_iters", C.c_int64),
                ("replace_every", C.c_int64), ("check_every", C.c_int32), ("device_ptrs", C.c_int32),
                ("use_u0", C.c_int32), ("use_graph", C.c_int32), ("stream", C.c_void_p)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int64), ("res_rec", C.c_double), ("res_true", C.c_double),
                ("converged", C.c_int32), ("replacements", C.c_int32), ("ms", C.c_double)]

    def asdict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class FactorInfo(C.Structure):
    _fields_ = [("star_factor_nnz", C.c_int64), ("star_rcm_nnz", C.c_int64), ("star_envelope", C.c_int64),
                ("star_stored", C.c_int64), ("star_blob_bytes", C.c_int64), ("star_index_bytes", C.c_int64),
                ("star_stream_bytes", C.c_int64), ("coarse_bytes", C.c_int64), ("device_bytes", C.c_int64),
                ("max_star_dofs", C.c_int32), ("max_band", C.c_int32), ("max_levels", C.c_int32),
                ("pad0", C.c_int32), ("factor_seconds", C.c_double), ("sweep_bytes", C.c_int64),
                ("sweep_bytes_sn", C.c_int64), ("spmv_bytes", C.c_int64), ("sweep_flops", C.c_int64),
                ("max_pivot_ratio", C.c_double), ("star_precision", C.c_int32), ("coarse_precision", C.c_int32),
                ("coarse_pivot_ratio", C.c_double)]

    def asdict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad0"}


class EngineInfo(C.Structure):
    _fields_ = [("star_sn", C.c_int32), ("star_waves_per_simd", C.c_int32), ("star_band_lds", C.c_int32),
                ("star_lds_bytes", C.c_int32), ("star_cols_per_wave", C.c_int32), ("star_waves", C.c_int32),
                ("star_big", C.c_int32), ("star_big_lds_bytes", C.c_int32), ("star_global", C.c_int32),
                ("star_band_prio", C.c_int32), ("star_global_waves", C.c_int32),
                ("star_big_index_global", C.c_int32), ("star_twins", C.c_int32), ("coarse_first", C.c_int32),
                ("coarse_kernel", C.c_int32),
                ("coarse_late", C.c_int32), ("star_band_queue", C.c_int32),
                ("sweep_bytes", C.c_int64), ("star_sweep_us", C.c_double),
                ("b_apply_us", C.c_double)]

    def asdict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class KernelStats(C.Structure):
    _fields_ = [("sweep_launches", C.c_int64), ("sweep_ms", C.c_double), ("iterations", C.c_int64),
                ("coarse_launches", C.c_int64), ("coarse_ms", C.c_double), ("coarse_flops", C.c_int64)]

    def asdict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerOpts(C.Structure):
    _fields_ = [("hbm_budget", C.c_int64), ("max_columns", C.c_int32), ("iters_per_tick", C.c_int32),
                ("precision", C.c_int32), ("use_graph", C.c_int32)]


# sn_alloc_fn / sn_free_fn of include/spnet.h
ALLOC_FN = C.CFUNCTYPE(_P, C.c_size_t, C.c_int, _P)
FREE_FN = C.CFUNCTYPE(None, _P, C.c_size_t, C.c_int, _P)


class SpnetError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"spnet status {code}: {msg}")
        self.code = code


_lib = None

# name -> (restype, argtypes); the exported surface of include/spnet.h
SIGNATURES = {
    "sn_last_error": (C.c_char_p, []),
    "sn_set_allocator": (C.c_int, [ALLOC_FN, FREE_FN, _P]),
    "sn_version": (C.c_char_p, []),
    "sn_network_from_segments": (C.c_int, [C.c_int, _i64, _P, _dbl, _dbl, C.c_int, C.c_int, _dbl, C.POINTER(_P)]),
    "sn_network_from_arrays": (C.c_int, [C.c_int, _i64, _P, _i64, _P, _P, C.POINTER(_P)]),
    "sn_network_info": (C.c_int, [_P, C.POINTER(C.c_int), C.POINTER(_i64), C.POINTER(_i64)]),
    "sn_network_export": (C.c_int, [_P, _P, _P, _P]),
    "sn_network_destroy": (None, [_P]),
    "sn_network_diagnostics": (C.c_int, [_P, C.c_int, _dbl, C.POINTER(_dbl), C.POINTER(_dbl), _P, _P]),
    "sn_assemble": (C.c_int, [_P, C.c_int, _P, C.POINTER(_P)]),
    "sn_assemble_beam": (C.c_int, [_P, C.c_int, _dbl, _dbl, C.POINTER(_P)]),
    "sn_system_apply_full": (C.c_int, [_P, _P, _P]),
    "sn_system_mass": (C.c_int, [_P, _P]),
    "sn_system_info": (C.c_int, [_P, C.POINTER(_i64), C.POINTER(_i64), C.POINTER(C.c_int), C.POINTER(_i64)]),
    "sn_system_export_csr": (C.c_int, [_P, _P, _P, _P]),
    "sn_system_free_nodes": (C.c_int, [_P, _P]),
    "sn_system_destroy": (None, [_P]),
    "sn_precond_build": (C.c_int, [_P, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(_P)]),
    "sn_precond_info": (C.c_int, [_P, C.POINTER(_i64), C.POINTER(_i64), C.POINTER(_i64)]),
    "sn_precond_export_stars": (C.c_int, [_P, _P, _P, _P]),
    "sn_precond_export_coarse": (C.c_int, [_P, _P]),
    "sn_precond_factor": (C.c_int, [_P, C.c_int]),
    "sn_precond_factor_info": (C.c_int, [_P, C.POINTER(FactorInfo)]),
    "sn_precond_destroy": (None, [_P]),
    "sn_solve_opts_default": (None, [C.POINTER(SolveOpts)]),
    "sn_solve": (C.c_int, [_P, C.c_int, _P, _P, C.POINTER(SolveOpts), C.POINTER(SolveInfo)]),
    "sn_precond_profile": (C.c_int, [_P, C.c_int]),
    "sn_precond_kernel_stats": (C.c_int, [_P, C.POINTER(KernelStats)]),
    "sn_precond_engine_info": (C.c_int, [_P, C.c_int, C.POINTER(EngineInfo)]),
    "sn_precond_set_star_split": (C.c_int, [_P, _i64]),
    "sn_precond_set_coarse_launch": (C.c_int, [_P, C.c_int]),
    "sn_precond_set_sn_beyond_lds": (C.c_int, [_P, C.c_int]),
    "sn_precond_set_band_twins": (C.c_int, [_P, _i64]),
    "sn_precond_set_band_queue": (C.c_int, [_P, _i32]),
    "sn_apply_K": (C.c_int, [_P, C.c_int, _P, _P, C.c_int, _P]),
    "sn_apply_B": (C.c_int, [_P, C.c_int, _P, _P, C.c_int, _P]),
    "sn_apply_K_noalloc": (C.c_int, [_P, C.c_int, _P, _P, _P]),
    "sn_server_opts_default": (None, [C.POINTER(ServerOpts)]),
    "sn_server_create": (C.c_int, [C.POINTER(ServerOpts), C.POINTER(_P)]),
    "sn_server_submit": (C.c_int, [_P, _P, C.c_int, _P, _dbl, _i64, C.POINTER(C.c_uint64)]),
    "sn_server_step": (C.c_int, [_P, C.POINTER(_i32), C.POINTER(_i32)]),
    "sn_server_poll": (C.c_int, [_P, C.c_uint64, _P, C.POINTER(SolveInfo)]),
    "sn_server_usage": (C.c_int, [_P, C.POINTER(_i64), C.POINTER(_i32)]),
    "sn_server_run": (C.c_int, [_P, C.c_int]),
    "sn_server_wait": (C.c_int, [_P, C.c_uint64, _dbl]),
    "sn_server_destroy": (None, [_P]),
}


def lib():
    """Load libspnet.so (built in-tree by build.py); fails loudly if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_2207_07488_amd.build` (or "
                              f"__graft_entry__.build()) first")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            if not hasattr(L, name):
                continue
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != SN_OK:
        raise SpnetError(rc, lib().sn_last_error().decode())
    return rc


def _np(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_P)


def _is_torch(x):
    return type(x).__module__.startswith("torch")


# the callbacks the library holds (ctypes frees a callback object that nothing references)
_allocator = None


def set_allocator(alloc=None, free=None):
    """sn_set_allocator: alloc(nbytes, device) -> device address (0 when out of memory) and
    free(address, nbytes, device) take the library's device buffers from now on; with both None
    the library returns to hipMalloc / hipFree."""
    global _allocator
    L = lib()
    if alloc is None and free is None:
        _check(L.sn_set_allocator(C.cast(None, ALLOC_FN), C.cast(None, FREE_FN), None))
        _allocator = None
        return
    if alloc is None or free is None:
        raise ValueError("alloc and free must both be given or both be None")

    def _a(nbytes, device, ctx):
        try:
            return int(alloc(int(nbytes), int(device)) or 0)
        except Exception:  # an exception cannot cross the C boundary: report out of memory
            return 0

    def _f(ptr, nbytes, device, ctx):
        free(int(ptr), int(nbytes), int(device))

    cbs = (ALLOC_FN(_a), FREE_FN(_f))
    _check(L.sn_set_allocator(cbs[0], cbs[1], None))
    _allocator = cbs


def use_torch_allocator(enable=True):
    """Give the library's device buffers from PyTorch's caching allocator (enable=False: hipMalloc)."""
    if not enable:
        set_allocator(None, None)
        return
    import torch

    def alloc(nbytes, device):
        return torch.cuda.caching_allocator_alloc(nbytes, device)

    def free(ptr, nbytes, device):
        torch.cuda.caching_allocator_delete(ptr)

    set_allocator(alloc, free)


class Network:
    """Spatial network G = (N, E) in the unit box with its Dirichlet set (Sec. 2.1)."""

    def __init__(self, handle, dim):
        self.h = handle
        self.dim = dim
        d, n, e = C.c_int(), _i64(), _i64()
        _check(lib().sn_network_info(self.h, C.byref(d), C.byref(n), C.byref(e)))
        self.n_nodes, self.n_edges = n.value, e.value

    @classmethod
    def from_segments(cls, dim, segments, contact_eps=0.0, merge_tol=1e-5, dir_lo=1, dir_hi=1, band=1e-3):
        seg = _np(segments, np.float64)
        h = _P()
        _check(lib().sn_network_from_segments(dim, seg.shape[0], _ptr(seg), contact_eps, merge_tol, dir_lo, dir_hi,
                                              band, C.byref(h)))
        return cls(h, dim)

    @classmethod
    def from_arrays(cls, coords, edges, dirichlet):
        x = _np(coords, np.float64)
        e = _np(edges, np.int32)
        d = _np(dirichlet, np.uint8)
        h = _P()
        _check(lib().sn_network_from_arrays(x.shape[1], x.shape[0], _ptr(x), e.shape[0], _ptr(e), _ptr(d),
                                            C.byref(h)))
        return cls(h, x.shape[1])

    def arrays(self):
        x = np.zeros((self.n_nodes, self.dim))
        e = np.zeros((self.n_edges, 2), dtype=np.int32)
        d = np.zeros(self.n_nodes, dtype=np.uint8)
        _check(lib().sn_network_export(self.h, _ptr(x), _ptr(e), _ptr(d)))
        return x, e, d

    def diagnostics(self, nb, r0=None):
        """Homogeneity and connectivity over nb^dim boxes (Assumption 3.4):
        (sigma, mu, density per box, mu per box); r0 None takes the longest edge."""
        nbox = int(nb) ** self.dim
        dens = np.zeros(nbox)
        mus = np.zeros(nbox)
        sig, mu = _dbl(), _dbl()
        _check(lib().sn_network_diagnostics(self.h, int(nb), 0.0 if r0 is None else float(r0), C.byref(sig),
                                            C.byref(mu), _ptr(dens), _ptr(mus)))
        return sig.value, mu.value, dens, mus

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.sn_network_destroy(self.h)
            self.h = None


class System:
    """K on the free dofs: heat model (eq. 3.3), truss model (eq. 3.4) or beam
    model (eq. 3.4 + eq. 3.5 with ncomp components, tensile stiffness gamma1 and
    wire radius r_w, Sec. 6.3)."""

    def __init__(self, net: Network, model=MODEL_HEAT, gamma=None, ncomp=3, gamma1=1.0, r_w=0.0):
        h = _P()
        if model == MODEL_BEAM:
            _check(lib().sn_assemble_beam(net.h, int(ncomp), float(gamma1), float(r_w), C.byref(h)))
        else:
            g = None if gamma is None else _np(gamma, np.float64)
            _check(lib().sn_assemble(net.h, model, _ptr(g), C.byref(h)))
        self.h, self.net, self.model = h, net, model
        n, nnz, nc, nf = _i64(), _i64(), C.c_int(), _i64()
        _check(lib().sn_system_info(self.h, C.byref(n), C.byref(nnz), C.byref(nc), C.byref(nf)))
        self.n, self.nnz, self.ncomp, self.n_free_nodes = n.value, nnz.value, nc.value, nf.value

    def csr(self):
        rp = np.zeros(self.n + 1, dtype=np.int64)
        ci = np.zeros(self.nnz, dtype=np.int32)
        v = np.zeros(self.nnz)
        _check(lib().sn_system_export_csr(self.h, _ptr(rp), _ptr(ci), _ptr(v)))
        return rp, ci, v

    def free_nodes(self):
        f = np.zeros(self.n_free_nodes, dtype=np.int32)
        _check(lib().sn_system_free_nodes(self.h, _ptr(f)))
        return f

    def apply_full(self, g):
        """Free rows of K applied to g on every node ((n_nodes, ncomp) or flat):
        the right-hand-side term of a non-zero Dirichlet lifting."""
        g = _np(g, np.float64).ravel()
        if g.size != self.net.n_nodes * self.ncomp:
            raise ValueError("g needs n_nodes x ncomp values")
        y = np.zeros(self.n)
        _check(lib().sn_system_apply_full(self.h, _ptr(g), _ptr(y)))
        return y

    def mass(self):
        """(M 1)(x) at every free node (eq. 2.1)."""
        m = np.zeros(self.n_free_nodes)
        _check(lib().sn_system_mass(self.h, _ptr(m)))
        return m

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.sn_system_destroy(self.h)
            self.h = None


class Precond:
    """Coarse space and local spaces (Sec. 2.3, 4.1), factored on the device."""

    def __init__(self, sys: System, nH: int, policy=STARS_ALL, dir_lo=1, dir_hi=1, precision=None):
        h = _P()
        _check(lib().sn_precond_build(sys.h, nH, policy, dir_lo, dir_hi, C.byref(h)))
        self.h, self.sys, self.nH = h, sys, nH
        m0, ns, tot = _i64(), _i64(), _i64()
        _check(lib().sn_precond_info(self.h, C.byref(m0), C.byref(ns), C.byref(tot)))
        self.m0, self.nstars, self.star_total = m0.value, ns.value, tot.value
        self.precision = None
        if precision is not None:
            self.factor(precision)

    def stars(self):
        sp = np.zeros(self.nstars + 1, dtype=np.int64)
        sd = np.zeros(self.star_total, dtype=np.int32)
        sv = np.zeros(self.nstars, dtype=np.int32)
        _check(lib().sn_precond_export_stars(self.h, _ptr(sp), _ptr(sd), _ptr(sv)))
        return sp, sd, sv

    def coarse_vertices(self):
        cv = np.zeros(self.m0 // self.sys.ncomp, dtype=np.int32)
        _check(lib().sn_precond_export_coarse(self.h, _ptr(cv)))
        return cv

    def factor(self, precision=FP64):
        _check(lib().sn_precond_factor(self.h, precision))
        self.precision = precision

    def factor_info(self):
        fi = FactorInfo()
        _check(lib().sn_precond_factor_info(self.h, C.byref(fi)))
        return fi.asdict()

    def engine_info(self, k=1):
        """Launch shape measured for batches of k columns (see sn_engine_info)."""
        ei = EngineInfo()
        _check(lib().sn_precond_engine_info(self.h, k, C.byref(ei)))
        d = ei.asdict()
        d["star_sweep_us"] = round(d["star_sweep_us"], 2)
        d["b_apply_us"] = round(d["b_apply_us"], 2)
        d["coarse_first"] = bool(d["coarse_first"])
        return d

    def set_star_split(self, n_sn):
        """Fix the stars on the supernodal path (the n_sn with most positions);
        n_sn < 0: measure it at the next solve."""
        _check(lib().sn_precond_set_star_split(self.h, int(n_sn)))

    def set_band_twins(self, min_positions):
        """Two-chain band sweeps for stars of at least min_positions (0 never, -1 measured)."""
        _check(lib().sn_precond_set_band_twins(self.h, int(min_positions)))

    def set_band_queue(self, waves):
        """Narrow band sweeps as one persistent launch of `waves` wavefronts (0 off, -1 measured)."""
        _check(lib().sn_precond_set_band_queue(self.h, int(waves)))

    def set_sn_beyond_lds(self, mode):
        """Supernodal stars beyond LDS: 0 global memory, 1 vectors in LDS, -1 measured."""
        _check(lib().sn_precond_set_sn_beyond_lds(self.h, int(mode)))

    def set_coarse_launch(self, mode):
        """Fix the coarse kernel and placement (kernel + 2 placement, see the C
        header); mode < 0: measure them when the next engine is created."""
        _check(lib().sn_precond_set_coarse_launch(self.h, int(mode)))

    # ---------------------------------------------------------------- solves
    def _block(self, a):
        """(array, k, is_device, keepalive)"""
        if _is_torch(a):
            import torch
            if a.is_cuda:
                t = a.contiguous()
                assert t.dtype == torch.float64
                k = 1 if t.dim() == 1 else t.shape[1]
                return t, k, True
            a = a.numpy()
        arr = _np(a, np.float64)
        k = 1 if arr.ndim == 1 else arr.shape[1]
        return arr, k, False

    @staticmethod
    def _addr(a, dev):
        return C.c_void_p(a.data_ptr()) if dev else _ptr(a)

    @staticmethod
    def _stream(dev):
        if not dev:
            return None
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)

    def solve(self, f, u0=None, rtol=1e-8, max_iter=1000, fixed_iters=0, replace_every=0, check_every=8,
              use_graph=False, raise_on_noconv=True):
        """Solve K u = f; f is (n,) or (n, k) numpy or a float64 torch tensor
        (device tensors stay on the device). Returns (u, [info dicts])."""
        fa, k, dev = self._block(f)
        if dev:
            import torch
            u = torch.zeros_like(fa) if u0 is None else u0.clone().contiguous()
        else:
            u = np.zeros_like(fa) if u0 is None else _np(u0, np.float64).copy()
        o = SolveOpts()
        lib().sn_solve_opts_default(C.byref(o))
        o.rtol, o.max_iter, o.fixed_iters, o.replace_every = rtol, max_iter, fixed_iters, replace_every
        o.check_every, o.device_ptrs, o.use_u0, o.use_graph = check_every, int(dev), int(u0 is not None), int(use_graph)
        o.stream = self._stream(dev)
        infos = (SolveInfo * k)()
        rc = lib().sn_solve(self.h, k, self._addr(fa, dev), self._addr(u, dev), C.byref(o), infos)
        if rc == SN_ENOCONV and not raise_on_noconv:
            pass
        else:
            _check(rc)
        return u, [i.asdict() for i in infos]

    def apply_K(self, x):
        xa, k, dev = self._block(x)
        y = (xa.new_zeros(xa.shape) if dev else np.zeros_like(xa))
        _check(lib().sn_apply_K(self.h, k, self._addr(xa, dev), self._addr(y, dev), int(dev), self._stream(dev)))
        return y

    def apply_K_noalloc(self, x, y):
        """y = K x through the library's fixed workspace (no allocation), queued
        on torch's current stream; x and y are float64 CUDA tensors (n,) or (n, k)."""
        assert _is_torch(x) and x.is_cuda and _is_torch(y) and y.is_cuda
        assert x.is_contiguous() and y.is_contiguous() and x.shape == y.shape
        k = 1 if x.dim() == 1 else x.shape[1]
        _check(lib().sn_apply_K_noalloc(self.h, k, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                        self._stream(True)))
        return y

    def apply_B(self, r):
        ra, k, dev = self._block(r)
        z = (ra.new_zeros(ra.shape) if dev else np.zeros_like(ra))
        _check(lib().sn_apply_B(self.h, k, self._addr(ra, dev), self._addr(z, dev), int(dev), self._stream(dev)))
        return z

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.sn_precond_destroy(self.h)
            self.h = None


class Server:
    """Continuous-batching solve server (sn_server_*): requests on factored or
    unfactored preconditioners iterate together, admitted by device memory."""

    def __init__(self, hbm_budget=None, max_columns=8, iters_per_tick=4, precision=FP32_STARS, use_graph=True):
        o = ServerOpts()
        lib().sn_server_opts_default(C.byref(o))
        if hbm_budget is not None:
            o.hbm_budget = int(hbm_budget)
        o.max_columns, o.iters_per_tick, o.precision, o.use_graph = max_columns, iters_per_tick, precision, int(use_graph)
        h = _P()
        _check(lib().sn_server_create(C.byref(o), C.byref(h)))
        self.h = h
        self._keep = {}  # ticket -> (precond, k)

    def submit(self, pre: "Precond", f, rtol=1e-8, max_iter=1000):
        fa = _np(f, np.float64)
        k = 1 if fa.ndim == 1 else fa.shape[1]
        t = C.c_uint64()
        _check(lib().sn_server_submit(self.h, pre.h, k, _ptr(fa), rtol, max_iter, C.byref(t)))
        self._keep[t.value] = (pre, k, fa.shape)
        return t.value

    def step(self):
        a, q = _i32(), _i32()
        _check(lib().sn_server_step(self.h, C.byref(a), C.byref(q)))
        return a.value, q.value

    def poll(self, ticket):
        """(u, [info]) when the request is done, None while it is pending."""
        pre, k, shape = self._keep[ticket]
        rc = lib().sn_server_poll(self.h, ticket, None, None)  # status only
        if rc == SN_EBUSY:
            return None
        if rc != SN_OK:  # a failed request reports its error once
            del self._keep[ticket]
            _check(rc)
        u = np.empty(shape)
        infos = (SolveInfo * k)()
        rc = lib().sn_server_poll(self.h, ticket, _ptr(u), infos)
        del self._keep[ticket]
        _check(rc)
        return u, [i.asdict() for i in infos]

    def usage(self):
        b, n = _i64(), _i32()
        _check(lib().sn_server_usage(self.h, C.byref(b), C.byref(n)))
        return b.value, n.value

    def run(self, enable=True):
        """Start (or stop) the server's own host thread that steps it."""
        _check(lib().sn_server_run(self.h, int(bool(enable))))

    def wait(self, ticket=0, timeout=60.0):
        """Block until `ticket` (0: any request) has a result, at most `timeout`
        seconds; True when a result is ready, False on timeout. The result stays
        for poll()."""
        rc = lib().sn_server_wait(self.h, int(ticket), float(timeout))
        if rc == SN_EBUSY:
            return False
        _check(rc)
        return True

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.sn_server_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


def build_fiber_problem(preset: dict, precision=FP64, policy=STARS_ALL, nH=None, model=None):
    """Network + system + factored preconditioner for a workload preset."""
    from . import workloads as W
    seg = W.fiber_segments(preset["dim"], preset["n_segments"], preset["length"], preset["seed"])
    net = Network.from_segments(preset["dim"], seg, contact_eps=preset.get("contact_eps", 0.0),
                                merge_tol=W.merge_tol(preset["length"]), dir_lo=preset["dir_lo"],
                                dir_hi=preset["dir_hi"], band=W.BAND)
    sys = System(net, preset.get("model", MODEL_HEAT) if model is None else model)
    pre = Precond(sys, preset["nH"] if nH is None else nH, policy, preset["dir_lo"], preset["dir_hi"])
    if precision is not None:
        pre.factor(precision)
    return net, sys, pre
