"""ctypes wrapper of the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the library. It does not import the
library either.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_SANITIZE=1 builds and loads an AddressSanitizer / UndefinedBehaviorSanitizer
# variant (run with LD_PRELOAD=$(gcc -print-file-name=libasan.so))
_SAN = os.environ.get("ORACLE_SANITIZE") == "1"
_SO = os.path.join(_HERE, "liboracle_san.so" if _SAN else "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

i64, i32, dbl, u8 = C.c_int64, C.c_int32, C.c_double, C.c_uint8
P = C.c_void_p


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (plain C11, -ffp-contract=off)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        san = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined"] if _SAN \
            else []
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-ffp-contract=off", "-fPIC", "-shared", *san,
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = C.CDLL(_SO)
        L.orc_last_error.restype = C.c_char_p
        L.orc_net_build.argtypes = [C.c_int, i64, P, dbl, dbl, C.c_int, C.c_int, dbl, C.c_int, C.POINTER(P)]
        L.orc_net_from_arrays.argtypes = [C.c_int, i64, P, i64, P, P, C.POINTER(P)]
        L.orc_net_sizes.argtypes = [P, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)]
        L.orc_net_get.argtypes = [P, P, P, P]
        L.orc_net_free.argtypes = [P]
        L.orc_sys_build.argtypes = [P, C.c_int, P, C.POINTER(P)]
        L.orc_sys_build_beam.argtypes = [P, C.c_int, dbl, dbl, C.POINTER(P)]
        L.orc_sys_apply_full.argtypes = [P, P, P]
        L.orc_sys_mass.argtypes = [P, P]
        L.orc_sys_sizes.argtypes = [P, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)]
        L.orc_sys_get_csr.argtypes = [P, P, P, P]
        L.orc_sys_get_free_nodes.argtypes = [P, P]
        L.orc_sys_free.argtypes = [P]
        L.orc_apply_K.argtypes = [P, P, P]
        L.orc_pre_build.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(P)]
        L.orc_pre_sizes.argtypes = [P, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)]
        L.orc_pre_get_stars.argtypes = [P, P, P, P]
        L.orc_pre_get_coarse_vertices.argtypes = [P, P]
        L.orc_pre_get_P_dense.argtypes = [P, P]
        L.orc_pre_factor.argtypes = [P]
        L.orc_pre_get_K0_dense.argtypes = [P, P]
        L.orc_pre_factor_nnz.argtypes = [P, C.POINTER(i64)]
        L.orc_pre_factor_nnz.restype = i64
        L.orc_pre_star_md_nnz.argtypes = [P]
        L.orc_pre_star_md_nnz.restype = i64
        L.orc_star_solve.argtypes = [P, i64, P, P]
        L.orc_apply_B.argtypes = [P, P, P]
        L.orc_pcg.argtypes = [P, P, P, dbl, i64, i64, P, P, P, C.POINTER(dbl)]
        L.orc_pcg.restype = i64
        L.orc_pre_free.argtypes = [P]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(P) if a is not None else None


class OracleError(RuntimeError):
    pass


def _check(rc):
    if rc < 0:
        raise OracleError(f"oracle status {rc}: {lib().orc_last_error().decode()}")
    return rc


class Network:
    """Spatial network (Sec. 2.1) built from raw segments or given arrays."""

    def __init__(self, handle):
        self.h = handle
        L = lib()
        n, e, s, r = i64(), i64(), i64(), i64()
        L.orc_net_sizes(self.h, C.byref(n), C.byref(e), C.byref(s), C.byref(r))
        self.n_nodes, self.n_edges, self.n_segments_kept, self.n_raw_nodes = n.value, e.value, s.value, r.value

    @classmethod
    def from_segments(cls, dim, seg, contact_eps=0.0, merge_tol=1e-5, dir_lo=1, dir_hi=1, band=1e-3,
                      brute=False):
        seg = np.ascontiguousarray(seg, dtype=np.float64)
        h = P()
        _check(lib().orc_net_build(dim, seg.shape[0], _ptr(seg), contact_eps, merge_tol, dir_lo, dir_hi, band,
                                   int(brute), C.byref(h)))
        obj = cls(h)
        obj.dim = dim
        return obj

    @classmethod
    def from_arrays(cls, coords, edges, dirichlet):
        coords = np.ascontiguousarray(coords, dtype=np.float64)
        edges = np.ascontiguousarray(edges, dtype=np.int32)
        dirichlet = np.ascontiguousarray(dirichlet, dtype=np.uint8)
        h = P()
        dim = coords.shape[1]
        _check(lib().orc_net_from_arrays(dim, coords.shape[0], _ptr(coords), edges.shape[0], _ptr(edges),
                                         _ptr(dirichlet), C.byref(h)))
        obj = cls(h)
        obj.dim = dim
        return obj

    def arrays(self):
        x = np.zeros((self.n_nodes, self.dim))
        e = np.zeros((self.n_edges, 2), dtype=np.int32)
        d = np.zeros(self.n_nodes, dtype=np.uint8)
        lib().orc_net_get(self.h, _ptr(x), _ptr(e), _ptr(d))
        return x, e, d

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_net_free(self.h)
            self.h = None


MODEL_HEAT, MODEL_TRUSS, MODEL_BEAM = 0, 1, 2


class System:
    """K restricted to the free dofs (model 0: heat eq. 3.3, model 1: truss eq.
    3.4, model 2: beams, eq. 3.4 + eq. 3.5 with ncomp components, tensile
    stiffness gamma1 and wire radius r_w as in Sec. 6.3)."""

    def __init__(self, net: Network, model: int = 0, gamma=None, ncomp=3, gamma1=1.0, r_w=0.0):
        self.net = net
        h = P()
        if model == MODEL_BEAM:
            _check(lib().orc_sys_build_beam(net.h, int(ncomp), float(gamma1), float(r_w), C.byref(h)))
        else:
            g = None if gamma is None else np.ascontiguousarray(gamma, dtype=np.float64)
            _check(lib().orc_sys_build(net.h, model, _ptr(g), C.byref(h)))
        self.h = h
        n, nnz, nf = i64(), i64(), i64()
        lib().orc_sys_sizes(self.h, C.byref(n), C.byref(nnz), C.byref(nf))
        self.n, self.nnz, self.n_free_nodes = n.value, nnz.value, nf.value
        self.model = model
        self.ncomp = {0: 1, 1: 3}.get(model, ncomp)

    def apply_full(self, g):
        """(K g) on the free rows for g on every node, shape (n_nodes, ncomp)
        or flat: the lifting term of non-zero Dirichlet data (Sec. 6.3)."""
        g = np.ascontiguousarray(g, dtype=np.float64).ravel()
        y = np.zeros(self.n)
        lib().orc_sys_apply_full(self.h, _ptr(g), _ptr(y))
        return y

    def mass(self):
        """(M 1)(x) at every free node (eq. 2.1)."""
        m = np.zeros(self.n_free_nodes)
        lib().orc_sys_mass(self.h, _ptr(m))
        return m

    def csr(self):
        rp = np.zeros(self.n + 1, dtype=np.int64)
        ci = np.zeros(self.nnz, dtype=np.int32)
        v = np.zeros(self.nnz)
        lib().orc_sys_get_csr(self.h, _ptr(rp), _ptr(ci), _ptr(v))
        return rp, ci, v

    def free_nodes(self):
        f = np.zeros(self.n_free_nodes, dtype=np.int32)
        lib().orc_sys_get_free_nodes(self.h, _ptr(f))
        return f

    def dense(self):
        rp, ci, v = self.csr()
        A = np.zeros((self.n, self.n))
        for i in range(self.n):
            A[i, ci[rp[i]:rp[i + 1]]] += v[rp[i]:rp[i + 1]]
        return A

    def apply_K(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.zeros(self.n)
        lib().orc_apply_K(self.h, _ptr(x), _ptr(y))
        return y

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_sys_free(self.h)
            self.h = None


class Precond:
    """Coarse space V_H and local spaces V_j (Sec. 2.3, 4.1) with their FP64 factors."""

    def __init__(self, sys: System, nH: int, policy: int = 0, dir_lo: int = 1, dir_hi: int = 1,
                 factor: bool = True):
        self.sys = sys
        h = P()
        _check(lib().orc_pre_build(sys.h, nH, policy, dir_lo, dir_hi, C.byref(h)))
        self.h = h
        m0, ns, tot = i64(), i64(), i64()
        lib().orc_pre_sizes(self.h, C.byref(m0), C.byref(ns), C.byref(tot))
        self.m0, self.nstars, self.star_total = m0.value, ns.value, tot.value
        self.nH = nH
        if factor:
            self.factor()

    def factor(self):
        _check(lib().orc_pre_factor(self.h))

    def stars(self):
        sp = np.zeros(self.nstars + 1, dtype=np.int64)
        sd = np.zeros(self.star_total, dtype=np.int32)
        sv = np.zeros(self.nstars, dtype=np.int32)
        lib().orc_pre_get_stars(self.h, _ptr(sp), _ptr(sd), _ptr(sv))
        return sp, sd, sv

    def coarse_vertices(self):
        cv = np.zeros(self.m0 // self.sys.ncomp, dtype=np.int32)
        lib().orc_pre_get_coarse_vertices(self.h, _ptr(cv))
        return cv

    def P_dense(self):
        Pd = np.zeros((self.sys.n, self.m0))
        lib().orc_pre_get_P_dense(self.h, _ptr(Pd))
        return Pd

    def K0_dense(self):
        K0 = np.zeros((self.m0, self.m0))
        _check(lib().orc_pre_get_K0_dense(self.h, _ptr(K0)))
        return K0

    def star_md_nnz(self):
        """Structural non-zeros of all local Cholesky factors under a minimum
        degree order (a measuring stick for factor sizes; not used in solves)."""
        return int(lib().orc_pre_star_md_nnz(self.h))

    def factor_nnz(self):
        c = i64()
        t = lib().orc_pre_factor_nnz(self.h, C.byref(c))
        return t, c.value

    def star_solve(self, st, g):
        g = np.ascontiguousarray(g, dtype=np.float64)
        z = np.zeros_like(g)
        _check(lib().orc_star_solve(self.h, st, _ptr(g), _ptr(z)))
        return z

    def apply_B(self, r):
        r = np.ascontiguousarray(r, dtype=np.float64)
        z = np.zeros(self.sys.n)
        _check(lib().orc_apply_B(self.h, _ptr(r), _ptr(z)))
        return z

    def pcg(self, f, u0=None, rtol=1e-8, max_iter=1000, fixed_iters=0, uref=None, history=False):
        """Returns (u, iters, info) with info = dict(true_res, hist_r, hist_e)."""
        n = self.sys.n
        f = np.ascontiguousarray(f, dtype=np.float64)
        u = np.zeros(n) if u0 is None else np.array(u0, dtype=np.float64)
        cap = (fixed_iters if fixed_iters > 0 else max_iter) + 1
        hr = np.zeros(cap) if history else None
        he = np.zeros(cap) if uref is not None else None
        ur = None if uref is None else np.ascontiguousarray(uref, dtype=np.float64)
        tr = dbl()
        it = lib().orc_pcg(self.h, _ptr(f), _ptr(u), rtol, max_iter, fixed_iters, _ptr(ur), _ptr(hr), _ptr(he),
                           C.byref(tr))
        _check(it)
        info = dict(true_res=tr.value,
                    hist_r=None if hr is None else hr[:it + 1],
                    hist_e=None if he is None else he[:it + 1])
        return u, it, info

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_pre_free(self.h)
            self.h = None
