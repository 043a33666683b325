"""ctypes binding of libpepsnet.so (argument marshalling only).

Every computation happens in the HIP library; this module converts numpy
arrays to the C ABI of ``include/pepsnet.h`` and back.  Loading fails loudly
if the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

BBP_KAGOME_OPEN, BBP_KAGOME_INF_HEX = 1, 2
BBP_OK, BBP_NOT_CONVERGED, BBP_PENDING = 0, 1, 2
BBP_EINVAL, BBP_ENOMEM, BBP_EDEVICE = -1, -2, -3
NOALLOC_MAX_BYTES = 128 << 20   # PEPSNET_NOALLOC_MAX_BYTES
BBP_FP64, BBP_FP32, BBP_BF16X3 = 0, 1, 2
BBP_SVD_FULL, BBP_SVD_RAND = 0, 1
ABI_VERSION = 4

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


class PepsnetError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pepsnet error {code}: {msg}")
        self.code = code


class Desc(C.Structure):
    _fields_ = [("abi_version", C.c_int32), ("lattice", C.c_int32),
                ("Lx", C.c_int32), ("Ly", C.c_int32), ("bLx", C.c_int32), ("bLy", C.c_int32),
                ("hex_N", C.c_int32), ("d", C.c_int32), ("D", C.c_int32),
                ("chi", C.c_int32), ("chi_env", C.c_int32), ("precision", C.c_int32),
                ("trunc", C.c_int32), ("rsvd_q", C.c_int32), ("rsvd_p", C.c_int32),
                ("seed", C.c_uint64), ("stream", C.c_void_p), ("hbm_budget_bytes", C.c_int64),
                ("swallow_order", C.c_int32), ("hermitize", C.c_int32),
                ("damping", C.c_double)]


def library_path():
    return os.path.join(_HERE, "libpepsnet.so")


def load_library():
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run paper_2603_13304_amd/build.py "
                          "(or __graft_entry__.build())")
    lib = C.CDLL(path)
    i32, i64, dbl, vp = C.c_int32, C.c_int64, C.c_double, C.c_void_p
    P = C.POINTER
    sig = {
        "pepsnet_create": (i32, [P(Desc), P(dbl), i64, P(vp)]),
        "pepsnet_set_sites": (i32, [vp, P(dbl), i64, i32]),
        "blockbp_sweep": (i32, [vp, i32, dbl, P(i32), P(dbl)]),
        "blockbp_sweep_noalloc": (i32, [vp, i32, dbl, P(i32), P(dbl)]),
        "blockbp_expect": (i32, [vp, i32, P(i32), i32, P(dbl), P(dbl), P(dbl), P(dbl), P(i32)]),
        "pepsnet_bonds": (i32, [vp, P(i32), i32, P(i32)]),
        "blockbp_rho_measures": (i32, [vp, i32, P(i32), P(dbl), P(dbl), P(dbl)]),
        "pepsnet_get_messages": (i32, [vp, P(dbl), i64, P(i64)]),
        "pepsnet_set_messages": (i32, [vp, P(dbl), i64]),
        "pepsnet_message_shape": (i32, [vp, i32, i32, P(i32), P(i32), P(i32), P(i32)]),
        "pepsnet_num_messages": (i32, [vp]),
        "pepsnet_stream": (vp, [vp]),
        "pepsnet_timing": (i32, [vp, i32, P(dbl), P(i64)]),
        "pepsnet_use_graph": (i32, [vp, i32]),
        "pepsnet_use_streams": (i32, [vp, i32]),
        "pepsnet_sweep_stats": (i32, [vp, P(dbl), P(dbl), P(i64)]),
        "pepsnet_profile_sweeps": (i32, [vp, i32, P(dbl), P(i64), P(dbl), P(dbl)]),
        "pepsnet_profile_launches": (i32, [vp, P(dbl), i64, P(i64)]),
        "pepsnet_destroy": (None, [vp]),
        "pepsnet_last_error": (C.c_char_p, []),
        "pepsnet_describe": (i32, [P(Desc), i32, i32, i32, i32, P(i32), P(i32), i64, P(i64)]),
        "pepsnet_batch_create": (i32, [P(vp), i32, vp, P(vp)]),
        "pepsnet_batch_use_graph": (i32, [vp, i32]),
        "blockbp_sweep_batch": (i32, [vp, i32, P(dbl), P(dbl)]),
        "pepsnet_batch_stats": (i32, [vp, P(dbl), P(i64)]),
        "pepsnet_batch_destroy": (None, [vp]),
        "pepsnet_memory": (i32, [vp, P(i64), P(i64)]),
        "pepsnet_autotune": (i32, [vp, C.c_char_p, P(i32), P(i32)]),
        "pepsnet_release_workspace": (i32, [vp]),
        "pepsnet_acquire_workspace": (i32, [vp]),
        "bbp_server_create": (i32, [i64, i32, P(vp)]),
        "bbp_server_submit": (i32, [vp, vp, P(dbl), i64, dbl, i32, P(C.c_uint64)]),
        "bbp_server_poll": (i32, [vp, C.c_uint64, i32, P(dbl), P(dbl), i32, P(i32), P(i32),
                                  P(dbl), P(dbl), P(dbl)]),
        "bbp_server_stats": (i32, [vp, P(i64), P(i32), P(i64), P(i32), P(i64)]),
        "bbp_server_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _LIB = lib
    return lib


def _check(rc):
    if rc < 0:
        raise PepsnetError(rc, _LIB.pepsnet_last_error().decode())
    return rc


def make_desc(lattice, D, chi, Lx=0, Ly=0, bLx=0, bLy=0, hex_N=0, chi_env=None,
              precision=BBP_FP64, trunc=BBP_SVD_FULL, q=2, p=8, seed=0, stream=None, d=2,
              hbm_budget_bytes=0, swallow_order=0, hermitize=False, damping=0.0):
    return Desc(ABI_VERSION, lattice, Lx, Ly, bLx, bLy, hex_N, d, D, chi,
                chi if chi_env is None else chi_env, precision, trunc, q, p, seed,
                stream if stream is None else C.c_void_p(stream), int(hbm_budget_bytes),
                int(swallow_order), int(bool(hermitize)), float(damping))


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _flatten_sites(tensors):
    return np.ascontiguousarray(np.concatenate(
        [np.ascontiguousarray(t, dtype=np.complex128).reshape(-1) for t in tensors])).view(np.float64)


def describe(desc, what, a=0, b=0, open_sites=()):
    lib = load_library()
    op = np.asarray(open_sites, dtype=np.int32)
    n = C.c_int64(0)
    _check(lib.pepsnet_describe(C.byref(desc), what, a, b, len(op),
                                op.ctypes.data_as(C.POINTER(C.c_int32)), None, 0, C.byref(n)))
    buf = np.zeros(max(n.value, 1), np.int32)
    _check(lib.pepsnet_describe(C.byref(desc), what, a, b, len(op),
                                op.ctypes.data_as(C.POINTER(C.c_int32)),
                                buf.ctypes.data_as(C.POINTER(C.c_int32)), n.value, C.byref(n)))
    return buf[:n.value]


class PepsNet:
    """Handle over ``pepsnet_t``: pepsnet_create / blockbp_sweep /
    blockbp_expect with numpy in and out."""

    def __init__(self, desc, tensors):
        self.lib = load_library()
        self.desc = desc
        self._sites = _flatten_sites(tensors)
        h = C.c_void_p()
        _check(self.lib.pepsnet_create(C.byref(desc), _dptr(self._sites), self._sites.size,
                                       C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.pepsnet_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_sites(self, tensors, reset_messages=False):
        s = _flatten_sites(tensors)
        _check(self.lib.pepsnet_set_sites(self.h, _dptr(s), s.size, int(reset_messages)))

    def blockbp_sweep(self, max_sweeps, tol=0.0):
        done, err = C.c_int32(0), C.c_double(0.0)
        rc = _check(self.lib.blockbp_sweep(self.h, max_sweeps, tol, C.byref(done), C.byref(err)))
        return done.value, err.value, rc

    def blockbp_sweep_noalloc(self, max_sweeps, tol=0.0):
        """blockbp_sweep through the library's fixed device workspace (no
        allocation; the handle's own workspace may be released)."""
        done, err = C.c_int32(0), C.c_double(0.0)
        rc = _check(self.lib.blockbp_sweep_noalloc(self.h, max_sweeps, tol, C.byref(done),
                                                   C.byref(err)))
        return done.value, err.value, rc

    def rho_measures(self, bond_ids=None, sigma=None):
        """(negativity, fidelity or None) per bond of the last expectation
        (Eq. res:negativity, Eq. metrics:fidelity against ``sigma``)."""
        n = C.c_int32(0)
        _check(self.lib.pepsnet_bonds(self.h, None, 0, C.byref(n)))
        ids = None if bond_ids is None else np.ascontiguousarray(bond_ids, np.int32)
        nb = n.value if ids is None else ids.size
        sg = None
        if sigma is not None:
            sg = np.ascontiguousarray(np.asarray(sigma, np.complex128).reshape(nb, 4, 4))
        neg, fid = np.zeros(nb), np.zeros(nb)
        _check(self.lib.blockbp_rho_measures(
            self.h, nb, None if ids is None else ids.ctypes.data_as(C.POINTER(C.c_int32)),
            None if sg is None else _dptr(sg.view(np.float64)), _dptr(neg),
            None if sg is None else _dptr(fid)))
        return neg, (fid if sg is not None else None)

    def blockbp_expect(self, bond_ids=None, ops=None):
        """(rho [n, 4, 4], values, energy).  values: <S.S> per bond (real)
        without ``ops``, else an [n, n_ops] complex array of <O_k>; energy is
        None for a bond subset."""
        n = C.c_int32(0)
        _check(self.lib.pepsnet_bonds(self.h, None, 0, C.byref(n)))
        ids = None
        if bond_ids is not None:
            ids = np.ascontiguousarray(bond_ids, np.int32)
        nb = n.value if ids is None else ids.size
        opa = None
        nops = 1
        if ops is not None:
            opa = np.ascontiguousarray(np.asarray(ops, np.complex128).reshape(-1, 4, 4))
            nops = opa.shape[0]
        rho = np.zeros(nb * 32, np.float64)
        out = np.zeros(nb * nops * 2, np.float64)
        e = C.c_double(0.0)
        _check(self.lib.blockbp_expect(
            self.h, nb, None if ids is None else ids.ctypes.data_as(C.POINTER(C.c_int32)),
            nops, None if opa is None else _dptr(opa.view(np.float64)), _dptr(out), _dptr(rho),
            C.byref(e) if ids is None else None, C.byref(n)))
        vals = out.view(np.complex128).reshape(nb, nops)
        vals = vals[:, 0].real.copy() if opa is None else vals.copy()
        return (rho.view(np.complex128).reshape(nb, 4, 4), vals,
                e.value if ids is None else None)

    def bonds(self):
        n = C.c_int32(0)
        _check(self.lib.pepsnet_bonds(self.h, None, 0, C.byref(n)))
        buf = np.zeros(2 * n.value, np.int32)
        _check(self.lib.pepsnet_bonds(self.h, buf.ctypes.data_as(C.POINTER(C.c_int32)),
                                      buf.size, C.byref(n)))
        return [(int(a), int(b)) for a, b in buf.reshape(-1, 2)]

    def num_messages(self):
        return self.lib.pepsnet_num_messages(self.h)

    def message_shapes(self, m):
        l, P, r, n = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(self.lib.pepsnet_message_shape(self.h, m, -1, None, None, None, C.byref(n)))
        out = []
        for j in range(n.value):
            _check(self.lib.pepsnet_message_shape(self.h, m, j, C.byref(l), C.byref(P),
                                                  C.byref(r), C.byref(n)))
            out.append((l.value, P.value, r.value))
        return out

    def get_messages(self):
        """List (per message slot) of lists of site arrays [l, P, r]."""
        n = C.c_int64(0)
        _check(self.lib.pepsnet_get_messages(self.h, None, 0, C.byref(n)))
        buf = np.zeros(n.value, np.float64)
        _check(self.lib.pepsnet_get_messages(self.h, _dptr(buf), buf.size, C.byref(n)))
        z = buf.view(np.complex128)
        out, o = [], 0
        for m in range(self.num_messages()):
            sites = []
            for (l, P, r) in self.message_shapes(m):
                sites.append(z[o:o + l * P * r].reshape(l, P, r).copy())
                o += l * P * r
            out.append(sites)
        return out

    def set_messages(self, msgs):
        flat = np.concatenate([np.ascontiguousarray(x, np.complex128).reshape(-1)
                               for sites in msgs for x in sites]).view(np.float64)
        _check(self.lib.pepsnet_set_messages(self.h, _dptr(flat), flat.size))

    def stream(self):
        return self.lib.pepsnet_stream(self.h)

    def timing(self, reset=False):
        ms, n = C.c_double(0.0), C.c_int64(0)
        _check(self.lib.pepsnet_timing(self.h, int(reset), C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def use_graph(self, on=True):
        _check(self.lib.pepsnet_use_graph(self.h, int(on)))

    def use_streams(self, n):
        """Streams a sweep may use (1-4): independent message updates run
        concurrently; 1 issues every launch on the handle's stream."""
        _check(self.lib.pepsnet_use_streams(self.h, int(n)))

    def memory(self):
        """(resident bytes, workspace bytes)."""
        r, w = C.c_int64(0), C.c_int64(0)
        _check(self.lib.pepsnet_memory(self.h, C.byref(r), C.byref(w)))
        return r.value, w.value

    def autotune(self, cache_path=None):
        """Pick the fastest GEMM tile shape per GEMM shape of the sweep plans
        (cached in ``cache_path``); returns (shapes timed now, shapes tuned)."""
        nt, ns = C.c_int32(0), C.c_int32(0)
        _check(self.lib.pepsnet_autotune(self.h, None if cache_path is None else
                                         os.fsencode(cache_path), C.byref(nt), C.byref(ns)))
        return nt.value, ns.value

    def release_workspace(self):
        _check(self.lib.pepsnet_release_workspace(self.h))

    def acquire_workspace(self):
        _check(self.lib.pepsnet_acquire_workspace(self.h))

    def sweep_stats(self):
        cf, gf, nl = C.c_double(0.0), C.c_double(0.0), C.c_int64(0)
        _check(self.lib.pepsnet_sweep_stats(self.h, C.byref(cf), C.byref(gf), C.byref(nl)))
        return cf.value, gf.value, nl.value

class Batch:
    """Batched sweeps over several handles (pepsnet_batch_*): one launch
    sequence serves the same stage of every handle's message updates."""

    def __init__(self, nets, stream=None):
        self.lib = load_library()
        self.nets = list(nets)          # keep the handles alive
        arr = (C.c_void_p * len(self.nets))(*[n.h.value for n in self.nets])
        h = C.c_void_p()
        _check(self.lib.pepsnet_batch_create(arr, len(self.nets),
                                             None if stream is None else C.c_void_p(stream),
                                             C.byref(h)))
        self.h = h

    def use_graph(self, on=True):
        _check(self.lib.pepsnet_batch_use_graph(self.h, int(on)))

    def sweep(self, n=1):
        errs = np.zeros(len(self.nets))
        ms = C.c_double(0.0)
        _check(self.lib.blockbp_sweep_batch(self.h, n, _dptr(errs), C.byref(ms)))
        return errs, ms.value

    def stats(self):
        gf, nl = C.c_double(0.0), C.c_int64(0)
        _check(self.lib.pepsnet_batch_stats(self.h, C.byref(gf), C.byref(nl)))
        return gf.value, nl.value

    def close(self):
        if getattr(self, "h", None):
            self.lib.pepsnet_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Serving loop (bbp_server_*): continuous batching of expectation
    requests on resident states under an HBM budget."""

    def __init__(self, hbm_budget_bytes, max_inflight):
        self.lib = load_library()
        h = C.c_void_p()
        _check(self.lib.bbp_server_create(int(hbm_budget_bytes), int(max_inflight), C.byref(h)))
        self.h = h
        self._keep = {}

    def submit(self, net, sites=None, tol=1e-8, max_sweeps=50):
        t = C.c_uint64(0)
        if sites is None:
            _check(self.lib.bbp_server_submit(self.h, net.h, None, 0, tol, max_sweeps, C.byref(t)))
        else:
            flat = _flatten_sites(sites)
            _check(self.lib.bbp_server_submit(self.h, net.h, _dptr(flat), flat.size, tol, max_sweeps,
                                              C.byref(t)))
        self._keep[t.value] = net
        return t.value

    def poll(self, ticket, wait=True):
        """None while pending, else a dict with the request's results."""
        e, err, lat = C.c_double(0.0), C.c_double(0.0), C.c_double(0.0)
        nb, sw = C.c_int32(0), C.c_int32(0)
        ss = np.zeros(256)
        win = np.zeros(2)
        rc = self.lib.bbp_server_poll(self.h, C.c_uint64(ticket), int(wait), C.byref(e), _dptr(ss),
                                      ss.size, C.byref(nb), C.byref(sw), C.byref(err), C.byref(lat),
                                      _dptr(win))
        if rc == BBP_PENDING:
            return None
        self._keep.pop(ticket, None)
        _check(rc)
        return {"rc": rc, "energy": e.value, "ss": ss[:nb.value].copy(), "sweeps": sw.value,
                "err": err.value, "latency_s": lat.value,
                "gpu_window_ms": (float(win[0]), float(win[1]))}

    def stats(self):
        pb, pi, done, q = C.c_int64(0), C.c_int32(0), C.c_int64(0), C.c_int32(0)
        na = C.c_int64(0)
        _check(self.lib.bbp_server_stats(self.h, C.byref(pb), C.byref(pi), C.byref(done), C.byref(q),
                                         C.byref(na)))
        return {"peak_bytes": pb.value, "peak_inflight": pi.value, "completed": done.value,
                "queued": q.value, "slot_allocations": na.value}

    def close(self):
        if getattr(self, "h", None):
            self.lib.bbp_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


PROFILE_KINDS = ["gemm", "transpose", "qr", "jacobi", "sketch", "norm", "pad", "msg_phase",
                 "split_gauge", "chol", "ksum"]
PREC_NAMES = ["fp64", "fp32", "bf16x3"]


def profile_sweeps(net, n_sweeps):
    """Per-kernel HIP-event timing of ``n_sweeps`` sweeps: dict slot name ->
    (ms, launches, flops, bytes)."""
    n = 33
    ms = np.zeros(n)
    nl = np.zeros(n, np.int64)
    fl = np.zeros(n)
    by = np.zeros(n)
    _check(net.lib.pepsnet_profile_sweeps(net.h, n_sweeps, _dptr(ms),
                                          nl.ctypes.data_as(C.POINTER(C.c_int64)),
                                          _dptr(fl), _dptr(by)))
    out = {}
    for k in range(n):
        if nl[k]:
            kind, prec = PROFILE_KINDS[k // 3], k % 3
            name = f"{kind}_{PREC_NAMES[prec]}" if kind == "gemm" else kind
            if kind == "qr" and prec == 1:
                name = "qr_tall"
            if kind == "jacobi" and prec == 1:
                name = "svd_bidiag"
            if kind == "jacobi" and prec == 2:
                name = "svd_top"
            out[name] = (float(ms[k]), int(nl[k]), float(fl[k]), float(by[k]))
    return out


def profile_launches(net):
    """One sweep timed launch by launch: array [n, 10] of (kind, precision,
    variant, items, M, N, K, flops, bytes, ms)."""
    n = C.c_int64(0)
    _check(net.lib.pepsnet_profile_launches(net.h, None, 0, C.byref(n)))
    rec = np.zeros(10 * n.value)
    _check(net.lib.pepsnet_profile_launches(net.h, _dptr(rec), rec.size, C.byref(n)))
    return rec.reshape(-1, 10)
