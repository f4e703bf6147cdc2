"""Thin ctypes binding of liblrh.so (argument marshalling only).

Every step of the message-passing path runs in the HIP library; this module only
converts arguments (numpy problem arrays, torch device tensors, the current HIP
stream) and unpacks the structure-of-arrays message layout for inspection.  The
functions carry the C names; `Problem` bundles them around one built problem.

PyTorch is used for device memory and streams only.  If the library is missing or
cannot be loaded, every entry point raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Dict, Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblrh.so")

LRH_SUBINTERVALS = 0x1
LRH_TWO_LEVEL = 0x2
LRH_F32 = 0x1
LRH_FUSED = 0x2
LRH_PACKED_COTANGENT = 0x4
LRH_MAX_BUCKETS = 8

STATUS = {0: "LRH_OK", 1: "LRH_E_INVALID", 2: "LRH_E_UNSUPPORTED", 3: "LRH_E_NOMEM",
          4: "LRH_E_DEVICE", 5: "LRH_E_NOCONV", 6: "LRH_E_NONFINITE"}


class LrhError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class ProblemDesc(C.Structure):
    _fields_ = [("n_sites", C.c_int32), ("site_dim", C.POINTER(C.c_int32)),
                ("n_terms", C.c_int32), ("term_ptr", C.POINTER(C.c_int64)),
                ("term_sites", C.POINTER(C.c_int32)), ("term_off", C.POINTER(C.c_int64)),
                ("term_re", C.POINTER(C.c_double)), ("term_im", C.POINTER(C.c_double)),
                ("n_top", C.c_int32), ("top_ptr", C.POINTER(C.c_int64)),
                ("top_sites", C.POINTER(C.c_int32)), ("site_instance", C.POINTER(C.c_int32)),
                ("flags", C.c_uint32), ("n_params", C.c_int32), ("term_param", C.POINTER(C.c_int32)),
                ("dterm_re", C.POINTER(C.c_double)), ("dterm_im", C.POINTER(C.c_double)),
                ("params", C.POINTER(C.c_double))]


class Layout(C.Structure):
    _fields_ = [("n_clusters", C.c_int64), ("n_msgs", C.c_int64), ("n_instances", C.c_int64),
                ("is_real", C.c_int32), ("max_D", C.c_int32), ("n_buckets", C.c_int32),
                ("bucket_D", C.c_int32 * LRH_MAX_BUCKETS),
                ("bucket_count", C.c_int64 * LRH_MAX_BUCKETS),
                ("bucket_comps", C.c_int64 * LRH_MAX_BUCKETS),
                ("bucket_offset", C.c_int64 * LRH_MAX_BUCKETS),
                ("nu_len", C.c_int64), ("marg_len", C.c_int64),
                ("Lambda_G", C.c_double), ("Gamma_G", C.c_double), ("max_sweeps", C.c_int32),
                ("n_params", C.c_int32)]


class NesterovState(C.Structure):
    _fields_ = [("k", C.c_int64), ("theta", C.c_double), ("beta", C.c_double), ("L", C.c_double)]


_lib = None

EXPORTS = ["lrh_build_clusters", "lrh_query", "lrh_export_clusters", "lrh_export_messages",
           "lrh_dual_eval", "lrh_step_subgrad", "lrh_step_nesterov", "lrh_certify", "lrh_check",
           "lrh_set_jacobi", "lrh_destroy", "lrh_last_error", "lrh_set_params", "lrh_dual_vjp",
           "lrh_unrolled_bound_grad", "lrh_autotune", "lrh_get_shapes", "lrh_set_shape", "lrh_time_buckets", "lrh_time_messages",
           "lrh_set_slab_limit", "lrh_build_info", "lrh_certify_noalloc", "lrh_measure_fp64_mfma",
           "lrh_certify_fallbacks", "lrh_set_certify_method"]


def load(path: str = LIB_PATH):
    """Load liblrh.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"liblrh.so not built ({path}); run __graft_entry__.build()")
    # torch ships its own HIP runtime under the same soname as the system one.  Whichever is
    # loaded first serves the whole process, so torch is imported before the library: both then
    # share torch's runtime.  Loaded the other way round, torch's own kernel launches run on a
    # runtime they were not built against and crash in the launch.
    import torch  # noqa: F401
    lib = C.CDLL(path)
    mapped = hip_runtimes_mapped()
    if len(mapped) != 1:
        raise RuntimeError(f"expected exactly one HIP runtime in the process, found {mapped}")
    vp, i32, i64, u32, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_double
    sig = {
        "lrh_build_clusters": (i32, [C.POINTER(ProblemDesc), C.c_int, C.POINTER(vp)]),
        "lrh_query": (i32, [vp, C.POINTER(Layout)]),
        "lrh_export_clusters": (i32, [vp, vp, vp, vp]),
        "lrh_export_messages": (i32, [vp, vp, vp, vp, vp]),
        "lrh_dual_eval": (i32, [vp, vp, u32, dbl, vp, vp, vp, vp]),
        "lrh_step_subgrad": (i32, [vp, vp, vp, vp, i64, i32, i32, dbl, vp, u32, vp]),
        "lrh_step_nesterov": (i32, [vp, vp, vp, C.POINTER(NesterovState), i32, u32, vp]),
        "lrh_certify": (i32, [vp, vp, u32, vp, vp, vp, vp]),
        "lrh_certify_noalloc": (i32, [vp, vp, u32, vp, vp, vp, vp]),
        "lrh_check": (i32, [vp, vp, C.POINTER(i64), C.POINTER(i64)]),
        "lrh_set_jacobi": (i32, [vp, i32, dbl]),
        "lrh_set_slab_limit": (i32, [vp, i64]),
        "lrh_certify_fallbacks": (i32, [vp, vp, C.POINTER(i64)]),
        "lrh_set_certify_method": (i32, [vp, i32]),
        "lrh_set_params": (i32, [vp, vp, vp]),
        "lrh_autotune": (i32, [vp, u32, C.c_char_p, vp]),
        "lrh_set_shape": (i32, [vp, i32, i32, i32, u32]),
        "lrh_time_buckets": (i32, [vp, vp, u32, C.c_double, i32, vp, vp]),
        "lrh_time_messages": (i32, [vp, vp, vp, u32, C.c_double, i32, vp, vp]),
        "lrh_get_shapes": (i32, [vp, i32, vp, vp, vp, vp, vp, vp, C.POINTER(i32)]),
        "lrh_dual_vjp": (i32, [vp, vp, u32, dbl, vp, vp, vp, vp, vp]),
        "lrh_unrolled_bound_grad": (i32, [vp, vp, dbl, dbl, i32, vp, vp, vp, vp, u32, vp]),
        "lrh_destroy": (None, [vp]),
        "lrh_last_error": (C.c_char_p, []),
        "lrh_build_info": (C.c_char_p, []),
        "lrh_measure_fp64_mfma": (i32, [C.c_int, C.POINTER(dbl), vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def hip_runtimes_mapped():
    """Distinct libamdhip64 files mapped into this process (Linux /proc/self/maps)."""
    with open("/proc/self/maps") as f:
        return sorted({ln.split()[-1] for ln in f if "libamdhip64" in ln and "/" in ln})


def runtime_info() -> dict:
    """The HIP release the library was compiled against, the one torch ships (and which serves
    the process once torch is imported first), and the runtime files mapped."""
    import torch
    lib = load()
    return dict(library=lib.lrh_build_info().decode(), torch_hip=torch.version.hip,
                mapped=hip_runtimes_mapped())


def _check(code: int):
    if code != 0:
        raise LrhError(code, load().lrh_last_error().decode())


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def _dptr(t) -> Optional[int]:
    """Device pointer of a torch tensor (None passes NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


# ---- C-name wrappers ---------------------------------------------------------------------

def lrh_build_clusters(desc, hip_device: int = 0):
    """Build a problem from an lrh_workloads.ProblemDesc; returns (handle, keep-alive arrays)."""
    lib = load()
    keep = dict(
        site_dim=np.ascontiguousarray(desc.site_dim, dtype=np.int32),
        term_ptr=np.ascontiguousarray(desc.term_ptr, dtype=np.int64),
        term_sites=np.ascontiguousarray(desc.term_sites, dtype=np.int32),
        term_off=np.ascontiguousarray(desc.term_off, dtype=np.int64),
        term_re=np.ascontiguousarray(desc.term_re, dtype=np.float64),
        term_im=None if desc.term_im is None else np.ascontiguousarray(desc.term_im, dtype=np.float64),
        top_ptr=np.ascontiguousarray(desc.top_ptr, dtype=np.int64),
        top_sites=np.ascontiguousarray(desc.top_sites, dtype=np.int32),
        site_instance=np.ascontiguousarray(desc.site_instance, dtype=np.int32),
    )
    npar = 0 if getattr(desc, "params", None) is None else len(desc.params)
    if npar:
        keep["term_param"] = np.ascontiguousarray(desc.term_param, dtype=np.int32)
        keep["dterm_re"] = np.ascontiguousarray(desc.dterm_re, dtype=np.float64)
        keep["dterm_im"] = None if desc.dterm_im is None else np.ascontiguousarray(desc.dterm_im, np.float64)
        keep["params"] = np.ascontiguousarray(desc.params, dtype=np.float64)
    d = ProblemDesc()
    d.n_sites = int(desc.n_sites)
    d.site_dim = _ptr(keep["site_dim"], C.c_int32)
    d.n_terms = int(desc.n_terms)
    d.term_ptr = _ptr(keep["term_ptr"], C.c_int64)
    d.term_sites = _ptr(keep["term_sites"], C.c_int32)
    d.term_off = _ptr(keep["term_off"], C.c_int64)
    d.term_re = _ptr(keep["term_re"], C.c_double)
    d.term_im = None if keep["term_im"] is None else _ptr(keep["term_im"], C.c_double)
    d.n_top = int(desc.n_top)
    d.top_ptr = _ptr(keep["top_ptr"], C.c_int64)
    d.top_sites = _ptr(keep["top_sites"], C.c_int32)
    d.site_instance = _ptr(keep["site_instance"], C.c_int32)
    d.flags = ((LRH_SUBINTERVALS if desc.subintervals else 0)
               | (LRH_TWO_LEVEL if getattr(desc, "two_level", False) else 0))
    d.n_params = npar
    if npar:
        d.term_param = _ptr(keep["term_param"], C.c_int32)
        d.dterm_re = _ptr(keep["dterm_re"], C.c_double)
        d.dterm_im = None if keep["dterm_im"] is None else _ptr(keep["dterm_im"], C.c_double)
        d.params = _ptr(keep["params"], C.c_double)
    h = C.c_void_p()
    _check(lib.lrh_build_clusters(C.byref(d), int(hip_device), C.byref(h)))
    return h


def lrh_query(h) -> Layout:
    out = Layout()
    _check(load().lrh_query(h, C.byref(out)))
    return out


def lrh_dual_eval(h, nu, flags, beta, q, grad=None, marg=None, stream=None):
    _check(load().lrh_dual_eval(h, _dptr(nu), flags, float(beta), _dptr(q), _dptr(grad), _dptr(marg),
                                _stream(stream)))


def lrh_step_subgrad(h, nu, nu_best, q_best, k0, n_iter, step_kind, step_scale, q_hist=None, flags=0,
                     stream=None):
    _check(load().lrh_step_subgrad(h, _dptr(nu), _dptr(nu_best), _dptr(q_best), int(k0), int(n_iter),
                                   int(step_kind), float(step_scale), _dptr(q_hist), flags,
                                   _stream(stream)))


def lrh_step_nesterov(h, nu, zeta, state: NesterovState, n_iter, flags=0, stream=None):
    _check(load().lrh_step_nesterov(h, _dptr(nu), _dptr(zeta), C.byref(state), int(n_iter), flags,
                                    _stream(stream)))


def lrh_certify(h, nu, flags, q, margin, lmin=None, stream=None):
    _check(load().lrh_certify(h, _dptr(nu), flags, _dptr(q), _dptr(margin), _dptr(lmin), _stream(stream)))


def lrh_certify_noalloc(h, nu, flags, q, margin, lmin=None, stream=None):
    _check(load().lrh_certify_noalloc(h, _dptr(nu), flags, _dptr(q), _dptr(margin), _dptr(lmin),
                                      _stream(stream)))


def lrh_check(h, stream=None) -> Tuple[int, int]:
    a, b = C.c_int64(0), C.c_int64(0)
    _check(load().lrh_check(h, _stream(stream), C.byref(a), C.byref(b)))
    return a.value, b.value


def lrh_set_jacobi(h, max_sweeps: int, rel_tol: float = 0.0):
    _check(load().lrh_set_jacobi(h, int(max_sweeps), float(rel_tol)))


def lrh_set_slab_limit(h, max_slabs: int):
    _check(load().lrh_set_slab_limit(h, int(max_slabs)))


def lrh_certify_fallbacks(h, stream=None) -> int:
    n = C.c_int64(0)
    _check(load().lrh_certify_fallbacks(h, _stream(stream), C.byref(n)))
    return int(n.value)


def lrh_set_certify_method(h, method: int):
    _check(load().lrh_set_certify_method(h, int(method)))


def lrh_set_params(h, params, stream=None):
    _check(load().lrh_set_params(h, _dptr(params), _stream(stream)))


def lrh_dual_vjp(h, nu, flags, beta, qbar=None, gbar=None, nu_bar=None, param_bar=None, stream=None):
    _check(load().lrh_dual_vjp(h, _dptr(nu), flags, float(beta), _dptr(qbar), _dptr(gbar), _dptr(nu_bar),
                               _dptr(param_bar), _stream(stream)))


def lrh_unrolled_bound_grad(h, nu0, beta, L, T, qbar, bound, param_bar=None, nu0_bar=None, flags=0,
                            stream=None):
    _check(load().lrh_unrolled_bound_grad(h, _dptr(nu0), float(beta), float(L), int(T), _dptr(qbar),
                                          _dptr(bound), _dptr(param_bar), _dptr(nu0_bar), flags,
                                          _stream(stream)))


def lrh_autotune(h, flags=0, cache_path: Optional[str] = None, stream=None):
    _check(load().lrh_autotune(h, flags, None if cache_path is None else cache_path.encode(), _stream(stream)))


def lrh_set_shape(h, De, block, W, flags=0):
    _check(load().lrh_set_shape(h, int(De), int(block), int(W), flags))


def lrh_time_buckets(h, nu, beta: float, reps: int = 3, stream=None):
    import torch
    cnt = C.c_int32(0)
    _check(load().lrh_get_shapes(h, 0, None, None, None, None, None, None, C.byref(cnt)))
    us = np.zeros(max(cnt.value, 1), np.float64)
    f32 = nu.dtype == torch.float32
    _check(load().lrh_time_buckets(h, _dptr(nu), LRH_F32 if f32 else 0, float(beta), int(reps), us.ctypes.data,
                                   _stream(stream)))
    return [float(u) for u in us[:cnt.value]]


def lrh_time_messages(h, nu, zeta, beta: float, n_buckets: int, reps: int = 3, stream=None):
    import torch
    us = np.zeros(max(n_buckets, 1), np.float64)
    f32 = nu.dtype == torch.float32
    _check(load().lrh_time_messages(h, _dptr(nu), _dptr(zeta), LRH_F32 if f32 else 0, float(beta), int(reps),
                                    us.ctypes.data, _stream(stream)))
    return [float(u) for u in us[:n_buckets]]


def lrh_get_shapes(h):
    cnt = C.c_int32(0)
    _check(load().lrh_get_shapes(h, 0, None, None, None, None, None, None, C.byref(cnt)))
    n = cnt.value
    De, Dc, blk, W = (np.zeros(n, np.int32) for _ in range(4))
    nn = np.zeros(n, np.int64)
    us = np.zeros(n, np.float64)
    _check(load().lrh_get_shapes(h, n, De.ctypes.data, Dc.ctypes.data, nn.ctypes.data, blk.ctypes.data,
                                 W.ctypes.data, us.ctypes.data, C.byref(cnt)))
    return [dict(De=int(De[i]), Dc=int(Dc[i]), n=int(nn[i]), block=int(blk[i]), W=int(W[i]), us=float(us[i]))
            for i in range(n)]


def lrh_measure_fp64_mfma(device: int = 0, stream=None) -> float:
    """Sustained FP64 matrix-core TFLOP/s of the device (see include/lrh.h)."""
    v = C.c_double(0.0)
    _check(load().lrh_measure_fp64_mfma(int(device), C.byref(v), _stream(stream)))
    return v.value


def lrh_destroy(h):
    if h:
        load().lrh_destroy(h)


# ---- convenience wrapper -----------------------------------------------------------------

class Problem:
    """A built problem on one device with torch-allocated state buffers.

    device = -1 builds the poset and layout on the host only (no compute calls)."""

    def __init__(self, desc, device: int = 0):
        if device >= 0:
            import torch
            self.torch = torch
            self.device = torch.device("cuda", device)
        self.desc = desc
        self.h = lrh_build_clusters(desc, device)
        lay = lrh_query(self.h)
        self.layout = lay
        self.n_clusters = int(lay.n_clusters)
        self.n_msgs = int(lay.n_msgs)
        self.n_inst = int(lay.n_instances)
        self.is_real = bool(lay.is_real)
        self.nu_len = int(lay.nu_len)
        self.marg_len = int(lay.marg_len)
        self.Lambda = float(lay.Lambda_G)
        self.Gamma = float(lay.Gamma_G)
        self.buckets = [dict(D=int(lay.bucket_D[b]), M=int(lay.bucket_count[b]),
                             comps=int(lay.bucket_comps[b]), offset=int(lay.bucket_offset[b]))
                        for b in range(lay.n_buckets)]
        ptr = np.zeros(self.n_clusters + 1, dtype=np.int64)
        load().lrh_export_clusters(self.h, ptr.ctypes.data, None, None)
        sites = np.zeros(int(ptr[-1]), dtype=np.int32)
        inst = np.zeros(self.n_clusters, dtype=np.int32)
        _check(load().lrh_export_clusters(self.h, ptr.ctypes.data, sites.ctypes.data, inst.ctypes.data))
        self.clusters = [tuple(int(x) for x in sites[ptr[c]:ptr[c + 1]]) for c in range(self.n_clusters)]
        self.cluster_instance = inst
        par = np.zeros(self.n_msgs, dtype=np.int32)
        chi = np.zeros(self.n_msgs, dtype=np.int32)
        bkt = np.zeros(self.n_msgs, dtype=np.int32)
        idx = np.zeros(self.n_msgs, dtype=np.int64)
        _check(load().lrh_export_messages(self.h, par.ctypes.data, chi.ctypes.data, bkt.ctypes.data,
                                          idx.ctypes.data))
        self.msg_parent, self.msg_child, self.msg_bucket, self.msg_index = par, chi, bkt, idx

    def close(self):
        if self.h:
            lrh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- buffers ----
    def dtype(self, f32: bool):
        return self.torch.float32 if f32 else self.torch.float64

    def zeros(self, f32: bool = False):
        return self.torch.zeros(self.nu_len, dtype=self.dtype(f32), device=self.device)

    def qbuf(self, fill: float = 0.0):
        return self.torch.full((self.n_inst,), fill, dtype=self.torch.float64, device=self.device)

    # ---- layout conversion (host side) ----
    def message_keys(self):
        return [(self.clusters[p], self.clusters[c]) for p, c in zip(self.msg_parent, self.msg_child)]

    def to_dense(self, nu) -> Dict[Tuple[Tuple[int, ...], Tuple[int, ...]], np.ndarray]:
        v = nu.detach().double().cpu().numpy() if hasattr(nu, "detach") else np.asarray(nu, np.float64)
        out = {}
        pos = 0
        for b in self.buckets:
            D, M, comps, off = b["D"], b["M"], b["comps"], b["offset"]
            blk = v[off:off + comps * M].reshape(comps, M)
            iu = np.triu_indices(D)
            ju = np.triu_indices(D, 1)
            ntri = D * (D + 1) // 2
            for m in range(M):
                A = np.zeros((D, D), dtype=np.complex128)
                A[iu] = blk[:ntri, m]
                if not self.is_real:
                    A[ju] += 1j * blk[ntri:, m]
                A = A + np.conj(np.triu(A, 1)).T
                key = (self.clusters[self.msg_parent[pos]], self.clusters[self.msg_child[pos]])
                out[key] = A
                pos += 1
        return out

    def from_dense(self, mats, f32: bool = False):
        v = self.from_dense_np(mats)
        return self.torch.from_numpy(v).to(device=self.device, dtype=self.dtype(f32))

    def from_dense_np(self, mats) -> np.ndarray:
        v = np.zeros(self.nu_len, dtype=np.float64)
        pos = 0
        for b in self.buckets:
            D, M, comps, off = b["D"], b["M"], b["comps"], b["offset"]
            blk = np.zeros((comps, M))
            iu = np.triu_indices(D)
            ju = np.triu_indices(D, 1)
            ntri = D * (D + 1) // 2
            for m in range(M):
                key = (self.clusters[self.msg_parent[pos]], self.clusters[self.msg_child[pos]])
                A = np.asarray(mats[key])
                blk[:ntri, m] = A.real[iu]
                if not self.is_real:
                    blk[ntri:, m] = A.imag[ju]
                pos += 1
            v[off:off + comps * M] = blk.reshape(-1)
        return v

    def marg_dense(self, marg) -> Dict[Tuple[int, ...], np.ndarray]:
        v = marg.detach().double().cpu().numpy()
        out = {}
        off = 0
        sd = np.asarray(self.desc.site_dim)
        for c, sites in enumerate(self.clusters):
            D = int(np.prod([int(sd[x]) for x in sites]))
            ntri = D * (D + 1) // 2
            n = D * D if not self.is_real else ntri
            blk = v[off:off + n]
            A = np.zeros((D, D), dtype=np.complex128)
            A[np.triu_indices(D)] = blk[:ntri]
            if not self.is_real:
                A[np.triu_indices(D, 1)] += 1j * blk[ntri:]
            out[sites] = A + np.conj(np.triu(A, 1)).T
            off += n
        return out

    # ---- compute calls ----
    def dual_eval(self, nu, beta: float, grad: bool = False, marg: bool = False, stream=None):
        f32 = nu.dtype == self.torch.float32
        q = self.qbuf()
        g = self.torch.empty_like(nu) if grad else None
        m = self.torch.empty(self.marg_len, dtype=nu.dtype, device=self.device) if marg else None
        lrh_dual_eval(self.h, nu, LRH_F32 if f32 else 0, beta, q, g, m, stream)
        return q, g, m

    def step_subgrad(self, nu, nu_best, q_best, k0: int, n_iter: int, step_kind: int = 0,
                     step_scale: float = 1.0, q_hist=None, stream=None):
        f32 = nu.dtype == self.torch.float32
        lrh_step_subgrad(self.h, nu, nu_best, q_best, k0, n_iter, step_kind, step_scale, q_hist,
                         LRH_F32 if f32 else 0, stream)

    def new_nesterov_state(self, beta: float, L: Optional[float] = None) -> NesterovState:
        st = NesterovState()
        st.k = 0
        st.theta = 1.0
        st.beta = float(beta)
        st.L = 0.0 if L is None else float(L)   # 0: the library's beta Lambda_G / 2
        return st

    def step_nesterov(self, nu, zeta, state: NesterovState, n_iter: int, fused: bool = False, stream=None):
        f32 = nu.dtype == self.torch.float32
        flags = (LRH_F32 if f32 else 0) | (LRH_FUSED if fused else 0)
        lrh_step_nesterov(self.h, nu, zeta, state, n_iter, flags, stream)

    def certify(self, nu, lmin: bool = False, stream=None):
        f32 = nu.dtype == self.torch.float32
        q = self.qbuf()
        mg = self.qbuf()
        lm = self.torch.empty(self.n_clusters, dtype=self.torch.float64, device=self.device) if lmin else None
        lrh_certify(self.h, nu, LRH_F32 if f32 else 0, q, mg, lm, stream)
        return q, mg, lm

    def check(self, stream=None):
        return lrh_check(self.h, stream)

    # ---- parameters and adjoint ----
    @property
    def n_params(self) -> int:
        return int(self.layout.n_params)

    def set_params(self, params, stream=None):
        lrh_set_params(self.h, params.contiguous(), stream)

    def dual_vjp(self, nu, beta: float, qbar=None, gbar=None, packed: bool = False, stream=None):
        nu_bar = self.torch.empty_like(nu)
        pbar = (self.torch.empty(self.n_params, dtype=self.torch.float64, device=self.device)
                if self.n_params else None)
        lrh_dual_vjp(self.h, nu, LRH_PACKED_COTANGENT if packed else 0, beta, qbar, gbar, nu_bar, pbar, stream)
        return nu_bar, pbar

    def unrolled_bound_grad(self, beta: float, T: int, L: Optional[float] = None, nu0=None, qbar=None,
                            want_nu0_bar: bool = False, packed: bool = False, stream=None):
        L = 0.0 if L is None else float(L)   # 0: the library's beta Lambda_G / 2
        bound = self.qbuf()
        pbar = (self.torch.empty(self.n_params, dtype=self.torch.float64, device=self.device)
                if self.n_params else None)
        n0b = self.zeros() if want_nu0_bar else None
        lrh_unrolled_bound_grad(self.h, nu0, beta, L, T, qbar, bound, pbar, n0b,
                                LRH_PACKED_COTANGENT if packed else 0, stream)
        return bound, pbar, n0b

    def set_jacobi(self, max_sweeps: int, rel_tol: float = 0.0):
        lrh_set_jacobi(self.h, max_sweeps, rel_tol)

    def set_slab_limit(self, max_slabs: int):
        lrh_set_slab_limit(self.h, max_slabs)

    def certify_fallbacks(self, stream=None) -> int:
        """Clusters (D_e >= 64) certified by the tridiagonalisation since the last call."""
        return lrh_certify_fallbacks(self.h, stream)

    def set_certify_method(self, method: int):
        """0: certificate at D_e = 256, tridiagonalisation at 64, 128 (default); 1: tridiagonalisation;
        3: certificate at every D_e >= 64; 2: fallback test hook (see lrh_set_certify_method)."""
        lrh_set_certify_method(self.h, method)

    def autotune(self, f32: bool = False, cache_path: Optional[str] = None, stream=None):
        lrh_autotune(self.h, LRH_F32 if f32 else 0, cache_path, stream)
        return self.shapes()

    def shapes(self):
        return lrh_get_shapes(self.h)

    def time_buckets(self, nu, beta: float, reps: int = 3, stream=None):
        """Per-bucket cluster-kernel launch durations (us), in shapes() order."""
        return lrh_time_buckets(self.h, nu, beta, reps, stream)

    def time_messages(self, nu, zeta, beta: float, reps: int = 3, stream=None):
        """Per-message-bucket durations (us) of the accelerated message update, run in place on
        nu and zeta (pass copies), in buckets order."""
        return lrh_time_messages(self.h, nu, zeta, beta, len(self.buckets), reps, stream)

    def force_shape(self, De: int, W: int, block: int = 64, f32=None):
        for flag in ([LRH_F32, 0] if f32 is None else [LRH_F32 if f32 else 0]):
            lrh_set_shape(self.h, De, block, W, flag)


def nesterov_schedule(beta0: float, beta_max: float, total_iters: int):
    """beta = beta0 * 2^s up to beta_max, iterations split evenly (remainder to the last)."""
    betas = []
    b = beta0
    while b <= beta_max * (1 + 1e-12):
        betas.append(b)
        b *= 2
    per = total_iters // len(betas)
    sched = [(bb, per) for bb in betas]
    sched[-1] = (betas[-1], total_iters - per * (len(betas) - 1))
    return sched


# ---- autograd wrappers (the arithmetic of both passes runs in the library) ------------------

def _autograd():
    import torch

    class SmoothedDual(torch.autograd.Function):
        """(nu, params) -> (Q_beta per instance, grad Q_beta).

        grad Q_beta is the Hermitian gradient matrix of every message (Frobenius inner product)
        stored in the message layout.  Cotangents follow torch's convention (with respect to the
        stored components); the library converts them (LRH_PACKED_COTANGENT).  Forward:
        lrh_set_params + lrh_dual_eval.  Backward: lrh_dual_vjp, which applies the
        Daleckii-Krein derivative of every Gibbs state."""

        @staticmethod
        def forward(ctx, nu, params, problem, beta):
            with_params = params is not None and problem.n_params > 0
            if with_params:
                problem.set_params(params.detach())
            q, g, _ = problem.dual_eval(nu.detach(), beta, grad=True)
            ctx.problem, ctx.beta, ctx.with_params = problem, beta, with_params
            if with_params:
                ctx.save_for_backward(nu.detach(), params.detach().clone())
            else:
                ctx.save_for_backward(nu.detach())
            return q, g

        @staticmethod
        def backward(ctx, qbar, gbar):
            P = ctx.problem
            if ctx.with_params:
                nu, params = ctx.saved_tensors
                P.set_params(params)   # the Hamiltonian of this forward, whatever was set since
            else:
                (nu,) = ctx.saved_tensors
            qb = None if qbar is None else qbar.contiguous().double()
            gb = None if gbar is None else gbar.contiguous().double()
            nu_bar, pbar = P.dual_vjp(nu, ctx.beta, qb, gb, packed=True)
            return nu_bar, (pbar if ctx.with_params else None), None, None

    class UnrolledBound(torch.autograd.Function):
        """params -> B_T per instance (T accelerated steps at fixed beta from zero messages,
        then Q).  Backward re-runs the forward and the reverse sweep in the library."""

        @staticmethod
        def forward(ctx, params, problem, beta, T, L):
            problem.set_params(params.detach())
            b, _, _ = problem.unrolled_bound_grad(beta, T, L)
            ctx.problem, ctx.beta, ctx.T, ctx.L = problem, beta, T, L
            ctx.save_for_backward(params.detach())
            return b

        @staticmethod
        def backward(ctx, bbar):
            (params,) = ctx.saved_tensors
            P = ctx.problem
            P.set_params(params)
            _, pbar, _ = P.unrolled_bound_grad(ctx.beta, ctx.T, ctx.L, qbar=bbar.contiguous().double())
            return pbar, None, None, None, None

    return SmoothedDual, UnrolledBound


def smoothed_dual(nu, params, problem, beta):
    return _autograd()[0].apply(nu, params, problem, beta)


def unrolled_bound(params, problem, beta, T, L=None):
    return _autograd()[1].apply(params, problem, beta, T, L)
