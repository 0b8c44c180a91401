"""ctypes binding of libtxe.so (the HIP/C++ Tucker-tensor exchange library).

Argument marshalling only: every step of the exchange computation runs in the
library's kernels.  torch supplies device memory (tensor data pointers) and
the current HIP stream.  There is no fallback: if the library is missing or a
call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtxe.so")

COMPUTE = {"f64": 0, "f32": 1, "bf16x3": 2, "bf16x6": 3}
DTYPE = {"f64": 0, "f32": 1}
FORM = {"core": 0, "collocation": 1}

_c_int = ctypes.c_int32
_c_dp = ctypes.POINTER(ctypes.c_double)


class SystemDesc(ctypes.Structure):
    _fields_ = [
        ("n", _c_int * 3),
        ("x", ctypes.c_void_p * 3),
        ("q", ctypes.c_void_p * 3),
        ("r", _c_int * 3),
        ("U", ctypes.c_void_p * 3),
        ("K", _c_int),
        ("w", ctypes.c_void_p),
        ("alpha", ctypes.c_void_p),
        ("C", ctypes.c_void_p * 3),
    ]


class ApplyArgs(ctypes.Structure):
    _fields_ = [
        ("compute", _c_int),
        ("dtype", _c_int),
        ("N", _c_int),
        ("psi", ctypes.c_void_p),
        ("symmetric", _c_int),
        ("i0", _c_int),
        ("Ni", _c_int),
        ("vxpsi", ctypes.c_void_p),
        ("out_scale", ctypes.c_void_p),
        ("out_weighted", _c_int),
        ("ex", ctypes.c_void_p),
        ("e_pairs", ctypes.c_void_p),
        ("e_orb", ctypes.c_void_p),
        ("pair_bases", _c_int),
        ("form", _c_int),
    ]


# every symbol include/txe.h declares, with its ctypes signature
SIGNATURES = {
    "txe_abi_version": (_c_int, []),
    "txe_status_string": (ctypes.c_char_p, [_c_int]),
    "txe_last_error": (ctypes.c_char_p, []),
    "txe_conv_matrix_1d": (_c_int, [_c_int, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p]),
    "txe_context_create": (_c_int, [_c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "txe_context_destroy": (_c_int, [ctypes.c_void_p]),
    "txe_context_set_stream": (_c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "txe_context_stream_changes": (_c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "txe_workspace_reserve": (_c_int, [ctypes.c_void_p, ctypes.c_size_t]),
    "txe_system_create": (_c_int, [ctypes.c_void_p, ctypes.POINTER(SystemDesc), ctypes.POINTER(ctypes.c_void_p)]),
    "txe_system_destroy": (_c_int, [ctypes.c_void_p]),
    "txe_system_conv": (_c_int, [ctypes.c_void_p, _c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "txe_fe_mesh_1d": (_c_int, [ctypes.c_void_p, _c_int, _c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "txe_hosvd_bases": (_c_int, [ctypes.c_void_p, ctypes.POINTER(_c_int), ctypes.POINTER(ctypes.c_void_p),
                                 ctypes.c_void_p, _c_int, _c_int, _c_int, _c_int, ctypes.POINTER(_c_int),
                                 ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p)]),
    "txe_fe_conv_matrices": (_c_int, [ctypes.c_void_p, _c_int, _c_int, ctypes.c_void_p, _c_int, ctypes.c_void_p]),
    "txe_workspace_query": (_c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ApplyArgs),
                                     ctypes.POINTER(ctypes.c_size_t)]),
    "txe_apply": (_c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ApplyArgs)]),
    "txe_apply_noalloc": (_c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ApplyArgs)]),
    "txe_profile_enable": (_c_int, [ctypes.c_void_p, _c_int]),
    "txe_profile_read": (_c_int, [ctypes.c_void_p, _c_int, ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_int64)]),
    "txe_kernel_name": (ctypes.c_char_p, [_c_int]),
    "txe_apply_batched": (_c_int, [ctypes.c_void_p, _c_int, ctypes.POINTER(ctypes.c_void_p),
                                   ctypes.POINTER(ApplyArgs), _c_int]),
    "txe_graph_capture_batched": (_c_int, [ctypes.c_void_p, _c_int, ctypes.POINTER(ctypes.c_void_p),
                                           ctypes.POINTER(ApplyArgs), _c_int, ctypes.POINTER(ctypes.c_void_p)]),
    "txe_graph_launch": (_c_int, [ctypes.c_void_p]),
    "txe_graph_destroy": (_c_int, [ctypes.c_void_p]),
    "txe_tune": (_c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ApplyArgs), _c_int,
                          ctypes.POINTER(ctypes.c_double)]),
    "txe_plan_get": (_c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ApplyArgs),
                              ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "txe_tune_save": (_c_int, [ctypes.c_void_p, ctypes.c_char_p]),
    "txe_tune_load": (_c_int, [ctypes.c_void_p, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32)]),
    "txe_measure_ceiling": (_c_int, [ctypes.c_void_p, _c_int, ctypes.POINTER(ctypes.c_double)]),
    "txe_ace_build": (_c_int, [ctypes.c_void_p, ctypes.c_void_p, _c_int, _c_int, ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "txe_ace_apply": (_c_int, [ctypes.c_void_p, ctypes.c_void_p, _c_int, ctypes.c_void_p, _c_int, _c_int,
                               ctypes.c_void_p, ctypes.c_void_p]),
}

KERNELS = ("proj12", "proj3", "core", "epair", "back", "energy")

_lib = None


class TxeError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"txe status {status}: {msg}")
        self.status = status


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2401_04189_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(st):
    if st != 0:
        L = lib()
        raise TxeError(st, f"{L.txe_status_string(st).decode()}: {L.txe_last_error().decode()}")


def conv_matrix_1d(x, alpha):
    """Host FP64 1-D convolution matrix of one Gaussian term (no GPU needed)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    C = np.empty((len(x), len(x)), dtype=np.float64)
    _check(lib().txe_conv_matrix_1d(len(x), x.ctypes.data, float(alpha), C.ctypes.data))
    return C


def fe_mesh_1d(edges, p):
    """Host FP64 nodes x and weights q of order-p Lagrange elements on the
    cells between `edges` (the domain ends held at zero; no GPU needed)."""
    edges = np.ascontiguousarray(edges, dtype=np.float64)
    n = (len(edges) - 1) * int(p) - 1
    x = np.empty(max(n, 0), dtype=np.float64)
    q = np.empty(max(n, 0), dtype=np.float64)
    _check(lib().txe_fe_mesh_1d(edges.ctypes.data, len(edges) - 1, int(p), x.ctypes.data, q.ctypes.data))
    return x, q


def fe_conv_matrices(edges, p, alpha):
    """Host FP64 convolution matrices [K][n][n] of the Gaussian terms with
    exponents `alpha` for order-p Lagrange elements (no GPU needed)."""
    edges = np.ascontiguousarray(edges, dtype=np.float64)
    alpha = np.ascontiguousarray(np.atleast_1d(alpha), dtype=np.float64)
    n = (len(edges) - 1) * int(p) - 1
    C = np.empty((len(alpha), max(n, 0), max(n, 0)), dtype=np.float64)
    _check(lib().txe_fe_conv_matrices(edges.ctypes.data, len(edges) - 1, int(p), alpha.ctypes.data, len(alpha),
                                      C.ctypes.data))
    return C


def hosvd_bases(ctx, psi, q, r, i0=0, Ni=None):
    """Shared q-orthonormal bases U_d (n_d x r_d) of the stacked pair densities
    of the orbitals `psi` (CUDA tensor N x n0 x n1 x n2), targets [i0, i0+Ni)
    against all orbitals, from the library's device HOSVD; returns (U, sv)."""
    import torch

    if not psi.is_cuda or not psi.is_contiguous():
        raise ValueError("psi must be a contiguous CUDA tensor")
    N = psi.shape[0]
    Ni = N - i0 if Ni is None else Ni
    n = tuple(psi.shape[1:])
    rr = tuple(r) if isinstance(r, (tuple, list)) else (r, r, r)
    qs = [np.ascontiguousarray(v, dtype=np.float64) for v in q]
    U = [np.empty((n[d], rr[d]), dtype=np.float64) for d in range(3)]
    sv = [np.empty(n[d], dtype=np.float64) for d in range(3)]
    ctx.set_stream(torch.cuda.current_stream(psi.device))
    _check(lib().txe_hosvd_bases(ctx.h, (_c_int * 3)(*n), (ctypes.c_void_p * 3)(*[v.ctypes.data for v in qs]),
                                 psi.data_ptr(), DTYPE["f64" if psi.dtype == torch.float64 else "f32"], N, int(i0),
                                 int(Ni), (_c_int * 3)(*rr), (ctypes.c_void_p * 3)(*[u.ctypes.data for u in U]),
                                 (ctypes.c_void_p * 3)(*[v.ctypes.data for v in sv])))
    return U, sv


def _stream_ptr(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


class Context:
    def __init__(self, device=0, stream=None):
        import torch

        self.device = int(device)
        torch.cuda.set_device(self.device)
        h = ctypes.c_void_p()
        _check(lib().txe_context_create(self.device, ctypes.c_void_p(_stream_ptr(stream)), ctypes.byref(h)))
        self.h = h

    def set_stream(self, stream):
        _check(lib().txe_context_set_stream(self.h, ctypes.c_void_p(_stream_ptr(stream))))

    def stream_changes(self):
        """Stream changes so far that were ordered after the previous stream."""
        n = ctypes.c_int64()
        _check(lib().txe_context_stream_changes(self.h, ctypes.byref(n)))
        return n.value

    def reserve(self, nbytes):
        _check(lib().txe_workspace_reserve(self.h, int(nbytes)))

    def profile(self, on=True):
        """Start (and reset) or stop per-kernel HIP-event timing."""
        _check(lib().txe_profile_enable(self.h, 1 if on else 0))

    def kernel_times(self):
        """{kernel name: (total ms, launches)} since profiling was enabled."""
        out = {}
        for k, name in enumerate(KERNELS):
            ms = ctypes.c_double()
            n = ctypes.c_int64()
            _check(lib().txe_profile_read(self.h, k, ctypes.byref(ms), ctypes.byref(n)))
            out[name] = (ms.value, n.value)
        return out

    def ceiling(self, kind):
        """Measured rate of this device: "f64", "f32", "bf16" MFMA (TFLOP/s) or "hbm" (GB/s)."""
        v = ctypes.c_double()
        _check(lib().txe_measure_ceiling(self.h, {"f64": 0, "f32": 1, "bf16": 2, "hbm": 3}[kind], ctypes.byref(v)))
        return v.value

    def close(self):
        if getattr(self, "h", None):
            lib().txe_context_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class System:
    """Fixed data of one exchange problem: grid (x_d, q_d), bases U_d, (w_k, alpha_k)."""

    def __init__(self, ctx: Context, x, q, U, w, alpha, C=None):
        """C: optional per-mode (K, n, n) 1-D convolution matrices (None = built-in)."""
        self.ctx = ctx
        self._keep = []
        d = SystemDesc()
        for m in range(3):
            if C is not None and C[m] is not None:
                Cm = np.ascontiguousarray(C[m], dtype=np.float64)
                if Cm.shape != (len(w), len(x[m]), len(x[m])):
                    raise ValueError(f"C[{m}] must have shape (K, n, n) = {(len(w), len(x[m]), len(x[m]))}")
                self._keep.append(Cm)
                d.C[m] = Cm.ctypes.data
        for m in range(3):
            xm = np.ascontiguousarray(x[m], dtype=np.float64)
            qm = np.ascontiguousarray(q[m], dtype=np.float64)
            Um = np.ascontiguousarray(U[m], dtype=np.float64)
            self._keep += [xm, qm, Um]
            d.n[m] = len(xm)
            d.r[m] = Um.shape[1]
            d.x[m] = xm.ctypes.data
            d.q[m] = qm.ctypes.data
            d.U[m] = Um.ctypes.data
        wk = np.ascontiguousarray(w, dtype=np.float64)
        ak = np.ascontiguousarray(alpha, dtype=np.float64)
        self._keep += [wk, ak]
        d.K = len(wk)
        d.w = wk.ctypes.data
        d.alpha = ak.ctypes.data
        self.n = tuple(d.n)
        self.r = tuple(d.r)
        self.K = d.K
        h = ctypes.c_void_p()
        _check(lib().txe_system_create(ctx.h, ctypes.byref(d), ctypes.byref(h)))
        self.h = h
        self._keep = []

    @classmethod
    def from_workload(cls, ctx, s):
        return cls(ctx, s.grid.x, s.grid.q, s.U, s.w, s.alpha)

    def conv(self, mode):
        """FP64 (C_k, Chat_k) tables of one mode, as built by the library."""
        n, r = self.n[mode], self.r[mode]
        C = np.empty((self.K, n, n))
        Ch = np.empty((self.K, r, r))
        _check(lib().txe_system_conv(self.h, mode, C.ctypes.data, Ch.ctypes.data))
        return C, Ch

    def close(self):
        if getattr(self, "h", None):
            lib().txe_system_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_args(psi, compute="f64", symmetric=True, i0=0, Ni=None, vx=None, ex=None, e_pairs=None,
              out_scale=None, out_weighted=False, e_orb=None, pair_bases=False, form="core"):
    import torch

    a = ApplyArgs()
    a.compute = COMPUTE[compute]
    a.dtype = DTYPE["f64" if psi.dtype == torch.float64 else "f32"]
    a.N = psi.shape[0]
    a.psi = psi.data_ptr()
    a.symmetric = 1 if symmetric else 0
    a.i0 = 0 if symmetric else int(i0)
    a.Ni = psi.shape[0] if symmetric else int(Ni)
    a.vxpsi = vx.data_ptr() if vx is not None else None
    a.out_scale = out_scale.data_ptr() if out_scale is not None else None
    a.out_weighted = 1 if out_weighted else 0
    a.ex = ex.data_ptr() if ex is not None else None
    a.e_pairs = e_pairs.data_ptr() if e_pairs is not None else None
    a.e_orb = e_orb.data_ptr() if e_orb is not None else None
    a.pair_bases = 1 if pair_bases else 0
    a.form = FORM[form]
    return a


def _prepare(sysm, psi, compute, symmetric, i0, Ni, want_vx, want_pairs, out_scale=None, out_weighted=False,
             vx_out=None, want_orb=False, pair_bases=False, form="core"):
    """ApplyArgs for one problem with freshly allocated outputs."""
    import torch

    if not psi.is_cuda or not psi.is_contiguous():
        raise ValueError("psi must be a contiguous CUDA tensor")
    if tuple(psi.shape[1:]) != sysm.n:
        raise ValueError(f"psi grid {tuple(psi.shape[1:])} does not match the system grid {sysm.n}")
    N = psi.shape[0]
    Ni = N if symmetric else (N - i0 if Ni is None else Ni)
    vx = None
    if want_vx:
        vx = vx_out if vx_out is not None else torch.empty((Ni,) + tuple(psi.shape[1:]), dtype=psi.dtype,
                                                             device=psi.device)
    ex = torch.empty((), dtype=torch.float64, device=psi.device)
    npairs = N * (N + 1) // 2 if symmetric else Ni * N
    ep = torch.empty(npairs, dtype=torch.float64, device=psi.device) if want_pairs else None
    eo = torch.empty(Ni, dtype=torch.float64, device=psi.device) if want_orb else None
    a = make_args(psi, compute, symmetric, i0, Ni, vx, ex, ep, out_scale, out_weighted, eo, pair_bases, form)
    if want_orb:
        return a, vx, ex, ep, eo
    return a, vx, ex, ep


def apply(ctx: Context, sysm: System, psi, compute="f64", symmetric=True, i0=0, Ni=None, want_vx=True,
          want_pairs=False, out_scale=None, out_weighted=False, vx_out=None, want_orb=False, pair_bases=False,
          form="core"):
    """Vx psi (targets) and E_x for the orbitals `psi` (a CUDA tensor N x n0 x n1 x n2).

    Returns (vx, ex, e_pairs): vx is None when want_vx is False; ex is a
    0-d float64 CUDA tensor; e_pairs is None unless want_pairs.  With
    want_orb a fourth entry holds the exchange-matrix diagonal
    <psi_i, Vx psi_i>_W of each target (FP64, from the library).  With
    pair_bases every pair uses its own Tucker bases (the sequentially
    truncated HOSVD of its density at the system's ranks).  form "core"
    evaluates the kernel sum in the Tucker core and back-projects it;
    "collocation" evaluates the 1-D convolutions at every node and
    reconstructs phi on the grid (FP64)."""
    import torch

    out = _prepare(sysm, psi, compute, symmetric, i0, Ni, want_vx, want_pairs, out_scale, out_weighted, vx_out,
                   want_orb, pair_bases, form)
    ctx.set_stream(torch.cuda.current_stream(psi.device))
    _check(lib().txe_apply(ctx.h, sysm.h, ctypes.byref(out[0])))
    return tuple(out[1:])


def apply_noalloc(ctx: Context, sysm: System, psi, compute="f64", symmetric=True, i0=0, Ni=None, want_vx=True,
                  want_pairs=False, out_scale=None, out_weighted=False, vx_out=None, want_orb=False):
    """As apply(), through txe_apply_noalloc: the library allocates nothing
    (its workspace is a fixed device array per GPU); the outputs are
    allocated here unless given."""
    import torch

    out = _prepare(sysm, psi, compute, symmetric, i0, Ni, want_vx, want_pairs, out_scale, out_weighted, vx_out,
                   want_orb)
    ctx.set_stream(torch.cuda.current_stream(psi.device))
    _check(lib().txe_apply_noalloc(ctx.h, sysm.h, ctypes.byref(out[0])))
    return tuple(out[1:])


def _batch(items, compute, want_vx, want_pairs):
    """Argument arrays of a batch of (System, psi) problems in symmetric mode."""
    args = (ApplyArgs * len(items))()
    systems = (ctypes.c_void_p * len(items))()
    outs = []
    for k, (sysm, psi) in enumerate(items):
        a, vx, ex, ep = _prepare(sysm, psi, compute, True, 0, None, want_vx, want_pairs)
        args[k] = a
        systems[k] = sysm.h
        outs.append((vx, ex, ep))
    return systems, args, outs


def apply_batched(ctx: Context, items, compute="f32", lanes=4, want_vx=True, want_pairs=False):
    """Symmetric-mode apply of several independent problems, items = [(System, psi), ...],
    enqueued as one batch over `lanes` concurrent streams.  Returns [(vx, ex, e_pairs)]."""
    import torch

    systems, args, outs = _batch(items, compute, want_vx, want_pairs)
    ctx.set_stream(torch.cuda.current_stream())
    _check(lib().txe_apply_batched(ctx.h, len(items), systems, args, int(lanes)))
    return outs


class Graph:
    """A batch captured once as a HIP graph; `launch()` replays it on the
    current stream.  The outputs (`outputs`, as in apply_batched) are the
    graph's own and are overwritten by every replay; the inputs are read
    where they were at capture time."""

    def __init__(self, ctx: Context, items, compute="f32", lanes=4, want_vx=True, want_pairs=False):
        self.ctx = ctx
        self.items = list(items)  # keeps systems and orbitals alive
        systems, args, self.outputs = _batch(self.items, compute, want_vx, want_pairs)
        h = ctypes.c_void_p()
        _check(lib().txe_graph_capture_batched(ctx.h, len(self.items), systems, args, int(lanes), ctypes.byref(h)))
        self.h = h

    def launch(self):
        import torch

        self.ctx.set_stream(torch.cuda.current_stream())
        _check(lib().txe_graph_launch(self.h))

    def close(self):
        if getattr(self, "h", None):
            lib().txe_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tune(ctx: Context, sysm: System, psi, compute="f32", symmetric=True, i0=0, Ni=None, want_vx=True, reps=3):
    """Search the launch shapes of this problem on the device; the context
    keeps the fastest.  Returns (mean ms of the chosen shape, knobs)."""
    import torch

    a, vx, ex, ep = _prepare(sysm, psi, compute, symmetric, i0, Ni, want_vx, False)
    ctx.set_stream(torch.cuda.current_stream(psi.device))
    ms = ctypes.c_double()
    _check(lib().txe_tune(ctx.h, sysm.h, ctypes.byref(a), int(reps), ctypes.byref(ms)))
    return ms.value, plan(ctx, sysm, psi, compute, symmetric, i0, Ni, want_vx)[0]


def plan(ctx: Context, sysm: System, psi, compute="f32", symmetric=True, i0=0, Ni=None, want_vx=True):
    """(knobs dict, tuned flag) an apply with these arguments would use."""
    a, vx, ex, ep = _prepare(sysm, psi, compute, symmetric, i0, Ni, want_vx, False)
    k = (ctypes.c_int32 * 5)()
    tuned = ctypes.c_int32()
    _check(lib().txe_plan_get(ctx.h, sysm.h, ctypes.byref(a), k, ctypes.byref(tuned)))
    return dict(ngs_mul=k[0], proj_gt=k[1], back_ncg=k[2], grid_cap=k[3], back_form=k[4]), bool(tuned.value)


def tune_save(ctx: Context, path):
    _check(lib().txe_tune_save(ctx.h, os.fsencode(path)))


def tune_load(ctx: Context, path):
    n = ctypes.c_int32()
    _check(lib().txe_tune_load(ctx.h, os.fsencode(path), ctypes.byref(n)))
    return n.value


def workspace_bytes(ctx, sysm, psi, compute="f64", symmetric=True, i0=0, Ni=None, want_vx=True):
    """Workspace bytes of one apply with these arguments (nothing is computed)."""
    N = psi.shape[0]
    Ni = N if symmetric else (N - i0 if Ni is None else Ni)
    a = make_args(psi, compute, symmetric, i0, Ni)
    # the query only inspects which outputs are requested; these addresses are
    # placeholders that are never dereferenced
    end = psi.data_ptr() + psi.numel() * psi.element_size()
    a.ex = end
    if want_vx:
        a.vxpsi = end + 256
    nb = ctypes.c_size_t()
    _check(lib().txe_workspace_query(ctx.h, sysm.h, ctypes.byref(a), ctypes.byref(nb)))
    return nb.value


def ace_build(ctx: Context, sysm: System, psi, W, want_factors=False):
    """ACE projection vectors xi (FP64, like psi's shape) from orbitals psi and
    W = Vx psi.  Returns (xi, info) or (xi, info, M, L) with want_factors;
    info is a 0-d int32 CUDA tensor (0 = success)."""
    import torch

    for t, name in ((psi, "psi"), (W, "W")):
        if not t.is_cuda or not t.is_contiguous() or tuple(t.shape[1:]) != sysm.n:
            raise ValueError(f"{name} must be a contiguous CUDA tensor N x {sysm.n}")
    if psi.shape != W.shape or psi.dtype != W.dtype:
        raise ValueError("psi and W must have the same shape and dtype")
    N = psi.shape[0]
    xi = torch.empty(psi.shape, dtype=torch.float64, device=psi.device)
    info = torch.empty((), dtype=torch.int32, device=psi.device)
    M = L = None
    if want_factors:
        M = torch.empty((N, N), dtype=torch.float64, device=psi.device)
        L = torch.empty((N, N), dtype=torch.float64, device=psi.device)
    ctx.set_stream(torch.cuda.current_stream(psi.device))
    _check(lib().txe_ace_build(ctx.h, sysm.h, N, DTYPE["f64" if psi.dtype == torch.float64 else "f32"],
                               psi.data_ptr(), W.data_ptr(), xi.data_ptr(), M.data_ptr() if M is not None else None,
                               L.data_ptr() if L is not None else None, info.data_ptr()))
    return (xi, info, M, L) if want_factors else (xi, info)


def ace_apply(ctx: Context, sysm: System, xi, phi):
    """V_ACE phi for trial functions phi (CUDA tensor Nphi x grid, f32 or f64)."""
    import torch

    if not phi.is_cuda or not phi.is_contiguous() or tuple(phi.shape[1:]) != sysm.n:
        raise ValueError(f"phi must be a contiguous CUDA tensor Nphi x {sysm.n}")
    if xi.dtype != torch.float64 or not xi.is_contiguous() or tuple(xi.shape[1:]) != sysm.n:
        raise ValueError("xi must be the FP64 tensor from ace_build")
    out = torch.empty_like(phi)
    ctx.set_stream(torch.cuda.current_stream(phi.device))
    _check(lib().txe_ace_apply(ctx.h, sysm.h, xi.shape[0], xi.data_ptr(), phi.shape[0],
                               DTYPE["f64" if phi.dtype == torch.float64 else "f32"], phi.data_ptr(),
                               out.data_ptr()))
    return out
