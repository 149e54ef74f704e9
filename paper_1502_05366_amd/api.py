"""Thin torch-facing wrappers of the C entry points in include/rsvd.h.

Inputs and outputs are torch tensors on a HIP device; each wrapper allocates
the outputs and the workspace with torch, passes raw device pointers and the
current torch stream to the library, and raises RsvdError on a non-zero
return code.  The numerical status words are returned as a 2-element int32
device tensor (read it with .cpu() when needed).
"""

import atexit
import ctypes

import torch

from . import _lib

F64 = 0
F32 = 1
BF16 = 2
F8E4M3 = 3

INFO_ORTH_FALLBACK = 1
INFO_JACOBI_CAP = 2
INFO_RANK = 4
INFO_NONFINITE = 8
INFO_BARRIER = 16

OP_SVD, OP_ID, OP_CUR = 1, 2, 4
OPT_JACOBI_MAX_SWEEPS, OPT_TEST_WAIT_GIVEUP = 1, 2


class RsvdError(RuntimeError):
    pass


_handles = {}


def _dev_index(device):
    d = torch.device(device)
    if d.type != "cuda":
        raise RsvdError("tensors must be on a HIP device, got %s" % d)
    return d.index if d.index is not None else torch.cuda.current_device()


def handle(device=None):
    """Per-device library handle (created once)."""
    lib = _lib.load()
    idx = _dev_index(device if device is not None else "cuda")
    h = _handles.get(idx)
    if h is None:
        p = ctypes.c_void_p()
        rc = lib.rsvd_create(ctypes.byref(p), idx)
        _check(rc, "rsvd_create")
        h = p
        _handles[idx] = h
    return h


def _release_handles():
    """At interpreter exit: wait for each device's work, then destroy its
    handle (its second stream and events) before the HIP runtime tears down."""
    if not _handles:
        return
    lib = _lib.load()
    for idx, h in list(_handles.items()):
        try:
            with torch.cuda.device(idx):
                torch.cuda.synchronize()
        except Exception:  # noqa: BLE001  (exit path: release what can be released)
            pass
        lib.rsvd_destroy(h)
        del _handles[idx]


atexit.register(_release_handles)


def set_option(option, value, device=None):
    """rsvd_set_option on the device's handle (OPT_JACOBI_MAX_SWEEPS,
    OPT_TEST_WAIT_GIVEUP)."""
    _check(_lib.load().rsvd_set_option(handle(device), int(option), int(value)), "rsvd_set_option")


def _check(rc, what):
    if rc != 0:
        msg = _lib.load().rsvd_status_string(rc).decode()
        raise RsvdError("%s failed: %s (code %d)" % (what, msg, rc))


def _dtype_code(t):
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.bfloat16:
        return BF16
    raise RsvdError("A must be float64, float32 or bfloat16, got %s" % t.dtype)


def _out_dtype(A):
    """Element type of U, V (and of the range-finder matrices) for a given A."""
    return torch.float32 if A.dtype == torch.bfloat16 else A.dtype


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _row_major(A):
    if A.dim() != 2:
        raise RsvdError("expected a matrix")
    if A.stride(1) != 1 or A.stride(0) < A.shape[1]:
        A = A.contiguous()
    if A.dtype == torch.bfloat16 and (A.stride(0) % 8 or A.data_ptr() % 16):
        # the BF16 passes read rows in 16-byte pieces: pad rows to 8 elements
        m, n = A.shape
        P = torch.zeros((m, (n + 7) // 8 * 8), dtype=A.dtype, device=A.device)
        P[:, :n] = A
        A = P[:, :n]
    return A


def _workspace(nbytes, device):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def workspace_bytes(ops, dtype, m, n, k, p, q):
    return int(_lib.load().rsvd_workspace_bytes(ops, dtype, m, n, k, p, q))


def decompose(A, k, p, q, seed, svd=True, id=True, cur=True):
    """One range finder, then the selected decompositions of the same B."""
    lib = _lib.load()
    A = _row_major(A)
    dev = A.device
    m, n = A.shape
    dt = _dtype_code(A)
    ops = (OP_SVD if svd else 0) | (OP_ID if id else 0) | (OP_CUR if cur else 0)
    wb = workspace_bytes(ops, dt, m, n, k, p, q)
    if wb == 0:
        raise RsvdError("invalid sizes")
    work = _workspace(wb, dev)
    info = torch.zeros(2, dtype=torch.int32, device=dev)
    out = {}
    U = S = V = J = T = Jr = Uc = None
    if svd:
        U = torch.empty((m, k), dtype=_out_dtype(A), device=dev)
        S = torch.empty(k, dtype=torch.float64, device=dev)
        V = torch.empty((n, k), dtype=_out_dtype(A), device=dev)
    if id or cur:
        J = torch.empty(n, dtype=torch.int64, device=dev)
        T = torch.empty((k, max(n - k, 1)), dtype=torch.float64, device=dev)
    if cur:
        Jr = torch.empty(k, dtype=torch.int64, device=dev)
        Uc = torch.empty((k, k), dtype=torch.float64, device=dev)
    rc = lib.rsvd_decompose(handle(dev), dt, m, n, k, p, q, seed, _ptr(A), A.stride(0),
                            _ptr(U), k if svd else 0, _ptr(S), _ptr(V), k if svd else 0,
                            _ptr(J), _ptr(T), max(n - k, 1) if J is not None else 0,
                            _ptr(Jr), _ptr(Uc), k if cur else 0,
                            _ptr(work), work.numel(), _ptr(info), _stream(dev))
    _check(rc, "rsvd_decompose")
    out["info"] = info
    if svd:
        out.update(U=U, S=S, V=V)
    if id or cur:
        out.update(J=J, T=T[:, :n - k])
    if cur:
        out.update(Jc=J[:k], Jr=Jr, Ucur=Uc)
    out["workspace"] = work
    return out


def svd(A, k, p, q, seed):
    """Rank-k randomized SVD: U (m x k), S (k, FP64, descending), V (n x k)."""
    lib = _lib.load()
    A = _row_major(A)
    dev = A.device
    m, n = A.shape
    dt = _dtype_code(A)
    wb = workspace_bytes(OP_SVD, dt, m, n, k, p, q)
    work = _workspace(wb, dev)
    info = torch.zeros(2, dtype=torch.int32, device=dev)
    U = torch.empty((m, k), dtype=_out_dtype(A), device=dev)
    S = torch.empty(k, dtype=torch.float64, device=dev)
    V = torch.empty((n, k), dtype=_out_dtype(A), device=dev)
    rc = lib.rsvd_svd(handle(dev), dt, m, n, k, p, q, seed, _ptr(A), A.stride(0), _ptr(U), k,
                      _ptr(S), _ptr(V), k, _ptr(work), work.numel(), _ptr(info), _stream(dev))
    _check(rc, "rsvd_svd")
    return U, S, V, info


def svd_noalloc(A, k, p, q, seed, out=None):
    """rsvd_svd_noalloc: the randomized SVD of `svd` with the library's static
    device scratch instead of a workspace.  `out` = (U, S, V, info) tensors to
    write into (allocated here when None)."""
    lib = _lib.load()
    A = _row_major(A)
    dev = A.device
    m, n = A.shape
    dt = _dtype_code(A)
    if out is None:
        out = (torch.empty((m, k), dtype=_out_dtype(A), device=dev),
               torch.empty(k, dtype=torch.float64, device=dev),
               torch.empty((n, k), dtype=_out_dtype(A), device=dev),
               torch.zeros(2, dtype=torch.int32, device=dev))
    U, S, V, info = out
    rc = lib.rsvd_svd_noalloc(handle(dev), dt, m, n, k, p, q, seed, _ptr(A), A.stride(0), _ptr(U),
                              U.stride(0), _ptr(S), _ptr(V), V.stride(0), _ptr(info), _stream(dev))
    _check(rc, "rsvd_svd_noalloc")
    return U, S, V, info


def id(A, k, p, q, seed):  # noqa: A001  (named after the C entry point)
    """Rank-k column ID: J (n; skeleton J[:k]), T (k x (n-k)), info."""
    lib = _lib.load()
    A = _row_major(A)
    dev = A.device
    m, n = A.shape
    dt = _dtype_code(A)
    work = _workspace(workspace_bytes(OP_ID, dt, m, n, k, p, q), dev)
    info = torch.zeros(2, dtype=torch.int32, device=dev)
    J = torch.empty(n, dtype=torch.int64, device=dev)
    ldt = max(n - k, 1)
    T = torch.empty((k, ldt), dtype=torch.float64, device=dev)
    rc = lib.rsvd_id(handle(dev), dt, m, n, k, p, q, seed, _ptr(A), A.stride(0), _ptr(J), _ptr(T),
                     ldt, _ptr(work), work.numel(), _ptr(info), _stream(dev))
    _check(rc, "rsvd_id")
    return J, T[:, :n - k], info


def id_left(A, k, p, q, seed):
    """Rank-k column ID from the left sample Y = Omega~ A (A^T A)^q (Alg. 6):
    J (n; skeleton J[:k]), T (k x (n-k)), info."""
    lib = _lib.load()
    A = _row_major(A)
    dev = A.device
    m, n = A.shape
    dt = _dtype_code(A)
    wb = lib.rsvd_id_left_workspace_bytes(dt, m, n, k, p, q)
    if wb == 0:
        raise RsvdError("invalid sizes")
    work = _workspace(wb, dev)
    info = torch.zeros(2, dtype=torch.int32, device=dev)
    J = torch.empty(n, dtype=torch.int64, device=dev)
    ldt = max(n - k, 1)
    T = torch.empty((k, ldt), dtype=torch.float64, device=dev)
    rc = lib.rsvd_id_left(handle(dev), dt, m, n, k, p, q, seed, _ptr(A), A.stride(0), _ptr(J),
                          _ptr(T), ldt, _ptr(work), work.numel(), _ptr(info), _stream(dev))
    _check(rc, "rsvd_id_left")
    return J, T[:, :n - k], info


def qb(A, b, M, q, tol, seed):
    """Blocked adaptive QB (Alg. 7) of an FP64 A, which is not modified (the
    library deflates a copy): Q (m x b*nblocks), B (b*nblocks x n), the
    residual ||A - Q B||_F, the deflated copy R = A - Q B, info."""
    lib = _lib.load()
    A = _row_major(A)
    dev = A.device
    m, n = A.shape
    dt = _dtype_code(A)
    wb = lib.rsvd_qb_workspace_bytes(dt, m, n, b, M, q)
    if wb == 0:
        raise RsvdError("invalid sizes or type")
    R = A.clone()
    work = _workspace(wb, dev)
    info = torch.zeros(2, dtype=torch.int32, device=dev)
    Q = torch.empty((m, b * M), dtype=torch.float64, device=dev)
    B = torch.empty((b * M, n), dtype=torch.float64, device=dev)
    nb = ctypes.c_int32(0)
    res = ctypes.c_double(0.0)
    rc = lib.rsvd_qb(handle(dev), dt, m, n, b, M, q, float(tol), seed, _ptr(R), R.stride(0),
                     _ptr(Q), Q.stride(0), _ptr(B), B.stride(0), ctypes.byref(nb),
                     ctypes.byref(res), _ptr(work), work.numel(), _ptr(info), _stream(dev))
    _check(rc, "rsvd_qb")
    k = b * nb.value
    return Q[:, :k], B[:k], res.value, R, info


def svd_grad(A, k, p, q, seed, dU=None, dS=None, dV=None, dres=None, outputs=False):
    """Reverse-mode derivative of the randomized SVD of an FP64 A (sketch fixed).

    dU (m x k), dS (k), dV (n x k) and dres (a 0-dim or 1-element tensor, the
    cotangent of ||A - Q Q^T A||_F^2) may be None for zero.  Returns dA, and
    with outputs=True the tuple (dA, U, S, V, resid2) of the recomputed
    forward.  With all cotangents None and outputs=True only the forward runs
    (dA is None)."""
    lib = _lib.load()
    A = _row_major(A)
    dev = A.device
    m, n = A.shape
    dt = _dtype_code(A)
    wb = lib.rsvd_svd_grad_workspace_bytes(dt, m, n, k, p, q)
    if wb == 0:
        raise RsvdError("invalid sizes or type")

    def cot(t, shape):
        if t is None:
            return None
        t = t.to(device=dev, dtype=torch.float64).reshape(shape)
        return t.contiguous()

    dU = cot(dU, (m, k))
    dS = cot(dS, (k,))
    dV = cot(dV, (n, k))
    dres = cot(dres, (1,))
    want_grad = any(t is not None for t in (dU, dS, dV, dres))
    dA = torch.empty((m, n), dtype=torch.float64, device=dev) if want_grad else None
    U = S = V = r2 = None
    if outputs:
        U = torch.empty((m, k), dtype=torch.float64, device=dev)
        S = torch.empty(k, dtype=torch.float64, device=dev)
        V = torch.empty((n, k), dtype=torch.float64, device=dev)
        r2 = torch.empty(1, dtype=torch.float64, device=dev)
    if dA is None and not outputs:
        raise RsvdError("nothing to compute: no cotangent and outputs=False")
    work = _workspace(wb, dev)
    info = torch.zeros(2, dtype=torch.int32, device=dev)
    rc = lib.rsvd_svd_grad(handle(dev), dt, m, n, k, p, q, seed, _ptr(A), A.stride(0), _ptr(dU),
                           k, _ptr(dS), _ptr(dV), k, _ptr(dres), _ptr(dA), n, _ptr(U), k, _ptr(S),
                           _ptr(V), k, _ptr(r2), _ptr(work), work.numel(), _ptr(info),
                           _stream(dev))
    _check(rc, "rsvd_svd_grad")
    if outputs:
        return dA, U, S, V, r2.reshape(())
    return dA


class _SvdFunction(torch.autograd.Function):
    """U, S, V and ||A - Q Q^T A||_F^2 of the randomized SVD as a
    differentiable function of A; the backward recomputes the forward."""

    @staticmethod
    def forward(ctx, A, k, p, q, seed):
        _, U, S, V, r2 = svd_grad(A, k, p, q, seed, outputs=True)
        ctx.save_for_backward(A)
        ctx.cfg = (k, p, q, seed)
        ctx.set_materialize_grads(False)
        return U, S, V, r2

    @staticmethod
    def backward(ctx, dU, dS, dV, dr2):
        (A,) = ctx.saved_tensors
        if all(t is None for t in (dU, dS, dV, dr2)):
            return None, None, None, None, None
        k, p, q, seed = ctx.cfg
        dA = svd_grad(A, k, p, q, seed, dU=dU, dS=dS, dV=dV, dres=dr2)
        return dA.to(A.dtype), None, None, None, None


def svd_diff(A, k, p, q, seed):
    """Differentiable randomized SVD of an FP64 A: (U, S, V, resid2) with
    resid2 = ||A - Q Q^T A||_F^2; gradients flow to A through the library's
    adjoint (sketch fixed)."""
    return _SvdFunction.apply(A, k, p, q, seed)


class BatchPlan:
    """Batched randomized SVD of FP32 matrices (rsvd_batch_*): the plan fixes
    the sizes; pack() lays the matrices out in one buffer, run() launches the
    persistent kernel (capturable in a CUDA/HIP graph once prepared), unpack()
    splits U, S, V per matrix."""

    def __init__(self, ms, ns, ks, p, q, device="cuda", variants=None):
        """variants: pass shape per matrix (an int for all, a sequence, or None
        for the autotuned table's choice; see batch_tune)."""
        import numpy as np
        from . import batch_tune
        lib = _lib.load()
        self.device = torch.device(device)
        self.count = len(ms)
        self.ms = np.asarray(ms, dtype=np.int64)
        self.ns = np.asarray(ns, dtype=np.int64)
        self.ks = np.asarray(ks, dtype=np.int32)
        if not (len(self.ns) == self.count == len(self.ks)):
            raise RsvdError("ms, ns, ks must have the same length")
        self.p, self.q = p, q
        plan = ctypes.c_void_p()
        rc = lib.rsvd_batch_create(handle(self.device), self.count,
                                   self.ms.ctypes.data_as(ctypes.c_void_p),
                                   self.ns.ctypes.data_as(ctypes.c_void_p),
                                   self.ks.ctypes.data_as(ctypes.c_void_p), p, q,
                                   ctypes.byref(plan))
        _check(rc, "rsvd_batch_create")
        self._plan = plan
        if variants is None:
            ls = np.minimum(self.ks.astype(np.int64) + p, np.minimum(self.ms, self.ns))
            variants = batch_tune.choose(self.ms, self.ns, ls)
        self.variants = np.ascontiguousarray(
            np.broadcast_to(np.asarray(variants, dtype=np.int32), (self.count,)))
        rc = lib.rsvd_batch_set_variants(plan, self.variants.ctypes.data_as(ctypes.c_void_p))
        _check(rc, "rsvd_batch_set_variants")
        tot = [ctypes.c_int64(0) for _ in range(4)]
        offs = [np.zeros(self.count, dtype=np.int64) for _ in range(5)]
        rc = lib.rsvd_batch_layout(plan, *[ctypes.byref(t) for t in tot],
                                   *[o.ctypes.data_as(ctypes.c_void_p) for o in offs])
        _check(rc, "rsvd_batch_layout")
        self.a_elems, self.u_elems, self.s_elems, self.v_elems = [t.value for t in tot]
        self.a_off, self.lda, self.u_off, self.s_off, self.v_off = offs
        self.work_bytes = int(lib.rsvd_batch_workspace_bytes(plan))
        self.work = _workspace(self.work_bytes, self.device)
        rc = lib.rsvd_batch_prepare(plan, _ptr(self.work), self.work.numel(),
                                    _stream(self.device))
        _check(rc, "rsvd_batch_prepare")

    def __del__(self):
        plan = getattr(self, "_plan", None)
        if plan is not None and _lib._lib is not None:
            _lib._lib.rsvd_batch_destroy(plan)
            self._plan = None

    def pack(self, As):
        """One FP32 buffer holding every A_i at its offset (rows padded to lda)."""
        buf = torch.zeros(self.a_elems + 4, dtype=torch.float32, device=self.device)
        for i, A in enumerate(As):
            m, n = int(self.ms[i]), int(self.ns[i])
            ld, off = int(self.lda[i]), int(self.a_off[i])
            view = buf[off:off + m * ld].view(m, ld)
            view[:, :n] = torch.as_tensor(A, device=self.device).to(torch.float32)
        return buf

    def outputs(self):
        dev = self.device
        return (torch.empty(max(self.u_elems, 1), dtype=torch.float32, device=dev),
                torch.empty(max(self.s_elems, 1), dtype=torch.float64, device=dev),
                torch.empty(max(self.v_elems, 1), dtype=torch.float32, device=dev),
                torch.zeros(2, dtype=torch.int32, device=dev))

    def run(self, A_packed, seed, out=None):
        """Launch the batch; out = (U, S, V, info) buffers from outputs() (new ones
        when None).  Returns the four buffers."""
        lib = _lib.load()
        if A_packed.dtype != torch.float32 or A_packed.numel() < self.a_elems:
            raise RsvdError("A_packed must be the FP32 buffer from pack()")
        U, S, V, info = self.outputs() if out is None else out
        rc = lib.rsvd_batch_svd(self._plan, seed, _ptr(A_packed), _ptr(U), _ptr(S), _ptr(V),
                                _ptr(self.work), self.work.numel(), _ptr(info),
                                _stream(self.device))
        _check(rc, "rsvd_batch_svd")
        return U, S, V, info

    def unpack(self, U, S, V):
        """Per-matrix views (U_i m_i x k_i, S_i k_i, V_i n_i x k_i)."""
        res = []
        for i in range(self.count):
            m, n, k = int(self.ms[i]), int(self.ns[i]), int(self.ks[i])
            uo, so, vo = int(self.u_off[i]), int(self.s_off[i]), int(self.v_off[i])
            res.append((U[uo:uo + m * k].view(m, k), S[so:so + k], V[vo:vo + n * k].view(n, k)))
        return res


def cur(A, k, p, q, seed):
    """Rank-k CUR: Jc (k), Jr (k), U (k x k FP64), info; A ~ A[:, Jc] U A[Jr, :]."""
    lib = _lib.load()
    A = _row_major(A)
    dev = A.device
    m, n = A.shape
    dt = _dtype_code(A)
    work = _workspace(workspace_bytes(OP_CUR, dt, m, n, k, p, q), dev)
    info = torch.zeros(2, dtype=torch.int32, device=dev)
    Jc = torch.empty(k, dtype=torch.int64, device=dev)
    Jr = torch.empty(k, dtype=torch.int64, device=dev)
    U = torch.empty((k, k), dtype=torch.float64, device=dev)
    rc = lib.rsvd_cur(handle(dev), dt, m, n, k, p, q, seed, _ptr(A), A.stride(0), _ptr(Jc),
                      _ptr(Jr), _ptr(U), k, _ptr(work), work.numel(), _ptr(info), _stream(dev))
    _check(rc, "rsvd_cur")
    return Jc, Jr, U, info


# ------------------------------------------------------------------ steps --

def sketch(n, l, seed, dtype=torch.float64, device="cuda", ldo=None):
    lib = _lib.load()
    ldo = l if ldo is None else ldo
    om = torch.empty((n, ldo), dtype=dtype, device=device)
    dt = F64 if dtype == torch.float64 else F32
    rc = lib.rsvd_sketch(handle(om.device), dt, seed, n, l, _ptr(om), ldo, _stream(om.device))
    _check(rc, "rsvd_sketch")
    return om


def philox(seed, stream_id, batch, first, count, device="cuda"):
    """Raw Philox words as an int32 tensor of shape (count, 4) (bit patterns)."""
    lib = _lib.load()
    out = torch.empty((count, 4), dtype=torch.int32, device=device)
    rc = lib.rsvd_philox(handle(out.device), seed, stream_id, batch, first, count, _ptr(out),
                         _stream(out.device))
    _check(rc, "rsvd_philox")
    return out


def quantize(A, dtype):
    """rsvd_quantize: the storage formats of the mixed-precision path from an
    FP64 A.  dtype BF16 -> a torch.bfloat16 matrix (rounded to nearest even
    from FP64); dtype F8E4M3 -> (codes, scales): uint8 E4M3 codes with a
    leading dimension padded to 16 bytes (a view of the first n columns) and
    the FP32 column scales, A ~ dec(codes) diag(scales)."""
    lib = _lib.load()
    A = _row_major(A)
    if A.dtype != torch.float64:
        raise RsvdError("quantize takes an FP64 matrix")
    m, n = A.shape
    dev = A.device
    if dtype == BF16:
        Aq = torch.empty((m, (n + 7) // 8 * 8), dtype=torch.bfloat16, device=dev)
        rc = lib.rsvd_quantize(handle(dev), BF16, m, n, _ptr(A), A.stride(0), _ptr(Aq),
                               Aq.stride(0), None, _stream(dev))
        _check(rc, "rsvd_quantize")
        return Aq[:, :n]
    if dtype == F8E4M3:
        Aq = torch.empty((m, (n + 15) // 16 * 16), dtype=torch.uint8, device=dev)
        sc = torch.empty(n, dtype=torch.float32, device=dev)
        rc = lib.rsvd_quantize(handle(dev), F8E4M3, m, n, _ptr(A), A.stride(0), _ptr(Aq),
                               Aq.stride(0), _ptr(sc), _stream(dev))
        _check(rc, "rsvd_quantize")
        return Aq[:, :n], sc
    raise RsvdError("quantize: dtype must be BF16 or F8E4M3")


def svd_ex(A, k, p, q, seed, scales=None, want_Q=False):
    """rsvd_svd_ex: the randomized SVD of `svd`, also for an FP8 A (uint8
    E4M3 codes with FP32 column scales), optionally returning the range
    finder's basis Q.  Returns U, S, V, info, Q (None unless want_Q)."""
    lib = _lib.load()
    dev = A.device
    if A.dtype == torch.uint8:
        if scales is None:
            raise RsvdError("an FP8 A needs its column scales")
        if A.stride(1) != 1 or A.stride(0) % 16 or A.data_ptr() % 16:
            raise RsvdError("FP8 A: rows must be contiguous with a leading dimension of 16k bytes")
        dt, ot = F8E4M3, torch.float32
    else:
        A = _row_major(A)
        dt, ot = _dtype_code(A), _out_dtype(A)
    m, n = A.shape
    l = min(k + p, m, n)
    wb = workspace_bytes(OP_SVD, dt, m, n, k, p, q)
    if wb == 0:
        raise RsvdError("invalid sizes")
    work = _workspace(wb, dev)
    info = torch.zeros(2, dtype=torch.int32, device=dev)
    U = torch.empty((m, k), dtype=ot, device=dev)
    S = torch.empty(k, dtype=torch.float64, device=dev)
    V = torch.empty((n, k), dtype=ot, device=dev)
    Qb = torch.empty((m, l), dtype=ot, device=dev) if want_Q else None
    rc = lib.rsvd_svd_ex(handle(dev), dt, m, n, k, p, q, seed, _ptr(A), A.stride(0),
                         _ptr(scales) if scales is not None else None, _ptr(U), k, _ptr(S),
                         _ptr(V), k, _ptr(Qb), l, _ptr(work), work.numel(), _ptr(info),
                         _stream(dev))
    _check(rc, "rsvd_svd_ex")
    return U, S, V, info, Qb


def pass_f8(A8, scales, X, trans=False, split=False):
    """rsvd_pass_f8: Y = A X or A^T X for A ~ dec(A8) diag(scales), X FP32."""
    lib = _lib.load()
    if A8.dtype != torch.uint8 or A8.stride(1) != 1 or A8.stride(0) % 16 or A8.data_ptr() % 16:
        raise RsvdError("A8: uint8 codes, rows contiguous, leading dimension a multiple of 16")
    X = _row_major(X)
    if X.dtype != torch.float32:
        raise RsvdError("X must be FP32")
    m, n = A8.shape
    l = X.shape[1]
    rows = n if trans else m
    Y = torch.empty((rows, l), dtype=torch.float32, device=A8.device)
    work = _workspace(lib.rsvd_pass_f8_workspace_bytes(int(trans), m, n, l), A8.device)
    rc = lib.rsvd_pass_f8(handle(A8.device), int(trans), m, n, l, _ptr(A8), A8.stride(0),
                          _ptr(scales), _ptr(X), X.stride(0), _ptr(Y), l, int(split), _ptr(work),
                          work.numel(), _stream(A8.device))
    _check(rc, "rsvd_pass_f8")
    return Y


def pass_(A, X, trans=False):
    """Y = A X (trans=False) or Y = A^T X (trans=True) on the matrix cores."""
    lib = _lib.load()
    A = _row_major(A)
    X = _row_major(X)
    m, n = A.shape
    l = X.shape[1]
    dt = _dtype_code(A)
    rows = n if trans else m
    Y = torch.empty((rows, l), dtype=_out_dtype(A), device=A.device)
    wb = lib.rsvd_pass_workspace_bytes(dt, int(trans), m, n, l)
    work = _workspace(wb, A.device)
    rc = lib.rsvd_pass(handle(A.device), dt, int(trans), m, n, l, _ptr(A), A.stride(0), _ptr(X),
                       X.stride(0), _ptr(Y), l, _ptr(work), work.numel(), _stream(A.device))
    _check(rc, "rsvd_pass")
    return Y


def orth(Y, seed=0, want_R=True):
    """Q, R, info with Y = Q R, Q orthonormal (CholeskyQR2, FP64 Gram)."""
    lib = _lib.load()
    Y = _row_major(Y)
    rows, l = Y.shape
    dt = _dtype_code(Y)
    Q = torch.empty((rows, l), dtype=Y.dtype, device=Y.device)
    R = torch.empty((l, l), dtype=torch.float64, device=Y.device) if want_R else None
    work = _workspace(lib.rsvd_orth_workspace_bytes(dt, rows, l), Y.device)
    info = torch.zeros(2, dtype=torch.int32, device=Y.device)
    rc = lib.rsvd_orth(handle(Y.device), dt, rows, l, _ptr(Y), Y.stride(0), _ptr(Q), l, _ptr(R),
                       l, seed, _ptr(work), work.numel(), _ptr(info), _stream(Y.device))
    _check(rc, "rsvd_orth")
    return Q, R, info


def small_svd(Rh, k):
    """S (k), Uh (l x k), Vh (l x k), info with Rh = Uh diag(S) Vh^T (top k)."""
    lib = _lib.load()
    Rh = _row_major(Rh)
    l = Rh.shape[0]
    S = torch.empty(k, dtype=torch.float64, device=Rh.device)
    Uh = torch.empty((l, k), dtype=torch.float64, device=Rh.device)
    Vh = torch.empty((l, k), dtype=torch.float64, device=Rh.device)
    work = _workspace(lib.rsvd_small_svd_workspace_bytes(l), Rh.device)
    info = torch.zeros(2, dtype=torch.int32, device=Rh.device)
    rc = lib.rsvd_small_svd(handle(Rh.device), l, k, _ptr(Rh), Rh.stride(0), _ptr(S), _ptr(Uh), k,
                            _ptr(Vh), k, _ptr(work), work.numel(), _ptr(info), _stream(Rh.device))
    _check(rc, "rsvd_small_svd")
    return S, Uh, Vh, info


def cpqr(Bcols, r, k):
    """k-step column-pivoted QR of the r x c matrix whose column j is row j of
    Bcols (c x >= r).  Returns J (c), T (k x (c-k)), pivot norms (k), info."""
    lib = _lib.load()
    Bcols = _row_major(Bcols)
    c = Bcols.shape[0]
    dt = _dtype_code(Bcols)
    dev = Bcols.device
    J = torch.empty(c, dtype=torch.int64, device=dev)
    ldt = max(c - k, 1)
    T = torch.empty((k, ldt), dtype=torch.float64, device=dev)
    pv = torch.empty(k, dtype=torch.float64, device=dev)
    work = _workspace(lib.rsvd_cpqr_workspace_bytes(r, c, k), dev)
    info = torch.zeros(2, dtype=torch.int32, device=dev)
    rc = lib.rsvd_cpqr(handle(dev), dt, r, c, k, _ptr(Bcols), Bcols.stride(0), _ptr(J), _ptr(T),
                       ldt, _ptr(pv), _ptr(work), work.numel(), _ptr(info), _stream(dev))
    _check(rc, "rsvd_cpqr")
    return J, T[:, :c - k], pv, info
