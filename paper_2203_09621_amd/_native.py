"""ctypes binding of libdmpt (the C ABI in include/dmpt.h).

Argument marshalling only: every step of the method runs in the HIP library.
If the shared library is missing the import of this module fails loudly;
there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_char_p, c_double, c_int8, c_int32, c_int64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdmpt.so")

DMPT_MAX_K = 8
DMPT_MAX_LAYERS = 256

STATUS = {0: "DMPT_OK", -1: "DMPT_EINVAL", -2: "DMPT_ENOMEM", -3: "DMPT_EHIP",
          -4: "DMPT_ENOCONV", -5: "DMPT_ENONFINITE", -6: "DMPT_EASYM", -7: "DMPT_ENOTSUP"}
PRECISION = {"fp64": 0, "fp32": 1, "split_bf16": 2, "split_fp16": 3}

# every entry point declared in include/dmpt.h
EXPORTS = ["dmpt_default_options", "dmpt_init", "dmpt_set_hamiltonian", "dmpt_response",
           "dmpt_response2", "dmpt_contract", "dmpt_contract_noalloc", "dmpt_inverse_factor", "dmpt_congruence",
           "dmpt_cpscf", "dmpt_adjoint", "dmpt_response_adjoint", "dmpt_destroy",
           "dmpt_batch_init", "dmpt_batch_response", "dmpt_batch_info", "dmpt_batch_destroy",
           "dmpt_status_str", "dmpt_last_error", "dmpt_layer_products", "dmpt_layer_trace",
           "dmpt_gershgorin", "dmpt_selftest_mfma", "dmpt_probe_mfma", "dmpt_plan_rounds",
           "dmpt_plan_layer"]


class DmptOptions(ctypes.Structure):
    _fields_ = [("precision", c_int32), ("max_layers", c_int32),
                ("check_symmetry", c_int32), ("poll_every", c_int32), ("timing", c_int32),
                ("ckpt_every", c_int32), ("graph", c_int32), ("tile_threshold", c_int32)]


class DmptStats(ctypes.Structure):
    _fields_ = [("layers", c_int32), ("d0_layer", c_int32),
                ("d1_layer", c_int32 * DMPT_MAX_K), ("k", c_int32), ("converged", c_int32),
                ("sigma", c_int8 * DMPT_MAX_LAYERS),
                ("eps1", c_double), ("epsN", c_double), ("n_s", c_double), ("idem0", c_double),
                ("idem1", c_double * DMPT_MAX_K), ("trace_p0", c_double),
                ("trace_p1", c_double * DMPT_MAX_K), ("ms", c_double),
                ("product_ms", c_double), ("product_launches", c_int32), ("x_layers", c_int32)]

    def as_dict(self) -> dict:
        k = self.k
        return {
            "layers": self.layers, "d0_layer": self.d0_layer,
            "d1_layer": list(self.d1_layer[:k]), "k": k, "converged": bool(self.converged),
            "sigma": list(self.sigma[:self.layers]), "eps1": self.eps1, "epsN": self.epsN,
            "n_s": self.n_s, "idem0": self.idem0, "idem1": list(self.idem1[:k]),
            "trace_p0": self.trace_p0, "trace_p1": list(self.trace_p1[:k]), "ms": self.ms,
            "product_ms": self.product_ms, "product_launches": self.product_launches,
            "x_layers": self.x_layers,
        }


class DmptProblemStats(ctypes.Structure):
    _fields_ = [("layers", c_int32), ("d0_layer", c_int32), ("converged", c_int32), ("k", c_int32),
                ("d1_layer", c_int32 * 3), ("pad", c_int32), ("idem0", c_double),
                ("idem1", c_double * 3)]

    def as_dict(self) -> dict:
        k = self.k
        return {"layers": self.layers, "d0_layer": self.d0_layer,
                "converged": bool(self.converged), "k": k, "d1_layer": list(self.d1_layer[:k]),
                "idem0": self.idem0, "idem1": list(self.idem1[:k])}


# induced-field callback of dmpt_cpscf: (user, P1, G, stream)
_FIELD_FN = ctypes.CFUNCTYPE(None, c_void_p, c_void_p, c_void_p, c_void_p)


class DmptError(RuntimeError):
    def __init__(self, status: int, message: str, stats: dict | None = None):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.stats = stats


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2203_09621_amd.build` (no fallback exists)")
    lib = ctypes.CDLL(LIB_PATH)
    lib.dmpt_default_options.argtypes = [POINTER(DmptOptions)]
    lib.dmpt_default_options.restype = None
    lib.dmpt_init.argtypes = [POINTER(c_void_p), c_void_p, c_int64, c_int64, c_int32,
                              POINTER(DmptOptions), c_void_p]
    lib.dmpt_init.restype = c_int32
    lib.dmpt_set_hamiltonian.argtypes = [c_void_p, c_void_p]
    lib.dmpt_set_hamiltonian.restype = c_int32
    lib.dmpt_response.argtypes = [c_void_p, POINTER(c_void_p), c_int32, c_void_p,
                                  POINTER(c_void_p), POINTER(DmptStats)]
    lib.dmpt_response.restype = c_int32
    lib.dmpt_response2.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                   POINTER(DmptStats)]
    lib.dmpt_response2.restype = c_int32
    lib.dmpt_contract.argtypes = [POINTER(c_void_p), c_int32, POINTER(c_void_p), c_int32, c_int64,
                                  POINTER(c_double), c_void_p]
    lib.dmpt_contract.restype = c_int32
    lib.dmpt_contract_noalloc.argtypes = lib.dmpt_contract.argtypes
    lib.dmpt_contract_noalloc.restype = c_int32
    lib.dmpt_cpscf.argtypes = [c_void_p, c_void_p, _FIELD_FN, c_void_p, c_double, c_double,
                               c_int32, c_void_p, c_void_p, c_void_p, POINTER(c_int32),
                               POINTER(c_double), POINTER(DmptStats)]
    lib.dmpt_cpscf.restype = c_int32
    lib.dmpt_inverse_factor.argtypes = [c_int32, c_void_p, c_int64, c_void_p, c_int32, c_double,
                                        POINTER(c_int32), POINTER(c_double), c_void_p]
    lib.dmpt_inverse_factor.restype = c_int32
    lib.dmpt_congruence.argtypes = [c_int32, c_int64, c_void_p, c_void_p, c_void_p, c_void_p]
    lib.dmpt_congruence.restype = c_int32
    lib.dmpt_adjoint.argtypes = [c_void_p, POINTER(c_void_p), c_int32, c_void_p, c_void_p,
                                 POINTER(c_void_p), POINTER(DmptStats)]
    lib.dmpt_adjoint.restype = c_int32
    lib.dmpt_response_adjoint.argtypes = [c_void_p, POINTER(c_void_p), c_int32, POINTER(c_void_p),
                                          c_void_p, c_void_p, POINTER(c_void_p), c_void_p,
                                          POINTER(c_void_p), POINTER(DmptStats)]
    lib.dmpt_response_adjoint.restype = c_int32
    lib.dmpt_batch_init.argtypes = [POINTER(c_void_p), c_int32, POINTER(c_int64), POINTER(c_int64),
                                    POINTER(c_int32), POINTER(DmptOptions), c_void_p]
    lib.dmpt_batch_init.restype = c_int32
    lib.dmpt_batch_response.argtypes = [c_void_p, POINTER(c_void_p), POINTER(c_void_p),
                                        POINTER(c_void_p), POINTER(c_void_p),
                                        POINTER(DmptProblemStats), POINTER(c_double)]
    lib.dmpt_batch_response.restype = c_int32
    lib.dmpt_batch_info.argtypes = [c_void_p, POINTER(c_int32), POINTER(c_int32), POINTER(c_int32)]
    lib.dmpt_batch_info.restype = c_int32
    lib.dmpt_batch_destroy.argtypes = [c_void_p]
    lib.dmpt_batch_destroy.restype = None
    lib.dmpt_destroy.argtypes = [c_void_p]
    lib.dmpt_destroy.restype = None
    lib.dmpt_status_str.argtypes = [c_int32]
    lib.dmpt_status_str.restype = c_char_p
    lib.dmpt_last_error.argtypes = []
    lib.dmpt_last_error.restype = c_char_p
    lib.dmpt_layer_products.argtypes = [c_int32, c_int64, c_void_p, c_void_p, c_void_p, c_void_p,
                                        c_void_p]
    lib.dmpt_layer_products.restype = c_int32
    lib.dmpt_layer_trace.argtypes = [c_int32, c_int64, c_void_p, c_void_p, c_void_p]
    lib.dmpt_layer_trace.restype = c_int32
    lib.dmpt_gershgorin.argtypes = [c_void_p, c_int64, POINTER(c_double), c_void_p]
    lib.dmpt_gershgorin.restype = c_int32
    lib.dmpt_selftest_mfma.argtypes = [POINTER(c_int32), c_void_p]
    lib.dmpt_selftest_mfma.restype = c_int32
    lib.dmpt_probe_mfma.argtypes = [c_int32, POINTER(c_double), POINTER(c_double), c_void_p]
    lib.dmpt_probe_mfma.restype = c_int32
    lib.dmpt_plan_rounds.argtypes = [POINTER(c_int64), c_int32, c_int32, c_int64,
                                     POINTER(c_int32), POINTER(c_int64)]
    lib.dmpt_plan_rounds.restype = c_int32
    lib.dmpt_plan_layer.argtypes = [c_int32, c_int32, c_int32, c_int32, POINTER(c_int64),
                                    POINTER(c_int64)]
    lib.dmpt_plan_layer.restype = c_int32
    return lib


LIB = _load()


def last_error() -> str:
    return LIB.dmpt_last_error().decode()


def _check(status: int, stats: dict | None = None):
    if status != 0:
        raise DmptError(status, last_error(), stats)


# ---------------------------------------------------------------- torch marshalling
def _torch():
    import torch
    return torch


def _dev(t, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != torch.float64 or not t.is_contiguous() or t.dim() != 2 or t.shape[0] != t.shape[1]:
        raise TypeError(f"{name} must be a contiguous square float64 tensor")
    return c_void_p(t.data_ptr())


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return c_void_p(s.cuda_stream)


def default_options() -> DmptOptions:
    o = DmptOptions()
    LIB.dmpt_default_options(byref(o))
    return o


# ---------------------------------------------------------------- entry points
def dmpt_init(H0, nocc: int, k_max: int = 1, precision: str = "split_fp16",
              max_layers: int = 100, check_symmetry: bool = False, poll_every: int = 0,
              timing: bool = False, ckpt_every: int = 0, stream=None) -> c_void_p:
    """dmpt_init: Gershgorin bounds and the normalised S0 of H0 (device FP64)."""
    o = default_options()
    o.ckpt_every = int(ckpt_every)
    o.precision = PRECISION[precision]
    o.max_layers = max_layers
    o.check_symmetry = int(check_symmetry)
    o.poll_every = poll_every
    o.timing = int(timing)
    ctx = c_void_p()
    _check(LIB.dmpt_init(byref(ctx), _dev(H0, "H0"), H0.shape[0], int(nocc), int(k_max),
                         byref(o), _stream(stream)))
    return ctx


def dmpt_set_hamiltonian(ctx: c_void_p, H0) -> None:
    """dmpt_set_hamiltonian: new H0 of the same size; no allocation."""
    _check(LIB.dmpt_set_hamiltonian(ctx, _dev(H0, "H0")))


def dmpt_response(ctx: c_void_p, H1s, P0=None, P1s=None):
    """dmpt_response: P0 and P1_k for the perturbations H1s (device FP64).
    Returns (P0, [P1_k], stats)."""
    torch = _torch()
    k = len(H1s)
    n = H1s[0].shape[0]
    if P1s is None:
        P1s = [torch.empty_like(h) for h in H1s]
    if P0 is None:
        P0 = torch.empty_like(H1s[0])
    h_arr = (c_void_p * k)(*[_dev(h, "H1").value for h in H1s])
    p_arr = (c_void_p * k)(*[_dev(p, "P1").value for p in P1s])
    st = DmptStats()
    status = LIB.dmpt_response(ctx, h_arr, k, _dev(P0, "P0"), p_arr, byref(st))
    stats = st.as_dict()
    _check(status, stats)
    del n
    return P0, P1s, stats


def dmpt_response2(ctx: c_void_p, H1, H2=None, P0=None, P1=None, P2=None):
    """dmpt_response2: P0, P1 and the second-order P2 of H0 + l H1 + l^2 H2
    (H2 may be None).  The context needs k_max >= 2.  Returns (P0, P1, P2,
    stats); stats index 1 of d1_layer / idem1 / trace_p1 refers to P2."""
    torch = _torch()
    P0 = torch.empty_like(H1) if P0 is None else P0
    P1 = torch.empty_like(H1) if P1 is None else P1
    P2 = torch.empty_like(H1) if P2 is None else P2
    h2 = _dev(H2, "H2") if H2 is not None else c_void_p(None)
    st = DmptStats()
    status = LIB.dmpt_response2(ctx, _dev(H1, "H1"), h2, _dev(P0, "P0"), _dev(P1, "P1"),
                                _dev(P2, "P2"), byref(st))
    stats = st.as_dict()
    _check(status, stats)
    return P0, P1, P2, stats


def dmpt_contract(As, Bs, stream=None):
    """dmpt_contract: the matrix Tr(A_a B_b) (B_b symmetric) of device FP64
    matrices, e.g. Pi_ab = Tr(H1_a P1_b).  Returns a numpy (na, nb) array."""
    import numpy as np
    na, nb = len(As), len(Bs)
    n = As[0].shape[0]
    for m in list(As) + list(Bs):
        if tuple(m.shape) != (n, n):
            raise ValueError("every matrix must be N x N")
    out = (c_double * (na * nb))()
    _check(LIB.dmpt_contract((c_void_p * na)(*[_dev(a, "A").value for a in As]), na,
                             (c_void_p * nb)(*[_dev(b, "B").value for b in Bs]), nb, n, out,
                             _stream(stream)))
    return np.array(out[:]).reshape(na, nb)


def dmpt_contract_noalloc(As, Bs, stream=None):
    """dmpt_contract_noalloc: as dmpt_contract, with the partial sums in the
    library's fixed device scratch (no allocation; at most 64 pairs)."""
    import numpy as np
    na, nb = len(As), len(Bs)
    n = As[0].shape[0]
    for m in list(As) + list(Bs):
        if tuple(m.shape) != (n, n):
            raise ValueError("every matrix must be N x N")
    out = (c_double * (na * nb))()
    _check(LIB.dmpt_contract_noalloc((c_void_p * na)(*[_dev(a, "A").value for a in As]), na,
                                     (c_void_p * nb)(*[_dev(b, "B").value for b in Bs]), nb, n,
                                     out, _stream(stream)))
    return np.array(out[:]).reshape(na, nb)


def dmpt_cpscf(ctx: c_void_p, H1, field, mix: float = 1.0, tol: float = 1e-8,
               max_iter: int = 50, P0=None, P1=None, G=None):
    """dmpt_cpscf: self-consistent first-order response P1 = DP[H1 + field(P1)].
    ``field(P1, G)`` writes the induced field into the tensor G (torch ops).
    Returns (P0, P1, iters, change, stats)."""
    torch = _torch()
    P0 = torch.empty_like(H1) if P0 is None else P0
    P1 = torch.empty_like(H1) if P1 is None else P1
    G = torch.empty_like(H1) if G is None else G
    errors = []

    def cb(user, p1, g, stream):
        try:
            torch.cuda.synchronize()        # P1 of the library's stream is complete
            field(P1, G)
            torch.cuda.synchronize()        # G is complete before the library reads it
        except Exception as exc:            # noqa: BLE001 - reported after the call
            errors.append(exc)
            G.fill_(float("nan"))           # the next response then stops with ENONFINITE
            torch.cuda.synchronize()

    fn = _FIELD_FN(cb)
    it, ch = c_int32(0), c_double(0.0)
    st = DmptStats()
    status = LIB.dmpt_cpscf(ctx, _dev(H1, "H1"), fn, None, mix, tol, max_iter, _dev(P0, "P0"),
                            _dev(P1, "P1"), _dev(G, "G"), byref(it), byref(ch), byref(st))
    if errors:
        raise errors[0]
    _check(status, {"iters": it.value, "change": ch.value})
    return P0, P1, it.value, ch.value, st.as_dict()


def dmpt_inverse_factor(O, precision: str = "fp64", max_iter: int = 60, tol: float = 1e-12,
                        Z=None, stream=None):
    """dmpt_inverse_factor: Z = O^{-1/2} (Z O Z = I).  Returns (Z, iters, err)."""
    torch = _torch()
    Z = torch.empty_like(O) if Z is None else Z
    it, err = c_int32(0), c_double(0.0)
    _check(LIB.dmpt_inverse_factor(PRECISION[precision], _dev(O, "O"), O.shape[0], _dev(Z, "Z"),
                                   max_iter, tol, byref(it), byref(err), _stream(stream)),
           {"iters": it.value, "err": err.value})
    return Z, it.value, err.value


def dmpt_congruence(Z, A, precision: str = "fp64", out=None, stream=None):
    """dmpt_congruence: Z A Z for symmetric Z and A (device FP64)."""
    torch = _torch()
    out = torch.empty_like(A) if out is None else out
    _check(LIB.dmpt_congruence(PRECISION[precision], A.shape[0], _dev(Z, "Z"), _dev(A, "A"),
                               _dev(out, "out"), _stream(stream)))
    return out


def solve_nonorth(H0, O, H1s, nocc: int, precision: str = "split_fp16",
                  ortho_precision: str = "fp64", **kw):
    """P0 and P1_k in a non-orthogonal basis with overlap O (all device FP64):
    Z = O^{-1/2}, H_perp = Z H Z, the response in the orthogonal basis, then
    P = Z P_perp Z (Sec. II.A).  Every step is a library call."""
    Z, _, _ = dmpt_inverse_factor(O, precision=ortho_precision)
    Hp = dmpt_congruence(Z, H0, precision=ortho_precision)
    H1p = [dmpt_congruence(Z, h, precision=ortho_precision) for h in H1s]
    P0p, P1ps, st = solve(Hp, H1p, nocc, precision=precision, **kw)
    P0 = dmpt_congruence(Z, P0p, precision=ortho_precision)
    P1s = [dmpt_congruence(Z, q, precision=ortho_precision) for q in P1ps]
    return P0, P1s, st


def dmpt_adjoint(ctx: c_void_p, Ws, W0=None, dH0=None, dH1s=None):
    """dmpt_adjoint: gradients of L = Tr(P0 W0) + sum_k Tr(P1_k W_k) for the
    last response (W0 may be None).  Returns (dL/dH0, [dL/dH1_k], stats)."""
    torch = _torch()
    k = len(Ws)
    if dH0 is None:
        dH0 = torch.empty_like(Ws[0])
    if dH1s is None:
        dH1s = [torch.empty_like(w) for w in Ws]
    w_arr = (c_void_p * k)(*[_dev(w, "W").value for w in Ws])
    g_arr = (c_void_p * k)(*[_dev(g, "dH1").value for g in dH1s])
    w0 = _dev(W0, "W0") if W0 is not None else c_void_p(None)
    st = DmptStats()
    _check(LIB.dmpt_adjoint(ctx, w_arr, k, w0, _dev(dH0, "dH0"), g_arr, byref(st)))
    return dH0, dH1s, st.as_dict()


def dmpt_response_adjoint(ctx: c_void_p, H1s, Ws, W0=None, P0=None, P1s=None, dH0=None,
                          dH1s=None):
    """dmpt_response_adjoint: forward and reverse in one call.  Returns
    (P0, [P1_k], dL/dH0, [dL/dH1_k], stats)."""
    torch = _torch()
    k = len(H1s)
    P0 = torch.empty_like(H1s[0]) if P0 is None else P0
    P1s = [torch.empty_like(h) for h in H1s] if P1s is None else P1s
    dH0 = torch.empty_like(H1s[0]) if dH0 is None else dH0
    dH1s = [torch.empty_like(h) for h in H1s] if dH1s is None else dH1s
    arr = lambda ts, nm: (c_void_p * k)(*[_dev(t, nm).value for t in ts])   # noqa: E731
    w0 = _dev(W0, "W0") if W0 is not None else c_void_p(None)
    st = DmptStats()
    status = LIB.dmpt_response_adjoint(ctx, arr(H1s, "H1"), k, arr(Ws, "W"), w0, _dev(P0, "P0"),
                                       arr(P1s, "P1"), _dev(dH0, "dH0"), arr(dH1s, "dH1"),
                                       byref(st))
    stats = st.as_dict()
    _check(status, stats)
    return P0, P1s, dH0, dH1s, stats


def dmpt_destroy(ctx: c_void_p) -> None:
    LIB.dmpt_destroy(ctx)


def dmpt_layer_products(S, S1=None, precision: str = "split_fp16", stream=None):
    """dmpt_layer_products: X = S^2 and X1 = S S1 + S1 S with the layer kernels."""
    torch = _torch()
    X = torch.empty_like(S)
    X1 = torch.empty_like(S) if S1 is not None else None
    _check(LIB.dmpt_layer_products(PRECISION[precision], S.shape[0], _dev(S, "S"),
                                   _dev(S1, "S1") if S1 is not None else None,
                                   _dev(X, "X"), _dev(X1, "X1") if X1 is not None else None,
                                   _stream(stream)))
    return X, X1


def dmpt_layer_trace(S, precision: str = "split_fp16", stream=None):
    """dmpt_layer_trace: per 32-row block, the FP64 sum of the diagonal of S^2
    as the split layers take it before their products.  Returns a device
    float64 tensor of ceil(N/32) entries."""
    torch = _torch()
    n = S.shape[0]
    part = torch.empty((n + 31) // 32, dtype=torch.float64, device=S.device)
    _check(LIB.dmpt_layer_trace(PRECISION[precision], n, _dev(S, "S"), c_void_p(part.data_ptr()),
                                _stream(stream)))
    return part


def dmpt_gershgorin(H, stream=None):
    eps = (c_double * 2)()
    _check(LIB.dmpt_gershgorin(_dev(H, "H"), H.shape[0], eps, _stream(stream)))
    return float(eps[0]), float(eps[1])


def dmpt_plan_rounds(costs, grid: int, cap: int = None):
    """dmpt_plan_rounds: the library's dealing plan of items with these costs
    over `grid` slots (host only).  Returns an int32 array: per position the
    item index or -1.  The default capacity holds any plan: every round places
    an item or raises the target, at most (n + largest cost) rounds."""
    import numpy as np
    c = np.ascontiguousarray(costs, dtype=np.int64)
    n = int(c.size)
    if cap is None:
        cap = (n + (int(c.max()) if n else 0) + 1) * max(int(grid), 1)
    out = np.empty(max(cap, 1), dtype=np.int32)
    used = c_int64(0)
    _check(LIB.dmpt_plan_rounds(c.ctypes.data_as(POINTER(c_int64)), n, int(grid), cap,
                                out.ctypes.data_as(POINTER(c_int32)), byref(used)))
    return out[:used.value].copy()


def dmpt_plan_layer(T: int, k: int, k_max: int, grid: int = 256):
    """dmpt_plan_layer: (item positions of the fused launch for k responses,
    partial-slot capacity of a context with k_max responses), host only."""
    npos, cap = c_int64(0), c_int64(0)
    _check(LIB.dmpt_plan_layer(int(T), int(k), int(k_max), int(grid), byref(npos), byref(cap)))
    return npos.value, cap.value


def dmpt_probe_mfma(precision: str = "split_fp16", stream=None):
    """dmpt_probe_mfma: (TFLOP/s, shader GHz) of back-to-back MFMAs on random operands,
    for the MFMA instruction of `precision`'s product kernels."""
    tf, ghz = c_double(0.0), c_double(0.0)
    _check(LIB.dmpt_probe_mfma(PRECISION[precision], byref(tf), byref(ghz), _stream(stream)))
    return tf.value, ghz.value


def dmpt_selftest_mfma(stream=None) -> int:
    detail = c_int32(0)
    status = LIB.dmpt_selftest_mfma(byref(detail), _stream(stream))
    if status not in (0, -7):
        _check(status)
    return detail.value


def dmpt_batch_init(Ns, noccs, ks, precision: str = "split_bf16", max_layers: int = 100,
                    graph: bool = True, stream=None, tile_threshold: int = -1) -> c_void_p:
    """dmpt_batch_init: workspace and tile tuning for a batch of problems
    (tile_threshold >= 0 fixes the tile classes instead of timing them)."""
    count = len(Ns)
    o = default_options()
    o.precision = PRECISION[precision]
    o.max_layers = max_layers
    o.graph = int(graph)
    o.tile_threshold = int(tile_threshold)
    b = c_void_p()
    _check(LIB.dmpt_batch_init(byref(b), count, (c_int64 * count)(*Ns), (c_int64 * count)(*noccs),
                               (c_int32 * count)(*ks), byref(o), _stream(stream)))
    return b


def dmpt_batch_response(batch: c_void_p, H0s, H1s, P0s=None, P1s=None):
    """dmpt_batch_response: H0s a list of device tensors, H1s a list (per problem)
    of lists of device tensors.  Returns (P0s, P1s, per-problem stats, ms)."""
    torch = _torch()
    count = len(H0s)
    flat_h1 = [h for hs in H1s for h in hs]
    if P0s is None:
        P0s = [torch.empty_like(h) for h in H0s]
    if P1s is None:
        P1s = [[torch.empty_like(h) for h in hs] for hs in H1s]
    flat_p1 = [p for ps in P1s for p in ps]
    st = (DmptProblemStats * count)()
    ms = c_double(0.0)
    status = LIB.dmpt_batch_response(
        batch, (c_void_p * count)(*[_dev(h, "H0").value for h in H0s]),
        (c_void_p * len(flat_h1))(*[_dev(h, "H1").value for h in flat_h1]),
        (c_void_p * count)(*[_dev(p, "P0").value for p in P0s]),
        (c_void_p * len(flat_p1))(*[_dev(p, "P1").value for p in flat_p1]), st, byref(ms))
    stats = [x.as_dict() for x in st]
    _check(status, {"problems": stats})
    return P0s, P1s, stats, ms.value


def dmpt_batch_info(batch: c_void_p):
    th, n256, n128 = c_int32(), c_int32(), c_int32()
    _check(LIB.dmpt_batch_info(batch, byref(th), byref(n256), byref(n128)))
    return th.value, n256.value, n128.value


def dmpt_batch_destroy(batch: c_void_p) -> None:
    LIB.dmpt_batch_destroy(batch)


def solve(H0, H1s, nocc: int, precision: str = "split_fp16", max_layers: int = 100, **kw):
    """One-shot dmpt_init + dmpt_response + dmpt_destroy."""
    ctx = dmpt_init(H0, nocc, k_max=len(H1s), precision=precision, max_layers=max_layers, **kw)
    try:
        return dmpt_response(ctx, H1s)
    finally:
        dmpt_destroy(ctx)


class _OwnedContext:
    """A library context with its checkpoints, released exactly once: by
    close(), or when the holder is garbage-collected (an autograd graph that is
    dropped without a backward pass)."""

    def __init__(self, ctx: c_void_p):
        self.ctx = ctx

    def close(self) -> None:
        ctx, self.ctx = self.ctx, None
        if ctx is not None and ctx.value:
            dmpt_destroy(ctx)

    def __del__(self):
        self.close()


def _autograd_function(with_p0: bool):
    torch = _torch()

    class DMPTResponse(torch.autograd.Function):
        @staticmethod
        def forward(fctx, H0, H1, nocc, precision="split_bf16", ckpt_every=8):
            grad = bool(fctx.needs_input_grad[0] or fctx.needs_input_grad[1])
            owned = _OwnedContext(dmpt_init(H0.detach().contiguous(), nocc, k_max=1,
                                            precision=precision,
                                            ckpt_every=ckpt_every if grad else 0))
            try:
                P0, (P1,), _ = dmpt_response(owned.ctx, [H1.detach().contiguous()])
            except Exception:
                owned.close()
                raise
            if grad:
                fctx.dmpt = owned
            else:
                owned.close()
            return (P0, P1) if with_p0 else P1

        @staticmethod
        def backward(fctx, *grads):
            gP0, gP1 = grads if with_p0 else (None, grads[0])
            owned = fctx.dmpt
            if owned is None or owned.ctx is None:
                raise RuntimeError("DMPTResponse: backward called twice (the context is released)")
            if gP1 is None:
                gP1 = torch.zeros_like(gP0)
            try:
                dH0, (dH1,), _ = dmpt_adjoint(owned.ctx, [gP1.contiguous()],
                                              W0=None if gP0 is None else gP0.contiguous())
            finally:
                owned.close()
            return dH0, dH1, None, None, None

    return DMPTResponse


def response_function():
    """torch.autograd.Function: P1 = DMPTResponse.apply(H0, H1, nocc, precision, ckpt_every).
    Its backward calls dmpt_adjoint; gradients follow the symmetric convention
    (dL = <G, dH> for symmetric dH).  The context (with its checkpoints) lives
    until the backward pass, or until the graph is dropped; when no input needs
    a gradient it is released at the end of the forward."""
    return _autograd_function(False)


def density_function():
    """torch.autograd.Function: (P0, P1) = DMPTDensity.apply(H0, H1, nocc, precision,
    ckpt_every); the backward takes upstream gradients of both (dL/dP0 enters
    dmpt_adjoint as W0).  Context lifetime as response_function."""
    return _autograd_function(True)
