"""Thin ctypes binding of libpimm (Pi_MatMul, Algorithm 1 of arXiv 2305.18396).

Argument marshalling only: every step of the protocol runs in the library's
HIP kernels.  PyTorch provides device memory (tensors are int64 storage; the
library reads and writes them as uint64) and the current stream.  The module
refuses to work without the built library: there is no fallback.

Call names match the C ABI in include/pimm.h (without the ``pimm_`` prefix on
the Python side where a class method is more natural).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpimm.so")

PIMM_OK = 0
ERRORS = {-1: "PIMM_E_ARG", -2: "PIMM_E_SHAPE", -3: "PIMM_E_PARAMS", -4: "PIMM_E_NOISE",
          -5: "PIMM_E_OOM", -6: "PIMM_E_DEVICE", -7: "PIMM_E_UNSUPPORTED",
          -8: "PIMM_E_WORKSPACE"}

# Stream tags of the randomness layout.
TAG_SK, TAG_PK_A, TAG_PK_E, TAG_ENC_A, TAG_ENC_E = 1, 2, 3, 4, 5
TAG_RR_U, TAG_RR_E1, TAG_RR_E2, TAG_MASK = 6, 7, 8, 9

# Every function include/pimm.h and include/pimm_probe.h declare.
EXPORTS = [
    "pimm_ctx_create", "pimm_ctx_destroy", "pimm_ctx_primes", "pimm_ctx_cdt",
    "pimm_params_primes", "pimm_cdt", "pimm_plan_rule", "pimm_noise_ok", "pimm_switch_ok",
    "pimm_plan_create", "pimm_plan_create_grouped", "pimm_plan_destroy", "pimm_plan_query", "pimm_plan_set_tuning",
    "pimm_plan_get_tuning", "pimm_plan_autotune", "pimm_plan_select", "pimm_batch_autotune",
    "pimm_keygen", "pimm_sk_destroy", "pimm_encode_input", "pimm_encrypt", "pimm_encrypt_input",
    "pimm_decrypt",
    "pimm_weights_create", "pimm_weights_destroy", "pimm_matmul", "pimm_mask_share",
    "pimm_matmul_share", "pimm_matmul_share_noalloc",
    "pimm_fc_complete",
    "pimm_weights_update",
    "pimm_encrypt_seeded",
    "pimm_ct_expand",
    "pimm_mod_switch", "pimm_decrypt_switched",
    "pimm_batch_create", "pimm_batch_destroy", "pimm_batch_query", "pimm_batch_set_schedule",
    "pimm_batch_get_schedule",
    "pimm_batch_matmul", "pimm_batch_status",
    "pimm_serve_create", "pimm_serve_destroy", "pimm_serve_footprint", "pimm_serve_run",
    "pimm_poly_mul", "pimm_poly_mul_workspace", "pimm_sample_poly",
    "pimm_profile_enable", "pimm_profile_select", "pimm_profile_read", "pimm_sync",
    "pimm_last_error",
    "pimm_probe",
]

# Device-rate probes (include/pimm_probe.h).
PROBE_READ, PROBE_COPY, PROBE_FMA64 = 0, 1, 2
PROBE_MODMUL_F64, PROBE_MODMUL_BARRETT, PROBE_MODMUL_SHOUP = 3, 4, 5
PROBE_READ8 = 6


class PimmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint32) for n in
                ("N", "L", "log2_t", "frac_bits", "prime_bits", "rerandomize")]


class PlanInfo(ctypes.Structure):
    _fields_ = ([(n, ctypes.c_uint32) for n in
                 ("n", "r", "m", "mb", "rb", "nb", "M", "R", "K", "I", "O", "Wb")] +
                [(n, ctypes.c_uint64) for n in
                 ("P", "pt_bytes", "ct_bytes", "acc_bytes", "c1_bytes", "c0s_bytes",
                  "share_bytes", "weights_bytes", "workspace_bytes")] +
                [("groups", ctypes.c_uint32)])

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """The loaded libpimm.so.  Raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                          "(python paper_2305_18396_amd/build.py)")
    L = ctypes.CDLL(LIB_PATH)
    vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    sig = {
        "pimm_ctx_create": [vp, i32, vp],
        "pimm_ctx_destroy": [vp],
        "pimm_ctx_primes": [vp, vp],
        "pimm_ctx_cdt": [vp, vp],
        "pimm_params_primes": [vp, vp],
        "pimm_cdt": [vp],
        "pimm_plan_rule": [vp, u32, u32, u32, u32, u32, u32, u32, vp],
        "pimm_noise_ok": [vp, vp, u64],
        "pimm_switch_ok": [vp, vp, u64],
        "pimm_mod_switch": [vp, vp, vp, vp, vp, vp, vp],
        "pimm_decrypt_switched": [vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp],
        "pimm_plan_create": [vp, u32, u32, u32, u32, u32, u32, u32, vp],
        "pimm_plan_create_grouped": [vp, u32, u32, u32, u32, u32, u32, u32, u32, vp],
        "pimm_plan_destroy": [vp],
        "pimm_plan_query": [vp, vp],
        "pimm_plan_set_tuning": [vp, i32, i32, i32],
        "pimm_plan_get_tuning": [vp, vp, vp],
        "pimm_plan_autotune": [vp, vp, vp, vp, vp, ctypes.c_size_t, i32, vp, vp],
        "pimm_plan_select": [vp, u32, u32, u32, vp, ctypes.c_double, vp, u32, i32, vp, vp, vp, vp],
        "pimm_batch_autotune": [vp, vp, ctypes.c_size_t, i32, vp, vp],
        "pimm_keygen": [vp, vp, vp, vp, vp],
        "pimm_sk_destroy": [vp],
        "pimm_encode_input": [vp, vp, vp, vp],
        "pimm_encrypt": [vp, vp, vp, u32, vp, vp, vp, ctypes.c_size_t, vp],
        "pimm_encrypt_input": [vp, vp, vp, u32, vp, vp, vp, ctypes.c_size_t, vp],
        "pimm_decrypt": [vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp],
        "pimm_weights_create": [vp, vp, vp, vp],
        "pimm_weights_destroy": [vp],
        "pimm_matmul": [vp, vp, vp, vp, vp, ctypes.c_size_t, vp],
        "pimm_mask_share": [vp, vp, vp, u32, vp, vp, vp, vp, vp, ctypes.c_size_t, vp],
        "pimm_matmul_share": [vp, vp, vp, vp, u32, vp, vp, vp, vp, vp, ctypes.c_size_t, vp],
        "pimm_matmul_share_noalloc": [vp, vp, vp, vp, u32, vp, vp, vp, vp, vp],
        "pimm_fc_complete": [vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp],
        "pimm_weights_update": [vp, vp, u64, vp],
        "pimm_encrypt_seeded": [vp, vp, vp, vp, u32, vp, vp, vp, ctypes.c_size_t, vp],
        "pimm_ct_expand": [vp, vp, u32, vp, vp, vp],
        "pimm_batch_create": [vp, u32, vp],
        "pimm_batch_destroy": [vp],
        "pimm_batch_query": [vp, vp, vp],
        "pimm_batch_set_schedule": [vp, i32, i32, i32, i32, u32],
        "pimm_batch_get_schedule": [vp, vp, vp, vp, vp, vp],
        "pimm_batch_matmul": [vp, vp, ctypes.c_size_t, vp],
        "pimm_batch_status": [vp, vp, vp],
        "pimm_serve_create": [vp, vp, vp],
        "pimm_serve_destroy": [vp],
        "pimm_serve_footprint": [vp, u32, vp],
        "pimm_serve_run": [vp, vp, u32, vp, vp],
        "pimm_poly_mul": [vp, vp, vp, vp, u32, vp, ctypes.c_size_t, vp],
        "pimm_poly_mul_workspace": [vp, u32],
        "pimm_probe": [i32, i32, u64, i32, vp],
        "pimm_sample_poly": [vp, i32, vp, u32, u32, u32, u32, vp, vp],
        "pimm_profile_enable": [i32],
        "pimm_profile_select": [ctypes.c_char_p],
        "pimm_profile_read": [ctypes.c_char_p, vp, vp],
        "pimm_sync": [vp],
        "pimm_last_error": [],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    L.pimm_poly_mul_workspace.restype = ctypes.c_uint64
    L.pimm_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(rc: int):
    if rc < 0:
        raise PimmError(rc, lib().pimm_last_error().decode())
    return rc


def _ptr(t: torch.Tensor | None):
    if t is None:
        return None
    assert t.is_contiguous(), "libpimm buffers must be contiguous"
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _seed(seed: bytes):
    assert len(seed) == 32
    return ctypes.create_string_buffer(bytes(seed), 32)


def _words(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(1, (int(nbytes) + 7) // 8), dtype=torch.int64, device=device)


def to_device_u64(a: np.ndarray, device="cuda") -> torch.Tensor:
    """numpy uint64/int64 array -> device int64 tensor with the same bytes."""
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint64:
        a = a.view(np.int64)
    return torch.from_numpy(a.astype(np.int64, copy=False)).to(device)


def to_host_u64(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint64)


# ---------------------------------------------------------------------------
# host-only queries
# ---------------------------------------------------------------------------

def make_params(N: int, L: int, log2_t: int, frac_bits: int, rerandomize: bool = True) -> Params:
    return Params(N, L, log2_t, frac_bits, 50, 1 if rerandomize else 0)


def params_primes(params: Params) -> list[int]:
    q = (ctypes.c_uint64 * params.L)()
    _check(lib().pimm_params_primes(ctypes.byref(params), q))
    return list(q)


def cdt() -> list[int]:
    t = (ctypes.c_uint64 * 19)()
    _check(lib().pimm_cdt(t))
    return list(t)


def plan_rule(params: Params, n, r, m, mb=0, rb=0, nb=0, d_fix=0) -> PlanInfo:
    info = PlanInfo()
    _check(lib().pimm_plan_rule(ctypes.byref(params), n, r, m, mb, rb, nb, d_fix,
                                ctypes.byref(info)))
    return info


def noise_ok(params: Params, info: PlanInfo, wmax: int) -> bool:
    return _check(lib().pimm_noise_ok(ctypes.byref(params), ctypes.byref(info), int(wmax))) == 1


def switch_ok(params: Params, info: PlanInfo, wmax: int) -> bool:
    return _check(lib().pimm_switch_ok(ctypes.byref(params), ctypes.byref(info), int(wmax))) == 1


# ---------------------------------------------------------------------------
# handles
# ---------------------------------------------------------------------------

class Context:
    """pimm_ctx: parameters, primes and NTT tables on one device."""

    def __init__(self, N: int, L: int, log2_t: int, frac_bits: int, rerandomize: bool = True,
                 device: int = 0):
        self.params = make_params(N, L, log2_t, frac_bits, rerandomize)
        self.device = torch.device("cuda", device)
        self.h = ctypes.c_void_p()
        _check(lib().pimm_ctx_create(ctypes.byref(self.params), device, ctypes.byref(self.h)))

    @property
    def N(self):
        return self.params.N

    @property
    def L(self):
        return self.params.L

    @property
    def ell(self):
        return self.params.log2_t

    def primes(self) -> list[int]:
        q = (ctypes.c_uint64 * self.params.L)()
        _check(lib().pimm_ctx_primes(self.h, q))
        return list(q)

    def cdt(self) -> list[int]:
        t = (ctypes.c_uint64 * 19)()
        _check(lib().pimm_ctx_cdt(self.h, t))
        return list(t)

    def close(self):
        if self.h:
            lib().pimm_ctx_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """pimm_plan: block plan and buffer sizes of Y[n][m] = X[n][r] W[r][m]; with groups = G > 1,
    G products of that shape run as one (X, W and the shares gain a leading dimension G)."""

    def __init__(self, ctx: Context, n: int, r: int, m: int, mb=0, rb=0, nb=0, d_fix=0, groups=1):
        self.ctx = ctx
        self.h = ctypes.c_void_p()
        if groups == 1:
            _check(lib().pimm_plan_create(ctx.h, n, r, m, mb, rb, nb, d_fix, ctypes.byref(self.h)))
        else:
            _check(lib().pimm_plan_create_grouped(ctx.h, n, r, m, mb, rb, nb, d_fix, groups,
                                                  ctypes.byref(self.h)))
        info = PlanInfo()
        _check(lib().pimm_plan_query(self.h, ctypes.byref(info)))
        self.info = info
        self._ws = None

    def __getattr__(self, k):
        info = self.__dict__.get("info")
        if info is not None and k in dict(PlanInfo._fields_):
            return getattr(info, k)
        raise AttributeError(k)

    def share_shape(self):
        """Shape of a share (and of X, W with (n, r), (r, m)): (n, m), or (G, n, m) when grouped."""
        f = self.info
        return (f.n, f.m) if f.groups == 1 else (f.groups, f.n, f.m)

    def lead(self, *shape):
        """shape with the group dimension in front when the plan is grouped."""
        return tuple(shape) if self.info.groups == 1 else (self.info.groups, *shape)

    def set_tuning(self, mac_rows: int = 8, mac_cols: int = 1, waves: int = 1):
        _check(lib().pimm_plan_set_tuning(self.h, mac_rows, mac_cols, waves))

    def tuning(self):
        """-> (mac_rows, mac_cols, waves) of the product schedule."""
        g, k, w = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().pimm_plan_get_tuning(self.h, ctypes.byref(g), ctypes.byref(k), ctypes.byref(w)))
        return g.value, k.value, w.value

    def autotune(self, w, ct, acc, reps: int = 3, stream=None) -> float:
        """Time every product schedule on these buffers; keep the fastest.  -> best ms."""
        ws = self.workspace()
        best = ctypes.c_double()
        _check(lib().pimm_plan_autotune(self.h, w.h, _ptr(ct), _ptr(acc), _ptr(ws), ws.numel() * 8,
                                        reps, _stream(stream), ctypes.byref(best)))
        return best.value

    def workspace(self) -> torch.Tensor:
        """A workspace tensor of the plan's size, allocated once by torch."""
        if self._ws is None:
            self._ws = _words(self.info.workspace_bytes, self.ctx.device)
        return self._ws

    def close(self):
        if self.h:
            lib().pimm_plan_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan_select(ctx: Context, n: int, r: int, m: int, W: torch.Tensor, link_bits_per_s: float,
                d_candidates, reps: int = 2, stream=None):
    """pimm_plan_select: time the server step for each candidate block area (0 = fewest-wire plan)
    and pick the one minimising server time + wire time at this link speed.
    -> (best d, [server ms per candidate], [wire bytes per candidate])."""
    assert W.dtype == torch.int64 and tuple(W.shape) == (r, m) and W.is_contiguous()
    cnt = len(d_candidates)
    ds = (ctypes.c_uint32 * cnt)(*d_candidates)
    ms = (ctypes.c_double * cnt)()
    wire = (ctypes.c_uint64 * cnt)()
    best = ctypes.c_uint32()
    _check(lib().pimm_plan_select(ctx.h, n, r, m, _ptr(W), float(link_bits_per_s), ds, cnt, reps,
                                  _stream(stream), ctypes.byref(best), ms, wire))
    return best.value, list(ms), list(wire)


class SecretKey:
    def __init__(self, ctx: Context, h):
        self.ctx, self.h = ctx, h

    def close(self):
        if self.h:
            lib().pimm_sk_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Weights:
    """pimm_weights: the server's weight cache (pi_A blocks in NTT form) for one plan."""

    def __init__(self, plan: Plan, W: torch.Tensor, stream=None):
        assert W.dtype == torch.int64 and tuple(W.shape) == plan.lead(plan.info.r, plan.info.m)
        self.plan = plan
        self.h = ctypes.c_void_p()
        _check(lib().pimm_weights_create(plan.h, _ptr(W), ctypes.byref(self.h), _stream(stream)))

    def update(self, W: torch.Tensor, wmax: int, stream=None):
        """pimm_weights_update: new weights of the same shape, |W| <= wmax, no sync."""
        assert W.dtype == torch.int64 and tuple(W.shape) == self.plan.lead(self.plan.info.r,
                                                                           self.plan.info.m)
        _check(lib().pimm_weights_update(self.h, _ptr(W), int(wmax), _stream(stream)))

    def close(self):
        if self.h:
            lib().pimm_weights_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# protocol calls
# ---------------------------------------------------------------------------

def keygen(ctx: Context, seed: bytes, stream=None):
    """-> (SecretKey, pk [2][L][N] or None)."""
    h = ctypes.c_void_p()
    pk = None
    if ctx.params.rerandomize:
        pk = torch.empty((2, ctx.L, ctx.N), dtype=torch.int64, device=ctx.device)
    _check(lib().pimm_keygen(ctx.h, _seed(seed), ctypes.byref(h), _ptr(pk), _stream(stream)))
    return SecretKey(ctx, h), pk


def encode_input(plan: Plan, X: torch.Tensor, pt: torch.Tensor | None = None, stream=None):
    f = plan.info
    if pt is None:
        pt = torch.empty((f.I, plan.ctx.N), dtype=torch.int64, device=plan.ctx.device)
    _check(lib().pimm_encode_input(plan.h, _ptr(X), _ptr(pt), _stream(stream)))
    return pt


def encrypt(plan: Plan, sk: SecretKey, seed: bytes, op_id: int, pt: torch.Tensor,
            ct: torch.Tensor | None = None, ws: torch.Tensor | None = None, stream=None):
    f, c = plan.info, plan.ctx
    if ct is None:
        ct = torch.empty((f.I, 2, c.L, c.N), dtype=torch.int64, device=c.device)
    ws = plan.workspace() if ws is None else ws
    _check(lib().pimm_encrypt(plan.h, sk.h, _seed(seed), op_id, _ptr(pt), _ptr(ct), _ptr(ws),
                              ws.numel() * 8, _stream(stream)))
    return ct


def encrypt_input(plan: Plan, sk: SecretKey, seed: bytes, op_id: int, X: torch.Tensor,
                  ct: torch.Tensor | None = None, ws: torch.Tensor | None = None, stream=None):
    """pimm_encrypt_input: encode_input and encrypt in one pass (X [n][r], or [G][n][r])."""
    f, c = plan.info, plan.ctx
    if ct is None:
        ct = torch.empty((f.I, 2, c.L, c.N), dtype=torch.int64, device=c.device)
    ws = plan.workspace() if ws is None else ws
    _check(lib().pimm_encrypt_input(plan.h, sk.h, _seed(seed), op_id, _ptr(X), _ptr(ct), _ptr(ws),
                                    ws.numel() * 8, _stream(stream)))
    return ct


def matmul(plan: Plan, w: Weights, ct: torch.Tensor, acc: torch.Tensor | None = None,
           ws: torch.Tensor | None = None, stream=None):
    f, c = plan.info, plan.ctx
    if acc is None:
        acc = torch.empty((f.O, 2, c.L, c.N), dtype=torch.int64, device=c.device)
    ws = plan.workspace() if ws is None else ws
    _check(lib().pimm_matmul(plan.h, w.h, _ptr(ct), _ptr(acc), _ptr(ws), ws.numel() * 8,
                             _stream(stream)))
    return acc


def mask_share(plan: Plan, pk: torch.Tensor | None, seed: bytes, op_id: int, acc: torch.Tensor,
               c1=None, c0s=None, share=None, ws=None, stream=None):
    """In place on acc.  -> (c1 [O][L][N], c0s [O][L][mb*nb], server_share [n][m])."""
    f, c = plan.info, plan.ctx
    dev = c.device
    if c1 is None:
        c1 = torch.empty((f.O, c.L, c.N), dtype=torch.int64, device=dev)
    if c0s is None:
        c0s = torch.empty((f.O, c.L, f.mb * f.nb), dtype=torch.int64, device=dev)
    if share is None:
        share = torch.empty(plan.share_shape(), dtype=torch.int64, device=dev)
    ws = plan.workspace() if ws is None else ws
    _check(lib().pimm_mask_share(plan.h, _ptr(pk), _seed(seed), op_id, _ptr(acc), _ptr(c1),
                                 _ptr(c0s), _ptr(share), _ptr(ws), ws.numel() * 8,
                                 _stream(stream)))
    return c1, c0s, share


def matmul_share(plan: Plan, w: Weights, pk, seed: bytes, op_id: int, ct: torch.Tensor, c1=None,
                 c0s=None, share=None, ws=None, stream=None):
    """pimm_matmul + pimm_mask_share in one pass.  -> (c1, c0s, server_share)."""
    f, c = plan.info, plan.ctx
    dev = c.device
    if c1 is None:
        c1 = torch.empty((f.O, c.L, c.N), dtype=torch.int64, device=dev)
    if c0s is None:
        c0s = torch.empty((f.O, c.L, f.mb * f.nb), dtype=torch.int64, device=dev)
    if share is None:
        share = torch.empty(plan.share_shape(), dtype=torch.int64, device=dev)
    ws = plan.workspace() if ws is None else ws
    _check(lib().pimm_matmul_share(plan.h, w.h, _ptr(pk), _seed(seed), op_id, _ptr(ct), _ptr(c1),
                                   _ptr(c0s), _ptr(share), _ptr(ws), ws.numel() * 8,
                                   _stream(stream)))
    return c1, c0s, share


def matmul_share_noalloc(plan: Plan, w: Weights, pk, seed: bytes, op_id: int, ct: torch.Tensor,
                         c1: torch.Tensor, c0s: torch.Tensor, share: torch.Tensor, stream=None):
    """pimm_matmul_share_noalloc: the fused server step on the library's static scratch (no
    workspace, no allocation; the caller passes the outputs).  -> (c1, c0s, server_share)."""
    f, c = plan.info, plan.ctx
    for t, shape in ((c1, (f.O, c.L, c.N)), (c0s, (f.O, c.L, f.mb * f.nb)), (share, plan.share_shape())):
        assert t.dtype == torch.int64 and tuple(t.shape) == shape and t.is_contiguous()
    _check(lib().pimm_matmul_share_noalloc(plan.h, w.h, _ptr(pk), _seed(seed), op_id, _ptr(ct),
                                           _ptr(c1), _ptr(c0s), _ptr(share), _stream(stream)))
    return c1, c0s, share


def encrypt_seeded(plan: Plan, sk: SecretKey, seed: bytes, a_seed: bytes, op_id: int,
                   pt: torch.Tensor, ct=None, ws=None, stream=None):
    """pimm_encrypt_seeded: c1 = a from the public a_seed, e from seed.  -> ct [I][2][L][N]
    (the upload is ct[:, 0] and a_seed)."""
    f, c = plan.info, plan.ctx
    if ct is None:
        ct = torch.empty((f.I, 2, c.L, c.N), dtype=torch.int64, device=c.device)
    ws = plan.workspace() if ws is None else ws
    _check(lib().pimm_encrypt_seeded(plan.h, sk.h, _seed(seed), _seed(a_seed), op_id, _ptr(pt),
                                     _ptr(ct), _ptr(ws), ws.numel() * 8, _stream(stream)))
    return ct


def ct_expand(plan: Plan, a_seed: bytes, op_id: int, c0: torch.Tensor, ct=None, stream=None):
    """pimm_ct_expand: the server rebuilds [I][2][L][N] from c0 [I][L][N] and a_seed."""
    f, c = plan.info, plan.ctx
    assert c0.dtype == torch.int64 and tuple(c0.shape) == (f.I, c.L, c.N) and c0.is_contiguous()
    if ct is None:
        ct = torch.empty((f.I, 2, c.L, c.N), dtype=torch.int64, device=c.device)
    _check(lib().pimm_ct_expand(plan.h, _seed(a_seed), op_id, _ptr(c0), _ptr(ct), _stream(stream)))
    return ct


def fc_complete(plan: Plan, w: Weights, x1: torch.Tensor, bias, share1: torch.Tensor, ws=None,
                stream=None):
    """pimm_fc_complete: share1 += x1 W + bias (mod 2^l), in place.  -> share1."""
    f = plan.info
    assert x1.dtype == torch.int64 and tuple(x1.shape) == (f.n, f.r)
    assert share1.dtype == torch.int64 and tuple(share1.shape) == (f.n, f.m)
    if bias is not None:
        assert bias.dtype == torch.int64 and tuple(bias.shape) == (f.m,)
    ws = plan.workspace() if ws is None else ws
    _check(lib().pimm_fc_complete(plan.h, w.h, _ptr(x1), _ptr(bias) if bias is not None else None,
                                  _ptr(share1), _ptr(ws), ws.numel() * 8, _stream(stream)))
    return share1


def decrypt(plan: Plan, sk: SecretKey, c1: torch.Tensor, c0s: torch.Tensor, share=None, ws=None,
            stream=None):
    f, c = plan.info, plan.ctx
    if share is None:
        share = torch.empty(plan.share_shape(), dtype=torch.int64, device=c.device)
    ws = plan.workspace() if ws is None else ws
    _check(lib().pimm_decrypt(plan.h, sk.h, _ptr(c1), _ptr(c0s), _ptr(share), _ptr(ws),
                              ws.numel() * 8, _stream(stream)))
    return share


def mod_switch(plan: Plan, w: Weights, c1: torch.Tensor, c0s: torch.Tensor, c1_out=None,
               c0s_out=None, stream=None):
    """pimm_mod_switch: the reply with its last prime dropped.
    -> (c1s [O][L-1][N], c0ss [O][L-1][mb*nb])."""
    f, c = plan.info, plan.ctx
    per = f.mb * f.nb
    assert tuple(c1.shape) == (f.O, c.L, c.N) and tuple(c0s.shape) == (f.O, c.L, per)
    if c1_out is None:
        c1_out = torch.empty((f.O, c.L - 1, c.N), dtype=torch.int64, device=c.device)
    if c0s_out is None:
        c0s_out = torch.empty((f.O, c.L - 1, per), dtype=torch.int64, device=c.device)
    _check(lib().pimm_mod_switch(plan.h, w.h, _ptr(c1), _ptr(c0s), _ptr(c1_out), _ptr(c0s_out),
                                 _stream(stream)))
    return c1_out, c0s_out


def decrypt_switched(plan: Plan, sk: SecretKey, c1s: torch.Tensor, c0ss: torch.Tensor, share=None,
                     ws=None, stream=None):
    """pimm_decrypt_switched: the client's share from a switched reply."""
    f, c = plan.info, plan.ctx
    if share is None:
        share = torch.empty(plan.share_shape(), dtype=torch.int64, device=c.device)
    ws = plan.workspace() if ws is None else ws
    _check(lib().pimm_decrypt_switched(plan.h, sk.h, _ptr(c1s), _ptr(c0ss), _ptr(share), _ptr(ws),
                                       ws.numel() * 8, _stream(stream)))
    return share


class BatchItem(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("weights", ctypes.c_void_p), ("ct", ctypes.c_void_p),
                ("acc", ctypes.c_void_p)]


PHASED, PERSISTENT = 0, 1


class Batch:
    """pimm_batch: many products of any shapes in one pass (three launches or one
    persistent launch).  items: list of (Plan, Weights, ct tensor, acc tensor)."""

    def __init__(self, items):
        self.items = list(items)  # keeps the tensors and handles alive
        arr = (BatchItem * len(items))()
        for k, (plan, w, ct, acc) in enumerate(items):
            arr[k] = BatchItem(plan.h.value, w.h.value, ct.data_ptr(), acc.data_ptr())
        self.h = ctypes.c_void_p()
        _check(lib().pimm_batch_create(arr, len(items), ctypes.byref(self.h)))
        self.ctx = items[0][0].ctx
        self._ws = None

    def query(self):
        ws, macs = ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().pimm_batch_query(self.h, ctypes.byref(ws), ctypes.byref(macs)))
        return ws.value, macs.value

    def set_schedule(self, schedule=PHASED, mac_rows=8, mac_cols=1, xcd_map=True, grid=0):
        _check(lib().pimm_batch_set_schedule(self.h, schedule, mac_rows, mac_cols,
                                             1 if xcd_map else 0, grid))
        need = self.query()[0]
        if self._ws is not None and self._ws.numel() * 8 < need:
            self._ws = None

    def get_schedule(self):
        """-> (schedule, mac_rows, mac_cols, xcd_map, grid) in force."""
        v = [ctypes.c_int() for _ in range(4)] + [ctypes.c_uint32()]
        _check(lib().pimm_batch_get_schedule(self.h, *[ctypes.byref(x) for x in v]))
        return tuple(x.value for x in v[:3]) + (bool(v[3].value), v[4].value)

    def workspace(self):
        if self._ws is None:
            self._ws = _words(self.query()[0], self.ctx.device)
        return self._ws

    def run(self, ws=None, stream=None):
        ws = self.workspace() if ws is None else ws
        _check(lib().pimm_batch_matmul(self.h, _ptr(ws), ws.numel() * 8, _stream(stream)))

    def autotune(self, reps: int = 3, stream=None) -> float:
        """Time each schedule candidate and keep the fastest.  -> best ms."""
        ws_need = max(self.query()[0], 1)
        ws = _words(ws_need * 2, self.ctx.device)
        best = ctypes.c_double()
        _check(lib().pimm_batch_autotune(self.h, _ptr(ws), ws.numel() * 8, reps, _stream(stream),
                                         ctypes.byref(best)))
        self._ws = None
        return best.value

    def status(self, ws=None, stream=None):
        ws = self.workspace() if ws is None else ws
        _check(lib().pimm_batch_status(self.h, _ptr(ws), _stream(stream)))

    def close(self):
        if self.h:
            lib().pimm_batch_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ServeConfig(ctypes.Structure):
    _fields_ = [("layers", ctypes.c_uint32), ("ops", ctypes.c_uint32),
                ("d_in", ctypes.POINTER(ctypes.c_uint32)), ("d_out", ctypes.POINTER(ctypes.c_uint32)),
                ("weights", ctypes.POINTER(ctypes.c_void_p)), ("d_fix", ctypes.c_uint32),
                ("hbm_budget", ctypes.c_uint64), ("max_active", ctypes.c_uint32),
                ("schedule", ctypes.c_int32), ("mac_rows", ctypes.c_uint32),
                ("mac_cols", ctypes.c_uint32), ("min_batch", ctypes.c_uint32)]


class Request(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("seq", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("arrival_s", ctypes.c_double), ("client_seed", ctypes.c_uint8 * 32),
                ("server_seed", ctypes.c_uint8 * 32)]


class RequestResult(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("arrival_s", ctypes.c_double),
                ("admit_s", ctypes.c_double), ("done_s", ctypes.c_double),
                ("pair_checksum", ctypes.c_uint64), ("sum_checksum", ctypes.c_uint64),
                ("useful_macs", ctypes.c_uint64), ("steps", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class Server:
    """pimm_server: replays request traces with continuous batching.
    shapes: [(d_in, d_out)] per op; weights: [layers * ops] Weights made with block area d_fix."""

    def __init__(self, ctx: Context, layers: int, shapes, weights, d_fix: int, hbm_budget: int,
                 max_active: int, schedule: int = PHASED, mac_rows: int = 8, mac_cols: int = 1,
                 min_batch: int = 0):
        self.ctx, self.weights = ctx, list(weights)
        ops = len(shapes)
        self._d_in = (ctypes.c_uint32 * ops)(*[r for r, _ in shapes])
        self._d_out = (ctypes.c_uint32 * ops)(*[m for _, m in shapes])
        self._w = (ctypes.c_void_p * len(self.weights))(*[w.h.value for w in self.weights])
        cfg = ServeConfig(layers, ops, self._d_in, self._d_out, self._w, d_fix, int(hbm_budget),
                          max_active, schedule, mac_rows, mac_cols, min_batch)
        self.h = ctypes.c_void_p()
        _check(lib().pimm_serve_create(ctx.h, ctypes.byref(cfg), ctypes.byref(self.h)))

    def footprint(self, seq: int) -> int:
        b = ctypes.c_uint64()
        _check(lib().pimm_serve_footprint(self.h, seq, ctypes.byref(b)))
        return b.value

    def run(self, requests, stream=None):
        """requests: [(id, seq, arrival_s, client_seed, server_seed)] -> list of result dicts."""
        arr = (Request * len(requests))()
        for k, (rid, seq, t, cs, ss) in enumerate(requests):
            arr[k].id, arr[k].seq, arr[k].arrival_s = rid, seq, t
            arr[k].client_seed[:] = list(cs)
            arr[k].server_seed[:] = list(ss)
        res = (RequestResult * len(requests))()
        _check(lib().pimm_serve_run(self.h, arr, len(requests), res, _stream(stream)))
        return [{k: getattr(r, k) for k, _ in RequestResult._fields_ if k != "reserved"}
                for r in res]

    def close(self):
        if self.h:
            lib().pimm_serve_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def poly_mul(ctx: Context, a: torch.Tensor, b: torch.Tensor, stream=None):
    """c = a * b mod (X^N + 1, q_l) for [count][L][N] residue tensors."""
    count = a.shape[0]
    c = torch.empty_like(a)
    ws = _words(lib().pimm_poly_mul_workspace(ctx.h, count), ctx.device)
    _check(lib().pimm_poly_mul(ctx.h, _ptr(a), _ptr(b), _ptr(c), count, _ptr(ws), ws.numel() * 8,
                               _stream(stream)))
    return c, ws


def sample_poly(ctx: Context, kind: int, seed: bytes, tag: int, prime: int, op_id: int, obj: int,
                stream=None):
    out = torch.empty(ctx.N, dtype=torch.int64, device=ctx.device)
    _check(lib().pimm_sample_poly(ctx.h, kind, _seed(seed), tag, prime, op_id, obj, _ptr(out),
                                  _stream(stream)))
    return out


def profile_enable(on: bool = True):
    _check(lib().pimm_profile_enable(1 if on else 0))


def profile_select(classes=None):
    """Record only these kernel classes (an iterable of names; None: every class)."""
    _check(lib().pimm_profile_select(",".join(classes).encode() if classes else None))


def profile_read(kernel: str):
    """-> (launches, total milliseconds) of one kernel class since the last read."""
    cnt, ms = ctypes.c_uint64(), ctypes.c_double()
    _check(lib().pimm_profile_read(kernel.encode(), ctypes.byref(cnt), ctypes.byref(ms)))
    return cnt.value, ms.value


def sync(stream=None):
    _check(lib().pimm_sync(_stream(stream)))


def probe(kind: int, size: int, reps: int = 5, device: int = 0) -> float:
    """Sustained device rate of one probe kind (PROBE_*): bytes/s, flop/s or products/s."""
    rate = ctypes.c_double()
    _check(lib().pimm_probe(device, kind, size, reps, ctypes.byref(rate)))
    return rate.value


class Party:
    """Both parties of one Pi_MatMul call in one process (the wire is device memory):
    the client's key and the server's weight cache for a plan."""

    def __init__(self, ctx: Context, plan: Plan, W: torch.Tensor, client_seed: bytes,
                 keys=None):
        self.ctx, self.plan = ctx, plan
        self.sk, self.pk = keys if keys is not None else keygen(ctx, client_seed)
        self.weights = Weights(plan, W)
        self.client_seed = client_seed

    def run(self, X: torch.Tensor, server_seed: bytes, op_id: int = 0, stream=None):
        """The whole protocol for Y = X W: -> (client_share, server_share), both [n][m]."""
        p = self.plan
        pt = encode_input(p, X, stream=stream)
        ct = encrypt(p, self.sk, self.client_seed, op_id, pt, stream=stream)
        acc = matmul(p, self.weights, ct, stream=stream)
        c1, c0s, y1 = mask_share(p, self.pk, server_seed, op_id, acc, stream=stream)
        y0 = decrypt(p, self.sk, c1, c0s, stream=stream)
        return y0, y1
